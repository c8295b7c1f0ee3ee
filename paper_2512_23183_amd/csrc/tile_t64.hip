// Tile-pass kernel with 64 threads per workgroup.
#include "tile_kernel.h"

namespace sv {
SV_TILE_INSTANTIATE(64)
}  // namespace sv
