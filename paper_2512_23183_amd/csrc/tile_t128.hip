// Tile-pass kernel with 128 threads per workgroup.
#include "tile_kernel.h"

namespace sv {
SV_TILE_INSTANTIATE(128)
}  // namespace sv
