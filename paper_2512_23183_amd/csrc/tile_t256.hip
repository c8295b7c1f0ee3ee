// Tile-pass kernel with 256 threads per workgroup.
#include "tile_kernel.h"

namespace sv {
SV_TILE_INSTANTIATE(256)
}  // namespace sv
