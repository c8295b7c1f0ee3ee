// Tile-pass kernel with 512 threads per workgroup.
#include "tile_kernel.h"

namespace sv {
SV_TILE_INSTANTIATE(512)
}  // namespace sv
