// Normal operator on the 2-D frequency grid with bfloat16 storage: maps
// (storage kind 1), or maps and the row-transformed coil planes (kind 2).
#include "grid2d_normal.h"

namespace pico {

hipError_t launch_grid_normal_bf16(int mode, const Grid2dArgs& a, hipStream_t s) {
  if (a.Tb) return grid_normal<2>(mode, a, s);
  return grid_normal<1>(mode, a, s);
}

}  // namespace pico
