// Separable Cartesian normal operator with bfloat16 map storage.
#include "cart1d_normal.h"

namespace pico {

hipError_t launch_cart1d_bf16(int mode, const Cart1dArgs& a, hipStream_t s) {
  return cart1d_dispatch<true>(mode, a, s);
}

}  // namespace pico
