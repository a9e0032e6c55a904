// Line-pass kernels of one element order, HOFEM_ORDER (1..9): the build
// compiles this file once per order.
#include "linepass.h"

#ifndef HOFEM_ORDER
#error "compile with -DHOFEM_ORDER=n, n = 1..9"
#endif

namespace hofem {

template <>
hipError_t launch_pass_order<HOFEM_ORDER>(int kind, int dt, const PassArgs& a, hipStream_t s) {
  return lp::launch_order<HOFEM_ORDER>(kind, dt, a, s);
}

}  // namespace hofem
