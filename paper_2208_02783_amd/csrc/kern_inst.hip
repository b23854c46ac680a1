// One (stencil radius, positions per thread) instance of the solver and apply
// kernels; compiled once per pair so the instances build in parallel.
#include "rst_precond.hpp"

#if !defined(RST_RAD) || !defined(RST_Q)
#error "RST_RAD and RST_Q must be defined"
#endif

#define RST_CAT2(a, b) a##b
#define RST_CAT(a, b) RST_CAT2(a, b)
#define RST_KPTR RST_CAT(RST_CAT(RST_CAT(rst_kptr_r, RST_RAD), _q), RST_Q)

extern "C" __attribute__((visibility("hidden"))) void* RST_KPTR(int which) {
  if (which == 0) return (void*)rst::k_bicgstab<RST_RAD, RST_Q, double>;
  if (which == 2) return (void*)rst::k_bicgstab_pc<RST_RAD, RST_Q, double>;
  return (void*)rst::k_apply<RST_RAD, RST_Q, double>;
}
