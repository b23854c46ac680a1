// One (stencil radius, positions per thread) instance of the solver and apply
// kernels; compiled once per pair so the instances build in parallel.
#include "rst_mixed.hpp"

#if !defined(RST_RAD) || !defined(RST_Q) || !defined(RST_KIND)
#error "RST_RAD, RST_Q and RST_KIND must be defined"
#endif

#define RST_CAT2(a, b) a##b
#define RST_CAT(a, b) RST_CAT2(a, b)
#define RST_KPTR RST_CAT(RST_CAT(RST_CAT(RST_CAT(RST_CAT(rst_kptr_k, RST_KIND), _r), RST_RAD), _q), RST_Q)

// RST_KIND: 0 plain solver, 1 apply, 2 preconditioned solver,
//           3 mixed-precision plain solver, 4 mixed-precision preconditioned solver,
//           5 batched plain solver, 6 batched preconditioned solver,
//           7 stand-alone preconditioner apply (blocked vectors)
extern "C" __attribute__((visibility("hidden"))) void* RST_KPTR() {
#if RST_KIND == 0
  return (void*)rst::k_bicgstab<RST_RAD, RST_Q, double, false>;
#elif RST_KIND == 1
  return (void*)rst::k_apply<RST_RAD, RST_Q, double>;
#elif RST_KIND == 2
  return (void*)rst::k_bicgstab_pc<RST_RAD, RST_Q, double, false>;
#elif RST_KIND == 3
  return (void*)rst::k_mixed<RST_RAD, RST_Q, false>;
#elif RST_KIND == 4
  return (void*)rst::k_mixed<RST_RAD, RST_Q, true>;
#elif RST_KIND == 5
  return (void*)rst::k_bicgstab<RST_RAD, RST_Q, double, true>;
#elif RST_KIND == 6
  return (void*)rst::k_bicgstab_pc<RST_RAD, RST_Q, double, true>;
#else
  return (void*)rst::k_pc_apply<RST_Q>;
#endif
}
