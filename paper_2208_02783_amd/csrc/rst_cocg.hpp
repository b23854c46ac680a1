// rst_cocg.hpp -- kernels of the conjugate orthogonal conjugate gradient
// method (COCG; van der Vorst and Melissen, IEEE Trans. Magn. 26, 1990) for a
// complex symmetric A = E - H_k + i Gamma, i.e. a real H_k (every Bloch phase
// +-1, the Gamma point among them), preconditioned by the (then also complex
// symmetric) free-electron + CAP operator M:
//   r = b - A x,  z = M^-1 r,  p = z,  rho = r^T z
//   repeat:  q = A p,  alpha = rho / (p^T q),  x += alpha p,  r -= alpha q,
//            z = M^-1 r,  rho' = r^T z,  p = z + (rho' / rho) p,  rho = rho'
// with the unconjugated bilinear form u^T v.  One operator apply per step.
// Vectors use the blocked layout of the flexible-GMRES kernels (fg::Shape);
// per-column scalars live on the device; every reduction is workgroup-local in
// a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>

#include "rst_fgmres.hpp"

namespace rst {
namespace cg {

using fg::Shape;

__device__ __forceinline__ double2 cdiv2(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ bool finite2(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// out[c] = sum_p u[c,p] v[c,p] (bilinear) or conj(u[c,p]) v[c,p]; one workgroup per block.
__global__ __launch_bounds__(256) void k_cg_dot(Shape S, const double2* U, const double2* V, int conj,
                                                double2* out, int ncolp) {
  __shared__ double2 red[256];
  const int blk = blockIdx.x;
  const double2* u = U + (size_t)blk * S.n * S.cw;
  const double2* v = V + (size_t)blk * S.n * S.cw;
  const long long tot = S.n * S.cw;
  double2 acc = make_double2(0.0, 0.0);
  for (long long t = threadIdx.x; t < tot; t += blockDim.x) {
    const double2 a = u[t], b = v[t];
    const double ay = conj ? -a.y : a.y;
    acc.x += a.x * b.x - ay * b.y;
    acc.y += a.x * b.y + ay * b.x;
  }
  // thread t met column t % cw only (256 is a multiple of cw)
  const double2 s = rst::col_reduce_c(red, S.cw, acc);
  if ((int)threadIdx.x < S.cw) {
    const int c = blk * S.cw + threadIdx.x;
    if (c < ncolp) out[c] = s;
  }
}

// alpha = rho / (p^T q) for active columns (0 otherwise); brk[c] = 1 if p^T q vanished
__global__ void k_cg_alpha(int ncolp, const double2* rho, const double2* pq, const int* act, double2* alpha,
                           int* brk) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncolp) return;
  double2 a = make_double2(0.0, 0.0);
  if (act[c]) {
    const double2 d = pq[c];
    if (d.x == 0.0 && d.y == 0.0) {
      brk[c] = 1;
    } else {
      a = cdiv2(rho[c], d);
      if (!finite2(a)) {
        a = make_double2(0.0, 0.0);
        brk[c] = 1;
      }
    }
  }
  alpha[c] = a;
}

// x += alpha p, r -= alpha q
__global__ void k_cg_xr(Shape S, double2* X, double2* R, const double2* Pv, const double2* Q,
                        const double2* alpha) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int c = (int)(j / (S.n * S.cw)) * S.cw + (int)(j % S.cw);
  const double2 a = alpha[c];
  if (a.x == 0.0 && a.y == 0.0) return;
  const double2 ap = fg::cmul_(a, Pv[j]), aq = fg::cmul_(a, Q[j]);
  X[j] = make_double2(X[j].x + ap.x, X[j].y + ap.y);
  R[j] = make_double2(R[j].x - aq.x, R[j].y - aq.y);
}

// beta = rho' / rho and rho = rho' for active columns (beta 0 otherwise); brk if rho vanished
__global__ void k_cg_beta(int ncolp, double2* rho, const double2* rho_new, const int* act, double2* beta,
                          int* brk) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncolp) return;
  double2 b = make_double2(0.0, 0.0);
  if (act[c]) {
    const double2 r0 = rho[c];
    if (r0.x == 0.0 && r0.y == 0.0) {
      brk[c] = 1;
    } else {
      b = cdiv2(rho_new[c], r0);
      if (!finite2(b)) {
        b = make_double2(0.0, 0.0);
        brk[c] = 1;
      }
    }
  }
  beta[c] = b;
  rho[c] = rho_new[c];
}

// p = z + beta p
__global__ void k_cg_p(Shape S, double2* Pv, const double2* Z, const double2* beta) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int c = (int)(j / (S.n * S.cw)) * S.cw + (int)(j % S.cw);
  const double2 bp = fg::cmul_(beta[c], Pv[j]);
  Pv[j] = make_double2(Z[j].x + bp.x, Z[j].y + bp.y);
}

// dst = src in the marked columns (restarts: r = b - A x, then p = z)
__global__ void k_cg_copy_marked(Shape S, double2* dst, const double2* src, const int* mark) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int c = (int)(j / (S.n * S.cw)) * S.cw + (int)(j % S.cw);
  if (mark[c]) dst[j] = src[j];
}
__global__ void k_cg_rho_set(int ncolp, double2* rho, const double2* rho_new, const int* mark) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncolp && mark[c]) rho[c] = rho_new[c];
}

}  // namespace cg
}  // namespace rst
