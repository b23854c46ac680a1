// rst_idr.hpp -- IDR(s) with biorthogonalisation over a block of columns, one
// kernel per step, for lateral planes of any size.
//
// Induced dimension reduction (Sonneveld and van Gijzen, SIAM J. Sci. Comput. 31,
// 2008; the biorthogonal variant of van Gijzen and Sonneveld, ACM TOMS 38, 2011),
// right-preconditioned by the free-electron + CAP operator M, on A x = b with
// A = E - H_k + i Gamma (the retarded Green's function of the transmission
// equation, paper Sec. II.A).  Per column, with an s-dimensional shadow space
// P (shared by all columns: n x s, random complex):
//   f = P^H r;  for k = 0..s-1:
//     c = M[k:s, k:s]^-1 f[k:s]                        (lower triangular)
//     v = r - sum_{i>=k} c_i g_i;  u_k = sum_{i>=k} c_i u_i + omega M^-1 v;  g_k = A u_k
//     alpha = M[0:k, 0:k]^-1 (P^H g_k)[0:k];  g_k -= sum_{i<k} alpha_i g_i;  u_k -= sum_{i<k} alpha_i u_i
//     M[j][k] = P_j^H g_k (j >= k);  beta = f_k / M[k][k];  r -= beta g_k;  x += beta u_k;
//     f[j] -= beta M[j][k] (j > k)
//   v = M^-1 r;  t = A v;  omega = (t, r)/(t, t), enlarged to |rho| = 0.7 when the
//   angle rho = (t, r)/(|t||r|) is smaller;  r -= omega t;  x += omega v
// (s + 1 operator applies per cycle).  The biorthogonalisation coefficients and
// the new column of M come from one pass of dot products with P (the s products
// of g_k before its update; M[j][k] then follows from the old M column entries).
// Vectors use the column-fastest layout of the many-column BiCGSTAB (rst_mk.hpp),
// g_i and u_i at G + i*vlen, U + i*vlen.  Per-column scalars and the small s x s
// systems live in IdrSt, one thread per column; reductions are partial sums over
// row ranges summed in a fixed order (deterministic for a given launch shape).
#pragma once
#include <hip/hip_runtime.h>

#include "rst_mk.hpp"

namespace rst {
namespace idr {

using mk::Shape;
using mk::c_add;
using mk::c_sub;
using mk::c_mul;
using mk::c_mulc;
using mk::c_div;
using mk::c_finite;
using mk::vld;
using mk::vst;

constexpr int SMAX = 8;

struct IdrSt {
  double2 M[SMAX][SMAX];  // M[j][i] = P_j^H g_i (lower triangular)
  double2 f[SMAX];        // P^H r (entries k.. are current during a cycle)
  double2 c[SMAX];        // coefficients of the current step (entries k..s-1)
  double2 al[SMAX];       // biorthogonalisation coefficients (entries 0..k-1)
  double2 omega, beta;
  double bb, rr, rrmin;
  int check, brk, its, restarts, done;
};

enum IdrStep { ID_INIT = 0, ID_C = 1, ID_D = 2, ID_CONV = 3, ID_OMEGA = 4, ID_END = 5, ID_RESTART = 6 };

// Partials of the s products (P_j, y) (conj(P_j) y) for j < s, stored as products
// 1..s of the partial array (product 0 is left to the caller); with NORM also
// ||y||^2 as product 0.
template <bool NORM, class VT = double2>
__global__ __launch_bounds__(256) void k_idr_pdots(Shape S, int s, const int* act, const double2* Pm,
                                                   const VT* Y, double2* part) {
  __shared__ double2 red[SMAX + 1][4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  double2 acc[SMAX + 1];
#pragma unroll
  for (int d = 0; d <= SMAX; ++d) acc[d] = make_double2(0.0, 0.0);
  if (act == nullptr || act[c]) {
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const double2 y = vld(Y, (size_t)gi * S.ld + c);
      if (NORM) acc[0].x += y.x * y.x + y.y * y.y;
#pragma unroll
      for (int j = 0; j < SMAX; ++j)
        if (j < s) acc[1 + j] = c_add(acc[1 + j], c_mulc(Pm[(size_t)gi * s + j], y));
    }
  }
#pragma unroll
  for (int d = 0; d <= SMAX; ++d) red[d][wv][lane] = acc[d];
  __syncthreads();
  if (wv == 0) {
    for (int d = NORM ? 0 : 1; d <= s; ++d) {
      double2 t = red[d][0][lane];
      t = c_add(t, red[d][1][lane]);
      t = c_add(t, red[d][2][lane]);
      t = c_add(t, red[d][3][lane]);
      part[((size_t)d * S.nsplit + blockIdx.y) * S.ld + c] = t;
    }
  }
}

// X = 0, R = b; G_i = U_i = 0 (all columns).
template <class VT = double2>
__global__ __launch_bounds__(256) void k_idr_init(Shape S, int s, mk::Rhs B, VT* X, VT* R, VT* G, VT* U) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long vlen = S.n * S.ld;
  if (t >= vlen) return;
  const int c = (int)(t % S.ld);
  const long long gi = t / S.ld;
  const double2 z = make_double2(0.0, 0.0);
  vst(X, t, z);
  vst(R, t, mk::rhs_at(B, gi, c));
  for (int i = 0; i < s; ++i) {
    vst(G, i * vlen + t, z);
    vst(U, i * vlen + t, z);
  }
}

// G_i = U_i = 0 for the marked columns (restart).
template <class VT = double2>
__global__ __launch_bounds__(256) void k_idr_zero(Shape S, int s, const int* mark, VT* G, VT* U) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long vlen = S.n * S.ld;
  if (t >= vlen) return;
  if (!mark[(int)(t % S.ld)]) return;
  for (int i = 0; i < s; ++i) {
    vst(G, i * vlen + t, make_double2(0.0, 0.0));
    vst(U, i * vlen + t, make_double2(0.0, 0.0));
  }
}

// The vector updates below run over a block's row range (grid (ld/64, nsplit),
// four waves striding the rows) with each column's coefficients loaded once into
// registers; columns that are not iterating are left untouched.

// V = R - sum_{i=k}^{s-1} c_i G_i.
template <class VT = double2>
__global__ __launch_bounds__(256) void k_idr_v(Shape S, int s, int k, const IdrSt* st, const int* act, const VT* R,
                                               const VT* G, VT* V) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  if (!act[c]) return;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  const long long vlen = S.n * S.ld;
  double2 cf[SMAX];
#pragma unroll
  for (int i = 0; i < SMAX; ++i) cf[i] = i >= k && i < s ? st[c].c[i] : make_double2(0.0, 0.0);
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t o = (size_t)gi * S.ld + c;
    double2 v = vld(R, o);
#pragma unroll
    for (int i = 0; i < SMAX; ++i)
      if (i >= k && i < s) v = c_sub(v, c_mul(cf[i], vld(G, i * vlen + o)));
    vst(V, o, v);
  }
}

// U_k = sum_{i=k}^{s-1} c_i U_i + omega VH.
template <class VT = double2>
__global__ __launch_bounds__(256) void k_idr_u(Shape S, int s, int k, const IdrSt* st, const int* act, const VT* VH,
                                               VT* U) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  if (!act[c]) return;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  const long long vlen = S.n * S.ld;
  double2 cf[SMAX];
#pragma unroll
  for (int i = 0; i < SMAX; ++i) cf[i] = i >= k && i < s ? st[c].c[i] : make_double2(0.0, 0.0);
  const double2 om = st[c].omega;
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t o = (size_t)gi * S.ld + c;
    double2 u = c_mul(om, vld(VH, o));
#pragma unroll
    for (int i = 0; i < SMAX; ++i)
      if (i >= k && i < s) u = c_add(u, c_mul(cf[i], vld(U, i * vlen + o)));
    vst(U, k * vlen + o, u);
  }
}

// G_k -= sum_{i<k} alpha_i G_i;  U_k -= sum_{i<k} alpha_i U_i;  R -= beta G_k;  X += beta U_k;
// partial ||R||^2 (product 0).
template <class VT = double2>
__global__ __launch_bounds__(256) void k_idr_upd(Shape S, int k, const IdrSt* st, const int* act, VT* G, VT* U, VT* R,
                                                 VT* X, double2* part) {
  __shared__ double2 red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  const long long vlen = S.n * S.ld;
  double rr = 0.0;
  if (act[c]) {
    const IdrSt& q = st[c];
    const double2 be = q.beta;
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const size_t o = (size_t)gi * S.ld + c;
      double2 g = vld(G, k * vlen + o), u = vld(U, k * vlen + o);
      for (int i = 0; i < k; ++i) {
        g = c_sub(g, c_mul(q.al[i], vld(G, i * vlen + o)));
        u = c_sub(u, c_mul(q.al[i], vld(U, i * vlen + o)));
      }
      vst(G, k * vlen + o, g);
      vst(U, k * vlen + o, u);
      const double2 r = c_sub(vld(R, o), c_mul(be, g));
      vst(R, o, r);
      vst(X, o, c_add(vld(X, o), c_mul(be, u)));
      rr += r.x * r.x + r.y * r.y;
    }
  }
  red[wv][lane] = make_double2(rr, 0.0);
  __syncthreads();
  if (wv == 0) {
    double2 t = red[0][lane];
    t = c_add(t, red[1][lane]);
    t = c_add(t, red[2][lane]);
    t = c_add(t, red[3][lane]);
    part[(size_t)blockIdx.y * S.ld + c] = t;
  }
}

// R -= omega T;  X += omega VH  (dimension-reduction step), with the partials of
// ||R||^2 (product 0) and P^H R (products 1..s) of the new residual, as k_idr_pdots<true>.
template <class VT = double2>
__global__ __launch_bounds__(256) void k_idr_rx(Shape S, int s, const IdrSt* st, const int* act, VT* R, VT* X,
                                                const VT* T, const VT* VH, const double2* Pm, double2* part) {
  __shared__ double2 red[SMAX + 1][4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  double2 acc[SMAX + 1];
#pragma unroll
  for (int d = 0; d <= SMAX; ++d) acc[d] = make_double2(0.0, 0.0);
  if (act[c]) {
    const double2 om = st[c].omega;
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const size_t o = (size_t)gi * S.ld + c;
      const double2 vh = vld(VH, o);  // read before R is written: VH may be R itself (no preconditioner)
      const double2 r = c_sub(vld(R, o), c_mul(om, vld(T, o)));
      vst(R, o, r);
      vst(X, o, c_add(vld(X, o), c_mul(om, vh)));
      acc[0].x += r.x * r.x + r.y * r.y;
#pragma unroll
      for (int j = 0; j < SMAX; ++j)
        if (j < s) acc[1 + j] = c_add(acc[1 + j], c_mulc(Pm[(size_t)gi * s + j], r));
    }
  }
#pragma unroll
  for (int d = 0; d <= SMAX; ++d) red[d][wv][lane] = acc[d];
  __syncthreads();
  if (wv == 0) {
    for (int d = 0; d <= s; ++d) {
      double2 t = red[d][0][lane];
      t = c_add(t, red[d][1][lane]);
      t = c_add(t, red[d][2][lane]);
      t = c_add(t, red[d][3][lane]);
      part[((size_t)d * S.nsplit + blockIdx.y) * S.ld + c] = t;
    }
  }
}

// Per-column scalar work after each reduction; one wavefront per column sums the
// partials, its first lane updates the state.
//  ID_INIT   : bb = ||b||^2 (product 0), f = P^H b (products 1..s), M = I, omega = 1.
//  ID_RESTART: for the marked columns, rr = ||r||^2, f = P^H r, M = I, omega = 1 (the true
//              residual is already in R).
//  ID_C      : c[k..s-1] = M[k:s, k:s]^-1 f[k:s] (forward substitution).
//  ID_D      : d = P^H g_k (products 1..s): alpha = M[0:k,0:k]^-1 d[0:k]; M[j][k] = d_j -
//              sum_{i<k} alpha_i M[j][i] (j >= k); beta = f_k / M[k][k]; f[j] -= beta M[j][k] (j > k).
//              A vanishing or non-finite M[k][k] is a breakdown.
//  ID_CONV   : rr = ||r||^2 after the step (product 0); its += 1; stop at the tolerance (true
//              residual check), at max_iter, on a non-finite rr or a 1e5-fold growth over the
//              smallest rr since the last restart.
//  ID_OMEGA  : omega = (t, r)/(t, t) from products 0 and 1, enlarged to an angle of 0.7.
//  ID_END    : as ID_CONV with f = P^H r (products 1..s).
// cap (nullable): per-column iteration limits in place of max_iter.
__global__ __launch_bounds__(64) void k_idr_scalar(Shape S, int step, int s, int k, IdrSt* st, int* act,
                                                   const int* mark, const double2* part, double tol, int max_iter,
                                                   const int* cap) {
  const int c = blockIdx.x;
  if (cap != nullptr) max_iter = cap[c];  // per-column iteration budget (inner solves of the refinement)
  if (step == ID_RESTART) {
    if (!mark[c]) return;
  } else if (step != ID_INIT && !act[c]) {
    return;
  }
  const int np = step == ID_C ? 0 : step == ID_CONV ? 1 : step == ID_OMEGA ? 2 : s + 1;
  double2 v[SMAX + 1];
  for (int d = 0; d <= SMAX; ++d) v[d] = make_double2(0.0, 0.0);
  for (int d = 0; d < np; ++d) {
    if (step == ID_D && d == 0) continue;  // no norm product in this pass
    v[d] = mk::sum_part_wave(S, part, d, c);
  }
  if (threadIdx.x != 0) return;
  IdrSt& q = st[c];
  auto reset = [&](double rr) {
    for (int j = 0; j < SMAX; ++j)
      for (int i = 0; i < SMAX; ++i) q.M[j][i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    for (int j = 0; j < s; ++j) q.f[j] = v[1 + j];
    q.omega = make_double2(1.0, 0.0);
    q.rr = rr;
    q.rrmin = rr;
  };
  auto conv = [&](double rr) {
    q.its += 1;
    q.rr = rr;
    q.rrmin = fmin(q.rrmin, rr);
    if (!isfinite(rr) || rr > 1e10 * q.rrmin) {
      q.brk = 1;
      act[c] = 0;
    } else if (rr <= tol * tol * q.bb || q.its >= max_iter) {
      q.check = 1;
      act[c] = 0;
    }
  };
  if (step == ID_INIT) {
    q.bb = v[0].x;
    q.check = q.brk = q.its = q.restarts = 0;
    reset(q.bb);
    act[c] = q.bb > 0.0 ? 1 : 0;
    q.done = q.bb > 0.0 ? 0 : 1;
  } else if (step == ID_RESTART) {
    reset(v[0].x);
  } else if (step == ID_C) {
    for (int j = k; j < s; ++j) {
      double2 t = q.f[j];
      for (int i = k; i < j; ++i) t = c_sub(t, c_mul(q.M[j][i], q.c[i]));
      q.c[j] = c_div(t, q.M[j][j]);
    }
  } else if (step == ID_D) {
    for (int i = 0; i < k; ++i) {
      double2 t = v[1 + i];
      for (int i2 = 0; i2 < i; ++i2) t = c_sub(t, c_mul(q.M[i][i2], q.al[i2]));
      q.al[i] = c_div(t, q.M[i][i]);
    }
    for (int j = k; j < s; ++j) {
      double2 t = v[1 + j];
      for (int i = 0; i < k; ++i) t = c_sub(t, c_mul(q.al[i], q.M[j][i]));
      q.M[j][k] = t;
    }
    const double2 mkk = q.M[k][k];
    const double2 be = c_div(q.f[k], mkk);
    if ((mkk.x == 0.0 && mkk.y == 0.0) || !c_finite(be)) {
      q.beta = make_double2(0.0, 0.0);
      q.its += 1;  // counted, so that repeated breakdowns end at max_iter
      q.brk = 1;
      act[c] = 0;
      return;
    }
    q.beta = be;
    for (int j = k + 1; j < s; ++j) q.f[j] = c_sub(q.f[j], c_mul(be, q.M[j][k]));
  } else if (step == ID_CONV) {
    conv(v[0].x);
  } else if (step == ID_OMEGA) {
    const double2 tr = v[0];
    const double tt = v[1].x;
    const double nr = sqrt(q.rr), nt = sqrt(tt);
    if (!(tt > 0.0)) {
      q.omega = make_double2(0.0, 0.0);
      q.brk = 1;
      act[c] = 0;
      return;
    }
    double2 om = make_double2(tr.x / tt, tr.y / tt);
    const double rho = sqrt(tr.x * tr.x + tr.y * tr.y) / (nt * nr);
    if (rho < 0.7 && rho > 0.0) om = make_double2(om.x * 0.7 / rho, om.y * 0.7 / rho);
    q.omega = c_finite(om) ? om : make_double2(0.0, 0.0);
    if (!c_finite(om) || (om.x == 0.0 && om.y == 0.0)) {
      q.brk = 1;
      act[c] = 0;
    }
  } else if (step == ID_END) {
    for (int j = 0; j < s; ++j) q.f[j] = v[1 + j];
    conv(v[0].x);
  }
}

// Normal complex shadow vectors: Pm[gi*s + j] with components N(0, 1/(2n)) from
// SplitMix64 of (seed, element) and the Box-Muller transform, so |P_j| is about 1.
__device__ __forceinline__ unsigned long long idr_mix(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

__global__ void k_idr_shadow(long long n, int s, unsigned long long seed, double2* Pm) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n * s) return;
  const unsigned long long h = idr_mix(seed ^ idr_mix((unsigned long long)j));
  const double u1 = ((double)(h >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
  const double u2 = (double)(idr_mix(h) >> 11) * (1.0 / 9007199254740992.0);
  const double rad = sqrt(-log(u1) / (double)n);  // |z|^2 ~ Exp(1)/n
  const double th = 6.283185307179586 * u2;
  Pm[j] = make_double2(rad * cos(th), rad * sin(th));
}

}  // namespace idr
}  // namespace rst
