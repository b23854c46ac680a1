// rst_cocg2.hpp -- COCG on the doubled, complex symmetric system of a Bloch
// vector k and its opposite -k, over blocks of column pairs, one kernel per step.
//
// A_k = E - H_k + i Gamma is not complex symmetric for a general k, but
// A_k^T = A_-k (real V and projectors, real diagonal Gamma; the Bloch-form
// equation, paper Sec. II.B-II.D: the doubled operator built from the k and -k
// blocks restores the symmetry), so
//     B = [[0, A_k], [A_-k, 0]]
// is complex symmetric, and B (y1, y2) = (b1, b2) solves A_k y2 = b1 and
// A_-k y1 = b2 together.  COCG (van der Vorst and Melissen, IEEE Trans. Magn. 26,
// 1990) runs on B with the symmetric preconditioner K = [[0, M_k], [M_-k, 0]]^-1,
// K (r1, r2) = (M_-k^-1 r2, M_k^-1 r1), with the unconjugated bilinear form
// u^T v.  A pair j of a block of 2m columns is column j (first halves, y1, r1,
// ...) and column m + j (second halves).  The operator and the preconditioner
// are applied to the whole block at once with per-column flags (an A_-k or
// M_-k column runs conjugated: A_-k x = conj((E - H_k - i Gamma) conj(x)))
// and give the halves swapped: Q = apply(p) holds A_-k p1 in column j and
// A_k p2 in column m + j, so q = (B p) = (Q[m + j], Q[j]); likewise the
// preconditioner.  The kernels below read the swapped partner where the
// recurrence needs q or z.  Per-pair scalars live in CdSt; reductions are
// per-(row range, column) partial sums, each pair summed by one wavefront.
#pragma once
#include <hip/hip_runtime.h>

#include "rst_mk.hpp"

namespace rst {
namespace cd {

using mk::Shape;
using mk::c_add;
using mk::c_sub;
using mk::c_mul;
using mk::c_div;
using mk::c_finite;

struct CdSt {
  double2 rho;    // r^T z
  double2 alpha, beta;
  double bb;      // ||b1||^2 + ||b2||^2
  double rr, rrmin;
  int its, restarts, check, brk, done;
};

enum CdStep { CD_INIT = 0, CD_RHO = 1, CD_ALPHA = 2, CD_CONV = 3, CD_BETA = 4, CD_RESTART = 5 };

__device__ __forceinline__ double2 c_dotu(double2 a, double2 b) {  // a * b (no conjugation)
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Rows of a block: grid (ld/64, nsplit), four waves striding the rows of the range.
#define RST_CD_ROWS                                                        \
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;                \
  const int c = blockIdx.x * 64 + lane;                                    \
  const long long r0 = (long long)blockIdx.y * S.rows;                     \
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;

// X = P = 0, R = b (both halves from the right-hand-side description); partial ||R||^2.
__global__ __launch_bounds__(256) void k_cd_init(Shape S, mk::Rhs B, double2* X, double2* R, double2* Pv,
                                                 double2* part) {
  RST_CD_ROWS
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t o = (size_t)gi * S.ld + c;
    const double2 b = mk::rhs_at(B, gi, c);
    X[o] = make_double2(0.0, 0.0);
    Pv[o] = make_double2(0.0, 0.0);
    R[o] = b;
    acc[0].x += b.x * b.x + b.y * b.y;
  }
  mk::store_partials<1>(S, acc, part);
}

// Partial bilinear products U^T V of each column with V's column (swapped: the
// partner column m + j <-> j); the pair's value is the sum of its two columns.
__global__ __launch_bounds__(256) void k_cd_dot(Shape S, int m, const int* act, const double2* U, const double2* V,
                                                int swap, double2* part) {
  RST_CD_ROWS
  const int cv = swap ? (c < m ? c + m : c - m) : c;
  double2 acc[1] = {make_double2(0.0, 0.0)};
  if (act[c]) {
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const size_t row = (size_t)gi * S.ld;
      acc[0] = c_add(acc[0], c_dotu(U[row + c], V[row + cv]));
    }
  }
  mk::store_partials<1>(S, acc, part);
}

// X += alpha P;  R -= alpha q with q = Q swapped;  partial ||R||^2.
__global__ __launch_bounds__(256) void k_cd_xr(Shape S, int m, const CdSt* st, const int* act, double2* X, double2* R,
                                               const double2* Pv, const double2* Q, double2* part) {
  RST_CD_ROWS
  const int j = c < m ? c : c - m;
  const int cq = c < m ? c + m : c - m;
  double2 acc[1] = {make_double2(0.0, 0.0)};
  if (act[c]) {
    const double2 al = st[j].alpha;
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const size_t row = (size_t)gi * S.ld;
      X[row + c] = c_add(X[row + c], c_mul(al, Pv[row + c]));
      const double2 r = c_sub(R[row + c], c_mul(al, Q[row + cq]));
      R[row + c] = r;
      acc[0].x += r.x * r.x + r.y * r.y;
    }
  }
  mk::store_partials<1>(S, acc, part);
}

// P = z + beta P with z = Z (swapped when the preconditioner produced it); beta = 0
// (first step, restart) gives P = z.
__global__ __launch_bounds__(256) void k_cd_p(Shape S, int m, const CdSt* st, const int* act, double2* Pv,
                                              const double2* Z, int swap) {
  RST_CD_ROWS
  const int j = c < m ? c : c - m;
  if (!act[c]) return;
  const int cz = swap ? (c < m ? c + m : c - m) : c;
  const double2 be = st[j].beta;
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t row = (size_t)gi * S.ld;
    Pv[row + c] = c_add(Z[row + cz], c_mul(be, Pv[row + c]));
  }
}

// True residual of the marked pairs: R = b - q, q = Q swapped (Q = apply(X)); partial ||R||^2.
__global__ __launch_bounds__(256) void k_cd_resid(Shape S, int m, mk::Rhs B, const int* mark, const double2* Q,
                                                  double2* R, double2* part) {
  RST_CD_ROWS
  const int cq = c < m ? c + m : c - m;
  double2 acc[1] = {make_double2(0.0, 0.0)};
  if (mark[c]) {
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const size_t row = (size_t)gi * S.ld;
      const double2 r = c_sub(mk::rhs_at(B, gi, c), Q[row + cq]);
      R[row + c] = r;
      acc[0].x += r.x * r.x + r.y * r.y;
    }
  }
  mk::store_partials<1>(S, acc, part);
}

// Pair sum of a one-product partial array: columns j and m + j.
__device__ __forceinline__ double2 pair_sum(const Shape& S, const double2* part, int j, int m) {
  const double2 a = mk::sum_part_wave(S, part, 0, j);
  const double2 b = mk::sum_part_wave(S, part, 0, j + m);
  return c_add(a, b);
}

// Per-pair scalar work, one wavefront per pair (its first lane updates the state);
// act and mark are per column, equal on the two columns j and m + j of a pair.
//  CD_INIT   : bb = ||b||^2; its = restarts = 0; pairs with b = 0 are done.
//  CD_RHO    : rho = r^T z (start or restart: beta = 0 so that p = z).
//  CD_ALPHA  : alpha = rho / p^T q; a vanishing or non-finite p^T q is a breakdown.
//  CD_CONV   : rr = ||r||^2; its += 1; stop at the tolerance (true residual check), at
//              max_iter, or on a non-finite rr or a 1e5-fold growth over the smallest.
//  CD_BETA   : rho' = r^T z, beta = rho'/rho, rho = rho'; a vanishing rho is a breakdown.
//  CD_RESTART: marked pairs: rr = ||r||^2 of the true residual now in R.
__global__ __launch_bounds__(64) void k_cd_scalar(Shape S, int m, int step, CdSt* st, int* act, const int* mark,
                                                  const double2* part, double tol, int max_iter) {
  const int j = blockIdx.x;
  if (step == CD_RESTART) {
    if (!mark[j]) return;
  } else if (step != CD_INIT && !act[j]) {
    return;
  }
  auto set_act = [&](int a) {
    act[j] = a;
    act[j + m] = a;
  };
  const double2 v = pair_sum(S, part, j, m);
  if (threadIdx.x != 0) return;
  CdSt& q = st[j];
  if (step == CD_INIT) {
    q.bb = v.x;
    q.its = q.restarts = q.check = q.brk = 0;
    q.rr = q.rrmin = v.x;
    set_act(v.x > 0.0 ? 1 : 0);
    q.done = v.x > 0.0 ? 0 : 1;
  } else if (step == CD_RESTART) {
    q.rr = q.rrmin = v.x;
  } else if (step == CD_RHO) {
    q.rho = v;
    q.beta = make_double2(0.0, 0.0);
    if ((v.x == 0.0 && v.y == 0.0) || !c_finite(v)) {
      q.brk = 1;
      set_act(0);
    }
  } else if (step == CD_ALPHA) {
    const double2 al = c_div(q.rho, v);
    if ((v.x == 0.0 && v.y == 0.0) || !c_finite(al)) {
      q.alpha = make_double2(0.0, 0.0);
      q.its += 1;  // counted, so that repeated breakdowns end at max_iter
      q.brk = 1;
      set_act(0);
      return;
    }
    q.alpha = al;
  } else if (step == CD_CONV) {
    q.its += 1;
    q.rr = v.x;
    q.rrmin = fmin(q.rrmin, v.x);
    if (!isfinite(v.x) || v.x > 1e10 * q.rrmin) {
      q.brk = 1;
      set_act(0);
    } else if (v.x <= tol * tol * q.bb || q.its >= max_iter) {
      q.check = 1;
      set_act(0);
    }
  } else if (step == CD_BETA) {
    const double rh2 = v.x * v.x + v.y * v.y;
    if (rh2 <= 1e-60 * q.bb * q.bb || !c_finite(v)) {
      q.brk = 1;
      set_act(0);
      return;
    }
    q.beta = c_div(v, q.rho);
    q.rho = v;
  }
}

#undef RST_CD_ROWS

}  // namespace cd
}  // namespace rst
