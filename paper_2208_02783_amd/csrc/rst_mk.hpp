// rst_mk.hpp -- right-preconditioned BiCGSTAB over a block of columns with one
// kernel per step, for lateral planes of any size.
//
// Solves A x = b, A = E - H_k + i Gamma (the retarded Green's function of the
// transmission equation, paper Sec. II.A) for `ld` columns at once, each with
// its own energy and right-hand side.  Vectors are complex128 in the
// column-fastest layout of the many-column apply: element (grid point gi,
// column c) at gi*ld + c, ld a multiple of 64, so a wavefront reads or writes
// one grid point's row of 64 columns (1 KB) per access.  The operator is the
// many-column apply (k_proj_mm + k_apply_cols, per-column energies); the
// right preconditioner is the free-electron + CAP operator M (the lateral FD
// Laplacian diagonal in the twisted lateral Fourier basis of the Bloch-form
// equation, the three-point z Laplacian, the cell-mean potential and the
// z-only CAP), applied here as two lateral DFT passes along a and b, one
// tridiagonal (Thomas) solve along z per lateral mode and column, and the two
// inverse passes.  Every pass works on whole 64-column rows, so no workgroup
// needs a whole lateral plane.
//
// Iteration (van der Vorst 1992, right preconditioning; r0h the shadow residual):
//   p = r + beta (p - omega v);  ph = M^-1 p;  v = A ph;  alpha = rho / (r0h, v)
//   s = r - alpha v;  sh = M^-1 s;  t = A sh;  omega = (t, s) / (t, t)
//   x += alpha ph + omega sh;  r = s - omega t;  rho' = (r0h, r);  beta = (rho'/rho)(alpha/omega)
// with (u, v) = sum conj(u) v.  s overwrites r in place.  Reductions are
// per-column partial sums over row ranges, summed in a fixed order by the
// scalar kernels (bitwise deterministic for a given launch shape).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rst {
namespace mk {

struct Shape {
  long long n;     // grid points
  int ld;          // columns in the block (multiple of 64)
  int nsplit;      // row ranges per 64-column chunk in the reducing kernels
  long long rows;  // rows per range
};

// Right-hand side of column c: a point source bsc[c] e_{src[c]} (src < 0: none),
// or, with dense != nullptr, dense[gi*dld + doff[c]] (doff < 0: zero column).
struct Rhs {
  const long long* src;
  const double* bsc;
  const double2* dense;
  long long dld;
  const long long* doff;
};

// Per-column solver state.  Whether a column iterates is kept apart, in an int
// array `act` (1: iterating), which the apply and preconditioner kernels take as
// their column mask.
struct ColSt {
  double2 rho, alpha, omega, beta;
  double bb;      // ||b||^2
  double rr;      // recursive ||r||^2
  double r0n;     // ||r0h||^2 of the shadow residual
  double rrmin;   // smallest recursive ||r||^2 since the last (re)start
  int check;      // 1: the recursive residual met the tolerance (true residual pending)
  int brk;        // 1: breakdown, restart from the true residual pending
  int its;        // iterations
  int restarts;
  int done;       // 1: converged on the true residual; 2: iteration cap
};

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_mulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 c_div(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ bool c_finite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// Vector storage: complex128 (double2) or, for the inner solves of the mixed-precision
// refinement, complex64 (float2); arithmetic is FP64 either way.  The Krylov vectors are
// streamed once per kernel, so their loads and stores are non-temporal (the two halves of
// an element merge into one 16-byte or 8-byte access).
__device__ __forceinline__ double2 vld(const double2* p, size_t i) {
  return make_double2(__builtin_nontemporal_load(&p[i].x), __builtin_nontemporal_load(&p[i].y));
}
__device__ __forceinline__ double2 vld(const float2* p, size_t i) {
  return make_double2(__builtin_nontemporal_load(&p[i].x), __builtin_nontemporal_load(&p[i].y));
}
__device__ __forceinline__ void vst(double2* p, size_t i, double2 v) {
  __builtin_nontemporal_store(v.x, &p[i].x);
  __builtin_nontemporal_store(v.y, &p[i].y);
}
__device__ __forceinline__ void vst(float2* p, size_t i, double2 v) {
  __builtin_nontemporal_store((float)v.x, &p[i].x);
  __builtin_nontemporal_store((float)v.y, &p[i].y);
}

__device__ __forceinline__ double2 cflip(double2 a, double sg) { return make_double2(a.x, sg * a.y); }

__device__ __forceinline__ double2 rhs_at(const Rhs& B, long long gi, int c) {
  if (B.dense) {
    const long long o = B.doff[c];
    return o >= 0 ? B.dense[gi * B.dld + o] : make_double2(0.0, 0.0);
  }
  return B.src[c] == gi ? make_double2(B.bsc[c], 0.0) : make_double2(0.0, 0.0);
}

// Row loop of the reducing kernels: grid (ld/64 chunks, nsplit ranges), 256
// threads; wave w of a workgroup takes rows r0 + w, r0 + w + 4, ... of its range,
// lane l column chunk*64 + l.  Partial sums of NDOT products per column are
// reduced over the four waves in wave order and stored at
// part[(d*nsplit + range)*ld + c].
template <int NDOT>
__device__ __forceinline__ void store_partials(const Shape& S, double2 (&acc)[NDOT], double2* part) {
  __shared__ double2 red[NDOT][4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < NDOT; ++d) red[d][wv][lane] = acc[d];
  __syncthreads();
  if (wv == 0) {
    const int c = blockIdx.x * 64 + lane;
#pragma unroll
    for (int d = 0; d < NDOT; ++d) {
      double2 s = red[d][0][lane];
      s = c_add(s, red[d][1][lane]);
      s = c_add(s, red[d][2][lane]);
      s = c_add(s, red[d][3][lane]);
      part[((size_t)d * S.nsplit + blockIdx.y) * S.ld + c] = s;
    }
  }
}

// X = 0, R = R0 = P = b; partial ||b||^2.
__global__ __launch_bounds__(256) void k_mk_init(Shape S, Rhs B, double2* X, double2* R, double2* R0, double2* P,
                                                 double2* part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t o = (size_t)gi * S.ld + c;
    const double2 b = rhs_at(B, gi, c);
    X[o] = make_double2(0.0, 0.0);
    R[o] = b;
    R0[o] = b;
    P[o] = b;
    acc[0].x += b.x * b.x + b.y * b.y;
  }
  store_partials<1>(S, acc, part);
}

// P = R + beta (P - omega V) for iterating columns.
// (Grid (ld/64, nsplit), four waves striding the block's rows, the column's scalars
// loaded once.)
__global__ __launch_bounds__(256) void k_mk_p(Shape S, const ColSt* st, const int* act, double2* P, const double2* R,
                                              const double2* V) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  if (!act[c]) return;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  const double2 be = st[c].beta, om = st[c].omega;
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t o = (size_t)gi * S.ld + c;
    P[o] = c_add(R[o], c_mul(be, c_sub(P[o], c_mul(om, V[o]))));
  }
}

// R = R - alpha V (s overwrites r) for iterating columns (grid as k_mk_p).
__global__ __launch_bounds__(256) void k_mk_s(Shape S, const ColSt* st, const int* act, double2* R, const double2* V) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  if (!act[c]) return;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  const double2 al = st[c].alpha;
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t o = (size_t)gi * S.ld + c;
    R[o] = c_sub(R[o], c_mul(al, V[o]));
  }
}

// Partial (U0, V0) and, with NDOT = 2, (U1, V1) over iterating columns.
template <int NDOT, class VT = double2>
__global__ __launch_bounds__(256) void k_mk_dots(Shape S, const int* act, const VT* U0, const VT* V0,
                                                 const VT* U1, const VT* V1, double2* part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  double2 acc[NDOT];
#pragma unroll
  for (int d = 0; d < NDOT; ++d) acc[d] = make_double2(0.0, 0.0);
  if (act[c]) {
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const size_t o = (size_t)gi * S.ld + c;
      acc[0] = c_add(acc[0], c_mulc(vld(U0, o), vld(V0, o)));
      if (NDOT > 1) acc[NDOT - 1] = c_add(acc[NDOT - 1], c_mulc(vld(U1, o), vld(V1, o)));
    }
  }
  store_partials<NDOT>(S, acc, part);
}

// X += alpha PH + omega SH;  R = R - omega T;  partial (R0, R) and (R, R).
__global__ __launch_bounds__(256) void k_mk_xr(Shape S, const ColSt* st, const int* act, double2* X, double2* R,
                                               const double2* R0,
                                               const double2* PH, const double2* SH, const double2* T,
                                               double2* part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  double2 acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  if (act[c]) {
    const double2 al = st[c].alpha, om = st[c].omega;
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const size_t o = (size_t)gi * S.ld + c;
      X[o] = c_add(X[o], c_add(c_mul(al, PH[o]), c_mul(om, SH[o])));
      const double2 rn = c_sub(R[o], c_mul(om, T[o]));
      R[o] = rn;
      acc[0] = c_add(acc[0], c_mulc(R0[o], rn));
      acc[1].x += rn.x * rn.x + rn.y * rn.y;
    }
  }
  store_partials<2>(S, acc, part);
}

// True residual of the marked columns: R = b - W (W = A X); partial ||R||^2.
__global__ __launch_bounds__(256) void k_mk_resid(Shape S, Rhs B, const int* mark, const double2* W, double2* R,
                                                  double2* part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  double2 acc[1] = {make_double2(0.0, 0.0)};
  if (mark[c]) {
    for (long long gi = r0 + wv; gi < r1; gi += 4) {
      const size_t o = (size_t)gi * S.ld + c;
      const double2 r = c_sub(rhs_at(B, gi, c), W[o]);
      R[o] = r;
      acc[0].x += r.x * r.x + r.y * r.y;
    }
  }
  store_partials<1>(S, acc, part);
}

// Mixed-precision refinement: X = 0, R = b for all columns; partial ||b||^2.
__global__ __launch_bounds__(256) void k_mk_rhs(Shape S, Rhs B, double2* X, double2* R, double2* part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t o = (size_t)gi * S.ld + c;
    const double2 b = rhs_at(B, gi, c);
    X[o] = make_double2(0.0, 0.0);
    R[o] = b;
    acc[0].x += b.x * b.x + b.y * b.y;
  }
  store_partials<1>(S, acc, part);
}

// Mixed-precision refinement: X += D (the complex64 correction) for the marked columns.
__global__ __launch_bounds__(256) void k_mk_addx(Shape S, const int* mark, double2* X, const float2* D) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  if (!mark[c]) return;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const size_t o = (size_t)gi * S.ld + c;
    X[o] = c_add(X[o], vld(D, o));
  }
}

// Restart of the marked columns from their true residual: R0 = P = R.
__global__ __launch_bounds__(256) void k_mk_restart(Shape S, const int* mark, const double2* R, double2* R0,
                                                    double2* P) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.n * S.ld) return;
  const int c = (int)(t % S.ld);
  if (!mark[c]) return;
  R0[t] = R[t];
  P[t] = R[t];
}

// Sum of the nsplit partials of product d for column c, by one wavefront: lane l
// adds partials l, l + 64, ... in order, then the 64 lane sums are combined by a
// butterfly of cross-lane shuffles (xor 32, 16, ..., 1); every lane holds the
// total.  The order is fixed, so the result is reproducible.
__device__ __forceinline__ double2 sum_part_wave(const Shape& S, const double2* part, int d, int c) {
  const int lane = threadIdx.x & 63;
  double2 s = make_double2(0.0, 0.0);
  for (int r = lane; r < S.nsplit; r += 64) s = c_add(s, part[((size_t)d * S.nsplit + r) * S.ld + c]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s.x += __shfl_xor(s.x, off, 64);
    s.y += __shfl_xor(s.y, off, 64);
  }
  return s;
}

enum ScalarStep { SC_INIT = 0, SC_ALPHA = 1, SC_OMEGA = 2, SC_BETA = 3 };

// Per-column scalars after each reduction: one wavefront per column sums the
// partials (sum_part_wave); its first lane updates the column's state.
//  SC_INIT : bb = ||b||^2, rho = rr = bb; columns with b = 0 are finished (x = 0).
//  SC_ALPHA: alpha = rho / (r0h, v); a vanishing or non-finite (r0h, v) is a breakdown.
//  SC_OMEGA: omega = (t, s) / (t, t); t = 0 means s = 0: omega = 0 and the step ends at x + alpha ph.
//  SC_BETA : rho' = (r0h, r), rr = (r, r), its += 1; rr <= tol^2 bb stops the column for a true-residual
//            check; a non-finite rr, |rho'| <= 1e-14 |r0h| |r|, omega = 0, or |r| grown 1e5-fold over its
//            smallest value since the last restart is a breakdown (restart from the true residual);
//            otherwise beta = (rho'/rho)(alpha/omega).
__global__ __launch_bounds__(64) void k_mk_scalar(Shape S, int step, ColSt* st, int* act, const double2* part,
                                                  double tol, int max_iter) {
  const int c = blockIdx.x;
  if (step != SC_INIT && !act[c]) return;  // uniform across the wave
  const double2 s0 = sum_part_wave(S, part, 0, c);
  const double2 s1 = (step == SC_OMEGA || step == SC_BETA) ? sum_part_wave(S, part, 1, c) : make_double2(0.0, 0.0);
  if (threadIdx.x != 0) return;
  ColSt& q = st[c];
  if (step == SC_INIT) {
    const double bb = s0.x;
    q.bb = bb;
    q.rr = bb;
    q.r0n = bb;
    q.rrmin = bb;
    q.rho = make_double2(bb, 0.0);
    q.alpha = q.omega = q.beta = make_double2(0.0, 0.0);
    q.check = q.brk = 0;
    q.its = q.restarts = 0;
    act[c] = bb > 0.0 ? 1 : 0;
    q.done = bb > 0.0 ? 0 : 1;
    return;
  }
  if (step == SC_ALPHA) {
    const double2 r0v = s0;
    const double2 a = c_div(q.rho, r0v);
    if (!c_finite(a) || (r0v.x == 0.0 && r0v.y == 0.0)) {
      q.alpha = make_double2(0.0, 0.0);
      q.omega = make_double2(0.0, 0.0);
      q.its += 1;  // counted, so that repeated breakdowns end at max_iter
      q.brk = 1;
      act[c] = 0;
      return;
    }
    q.alpha = a;
  } else if (step == SC_OMEGA) {
    const double2 ts = s0;
    const double tt = s1.x;
    q.omega = tt > 0.0 ? make_double2(ts.x / tt, ts.y / tt) : make_double2(0.0, 0.0);
    if (!c_finite(q.omega)) q.omega = make_double2(0.0, 0.0);
  } else {
    const double2 rho_n = s0;
    const double rr = s1.x;
    q.its += 1;
    q.rr = rr;
    if (!isfinite(rr)) {
      q.brk = 1;
      act[c] = 0;
      return;
    }
    if (rr <= tol * tol * q.bb) {
      q.check = 1;
      act[c] = 0;
      return;
    }
    if (q.its >= max_iter) {
      q.check = 1;  // final true residual, then reported as not converged
      act[c] = 0;
      return;
    }
    const double om2 = q.omega.x * q.omega.x + q.omega.y * q.omega.y;
    const double rh2 = rho_n.x * rho_n.x + rho_n.y * rho_n.y;
    q.rrmin = fmin(q.rrmin, rr);
    if (om2 == 0.0 || rh2 <= 1e-28 * rr * q.r0n || !c_finite(rho_n) || rr > 1e10 * q.rrmin) {
      q.brk = 1;
      act[c] = 0;
      return;
    }
    q.beta = c_mul(c_div(rho_n, q.rho), c_div(q.alpha, q.omega));
    q.rho = rho_n;
  }
}

// ---------------------------------------------------------------------------
// Free-electron + CAP preconditioner on column-fastest blocks
// ---------------------------------------------------------------------------

// One DFT pass along a lateral axis: out[line][j] = post[j] sum_i w[j]^i in[line][i]
// for every line of N points along the axis and every column.  Forward passes use
// w[j] = exp(-i(2 pi j/N + k h)) (the Bloch twist folded into the kernel) and
// post = 1; inverse passes w[j] = exp(+2 pi i j/N) and post[j] = exp(+i k h j)/N.
// The sum is evaluated by Horner's rule from i = N-1 down (acc = acc w + in[i]),
// so no twiddle table is read in the loop.  Axis a: a line is (z, b), stride 1;
// axis b: a line is (z, a), stride na.  Workgroup: one (line, 64-column chunk),
// four waves; the line's N rows and the w and post tables are staged in LDS, wave
// q forms outputs j = q, q + 4, ..., q + 4(R-1) (R = ceil(N/4) <= RW, the rest
// of a block of 4*RW outputs in later rounds).
struct DftPass {
  const void* in;      // n x ld vectors of the kernel's storage type
  void* out;
  const double2* w;    // [N] (direct evaluation)
  const double2* post; // [N]
  const double2* pre;  // [N] (factored evaluation): pre[i] = (w[j] / root^j)^i, the twist
  const double2* root; // [N] (factored evaluation): root^m, root = w[1] / w[0]
  const int* act;      // [ld] columns to transform (others untouched); nullable = all
  const int* cfl;      // [ld] (nullable) flagged columns: conjugated on load (cin) and on store (cout)
  int cin, cout;
  int N;               // points along the axis
  int stride;          // grid-index stride along the axis
  int nline_inner;     // lines per plane (axis a: nb; axis b: na)
  int inner_mul;       // grid-index step between consecutive lines of a plane (axis a: na; axis b: 1)
  int P, nz, ld;
};

// CJ: the instance honours the conjugation flags (cfl, cin, cout); the others ignore them (reading
// them measurably slowed the pass).
template <int RW, class VT = double2, bool CJ = false>
__global__ __launch_bounds__(256) void k_mk_dft(DftPass D) {
  const VT* in = (const VT*)D.in;
  VT* out = (VT*)D.out;
  extern __shared__ double2 lds_dft[];  // [N][64] line, then w[N], post[N]
  double2* lin = lds_dft;
  double2* tw = lds_dft + (size_t)D.N * 64;
  double2* tp = tw + D.N;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int N = D.N;
  const int nchunk = D.ld / 64;
  const long long line = blockIdx.x / nchunk;
  const int chunk = (int)(blockIdx.x % nchunk);
  const int c = chunk * 64 + lane;
  const int z = (int)(line / D.nline_inner), li = (int)(line % D.nline_inner);
  const long long base = (long long)z * D.P + (long long)li * D.inner_mul;
  const bool on = D.act == nullptr || D.act[c];
  const bool cfc = CJ && D.cfl != nullptr && D.cfl[c] != 0;
  const double cjin = cfc && D.cin ? -1.0 : 1.0, cjout = cfc && D.cout ? -1.0 : 1.0;  // imaginary-part signs
  for (int i = wv; i < N; i += 4)
    lin[i * 64 + lane] = on ? cflip(vld(in, (size_t)(base + (long long)i * D.stride) * D.ld + c), cjin)
                            : make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    tw[i] = D.w[i];
    tp[i] = D.post[i];
  }
  __syncthreads();
  if (!on) return;
  for (int jb = 0; jb < N; jb += 4 * RW) {
    double2 wr[RW], acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int j = jb + wv + 4 * r;
      wr[r] = j < N ? tw[j] : make_double2(0.0, 0.0);
      acc[r] = make_double2(0.0, 0.0);
    }
    for (int i = N - 1; i >= 0; --i) {
      const double2 x = lin[i * 64 + lane];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const double ax = acc[r].x, ay = acc[r].y;
        acc[r].x = fma(ax, wr[r].x, fma(-ay, wr[r].y, x.x));
        acc[r].y = fma(ax, wr[r].y, fma(ay, wr[r].x, x.y));
      }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int j = jb + wv + 4 * r;
      if (j < N) vst(out, (size_t)(base + (long long)j * D.stride) * D.ld + c, cflip(c_mul(tp[j], acc[r]), cjout));
    }
  }
}

// The same pass factored (Cooley-Tukey, one twiddle stage) for N = N1 N2, where
// w[j] = w[0] root^j with root an N-th root of unity: then w[j]^i = pre[i] root^(ij)
// with pre[i] = w[0]^i, and with i = N2 n1 + n2 (n1 < N1, n2 < N2), j = k1 + N1 k2,
//   Y[k1][n2]      = root^(n2 k1) sum_n1 pre[i] in[i] root^(N2 n1 k1)   (N2 transforms of length N1)
//   out[k1 + N1 k2] = post[j] sum_n2 Y[k1][n2] root^(N1 n2 k2)          (N1 transforms of length N2)
// N1 + N2 + 2 complex products per point instead of N.  The first stage reads its
// inputs straight from global memory (all of a wave's rows requested before the
// first is used) and leaves Y[k1][n2] in LDS slot N2 k1 + n2; after one barrier
// the second stage reads N2 consecutive slots and writes the outputs.  Workgroup:
// one (line, 64-column chunk), NW waves; wave q takes n2 = q, q + NW, ... in the
// first stage and k1 = q, q + NW, ... in the second.  MINW: waves per SIMD asked of
// the register allocator.
template <int N1, int N2, int NW, int MINW, class VT = double2, bool CJ = false>
__global__ __launch_bounds__(64 * NW, MINW) void k_mk_fft(DftPass D) {
  constexpr int N = N1 * N2;
  const VT* in = (const VT*)D.in;
  VT* out = (VT*)D.out;
  __shared__ double2 ys[N * 64];
  __shared__ double2 troot[N], tpre[N], tpost[N];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nchunk = D.ld / 64;
  const long long line = blockIdx.x / nchunk;
  const int chunk = (int)(blockIdx.x % nchunk);
  const int c = chunk * 64 + lane;
  const int z = (int)(line / D.nline_inner), li = (int)(line % D.nline_inner);
  const long long base = (long long)z * D.P + (long long)li * D.inner_mul;
  const bool on = D.act == nullptr || D.act[c];
  const bool cfc = CJ && D.cfl != nullptr && D.cfl[c] != 0;
  const double cjin = cfc && D.cin ? -1.0 : 1.0, cjout = cfc && D.cout ? -1.0 : 1.0;  // imaginary-part signs
  for (int i = threadIdx.x; i < N; i += 64 * NW) {
    troot[i] = D.root[i];
    tpre[i] = D.pre[i];
    tpost[i] = D.post[i];
  }
  __syncthreads();
  constexpr int G1 = (N2 + NW - 1) / NW;  // first-stage transforms per wave
  double2 v[G1][N1];
#pragma unroll
  for (int g = 0; g < G1; ++g) {
    const int n2 = wv + g * NW;
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1)
      v[g][n1] = on && n2 < N2 ? cflip(vld(in, (size_t)(base + (long long)(N2 * n1 + n2) * D.stride) * D.ld + c), cjin)
                               : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int g = 0; g < G1; ++g) {
    const int n2 = wv + g * NW;
    if (n2 >= N2) break;
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[g][n1] = c_mul(v[g][n1], tpre[N2 * n1 + n2]);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      double2 acc = v[g][0];
#pragma unroll
      for (int n1 = 1; n1 < N1; ++n1) {
        const double2 r = troot[(N2 * n1 * k1) % N];
        acc.x = fma(v[g][n1].x, r.x, fma(-v[g][n1].y, r.y, acc.x));
        acc.y = fma(v[g][n1].x, r.y, fma(v[g][n1].y, r.x, acc.y));
      }
      ys[(N2 * k1 + n2) * 64 + lane] = c_mul(acc, troot[(n2 * k1) % N]);
    }
  }
  __syncthreads();
  if (!on) return;
  for (int k1 = wv; k1 < N1; k1 += NW) {
    double2 u[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[n2] = ys[(N2 * k1 + n2) * 64 + lane];
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      double2 acc = u[0];
#pragma unroll
      for (int n2 = 1; n2 < N2; ++n2) {
        const double2 r = troot[(N1 * n2 * k2) % N];
        acc.x = fma(u[n2].x, r.x, fma(-u[n2].y, r.y, acc.x));
        acc.y = fma(u[n2].x, r.y, fma(u[n2].y, r.x, acc.y));
      }
      const int j = k1 + N1 * k2;
      vst(out, (size_t)(base + (long long)j * D.stride) * D.ld + c, cflip(c_mul(tpost[j], acc), cjout));
    }
  }
}

// Banded z part of the preconditioner.  Per energy e and lateral mode m the z
// operator is the complex symmetric band matrix (half bandwidth M, the stencil
// radius) T_m = diag(E - Vref(z) - eps_perp(m) + cz[0] + i (Gamma(z) + shift)) + sum_j cz[j]
// (shift by +-j), cz[j] = c_j / (2 hz^2) from the operator's own order-2M
// second-derivative weights, factored without pivoting as T = L D L^T (L unit lower,
// the CAP keeps every pivot off zero).  Row-oriented: for row z,
//   L[z][k] = (T[z][z-k] - sum_{j=k+1..M} L[z][j] L[z-k][j-k] D[z-j]) / D[z-k],  k = M..1,
//   D[z]    = T[z][z] - sum_{k=1..M} L[z][k]^2 D[z-k]
// with L[z][k] the entry (z, z-k).  Stored per (e, z, m): L[.][1..M] and 1/D.
struct Band {
  double2* L;       // [ne][nz][P][M]
  double2* dinv;    // [ne][nz][P]
  const double* energies;
  const double* eps;   // [P] lateral mode energies
  const double* vz;    // [nz] reference potential per plane
  const double* gz;    // [nz] Gamma_L + Gamma_R
  double cz[7];        // c_j / (2 hz^2), j = 0..M
  double shift;        // imaginary shift added to the CAP (Ha)
  int M, P, nz, ne;
  int neg_from;        // energy entries e >= neg_from factor the conjugate-space operator: imaginary
                       // part -(Gamma + shift) (the -k half of the doubled COCG); ne: none
};

__global__ __launch_bounds__(256) void k_mk_band_factor(Band B) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B.ne * B.P) return;
  const int e = (int)(t / B.P), m = (int)(t % B.P);
  const int M = B.M, P = B.P;
  const double d0 = B.energies[e] - B.eps[m] + B.cz[0];
  double2* L = B.L + (size_t)e * B.nz * P * M;
  double2* Di = B.dinv + (size_t)e * B.nz * P;
  double2 D[7];  // D[z-1..z-M] in a ring: D[j] = D_{z-j}
  for (int j = 0; j <= M; ++j) D[j] = make_double2(1.0, 0.0);
  for (int z = 0; z < B.nz; ++z) {
    double2 Lr[7];  // this row's L[z][k], k = 1..M
    for (int k = M; k >= 1; --k) {
      if (z - k < 0) {
        Lr[k] = make_double2(0.0, 0.0);
        continue;
      }
      double2 acc = make_double2(B.cz[k], 0.0);
      const double2* Lp = L + ((size_t)(z - k) * P + m) * M;  // row z-k
      for (int j = k + 1; j <= M; ++j) {
        if (z - j < 0) break;
        acc = c_sub(acc, c_mul(c_mul(Lr[j], Lp[j - k - 1]), D[j]));
      }
      Lr[k] = c_div(acc, D[k]);
    }
    double2 dz = make_double2(d0 - B.vz[z], (e >= B.neg_from ? -1.0 : 1.0) * (B.gz[z] + B.shift));
    for (int k = 1; k <= M; ++k)
      if (z - k >= 0) dz = c_sub(dz, c_mul(c_mul(Lr[k], Lr[k]), D[k]));
    double2* Lo = L + ((size_t)z * P + m) * M;
    for (int k = 1; k <= M; ++k) Lo[k - 1] = Lr[k];
    Di[(size_t)z * P + m] = c_div(make_double2(1.0, 0.0), dz);
    for (int j = M; j >= 2; --j) D[j] = D[j - 1];
    D[1] = dz;
  }
}

// z solve per (lateral mode m, column c): forward y_z = f_z - sum_k L[z][k] y_{z-k},
// w_z = y_z / D_z (into W), backward x_z = w_z - sum_j L[z+j][j] x_{z+j} (into io,
// which held f).  The last M values of y (forward) and x (backward) stay in
// registers.  RM: the stencil radius.
template <int RM, class VT = double2>
__global__ __launch_bounds__(256) void k_mk_band_solve(VT* io, VT* W, const double2* Lb,
                                                       const double2* dinv, const int* eidx, const int* act, int P,
                                                       int nz, int ld) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)P * ld) return;
  const int c = (int)(t % ld);
  const int m = (int)(t / ld);
  if (act != nullptr && !act[c]) return;
  const size_t eo = (size_t)eidx[c] * nz * P;
  const double2* L = Lb + eo * RM;
  const double2* di = dinv + eo;
  const size_t zs = (size_t)P * ld;
  double2 win[RM];  // win[k-1] = y_{z-k} (forward), x_{z+k} (backward)
#pragma unroll
  for (int k = 0; k < RM; ++k) win[k] = make_double2(0.0, 0.0);
  // both sweeps go BZ planes at a time, the block's loads (vector rows, factor rows, pivots)
  // requested before the first is used
  constexpr int BZ = 4;
  const size_t o0 = (size_t)m * ld + c;
  for (int zb = 0; zb < nz; zb += BZ) {
    double2 xin[BZ], dv[BZ], Lz[BZ][RM];
#pragma unroll
    for (int q = 0; q < BZ; ++q) {
      const int z = zb + q < nz ? zb + q : nz - 1;
      xin[q] = vld(io, o0 + (size_t)z * zs);
      dv[q] = di[(size_t)z * P + m];
#pragma unroll
      for (int k = 0; k < RM; ++k) Lz[q][k] = L[((size_t)z * P + m) * RM + k];
    }
#pragma unroll
    for (int q = 0; q < BZ; ++q) {
      if (zb + q >= nz) break;
      double2 y = xin[q];
#pragma unroll
      for (int k = 1; k <= RM; ++k) y = c_sub(y, c_mul(Lz[q][k - 1], win[k - 1]));
#pragma unroll
      for (int k = RM - 1; k >= 1; --k) win[k] = win[k - 1];
      win[0] = y;
      vst(W, o0 + (size_t)(zb + q) * zs, c_mul(y, dv[q]));
    }
  }
#pragma unroll
  for (int k = 0; k < RM; ++k) win[k] = make_double2(0.0, 0.0);
  // backward: x_z = W_z - sum_j L[z+j][j] x_{z+j}; the block z = zt, zt-1, ..., zt-BZ+1 needs the
  // factor rows z+1 .. z+RM, i.e. rows zt-BZ+2 .. zt+RM (clamped; entries past nz-1 unused)
  for (int zt = nz - 1; zt >= 0; zt -= BZ) {
    double2 w[BZ], Lz[BZ][RM];
#pragma unroll
    for (int q = 0; q < BZ; ++q) {
      const int z = zt - q >= 0 ? zt - q : 0;
      w[q] = vld(W, o0 + (size_t)z * zs);
#pragma unroll
      for (int j = 1; j <= RM; ++j) {
        const int zr = z + j < nz ? z + j : nz - 1;
        Lz[q][j - 1] = L[((size_t)zr * P + m) * RM + (j - 1)];
      }
    }
#pragma unroll
    for (int q = 0; q < BZ; ++q) {
      const int z = zt - q;
      if (z < 0) break;
      double2 x = w[q];
#pragma unroll
      for (int j = 1; j <= RM; ++j)
        if (z + j < nz) x = c_sub(x, c_mul(Lz[q][j - 1], win[j - 1]));
#pragma unroll
      for (int k = RM - 1; k >= 1; --k) win[k] = win[k - 1];
      win[0] = x;
      vst(io, o0 + (size_t)z * zs, x);
    }
  }
}

// T accumulation: T_c = 4 sum over the points of gdst[z] |x|^2 (partials; real part).
__global__ __launch_bounds__(256) void k_mk_tacc(Shape S, int P, const double* gdst, const double2* X,
                                                 double2* part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * S.rows;
  const long long r1 = r0 + S.rows < S.n ? r0 + S.rows : S.n;
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (long long gi = r0 + wv; gi < r1; gi += 4) {
    const double gz = gdst[gi / P];
    if (gz > 0.0) {
      const double2 x = X[(size_t)gi * S.ld + c];
      acc[0].x += 4.0 * gz * (x.x * x.x + x.y * x.y);
    }
  }
  store_partials<1>(S, acc, part);
}

// Final per-column sums of a one-product partial array into out[c] (real part);
// one wavefront per column.
__global__ __launch_bounds__(64) void k_mk_sum(Shape S, const double2* part, double* out) {
  const double2 s = sum_part_wave(S, part, 0, blockIdx.x);
  if (threadIdx.x == 0) out[blockIdx.x] = s.x;
}

// Export of nc columns from column c0 on: xout[gi*xld + it0 + c] = X[gi*ld + c0 + c].
__global__ __launch_bounds__(256) void k_mk_export(Shape S, int nc, const double2* X, double2* xout, long long xld,
                                                   long long it0, int c0) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.n * S.ld) return;
  const int c = (int)(t % S.ld) - c0;
  if (c < 0 || c >= nc) return;
  const long long gi = t / S.ld;
  xout[gi * xld + it0 + c] = X[t];
}

}  // namespace mk
}  // namespace rst
