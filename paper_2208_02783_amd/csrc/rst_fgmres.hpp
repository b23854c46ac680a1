// rst_fgmres.hpp -- kernels of restarted flexible GMRES (FGMRES(m), Saad 1993)
// over a chunk of columns, the outer solver of the learned preconditioner.
//
// Vectors are complex128 in blocked layout: column c of a chunk is column
// c % cw of block c / cw, element (c, grid point p) at (blk*n + p)*cw + c%cw,
// so a block is exactly the vector set one workgroup of the stencil and
// preconditioner kernels owns.  The basis V_0..V_m and the preconditioned
// directions Z_0..Z_{m-1} are consecutive vectors `vstride` elements apart.
// Orthogonalisation is classical Gram-Schmidt applied twice (CGS2).  The
// Hessenberg matrix, its Givens rotations and the rotated right-hand side are
// kept per column on the device; one thread per column updates them.  All
// reductions are workgroup-local and in a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>

#include "rst_kernels.hpp"

namespace rst {
namespace fg {

struct Shape {
  long long n;  // grid points
  int cw;       // columns per block
  int nblk;     // blocks
  int ncol;     // valid columns (the rest of the last block is padding)
  int m;        // restart length
};

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cmulc_(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cmul_(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// X = 0 and R = b with b_c = bsc[c] e_{src[c]} (zero columns past ncol).
__global__ void k_fg_init(Shape S, const long long* src, const double* bsc, double2* X, double2* R) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int cc = (int)(j % S.cw);
  const long long p = (j / S.cw) % S.n;
  const int c = (int)(j / S.cw / S.n) * S.cw + cc;
  X[j] = make_double2(0.0, 0.0);
  R[j] = (c < S.ncol && p == src[c]) ? make_double2(bsc[c], 0.0) : make_double2(0.0, 0.0);
}

// out[i*ncolp + c] = sum_p conj(V_i[c, p]) W[c, p] for i < nv: one workgroup per
// (block, i); thread t always meets column t % cw (256 is a multiple of cw).
__global__ __launch_bounds__(256) void k_fg_dots(Shape S, const double2* V, long long vstride, int nv,
                                                 const double2* W, double2* out, int ncolp) {
  __shared__ double2 red[256];
  const int blk = blockIdx.x, i = blockIdx.y;
  const double2* v = V + (size_t)i * vstride + (size_t)blk * S.n * S.cw;
  const double2* w = W + (size_t)blk * S.n * S.cw;
  const long long tot = S.n * S.cw;
  double2 acc = make_double2(0.0, 0.0);
  for (long long t = threadIdx.x; t < tot; t += blockDim.x) acc = cadd(acc, cmulc_(v[t], w[t]));
  // thread t met column t % cw only (256 is a multiple of cw)
  const double2 s = rst::col_reduce_c(red, S.cw, acc);
  if ((int)threadIdx.x < S.cw) {
    const int c = blk * S.cw + threadIdx.x;
    if (c < ncolp) out[(size_t)i * ncolp + c] = s;
  }
  (void)nv;
}

// W[c] += sign * sum_{i < nv} V_i[c] h[i*ncolp + c]
__global__ void k_fg_update(Shape S, double2* W, const double2* V, long long vstride, int nv, const double2* h,
                            int ncolp, double sign) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int c = (int)(j / (S.n * S.cw)) * S.cw + (int)(j % S.cw);
  double2 s = make_double2(0.0, 0.0);
  for (int i = 0; i < nv; ++i) s = cadd(s, cmul_(V[(size_t)i * vstride + j], h[(size_t)i * ncolp + c]));
  W[j] = make_double2(W[j].x + sign * s.x, W[j].y + sign * s.y);
}

// V = W * scal[c]
__global__ void k_fg_scale(Shape S, double2* V, const double2* W, const double* scal) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int c = (int)(j / (S.n * S.cw)) * S.cw + (int)(j % S.cw);
  const double a = scal[c];
  V[j] = make_double2(W[j].x * a, W[j].y * a);
}

// Per-column Hessenberg state of one cycle, column-major per column:
// H[c][(m+1)*j + i], cs[c][j], sn[c][j], g[c][i].
struct Hess {
  double2* H;
  double* cs;
  double2* sn;
  double2* g;
  double* inv;       // [ncolp] scaling of the next basis vector
  double* est;       // [ncolp] |g_{j+1}|: the cycle's residual-norm estimate
  const int* active; // [ncolp] 1 while the column iterates
  int* iters;        // [ncolp] Arnoldi steps taken
};

// Starts a cycle: beta = sqrt(nrm2[c]), g = (beta, 0...), inv = 1 / beta.
__global__ void k_fg_start(Shape S, const double2* nrm2, Hess Hs, int ncolp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncolp) return;
  const double beta = sqrt(nrm2[c].x);
  for (int i = 0; i <= S.m; ++i) Hs.g[(size_t)c * (S.m + 1) + i] = make_double2(0.0, 0.0);
  Hs.g[(size_t)c * (S.m + 1)] = make_double2(beta, 0.0);
  Hs.inv[c] = (Hs.active[c] && beta > 0.0) ? 1.0 / beta : 0.0;
  Hs.est[c] = beta;
}

// Arnoldi step j of every column: H[0..j][j] = h1 + h2 (the two CGS passes),
// H[j+1][j] = ||w||, previous rotations applied, new rotation from
// (H[j][j], H[j+1][j]), g rotated; est = |g[j+1]|, inv = 1 / H[j+1][j].
__global__ void k_fg_arnoldi(Shape S, int j, const double2* h1, const double2* h2, const double2* wn2, Hess Hs,
                             int ncolp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncolp) return;
  const int m1 = S.m + 1;
  double2* Hc = Hs.H + (size_t)c * m1 * S.m + (size_t)m1 * j;
  double* cs = Hs.cs + (size_t)c * S.m;
  double2* sn = Hs.sn + (size_t)c * S.m;
  double2* g = Hs.g + (size_t)c * m1;
  if (!Hs.active[c]) {
    for (int i = 0; i <= S.m; ++i) Hc[i] = make_double2(0.0, 0.0);
    Hc[j] = make_double2(1.0, 0.0);  // identity column: the column's update is zero
    cs[j] = 1.0;
    sn[j] = make_double2(0.0, 0.0);
    Hs.inv[c] = 0.0;
    return;
  }
  for (int i = 0; i <= j; ++i) Hc[i] = cadd(h1[(size_t)i * ncolp + c], h2[(size_t)i * ncolp + c]);
  const double hn = sqrt(wn2[c].x);
  Hc[j + 1] = make_double2(hn, 0.0);
  for (int i = 0; i <= S.m; ++i)
    if (i > j + 1) Hc[i] = make_double2(0.0, 0.0);
  // previous rotations: [c s; -conj(s) c] on rows (i, i+1)
  for (int i = 0; i < j; ++i) {
    const double2 a = Hc[i], b = Hc[i + 1];
    const double2 ta = cadd(make_double2(cs[i] * a.x, cs[i] * a.y), cmul_(sn[i], b));
    const double2 tb = cadd(make_double2(-(sn[i].x * a.x + sn[i].y * a.y), -(sn[i].x * a.y - sn[i].y * a.x)),
                            make_double2(cs[i] * b.x, cs[i] * b.y));
    Hc[i] = ta;
    Hc[i + 1] = tb;
  }
  // new rotation zeroing H[j+1][j]: c = |a| / r, s = (a / |a|) conj(b) / r
  const double2 a = Hc[j];
  const double an = hypot(a.x, a.y);
  const double r = hypot(an, hn);
  double cj = 1.0;
  double2 sj = make_double2(0.0, 0.0);
  if (r > 0.0) {
    if (an == 0.0) {
      cj = 0.0;
      sj = make_double2(1.0, 0.0);
    } else {
      cj = an / r;
      sj = make_double2(a.x / an * hn / r, a.y / an * hn / r);
    }
  }
  cs[j] = cj;
  sn[j] = sj;
  Hc[j] = (an == 0.0) ? make_double2(r, 0.0) : make_double2(a.x / an * r, a.y / an * r);
  Hc[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = g[j];
  g[j] = make_double2(cj * gj.x, cj * gj.y);
  g[j + 1] = make_double2(-(sj.x * gj.x + sj.y * gj.y), -(sj.x * gj.y - sj.y * gj.x));
  Hs.est[c] = hypot(g[j + 1].x, g[j + 1].y);
  Hs.inv[c] = hn > 0.0 ? 1.0 / hn : 0.0;
  Hs.iters[c] += 1;
}

// y = R^-1 g over the first k rows (back substitution), y[i*ncolp + c]; zero
// for inactive columns.
__global__ void k_fg_trisolve(Shape S, int k, Hess Hs, double2* y, int ncolp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncolp) return;
  const int m1 = S.m + 1;
  const double2* H = Hs.H + (size_t)c * m1 * S.m;
  const double2* g = Hs.g + (size_t)c * m1;
  for (int i = k - 1; i >= 0; --i) {
    double2 s = g[i];
    for (int l = i + 1; l < k; ++l) {
      const double2 t = cmul_(H[(size_t)m1 * l + i], y[(size_t)l * ncolp + c]);
      s = make_double2(s.x - t.x, s.y - t.y);
    }
    const double2 d = H[(size_t)m1 * i + i];
    const double dd = d.x * d.x + d.y * d.y;
    y[(size_t)i * ncolp + c] =
        (Hs.active[c] && dd > 0.0) ? make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd)
                                   : make_double2(0.0, 0.0);
  }
}

// R = b - W (W = A X), b_c = bsc[c] e_{src[c]}
__global__ void k_fg_resid(Shape S, const long long* src, const double* bsc, const double2* W, double2* R) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int cc = (int)(j % S.cw);
  const long long p = (j / S.cw) % S.n;
  const int c = (int)(j / S.cw / S.n) * S.cw + cc;
  double2 r = make_double2(-W[j].x, -W[j].y);
  if (c < S.ncol && p == src[c]) r.x += bsc[c];
  R[j] = r;
}

// Network input x[c][p] = (Re v, Im v, Re m, Im m) (FP32) for c < ncol.
__global__ void k_fg_features(Shape S, const double2* Vj, const double2* Mj, float* x) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.ncol * S.n;
  if (j >= tot) return;
  const int c = (int)(j / S.n);
  const long long p = j % S.n;
  const size_t e = ((size_t)(c / S.cw) * S.n + p) * S.cw + c % S.cw;
  const double2 v = Vj[e], mm = Mj[e];
  x[4 * j] = (float)v.x;
  x[4 * j + 1] = (float)v.y;
  x[4 * j + 2] = (float)mm.x;
  x[4 * j + 3] = (float)mm.y;
}

// Z = M + use[c] * f (f the network output [c][p][2]).
__global__ void k_fg_combine(Shape S, const double2* Mj, const float* f, const int* use, double2* Z) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int cc = (int)(j % S.cw);
  const long long p = (j / S.cw) % S.n;
  const int c = (int)(j / S.cw / S.n) * S.cw + cc;
  double2 z = Mj[j];
  if (c < S.ncol && use[c]) {
    const size_t o = ((size_t)c * S.n + p) * 2;
    z.x += (double)f[o];
    z.y += (double)f[o + 1];
  }
  Z[j] = z;
}

// T accumulator per column: out[c] = sum_p gdst[z(p)] |X[c, p]|^2.
__global__ __launch_bounds__(256) void k_fg_tacc(Shape S, const double2* X, const double* gdst, long long P,
                                                 double* out) {
  __shared__ double red[256];
  const int blk = blockIdx.x;
  const double2* x = X + (size_t)blk * S.n * S.cw;
  const long long tot = S.n * S.cw;
  double acc = 0.0;
  for (long long t = threadIdx.x; t < tot; t += blockDim.x) {
    const double gd = gdst[(t / S.cw) / P];
    if (gd != 0.0) acc += gd * (x[t].x * x[t].x + x[t].y * x[t].y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < S.cw) {
    double s = 0.0;
    for (int k = threadIdx.x; k < (int)blockDim.x; k += S.cw) s += red[k];
    const int c = blk * S.cw + threadIdx.x;
    if (c < S.ncol) out[c] = s;
  }
}

// Standard complex normal entries (E|z|^2 = 1) for the valid columns of a
// blocked vector, from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) of
// (seed, element index) and the Box-Muller transform; padding columns zero.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

__global__ void k_fg_randn(Shape S, unsigned long long seed, double2* out) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.n * S.cw;
  if (j >= tot) return;
  const int c = (int)(j / (S.n * S.cw)) * S.cw + (int)(j % S.cw);
  if (c >= S.ncol) {
    out[j] = make_double2(0.0, 0.0);
    return;
  }
  const unsigned long long h = splitmix64(seed ^ splitmix64((unsigned long long)j));
  const double u1 = ((double)(h >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
  const double u2 = (double)(splitmix64(h) >> 11) * (1.0 / 9007199254740992.0);
  const double rad = sqrt(-log(u1));  // |z|^2 ~ Exp(1)
  const double th = 6.283185307179586 * u2;
  out[j] = make_double2(rad * cos(th), rad * sin(th));
}

// Training target of one pair: tgt[c][p] = s_c (e - m) with m = M^-1 r already
// scaled by s_c (FP32, 2 channels).
__global__ void k_fg_target(Shape S, const double2* E, const double2* Ms, const double* s, float* tgt) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.ncol * S.n;
  if (j >= tot) return;
  const int c = (int)(j / S.n);
  const long long p = j % S.n;
  const size_t e = ((size_t)(c / S.cw) * S.n + p) * S.cw + c % S.cw;
  tgt[2 * j] = (float)(s[c] * E[e].x - Ms[e].x);
  tgt[2 * j + 1] = (float)(s[c] * E[e].y - Ms[e].y);
}

// Solver-generated training pairs: from the column-fastest n x B blocks of an iterate x_j and the
// converged x*, the blocked x_j (into Xb) and error e_j = x* - x_j (into Eb); padding columns zero.
__global__ void k_fg_pairs(Shape S, int B, const double2* Xs, const double2* Xj, double2* Xb, double2* Eb) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.cw * S.n;
  if (t >= tot) return;
  const int c = (int)(t / S.n);
  const long long p = t % S.n;
  const size_t e = ((size_t)(c / S.cw) * S.n + p) * S.cw + c % S.cw;
  if (c >= B) {
    Xb[e] = make_double2(0.0, 0.0);
    Eb[e] = make_double2(0.0, 0.0);
    return;
  }
  const double2 xj = Xj[(size_t)p * B + c], xs = Xs[(size_t)p * B + c];
  Xb[e] = xj;
  Eb[e] = make_double2(xs.x - xj.x, xs.y - xj.y);
}

// R = b - R for unit right-hand sides b = e_{cols[c]} (blocked layout); padding columns zero.
__global__ void k_fg_bsub(Shape S, int B, const long long* cols, double2* R) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)S.nblk * S.cw * S.n;
  if (t >= tot) return;
  const int c = (int)(t / S.n);
  const long long p = t % S.n;
  const size_t e = ((size_t)(c / S.cw) * S.n + p) * S.cw + c % S.cw;
  if (c >= B) {
    R[e] = make_double2(0.0, 0.0);
    return;
  }
  const double2 ax = R[e];
  R[e] = make_double2((p == cols[c] ? 1.0 : 0.0) - ax.x, -ax.y);
}

// s[c] = 1 / sqrt(nrm2[c]) (0 for a zero column)
__global__ void k_fg_rsqrt(const double2* nrm2, double* s, int ncolp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncolp) return;
  s[c] = nrm2[c].x > 0.0 ? 1.0 / sqrt(nrm2[c].x) : 0.0;
}

}  // namespace fg
}  // namespace rst
