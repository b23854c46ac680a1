// rst_lowrank.hpp -- kernels of the low-rank transmission.
//
// T = 4 Tr[Gamma_L G Gamma_R G^+] = 4 ||M||_F^2 with M = Gamma_L^1/2 G Gamma_R^1/2
// restricted to the left-CAP rows and right-CAP columns (transmission
// equation).  M has small numerical rank (open channels plus modes decaying
// across the slab), so a randomised range finder (Halko, Martinsson and Tropp,
// SIAM Review 53, 2011) replaces the |R| column solves:
//   Y = M Omega            s + p solves with Gaussian right-hand sides on R,
//   Q = orth(Y[:, :s])     Cholesky QR applied twice,
//   tail = mean_j ||(I - QQ^H) y_j||^2 over the p held-out probes,
//                          an unbiased estimate of ||(I - QQ^H) M||_F^2,
//   Z = G_{-k} Gamma_L^1/2 conj(Q)   s solves at -k, since G_k^H = conj(G_{-k})
//                          for H_{-k} = conj(H_k),
//   T_Q = 4 ||Gamma_R^1/2 Z|_R||_F^2 = 4 ||Q^H M||_F^2 = T - 4 ||(I - QQ^H) M||_F^2.
// Matrices of one energy: Y and Q are nL x (s + p) column-major ([e][col][row]).
#pragma once
#include <hip/hip_runtime.h>

namespace rst {
namespace lr {

__device__ __forceinline__ unsigned long long smix(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

// Probe right-hand sides (n x ncol, column fastest): standard complex normal
// times sqrt(Gamma_R(z)) on the planes where Gamma_R > 0, zero elsewhere
// (SplitMix64 of (seed, element) and Box-Muller).
__global__ void k_lr_probes(long long n, int P, int ncol, const double* gsrc, unsigned long long seed,
                            double2* out) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n * ncol) return;
  const long long gi = j / ncol;
  const double g = gsrc[gi / P];
  if (!(g > 0.0)) {
    out[j] = make_double2(0.0, 0.0);
    return;
  }
  const unsigned long long h = smix(seed ^ smix((unsigned long long)j));
  const double u1 = ((double)(h >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (double)(smix(h) >> 11) * (1.0 / 9007199254740992.0);
  const double r = sqrt(-log(u1)) * sqrt(g);
  const double th = 6.283185307179586 * u2;
  out[j] = make_double2(r * cos(th), r * sin(th));
}

// Y[e][col][i] = sqrt(Gamma_L(z_i)) X[L_i, e*ncol + col]  (X: n x ne*ncol)
__global__ void k_lr_gather_left(const double2* X, int ne, int ncol, const long long* L, int nL, int P,
                                 const double* gdst, double2* Y) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)ne * ncol * nL;
  if (j >= tot) return;
  const int i = (int)(j % nL);
  const long long ec = j / nL;  // e*ncol + col
  const long long gi = L[i];
  const double w = sqrt(gdst[gi / P]);
  const double2 v = X[gi * ((long long)ne * ncol) + ec];
  Y[j] = make_double2(w * v.x, w * v.y);
}

// Gram blocks G[e][a][b] = sum_i conj(A[e][a][i]) B[e][b][i] for a < na, b < nb;
// A, B with column stride lda = ldb = nL and energy strides sa, sb.  One
// workgroup per (a, b, e); fixed-order reduction.
__global__ __launch_bounds__(256) void k_lr_gram(const double2* A, long long sa, const double2* B, long long sb,
                                                 int nL, int na, int nb, double2* G) {
  __shared__ double2 red[256];
  const int a = blockIdx.x, b = blockIdx.y, e = blockIdx.z;
  const double2* x = A + e * sa + (long long)a * nL;
  const double2* y = B + e * sb + (long long)b * nL;
  double sx = 0.0, sy = 0.0;
  for (int i = threadIdx.x; i < nL; i += blockDim.x) {
    sx += x[i].x * y[i].x + x[i].y * y[i].y;
    sy += x[i].x * y[i].y - x[i].y * y[i].x;
  }
  red[threadIdx.x] = make_double2(sx, sy);
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[threadIdx.x].x += red[threadIdx.x + h].x;
      red[threadIdx.x].y += red[threadIdx.x + h].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) G[((long long)e * na + a) * nb + b] = red[0];
}

// Per energy (one thread): Cholesky G = R^H R of the s x s Gram matrix and
// W = R^-1 (upper triangular), W[e][a][b] row a, column b.  A pivot below
// 1e-28 times the largest diagonal marks a numerically dependent column: its
// row of R^-1 is zero (the column drops out of Q).
__global__ void k_lr_chol_inv(const double2* G, int s, int ne, double2* Rm, double2* W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double2* g = G + (long long)e * s * s;
  double2* R = Rm + (long long)e * s * s;
  double2* w = W + (long long)e * s * s;
  double dmax = 0.0;
  for (int a = 0; a < s; ++a) dmax = fmax(dmax, g[a * s + a].x);
  for (int a = 0; a < s * s; ++a) R[a] = make_double2(0.0, 0.0);
  for (int j = 0; j < s; ++j) {
    // R[j][j] = sqrt(G[j][j] - sum_k |R[k][j]|^2)
    double d = g[j * s + j].x;
    for (int k = 0; k < j; ++k) d -= R[k * s + j].x * R[k * s + j].x + R[k * s + j].y * R[k * s + j].y;
    if (!(d > 1e-28 * dmax)) {
      R[j * s + j] = make_double2(0.0, 0.0);
      continue;
    }
    const double rjj = sqrt(d);
    R[j * s + j] = make_double2(rjj, 0.0);
    // R[j][m] = (G[j][m] - sum_k conj(R[k][j]) R[k][m]) / R[j][j], m > j
    for (int m = j + 1; m < s; ++m) {
      double2 t = g[j * s + m];
      for (int k = 0; k < j; ++k) {
        const double2 u = R[k * s + j], v = R[k * s + m];
        t.x -= u.x * v.x + u.y * v.y;
        t.y -= u.x * v.y - u.y * v.x;
      }
      R[j * s + m] = make_double2(t.x / rjj, t.y / rjj);
    }
  }
  // W = R^-1 by back substitution, column by column: R W[:, b] = e_b
  for (int a = 0; a < s * s; ++a) w[a] = make_double2(0.0, 0.0);
  for (int b = 0; b < s; ++b) {
    for (int a = b; a >= 0; --a) {
      const double2 raa = R[a * s + a];
      if (raa.x == 0.0) {
        w[a * s + b] = make_double2(0.0, 0.0);
        continue;
      }
      double2 t = make_double2(a == b ? 1.0 : 0.0, 0.0);
      for (int m = a + 1; m <= b; ++m) {
        const double2 u = R[a * s + m], v = w[m * s + b];
        t.x -= u.x * v.x - u.y * v.y;
        t.y -= u.x * v.y + u.y * v.x;
      }
      w[a * s + b] = make_double2(t.x / raa.x, t.y / raa.x);
    }
  }
}

// Qout[e][b][i] = sum_{a <= b} Y[e][a][i] W[e][a][b]
__global__ void k_lr_right_mul(const double2* Y, long long sy, const double2* W, int s, int nL, int ne,
                               double2* Qout) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)ne * s * nL;
  if (j >= tot) return;
  const int i = (int)(j % nL);
  const int b = (int)((j / nL) % s);
  const int e = (int)(j / nL / s);
  const double2* y = Y + e * sy;
  const double2* w = W + (long long)e * s * s;
  double qx = 0.0, qy = 0.0;
  for (int a = 0; a <= b; ++a) {
    const double2 u = y[(long long)a * nL + i], v = w[a * s + b];
    qx += u.x * v.x - u.y * v.y;
    qy += u.x * v.y + u.y * v.x;
  }
  Qout[j] = make_double2(qx, qy);
}

// Adjoint right-hand sides (n x ne*s, column e*s + b): sqrt(Gamma_L) conj(Q[e][b][i])
// at the left-CAP points, zero elsewhere.
__global__ void k_lr_adjoint_rhs(const double2* Q, int ne, int s, const long long* L, int nL, int P,
                                 const double* gdst, long long n, double2* out) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)ne * s * nL;
  if (j >= tot) return;
  const int i = (int)(j % nL);
  const long long eb = j / nL;
  const long long gi = L[i];
  const double w = sqrt(gdst[gi / P]);
  const double2 q = Q[j];
  out[gi * ((long long)ne * s) + eb] = make_double2(w * q.x, -w * q.y);
  (void)n;
}

// T_Q[e] partial: 4 sum_b sum_{i in R} Gamma_R(z_i) |Z[R_i, e*s + b]|^2; one
// workgroup per energy, fixed-order reduction.
__global__ __launch_bounds__(256) void k_lr_tq(const double2* Z, int ne, int s, const long long* R, int nR, int P,
                                               const double* gsrc, double* out) {
  __shared__ double red[256];
  const int e = blockIdx.x;
  double acc = 0.0;
  for (long long t = threadIdx.x; t < (long long)nR * s; t += blockDim.x) {
    const int i = (int)(t / s), b = (int)(t % s);
    const long long gi = R[i];
    const double2 z = Z[gi * ((long long)ne * s) + (long long)e * s + b];
    acc += gsrc[gi / P] * (z.x * z.x + z.y * z.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[e] = 4.0 * red[0];
}

}  // namespace lr
}  // namespace rst
