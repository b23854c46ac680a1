// rst_eig.hpp -- kernels of the eigen route: dense blocks of vectors in the
// column-fastest layout (element (grid point g, column a) at g*ld + a).
//
// The eigen route (paper Sec. II.A: the transmission trace in the eigenbasis of
// G^-1; Sec. II.B-II.D and the Appendix: eigenpairs of +k and -k matched)
// finds the eigenpairs of K_k = H_k - i Gamma nearest a target energy by
// shift-invert subspace iteration (blocks of solves with G(sigma) = (sigma -
// K)^-1) and Rayleigh-Ritz, takes the left eigenvectors from the right ones at
// -k (K_k^T = K_{-k}), transforms the CAPs into the eigenbasis and sums the
// trace for every energy.  These kernels do the block algebra on the device:
// Gram matrices (optionally weighted by a plane-dependent CAP), right products
// with small host matrices, residual norms and the left-vector assembly.
// Every reduction is one workgroup per output entry in a fixed order.
#pragma once
#include <hip/hip_runtime.h>

namespace rst {
namespace eig {

__device__ __forceinline__ unsigned long long emix(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

// Q (n x m, column fastest): standard complex normal entries from SplitMix64 of
// (seed, element) and the Box-Muller transform.
__global__ void k_eig_randn(long long n, int m, unsigned long long seed, double2* Q) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n * m) return;
  const unsigned long long h = emix(seed ^ emix((unsigned long long)j));
  const double u1 = ((double)(h >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (double)(emix(h) >> 11) * (1.0 / 9007199254740992.0);
  const double r = sqrt(-log(u1));
  const double th = 6.283185307179586 * u2;
  Q[j] = make_double2(r * cos(th), r * sin(th));
}

// G[a + b*ma] = sum_g w(g) c(X[g*ldx + a]) Y[g*ldy + b], c = conj (cj != 0) or the
// identity (the bilinear product); w(g) = wz[g / P] if wz, else 1.  One
// workgroup per (a, b), 256 threads, tree reduction in LDS.
__global__ __launch_bounds__(256) void k_eig_gram(const double2* X, int ldx, const double2* Y, int ldy, long long n,
                                                  int ma, int mb, int cj, const double* wz, int P, double2* G) {
  __shared__ double2 red[256];
  const int a = blockIdx.x % ma, b = blockIdx.x / ma;
  double sx = 0.0, sy = 0.0;
  for (long long g = threadIdx.x; g < n; g += blockDim.x) {
    const double w = wz ? wz[g / P] : 1.0;
    if (w == 0.0) continue;
    const double2 x = X[g * ldx + a], y = Y[g * ldy + b];
    const double xy = cj ? -x.y : x.y;
    sx += w * (x.x * y.x - xy * y.y);
    sy += w * (x.x * y.y + xy * y.x);
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
  if (threadIdx.x == 0) G[a + (size_t)b * ma] = red[0];
}

// Z[g*ldz + b] = alpha sum_{a < mi} X[g*ldx + a] S[a + b*mi]   (b < mo; S column-major mi x mo)
__global__ void k_eig_rmul(const double2* X, int ldx, long long n, int mi, const double2* S, int mo, double alpha,
                           double2* Z, int ldz) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * mo) return;
  const long long g = t / mo;
  const int b = (int)(t % mo);
  double zx = 0.0, zy = 0.0;
  const double2* x = X + g * ldx;
  const double2* s = S + (size_t)b * mi;
  for (int a = 0; a < mi; ++a) {
    const double2 u = x[a], v = s[a];
    zx += u.x * v.x - u.y * v.y;
    zy += u.x * v.y + u.y * v.x;
  }
  Z[g * ldz + b] = make_double2(alpha * zx, alpha * zy);
}

// out[b] = || KX[:, b] - theta_b X[:, b] ||^2; one workgroup per column.
__global__ __launch_bounds__(256) void k_eig_resid(const double2* KX, const double2* X, int ld, long long n,
                                                   const double2* theta, double* out) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  const double2 th = theta[b];
  double s = 0.0;
  for (long long g = threadIdx.x; g < n; g += blockDim.x) {
    const double2 kx = KX[g * ld + b], x = X[g * ld + b];
    const double rx = kx.x - (th.x * x.x - th.y * x.y), ry = kx.y - (th.x * x.y + th.y * x.x);
    s += rx * rx + ry * ry;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0];
}

// Left eigenvectors from the right ones at -k: L[g*p + i] = conj(Rm[g*ldr + map[i]] * scale[i]).
__global__ void k_eig_left(const double2* Rm, int ldr, long long n, int p, const int* map, const double2* scale,
                           double2* L) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * p) return;
  const long long g = t / p;
  const int i = (int)(t % p);
  const double2 r = Rm[g * ldr + map[i]], s = scale[i];
  L[t] = make_double2(r.x * s.x - r.y * s.y, -(r.x * s.y + r.y * s.x));
}

}  // namespace eig
}  // namespace rst
