// rst_cnn.hpp -- kernels of the learned correction network (3D U-Net, 16
// channels, 3x3x3 convolutions without biases, ReLU, 2x2x2 mean pooling,
// nearest upsampling with additive skips) on FP32 matrix cores.
//
// Tensors are channel-last FP32: element (column c, grid point p, channel ch)
// of a tensor with C channels on a level with n points is at (c*n + p)*C + ch;
// p = (z*nb + b)*na + a.  Convolutions are cross-correlations, periodic in the
// two lateral directions (plain wrap at every level) and zero beyond the first
// and last plane along z.
//
// A convolution is an implicit GEMM, out[p][o] = sum_{t, i} in[p + t][i] W[t][i][o]:
// one wave owns 16 consecutive points x 16 output channels and runs
// v_mfma_f32_16x16x4f32 over K = 27 taps x input channels.  Lane l holds A
// element (point l%16, k = l/16) and B element (k = l/16, out channel l%16);
// the accumulator holds D(point 4*(l/16) + r, out channel l%16), r = 0..3.  For
// 16 input channels a lane loads 4 consecutive channels of its point once per
// tap; MFMA r of the tap takes channel 4*(l/16) + r, i.e. K is permuted the
// same way in A and B.  The weights of the layer sit in LDS.
//
// The weight gradient sum_p in[p + t][i] gy[p][o] is the same instruction with
// K running over points: a wave accumulates all 27 taps over a chunk of
// points and writes one partial 27x16x16 block; a second kernel adds the
// partial blocks in a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rst {
namespace cnn {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int CH = 16;
constexpr int NLAYER = 9;
constexpr int NTAP = 27;

enum ConvIn { CIN_PLAIN = 0, CIN_UPADD = 1, CIN_MASK = 2 };

struct Lvl {
  int nz, nb, na;
  long long n;
};

struct ConvArgs {
  const float* X;  // [ncol][n][CIN]
  const float* Y;  // CIN_UPADD: coarse skip source [ncol][nc][16]; CIN_MASK: mask [ncol][n][CIN]
  const float* W;  // [27][CIN][16]
  float* out;      // [ncol][n][COUT]
  Lvl L, Lc;       // level and (CIN_UPADD) its coarse level
  int ncol;
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// out = act(conv(in, W)) (+ out if ACCUM); in per MODE: X, X + up(Y), or X * (Y > 0).
template <int CIN, int COUT, int MODE, bool RELU, bool ACCUM>
__global__ __launch_bounds__(256) void k_conv(ConvArgs A) {
  static_assert(CIN == 4 || CIN == 16, "input channels");
  __shared__ float Ws[NTAP * CIN * 16];
  for (int i = threadIdx.x; i < NTAP * CIN * 16; i += blockDim.x) Ws[i] = A.W[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const long long tile = ((long long)blockIdx.x * 4 + wave) * 16;
  const int col = blockIdx.y;
  const long long n = A.L.n;
  const int nz = A.L.nz, nb = A.L.nb, na = A.L.na;
  const long long p = tile + i16;
  const bool valid = p < n;
  int z = 0, b = 0, a = 0;
  if (valid) {
    a = (int)(p % na);
    const long long r = p / na;
    b = (int)(r % nb);
    z = (int)(r / nb);
  }
  const float* Xc = A.X + (size_t)col * n * CIN;
  const float* Yc = nullptr;
  if (MODE == CIN_UPADD) Yc = A.Y + (size_t)col * A.Lc.n * 16;
  if (MODE == CIN_MASK) Yc = A.Y + (size_t)col * n * CIN;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  int t = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = z + dz;
    const bool zok = valid && zz >= 0 && zz < nz;
    for (int db = -1; db <= 1; ++db) {
      const int bb = wrapi(b + db, nb);
      for (int da = -1; da <= 1; ++da, ++t) {
        const int aa = wrapi(a + da, na);
        const long long q = ((long long)zz * nb + bb) * na + aa;
        if constexpr (CIN == 16) {
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (zok) {
            v = ld4(Xc + q * 16 + 4 * kq);
            if constexpr (MODE == CIN_UPADD) {
              const long long qc = ((long long)(zz >> 1) * A.Lc.nb + (bb >> 1)) * A.Lc.na + (aa >> 1);
              const float4 u = ld4(Yc + qc * 16 + 4 * kq);
              v.x += u.x;
              v.y += u.y;
              v.z += u.z;
              v.w += u.w;
            } else if constexpr (MODE == CIN_MASK) {
              const float4 m = ld4(Yc + q * 16 + 4 * kq);
              v.x = m.x > 0.f ? v.x : 0.f;
              v.y = m.y > 0.f ? v.y : 0.f;
              v.z = m.z > 0.f ? v.z : 0.f;
              v.w = m.w > 0.f ? v.w : 0.f;
            }
          }
          const float* wr = Ws + (t * 16 + 4 * kq) * 16 + i16;
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.x, wr[0], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.y, wr[16], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.z, wr[32], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.w, wr[48], acc, 0, 0, 0);
        } else {
          float v = 0.f;
          if (zok) {
            v = Xc[q * 4 + kq];
            if constexpr (MODE == CIN_MASK) v = Yc[q * 4 + kq] > 0.f ? v : 0.f;
          }
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v, Ws[(t * 4 + kq) * 16 + i16], acc, 0, 0, 0);
        }
      }
    }
  }
  if (i16 < COUT) {
    float* oc = A.out + (size_t)col * n * COUT;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long pt = tile + 4 * kq + r;
      if (pt < n) {
        float y = acc[r];
        if (RELU) y = y > 0.f ? y : 0.f;
        float* d = oc + pt * COUT + i16;
        if (ACCUM) y += *d;
        *d = y;
      }
    }
  }
}

struct BwArgs {
  const float* X;  // layer input [ncol][n][CIN]
  const float* Y;  // CIN_UPADD: coarse skip source [ncol][nc][16]
  const float* G;  // gradient of the layer output [ncol][n][GC]
  const float* M;  // mask (the layer's ReLU output) [ncol][n][16], or null
  float* part;     // [nwaves][27][16][16] partial weight gradients
  Lvl L, Lc;
  int ncol;
  long long chunk;  // points per wave (multiple of 4)
  long long total;  // ncol * n
};

// Partial weight gradients part[w][t][i][o] = sum over the wave's points of
// in[p + t][i] * gy[p][o] (gy masked by M > 0 when M is given).
template <int CIN, int GC, int MODE>
__global__ __launch_bounds__(256) void k_conv_bwdw(BwArgs A) {
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15, kq = lane >> 4;
  const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long long g0 = w * A.chunk;
  const long long g1 = g0 + A.chunk < A.total ? g0 + A.chunk : A.total;
  const long long n = A.L.n;
  const int nz = A.L.nz, nb = A.L.nb, na = A.L.na;
  v4f acc[NTAP];
#pragma unroll
  for (int t = 0; t < NTAP; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  for (long long k4 = g0; k4 < g1; k4 += 4) {
    const long long g = k4 + kq;  // this lane's point for both operands
    const bool gv = g < g1;
    float bv = 0.f;
    int col = 0, z = 0, b = 0, a = 0;
    if (gv) {
      col = (int)(g / n);
      const long long p = g - (long long)col * n;
      a = (int)(p % na);
      const long long r = p / na;
      b = (int)(r % nb);
      z = (int)(r / nb);
      if (i16 < GC) {
        bv = A.G[g * GC + i16];
        if (A.M != nullptr && !(A.M[g * 16 + i16] > 0.f)) bv = 0.f;
      }
    }
    const float* Xc = A.X + (size_t)col * n * CIN;
#pragma unroll
    for (int t = 0; t < NTAP; ++t) {
      const int dz = t / 9 - 1, db = (t / 3) % 3 - 1, da = t % 3 - 1;
      const int zz = z + dz;
      const bool zok = gv && zz >= 0 && zz < nz && i16 < CIN;
      const int bb = wrapi(b + db, nb);
      const int aa = wrapi(a + da, na);
      float av = 0.f;
      if (zok) {
        const long long q = ((long long)zz * nb + bb) * na + aa;
        av = Xc[q * CIN + i16];
        if constexpr (MODE == CIN_UPADD) {
          const long long qc = ((long long)(zz >> 1) * A.Lc.nb + (bb >> 1)) * A.Lc.na + (aa >> 1);
          av += A.Y[((size_t)col * A.Lc.n + qc) * 16 + i16];
        }
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
    }
  }
  float* pw = A.part + (size_t)w * NTAP * 256;
#pragma unroll
  for (int t = 0; t < NTAP; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) pw[t * 256 + (4 * kq + r) * 16 + i16] = acc[t][r];
}

// gw[j] = sum_w part[w][j] for j < 27*16*16, then scattered into the packed
// [27][cin][16] layout (rows i >= cin dropped).
__global__ void k_bwdw_reduce(const float* part, long long nw, int cin, float* gw) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= NTAP * 256) return;
  float s = 0.f;
  for (long long w = 0; w < nw; ++w) s += part[w * NTAP * 256 + j];
  const int t = j / 256, i = (j / 16) % 16, o = j % 16;
  if (i < cin) gw[(t * cin + i) * 16 + o] = s;
}

// Mean pooling over the existing children.
__global__ void k_pool(const float* x, float* y, Lvl f, Lvl c, int ncol) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)ncol * c.n * 16;
  if (j >= tot) return;
  const int ch = (int)(j % 16);
  const long long cp = (j / 16) % c.n;
  const int col = (int)(j / 16 / c.n);
  const int A_ = (int)(cp % c.na), B_ = (int)((cp / c.na) % c.nb), Z_ = (int)(cp / c.na / c.nb);
  float s = 0.f;
  int cnt = 0;
  for (int oz = 0; oz < 2; ++oz) {
    const int z = 2 * Z_ + oz;
    if (z >= f.nz) continue;
    for (int ob = 0; ob < 2; ++ob) {
      const int b = 2 * B_ + ob;
      if (b >= f.nb) continue;
      for (int oa = 0; oa < 2; ++oa) {
        const int a = 2 * A_ + oa;
        if (a >= f.na) continue;
        s += x[(((size_t)col * f.n) + ((long long)z * f.nb + b) * f.na + a) * 16 + ch];
        ++cnt;
      }
    }
  }
  y[j] = s / (float)cnt;
}

// gc[parent] = (gc +) sum over children of gf (adjoint of nearest upsampling).
__global__ void k_up_adj(const float* gf, float* gc, Lvl f, Lvl c, int ncol, int accum) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)ncol * c.n * 16;
  if (j >= tot) return;
  const int ch = (int)(j % 16);
  const long long cp = (j / 16) % c.n;
  const int col = (int)(j / 16 / c.n);
  const int A_ = (int)(cp % c.na), B_ = (int)((cp / c.na) % c.nb), Z_ = (int)(cp / c.na / c.nb);
  float s = 0.f;
  for (int oz = 0; oz < 2; ++oz) {
    const int z = 2 * Z_ + oz;
    if (z >= f.nz) continue;
    for (int ob = 0; ob < 2; ++ob) {
      const int b = 2 * B_ + ob;
      if (b >= f.nb) continue;
      for (int oa = 0; oa < 2; ++oa) {
        const int a = 2 * A_ + oa;
        if (a >= f.na) continue;
        s += gf[(((size_t)col * f.n) + ((long long)z * f.nb + b) * f.na + a) * 16 + ch];
      }
    }
  }
  gc[j] = accum ? gc[j] + s : s;
}

// gf[p] += gc[parent(p)] / children(parent(p)) (adjoint of mean pooling).
__global__ void k_pool_adj_acc(const float* gc, float* gf, Lvl f, Lvl c, int ncol) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)ncol * f.n * 16;
  if (j >= tot) return;
  const int ch = (int)(j % 16);
  const long long p = (j / 16) % f.n;
  const int col = (int)(j / 16 / f.n);
  const int a = (int)(p % f.na), b = (int)((p / f.na) % f.nb), z = (int)(p / f.na / f.nb);
  const int Z_ = z >> 1, B_ = b >> 1, A_ = a >> 1;
  const int cnt = (2 * Z_ + 1 < f.nz ? 2 : 1) * (2 * B_ + 1 < f.nb ? 2 : 1) * (2 * A_ + 1 < f.na ? 2 : 1);
  const long long cp = ((long long)Z_ * c.nb + B_) * c.na + A_;
  gf[j] += gc[((size_t)col * c.n + cp) * 16 + ch] / (float)cnt;
}

// Loss partial sums and output gradient: d = out - tgt over 2 channels;
// gout (4 channels, the last two zero) = 2 d / ncol; lossp[block] = sum d^2.
__global__ void k_loss(const float* out, const float* tgt, float* gout, double* lossp, long long npts,
                       float inv_ncol) {
  __shared__ double red[256];
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (j < npts) {
    const float d0 = out[2 * j] - tgt[2 * j], d1 = out[2 * j + 1] - tgt[2 * j + 1];
    s = (double)d0 * d0 + (double)d1 * d1;
    gout[4 * j] = 2.f * d0 * inv_ncol;
    gout[4 * j + 1] = 2.f * d1 * inv_ncol;
    gout[4 * j + 2] = 0.f;
    gout[4 * j + 3] = 0.f;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[blockIdx.x] = red[0];
}

// Adam (Kingma and Ba 2015, Algorithm 1), t counted from 1.
__global__ void k_adam(float* w, const float* g, float* m, float* v, int count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.f - b1) * gj;
  const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  w[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// gout4[p] = (g[p][0], g[p][1], 0, 0): a two-channel output gradient widened
// to the four input channels of the last layer's adjoint convolution.
__global__ void k_pad24(const float* g, float* g4, long long npts) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npts) return;
  g4[4 * j] = g[2 * j];
  g4[4 * j + 1] = g[2 * j + 1];
  g4[4 * j + 2] = 0.f;
  g4[4 * j + 3] = 0.f;
}

// Weights of the adjoint convolution: Wt[26 - t][o][i] = W[t][i][o] (taps
// mirrored, channel roles swapped), cout rows padded to coutp.
__global__ void k_flip(const float* W, int cin, int cout, int coutp, float* Wt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= NTAP * coutp * 16) return;
  const int t2 = j / (coutp * 16), o = (j / 16) % coutp, i = j % 16;
  const int t = NTAP - 1 - t2;
  Wt[j] = (o < cout && i < cin) ? W[(t * cin + i) * 16 + o] : 0.f;
}

}  // namespace cnn
}  // namespace rst
