// rst_projmm.hpp -- batched projector gather on FP64 matrix cores.
//
// For many columns X (n x ncol, column fastest) the projections of one group
// of projectors sharing their sphere entries (one atom: 9 projectors, about a
// thousand grid points) form a dense product
//     P_g (nm x ncol) = h^3 * beta_g^T (nm x E_g) * Xt_g (E_g x ncol),
//     Xt_g[e][c] = conj(exp(i k.R_e)) X[gi_e][c],
// with real beta.  Products for 64 columns are formed with
// v_mfma_f64_16x16x4f64 (M = 16 projector rows, nm <= 16 valid; N = 16
// columns per block, four blocks; K = 4 entries per step), the real and the
// imaginary part of Xt as two products sharing the beta operand.  Lane l holds
// A element (row l%16, k = l/16), B element (k = l/16, column l%16) and the
// accumulator D(row 4*r + l/16, column l%16), r = 0..3 (the FP64 layout,
// measured on the device; it differs from the FP32 instruction's).  A
// workgroup of four waves takes one (group, 64 columns) tile and splits the
// entries between its waves (wave w takes the steps k0 = 4w, 4w + 16, ...); the
// four partial products are summed in LDS in wave order, so the result does not
// depend on scheduling.
#pragma once
#include <hip/hip_runtime.h>

namespace rst {

typedef double v4d __attribute__((ext_vector_type(4)));

struct ProjMMArgs {
  const void* X;          // n x ncol, complex128 or complex64 (the kernel's XT)
  double2* P;             // nproj x ncol: P[p*ncol + c]
  const int* grp_e0;      // [ngroup] first entry of the group (group-major entry order)
  const int* grp_ne;      // [ngroup] entries of the group
  const int* grp_pbase;   // [ngroup] first projector
  const int* grp_nm;      // [ngroup] projectors
  const int* ent_gi;      // [nent] grid index of the entry
  const double2* eph;     // [nent] exp(+i k.R_e)
  const double* beta;     // [nent*nm] beta[e*nm + m]
  int nm, ngroup, ncol;
  double h3;
  // blocked layout (cw > 0): X holds blocks of cw columns, block b at b*n*cw with
  // (gi, c) at gi*cw + c, and P is written per block at b*p_stride + p*cw + c
  // (the solvers' per-workgroup projection arrays); cw == 0: column fastest
  int cw;
  long long n;
  size_t p_stride;
  const int* cfl;         // [ncol] (nullable, column-fastest only): the column's x enters conjugated
};

// XT: element type of X (double2, or float2 for a complex64 apply: widened to FP64 on load)
template <class XT>
__global__ __launch_bounds__(256) void k_proj_mm(ProjMMArgs A) {
  const XT* X = (const XT*)A.X;
  __shared__ double red[3][32][64];  // partial products of waves 1..3: [wave-1][slot][lane]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ntile = (A.ncol + 63) / 64;
  const int g = (int)(blockIdx.x / ntile);
  const int c0 = (int)(blockIdx.x % ntile) * 64;
  const int e0 = A.grp_e0[g], ne = A.grp_ne[g], nmg = A.grp_nm[g];
  const int i16 = lane & 15, kq = lane >> 4;
  v4d re[4], im[4];
  double ysg[4];  // -1 for conjugate-space columns (their x enters conjugated)
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    re[b] = v4d{0.0, 0.0, 0.0, 0.0};
    im[b] = v4d{0.0, 0.0, 0.0, 0.0};
    const int col = c0 + 16 * b + i16;
    ysg[b] = A.cfl != nullptr && col < A.ncol && A.cfl[col] != 0 ? -1.0 : 1.0;
  }
  for (int k0 = 4 * wv; k0 < ne; k0 += 16) {
    const int k = k0 + kq;
    double a = 0.0;
    double2 ph = make_double2(0.0, 0.0);
    long long gi = 0;
    if (k < ne) {
      const int e = e0 + k;
      if (i16 < nmg) a = A.beta[(size_t)e * A.nm + i16];
      ph = A.eph[e];
      gi = A.ent_gi[e];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int col = c0 + 16 * b + i16;
      double xr = 0.0, xi = 0.0;
      if (k < ne && col < A.ncol) {
        const size_t xo = A.cw ? ((size_t)(col / A.cw) * A.n + gi) * A.cw + col % A.cw : (size_t)gi * A.ncol + col;
        const XT xv = X[xo];
        const double2 x = make_double2((double)xv.x, ysg[b] * (double)xv.y);
        xr = ph.x * x.x + ph.y * x.y;  // conj(ph) * x
        xi = ph.x * x.y - ph.y * x.x;
      }
      re[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xr, re[b], 0, 0, 0);
      im[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xi, im[b], 0, 0, 0);
    }
  }
  if (wv > 0) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        red[wv - 1][4 * b + r][lane] = re[b][r];
        red[wv - 1][16 + 4 * b + r][lane] = im[b][r];
      }
  }
  __syncthreads();
  if (wv != 0) return;
  const int pb = A.grp_pbase[g];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int col = c0 + 16 * b + i16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double sr = re[b][r], si = im[b][r];
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        sr += red[w][4 * b + r][lane];
        si += red[w][16 + 4 * b + r][lane];
      }
      const int m = 4 * r + kq;
      if (m < nmg && col < A.ncol) {
        const size_t pi = A.cw ? (size_t)(col / A.cw) * A.p_stride + (size_t)(pb + m) * A.cw + col % A.cw
                               : (size_t)(pb + m) * A.ncol + col;
        A.P[pi] = make_double2(A.h3 * sr, A.h3 * si);
      }
    }
  }
}

}  // namespace rst
