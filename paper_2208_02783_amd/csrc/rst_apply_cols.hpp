// rst_apply_cols.hpp -- y = (E - H_k + i Gamma) x for many columns in the
// column-fastest layout (x, y: n x ncol, element (gi, c) at gi*ncol + c).
//
// H_k is the order-2M finite-difference Laplacian with Bloch-phase lateral
// wraps, the local potential and the KB projectors (Bloch-form equation,
// Kleinman-Bylander form); Gamma is the z-only CAP.  One wave owns one lateral
// grid point and 64 consecutive columns (one lane per column), so every load
// and store of a grid point's row is 1 KB contiguous.  The wave streams z:
// its own rows sit in a (2M+1)-deep register queue (the z part of the
// stencil), the 4M lateral neighbours of the current plane are read from the
// rows other waves of the same column chunk stream at the same time (L2), and
// the projector part uses the projections P = h^3 B^H x of all columns
// computed beforehand (k_proj_mm).  The point is uniform across the wave, so
// neighbour indices, wrap phases, V and the projector tables are scalar.
//
// A wave covers one segment of zseg planes (its queue starts from the rows
// below and above the segment), so the waves that share lateral rows stay
// within a few planes of each other.  Workgroup b takes (chunk, segment,
// point).  The eight XCDs receive workgroups round robin (b mod 8) and each has
// its own L2, so the (chunk, segment) groups, segment fastest, are split into
// eight contiguous runs, one per XCD: every lateral neighbour row a wave reads
// was streamed on its own XCD, and consecutive segments of a chunk (which share
// their z halo rows) run back to back (a remainder of fewer than eight groups
// keeps plain order).  Inside a group the points go in strips of `strip`
// a-columns, a fastest, so a point's b neighbours are dispatched within a few
// strip widths of it and are still in L2 when it reads them (on wide planes a
// plain row-major order puts them a whole b-row apart per step).
//
// Instruction budget: the kernel is bound by issue and latency more than by
// HBM, so a plane costs as few instructions as possible.  Row requests are raw
// buffer loads (plane base in the descriptor, a per-wave constant byte offset per
// neighbour in a VGPR: no address arithmetic per request), every lane loads
// (masked and ragged columns are dropped at the store), uniform tables are read
// through the scalar cache, and the projector slot's weights come premultiplied
// (beta_m E_p, zero-padded rows).  Planes of rows or projection arrays past 2^31
// bytes take k_apply_cols_wide (64-bit addresses, same arithmetic).
//
// F is the arithmetic and storage type: double (complex128 x, y) or float
// (complex64 x, y: the stencil in FP32; the projector sum, from the FP64
// projections and tables, in FP64 and rounded once when subtracted).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rst_kernels.hpp"

namespace rst {

// Planes per wave (measured on config 2 at 1024-4096 columns: 8 and 16 best,
// 32 slightly and 170 (whole columns) 20-30% slower).
constexpr int APPLY_ZSEG = 16;
// a-columns per strip of the point order on planes wider than the waves in flight
constexpr int APPLY_STRIP = 6;

struct ColApplyArgs {
  const void* x;      // n x ncol, complex128 or complex64 (the kernel's F)
  void* y;
  int ncol;
  Geo g;
  const double* V;    // [n]
  const double* gz;   // [nz] Gamma_L + Gamma_R
  double energy;
  // projector part: y -= sum_p beta_p (E_p P_p), P from k_proj_mm (h^3 included)
  Proj pj;
  const double2* P;   // [nproj*ncol]
  int zseg;           // planes per wave (>= 1)
  int strip;          // a-columns per strip of the point order (1..na; na: row-major)
  const double* ecol; // [ncol] energy of each column (nullable: `energy` for all)
  const int* mask;    // [ncol] columns to apply (nullable: all); others are left untouched
  const int* cfl;     // [ncol] (nullable) columns given as conj(x) of a -k system: y = conj((E - H_k - i Gamma)
                      // conj(x)) = (E - H_-k + i Gamma) x for real V and projectors, i.e. A_-k x
};

template <class V2>
__device__ __forceinline__ V2 cmul2(V2 a, V2 b) {
  return V2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// NMU: compile-time bound on the projectors per group (9 for l <= 2, else 16),
// so a point's projection rows are all requested before the first is used.
// Occupancy request of the 64-bit addressed kernel (minimum waves per SIMD): 4
// for its complex64 instances with up to 9 projectors per group (at most 128
// VGPRs, a few spills); the others are left free (the 16-projector one would
// spill heavily).
template <class F, int NMU>
struct ApplyMinWaves {
  static constexpr int value = std::is_same<F, float>::value && NMU <= 9 ? 4 : 1;
};

// (chunk, segment, lateral point) of workgroup b: the (chunk, segment) groups,
// segment fastest, in eight contiguous runs, one per XCD (b mod 8); inside a
// group the points in strips of `strip` a-columns, a fastest.
__device__ __forceinline__ void apply_place(const ColApplyArgs& A, long long b, int& chunk, int& seg, int& ia,
                                            int& ib) {
  const int P = A.g.P, na = A.g.na, nb = A.g.nb;
  const int nchunk = (A.ncol + 63) / 64;
  const int nseg = (A.g.nz + A.zseg - 1) / A.zseg;
  const long long g8 = (long long)nchunk * nseg / 8;  // groups per XCD in the balanced part
  long long grp, pi;
  if (b < g8 * 8 * P) {
    const long long i = b / 8;  // position in this XCD's sequence
    grp = (b % 8) * g8 + i / P;
    pi = i % P;
  } else {
    const long long r = b - g8 * 8 * P;
    grp = g8 * 8 + r / P;
    pi = r % P;
  }
  chunk = (int)(grp / nseg);
  seg = (int)(grp % nseg);
  // point pi of the group: strip s of W a-columns (the last one narrower), b-rows of w points
  const int W = A.strip;
  const int s0 = (int)(pi / ((long long)W * nb));
  const int r0 = (int)(pi - (long long)s0 * W * nb);
  const int w0 = min(W, na - s0 * W);
  ib = r0 / w0;
  ia = s0 * W + r0 % w0;
}

// Raw buffer loads: the descriptor holds a (uniform) base address and a record
// count in bytes, and the request adds a 32-bit VGPR offset (the row's and the
// lane's column offset, fixed for the wave) and an SGPR offset, so a row request
// costs no address arithmetic.  A lane whose VGPR offset is at or past the record
// count reads zero without a memory access (offset = the record count itself,
// so the address would be the first byte past the described range).  Descriptor
// word 3 for gfx9-family chips (32-bit data format, no swizzle).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
template <class V2>
__device__ __forceinline__ V2 buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff);
template <>
__device__ __forceinline__ double2 buf_ld<double2>(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  return make_double2(__builtin_bit_cast(double, (unsigned long long)v.x | ((unsigned long long)v.y << 32)),
                      __builtin_bit_cast(double, (unsigned long long)v.z | ((unsigned long long)v.w << 32)));
}
// (two dword loads at adjacent offsets, which the backend merges into one dwordx2 load)
template <>
__device__ __forceinline__ float2 buf_ld<float2>(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  const unsigned a = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
  const unsigned b = __builtin_amdgcn_raw_buffer_load_b32(r, voff + 4u, soff, 0);
  return make_float2(__builtin_bit_cast(float, a), __builtin_bit_cast(float, b));
}

// Uniform read of a table that no kernel of the launch writes, through the
// scalar data cache (a constant-address-space load) instead of a vector load and
// a lane read-back.
template <class T>
__device__ __forceinline__ T sld(const T* p, long long i) {
  return ((const __attribute__((address_space(4))) T*)p)[i];
}
__device__ __forceinline__ double2 sld(const double2* p, long long i) {
  return make_double2(sld((const double*)p, 2 * i), sld((const double*)p, 2 * i + 1));
}
__device__ __forceinline__ int2 sld(const int2* p, long long i) {
  return make_int2(sld((const int*)p, 2 * i), sld((const int*)p, 2 * i + 1));
}

// Bytes of the projection array P (nproj x ncol complex128).
__device__ __forceinline__ int pj_bytes(const Proj& pj, int ncol) { return pj.nproj * ncol * 16; }

// Largest byte offset the buffer path addresses: a lateral plane of rows and the
// projection array must each stay below 2^31 bytes (offsets from one descriptor
// base are 32-bit); larger launches take k_apply_cols_wide.
constexpr long long APPLY_BUF_MAX = 0x7fffffffLL;

// CJ: the instance honours the conjugate-space flags (cfl); the others ignore them, so the hot
// instances carry no extra work.
//
// The row requests of a plane are one unconditional group: a masked lane (or one
// past ncol, which uses the last column's addresses) has its stencil row offsets
// set to the record count, so it reads zeros without memory traffic, and stores
// nothing; a wave whose 64 columns are all masked returns at once.  The 4M lateral neighbour offsets and their wrap flags depend only on
// the wave's point and are computed once; per plane the kernel advances one
// descriptor base.  The point's projector slot is read one plane ahead, so the
// projection rows are requested together with the stencil rows.
template <int RAD, int NMU, class F, bool CJ = false>
__global__ __launch_bounds__(64) void k_apply_cols(ColApplyArgs A) {
  using V2 = typename std::conditional<std::is_same<F, double>::value, double2, float2>::type;
  static_assert(SC_SLOTS == 1, "one scatter slot per point");
  constexpr int NQ = 2 * RAD + 1;
  constexpr unsigned ESZ = sizeof(V2);
  const V2* X = (const V2*)A.x;
  V2* Y = (V2*)A.y;
  const Geo& g = A.g;
  const int P = g.P, na = g.na, nb = g.nb, nz = g.nz, ncol = A.ncol;
  int chunk, seg, ia, ib;
  apply_place(A, blockIdx.x, chunk, seg, ia, ib);
  const int p = ia + na * ib;
  const int z0 = seg * A.zseg, z1 = min(nz, z0 + A.zseg);
  const int c = chunk * 64 + (int)threadIdx.x;
  const int cc = c < ncol ? c : ncol - 1;
  const bool ok = c < ncol && (A.mask == nullptr || A.mask[c] != 0);
  if (__builtin_amdgcn_ballot_w64(ok) == 0) return;  // no column of this chunk to apply
  const double ec = A.ecol != nullptr ? A.ecol[cc] : A.energy;
  const F ysg = CJ && A.cfl != nullptr && A.cfl[cc] != 0 ? (F)-1 : (F)1;
  const V2 pha{(F)g.pha_x, (F)g.pha_y}, phac{(F)g.pha_x, (F)-g.pha_y};
  const V2 phb{(F)g.phb_x, (F)g.phb_y}, phbc{(F)g.phb_x, (F)-g.phb_y};
  const V2 zero{(F)0, (F)0};

  // lateral neighbours of the point (a+j, a-j, b+j, b-j for j = 1..M): byte
  // offsets of their rows within a plane, and which of them wrap
  const int rowb = ncol * (int)ESZ;
  const unsigned voff = (unsigned)cc * ESZ;
  const int plane_bytes = P * rowb;                             // at most APPLY_BUF_MAX (host check)
  const unsigned oob = (unsigned)plane_bytes;
  unsigned off[4 * RAD];  // lane byte offset of each neighbour row within a plane
  unsigned wrap = 0;
#pragma unroll
  for (int j = 1; j <= RAD; ++j) {
    int ap = ia + j, am = ia - j, bp = ib + j, bm = ib - j;
    const int k = 4 * (j - 1);
    if (ap >= na) { ap -= na; wrap |= 1u << k; }
    if (am < 0) { am += na; wrap |= 2u << k; }
    if (bp >= nb) { bp -= nb; wrap |= 4u << k; }
    if (bm < 0) { bm += nb; wrap |= 8u << k; }
    // a masked lane's requests fall past the record count: zeros, no memory traffic
    off[k] = ok ? (unsigned)((ib * na + ap) * rowb) + voff : oob;
    off[k + 1] = ok ? (unsigned)((ib * na + am) * rowb) + voff : oob;
    off[k + 2] = ok ? (unsigned)((bp * na + ia) * rowb) + voff : oob;
    off[k + 3] = ok ? (unsigned)((bm * na + ia) * rowb) + voff : oob;
  }
  const unsigned voffp = (unsigned)cc * (unsigned)sizeof(double2);  // projection rows: every lane reads
  const size_t plane = (size_t)P * ncol;  // elements per plane

  V2 q[NQ];  // q[RAD + d] = row of plane z + d
#pragma unroll
  for (int s = 0; s < NQ; ++s) {
    const int zs = z0 - RAD + s;
    V2 v = (zs >= 0 && zs < nz) ? X[((size_t)zs * P + p) * ncol + cc] : zero;
    if (CJ) v.y *= ysg;
    q[s] = v;
  }

  const Proj& pj = A.pj;
  const __amdgpu_buffer_rsrc_t rP = buf_rsrc(A.P, pj_bytes(pj, ncol));
  const char* xz = (const char*)A.x + (size_t)z0 * plane * ESZ;
  const V2* xn = X + ((size_t)(z0 + RAD + 1) * P + p) * ncol + cc;  // z-queue row of plane z + M + 1
  V2* yp = Y + ((size_t)z0 * P + p) * ncol + cc;
  int pbn = pj.nproj ? sld(pj.sc_pb, (long long)z0 * P + p) : -1;

  for (int z = z0; z < z1; ++z) {
    const long long gi = (long long)z * P + p;
    const int pb = pbn;
    if (pj.nproj) pbn = z + 1 < z1 ? sld(pj.sc_pb, gi + P) : -1;
    const __amdgpu_buffer_rsrc_t rx = buf_rsrc(xz, plane_bytes);
    V2 xl[4 * RAD];
#pragma unroll
    for (int k = 0; k < 4 * RAD; ++k) xl[k] = buf_ld<V2>(rx, off[k], 0);
    V2 nxt = z + RAD + 1 < nz ? *xn : zero;
    // projector slot: sum_m beta_m E_{pb+m} P_{pb+m}, times exp(+i k.R) of the entry
    double sx = 0.0, sy = 0.0;
    if (pb >= 0) {
      const size_t si = (size_t)gi;
      const int nv = min(pj.nm, pj.nproj - pb);  // rows past the projector array are not read
      const double* wr = pj.sc_w + si * NMU;     // beta_m E_{pb+m}, zero past the group
      double w[NMU];
      double2 pv[NMU];
#pragma unroll
      for (int m = 0; m < NMU; ++m) {
        const int mm = min(m, nv - 1);  // clamped row: in bounds, its weight zero
        w[m] = sld(wr, m);
        pv[m] = buf_ld<double2>(rP, voffp, (pb + mm) * ncol * (int)sizeof(double2));
      }
      const double2 ph = sld(pj.sc_eph, (long long)si);
      double tx = 0.0, ty = 0.0;
#pragma unroll
      for (int m = 0; m < NMU; ++m) {
        tx += w[m] * pv[m].x;
        ty += w[m] * pv[m].y;
      }
      sx = ph.x * tx - ph.y * ty;
      sy = ph.x * ty + ph.y * tx;
    }
    if (pj.has_overflow) {
      const int k0 = sld(pj.pe_offs, gi), k1 = sld(pj.pe_offs, gi + 1);
      for (int k = k0; k < k1; ++k) {
        const int2 ge = sld(pj.pe, (long long)k);
        const int nmg = sld(pj.grp_nm, (long long)ge.x);
        const int pb2 = sld(pj.grp_pbase, (long long)ge.x);
        const double2 ph = sld(pj.eph, (long long)ge.y);
        double tx = 0.0, ty = 0.0;
        for (int m = 0; m < nmg; ++m) {
          const double w = sld(pj.beta, (long long)ge.y * pj.nm + m) * sld(pj.ekb, (long long)pb2 + m);
          const double2 pv = A.P[(size_t)(pb2 + m) * ncol + cc];
          tx += w * pv.x;
          ty += w * pv.y;
        }
        sx += ph.x * tx - ph.y * ty;
        sy += ph.x * ty + ph.y * tx;
      }
    }
    const V2 u = q[RAD];
    const F dr = (F)(ec - sld(A.V, gi) + g.diag0);
    const double gzd = sld(A.gz, (long long)z);
    const F gzz = CJ ? (F)gzd * ysg : (F)gzd;
    V2 y{dr * u.x - gzz * u.y, dr * u.y + gzz * u.x};
#pragma unroll
    for (int j = 1; j <= RAD; ++j) {
      const int k = 4 * (j - 1);
      // a wrap across the +face carries exp(+i k L), across the -face its conjugate
      V2 xap = xl[k], xam = xl[k + 1], xbp = xl[k + 2], xbm = xl[k + 3];
      if (CJ) {
        xap.y *= ysg;
        xam.y *= ysg;
        xbp.y *= ysg;
        xbm.y *= ysg;
      }
      // (uniform branches, taken by few waves; kept as branches rather than selects)
      if (__builtin_expect((wrap >> k) & 1u, 0)) xap = cmul2(xap, pha);
      if (__builtin_expect((wrap >> (k + 1)) & 1u, 0)) xam = cmul2(xam, phac);
      if (__builtin_expect((wrap >> (k + 2)) & 1u, 0)) xbp = cmul2(xbp, phb);
      if (__builtin_expect((wrap >> (k + 3)) & 1u, 0)) xbm = cmul2(xbm, phbc);
      const V2 zz{q[RAD + j].x + q[RAD - j].x, q[RAD + j].y + q[RAD - j].y};
      const V2 aa{xap.x + xam.x, xap.y + xam.y};
      const V2 bb{xbp.x + xbm.x, xbp.y + xbm.y};
      const F cz = (F)g.cz[j], ca = (F)g.ca[j], cb = (F)g.cb[j];
      y.x += cz * zz.x + ca * aa.x + cb * bb.x;
      y.y += cz * zz.y + ca * aa.y + cb * bb.y;
    }
    y.x -= (F)sx;
    y.y -= (F)sy;
    if (CJ) y.y *= ysg;
    if (ok) {  // streaming store: the output row is not read again by this launch
      __builtin_nontemporal_store(y.x, &yp->x);
      __builtin_nontemporal_store(y.y, &yp->y);
    }
    if (CJ) nxt.y *= ysg;
#pragma unroll
    for (int s = 0; s < NQ - 1; ++s) q[s] = q[s + 1];
    q[NQ - 1] = nxt;
    xz += plane * ESZ;
    xn += plane;
    yp += plane;
  }
}

// The same operator with 64-bit addressing throughout, for launches whose plane
// of rows or projection array exceeds the buffer path's offsets.  Lanes past
// ncol and masked lanes load zeros and store nothing.
template <int RAD, int NMU, class F, bool CJ = false>
__global__ __launch_bounds__(64, (ApplyMinWaves<F, NMU>::value)) void k_apply_cols_wide(ColApplyArgs A) {
  using V2 = typename std::conditional<std::is_same<F, double>::value, double2, float2>::type;
  constexpr int NQ = 2 * RAD + 1;
  const V2* X = (const V2*)A.x;
  V2* Y = (V2*)A.y;
  const Geo& g = A.g;
  const int P = g.P, na = g.na, nb = g.nb, nz = g.nz, ncol = A.ncol;
  int chunk, seg, ia, ib;
  apply_place(A, blockIdx.x, chunk, seg, ia, ib);
  const int p = ia + na * ib;
  const int z0 = seg * A.zseg, z1 = min(nz, z0 + A.zseg);
  const int c = chunk * 64 + (int)threadIdx.x;
  const bool ok = c < ncol && (A.mask == nullptr || A.mask[c] != 0);
  const double ec = A.ecol != nullptr && c < ncol ? A.ecol[c] : A.energy;
  // conjugate-space columns: sign of the imaginary parts of the loaded and stored rows and of the CAP
  // (a multiply, no branch, so the row loads below stay one unconditional group)
  const F ysg = CJ && A.cfl != nullptr && c < ncol && A.cfl[c] != 0 ? (F)-1 : (F)1;
  const V2 pha{(F)g.pha_x, (F)g.pha_y}, phac{(F)g.pha_x, (F)-g.pha_y};
  const V2 phb{(F)g.phb_x, (F)g.phb_y}, phbc{(F)g.phb_x, (F)-g.phb_y};
  const V2 zero{(F)0, (F)0};
  const double2 zero64 = make_double2(0.0, 0.0);

  auto row = [&](long long gi) -> V2 {
    V2 v = ok ? X[gi * ncol + c] : zero;
    if (CJ) v.y *= ysg;
    return v;
  };

  V2 q[NQ];  // q[RAD + d] = row of plane z + d
#pragma unroll
  for (int s = 0; s < NQ; ++s) {
    const int zs = z0 - RAD + s;
    q[s] = (zs >= 0 && zs < nz) ? row((long long)zs * P + p) : zero;
  }

  for (int z = z0; z < z1; ++z) {
    const int zl = z + RAD + 1;
    const V2 nxt = zl < nz ? row((long long)zl * P + p) : zero;
    const long long base = (long long)z * P;
    const long long gi = base + p;
    const V2 u = q[RAD];
    const F dr = (F)(ec - A.V[gi] + g.diag0);
    const F gzz = CJ ? (F)A.gz[z] * ysg : (F)A.gz[z];
    V2 y{dr * u.x - gzz * u.y, dr * u.y + gzz * u.x};
#pragma unroll
    for (int j = 1; j <= RAD; ++j) {
      // lateral neighbours: a wrap across the +face carries exp(+i k L), across the -face its conjugate
      int ap = ia + j, am = ia - j, bp = ib + j, bm = ib - j;
      V2 xap = row(base + (long long)ib * na + (ap >= na ? ap - na : ap));
      V2 xam = row(base + (long long)ib * na + (am < 0 ? am + na : am));
      V2 xbp = row(base + (long long)(bp >= nb ? bp - nb : bp) * na + ia);
      V2 xbm = row(base + (long long)(bm < 0 ? bm + nb : bm) * na + ia);
      if (ap >= na) xap = cmul2(xap, pha);
      if (am < 0) xam = cmul2(xam, phac);
      if (bp >= nb) xbp = cmul2(xbp, phb);
      if (bm < 0) xbm = cmul2(xbm, phbc);
      const V2 zz{q[RAD + j].x + q[RAD - j].x, q[RAD + j].y + q[RAD - j].y};
      const V2 aa{xap.x + xam.x, xap.y + xam.y};
      const V2 bb{xbp.x + xbm.x, xbp.y + xbm.y};
      const F cz = (F)g.cz[j], ca = (F)g.ca[j], cb = (F)g.cb[j];
      y.x += cz * zz.x + ca * aa.x + cb * bb.x;
      y.y += cz * zz.y + ca * aa.y + cb * bb.y;
    }
    if (A.pj.nproj) {
      // sum over the point's (group, entry) pairs of exp(+i k.R_e) sum_m beta_e,m E_p P_p, p = first + m
      const Proj& pj = A.pj;
      double sx = 0.0, sy = 0.0;
      for (int sl = 0; sl < SC_SLOTS; ++sl) {
        const size_t si = (size_t)gi * SC_SLOTS + sl;
        const int pb = pj.sc_pb[si];
        if (pb < 0) continue;
        const double2 ph = pj.sc_eph[si];
        const int nv = min(pj.nm, pj.nproj - pb);  // values past the group's projectors are zero
        double w[NMU];
        double2 pv[NMU];
#pragma unroll
        for (int m = 0; m < NMU; ++m) {
          const int mm = min(m, nv - 1);  // clamped: every load in bounds, the extra weights zero
          const double bw = pj.sc_beta[si * pj.nm + mm] * pj.ekb[pb + mm];
          w[m] = m < nv ? bw : 0.0;
          pv[m] = ok ? A.P[(size_t)(pb + mm) * ncol + c] : zero64;
        }
        double tx = 0.0, ty = 0.0;
#pragma unroll
        for (int m = 0; m < NMU; ++m) {
          tx += w[m] * pv[m].x;
          ty += w[m] * pv[m].y;
        }
        sx += ph.x * tx - ph.y * ty;
        sy += ph.x * ty + ph.y * tx;
      }
      if (pj.has_overflow) {
        const int k0 = pj.pe_offs[gi], k1 = pj.pe_offs[gi + 1];
        for (int k = k0; k < k1; ++k) {
          const int2 ge = pj.pe[k];
          const int nmg = pj.grp_nm[ge.x];
          const int pb = pj.grp_pbase[ge.x];
          const double2 ph = pj.eph[ge.y];
          double tx = 0.0, ty = 0.0;
          for (int m = 0; m < nmg; ++m) {
            const double w = pj.beta[(size_t)ge.y * pj.nm + m] * pj.ekb[pb + m];
            const double2 pv = ok ? A.P[(size_t)(pb + m) * ncol + c] : zero64;
            tx += w * pv.x;
            ty += w * pv.y;
          }
          sx += ph.x * tx - ph.y * ty;
          sy += ph.x * ty + ph.y * tx;
        }
      }
      y.x -= (F)sx;
      y.y -= (F)sy;
    }
    if (CJ) y.y *= ysg;
    if (ok) Y[gi * ncol + c] = y;
#pragma unroll
    for (int s = 0; s < NQ - 1; ++s) q[s] = q[s + 1];
    q[NQ - 1] = nxt;
  }
}

}  // namespace rst
