// rst_sweep.hpp -- the z-streaming sweep shared by the solver and apply kernels.
#pragma once
#include <type_traits>

#include "rst_kernels.hpp"

namespace rst {

template <class R>
struct SweepCtx {
  const Geo* g;
  const Proj* pj;
  const double* V;
  const double* gz;
  int cw;
  Vecs<R> vec;
  const double2* xext;   // IN_EXT source, (n x ext_ld) column-fastest
  double2* yext;         // OUT_EXT destination
  int ext_ld, ext_c0, ext_ncol;
  Lds<R> L;
  ColState* S;
  cx<double>* acc;       // gather accumulator of the output (nullptr: no gather)
  cx<R>* pcsrc;          // IN_PC source (preconditioned vector)
  cx<R>* pcs;            // OUT_TS: s for the (t, s) product
  cx<float>* r32;        // OUT_RES32 destination (FP32 copy of the FP64 residual)
  // dense right-hand side: column c of the block is rhs[gi*rhs_ld + rhs_c0 + c]
  // (null: the point source bsc e_src of the column)
  const double2* rhs;
  long long rhs_ld;
  long long rhs_c0;
  int rhs_nc;            // valid columns of the block
};

// Right-hand side b(gi) of column c.
template <class R>
__device__ __forceinline__ cx<R> rhs_at(const SweepCtx<R>& C, long long gi, int c) {
  if (C.rhs) {
    if (c >= C.rhs_nc) return mkc<R>((R)0, (R)0);
    const double2 v = C.rhs[gi * C.rhs_ld + C.rhs_c0 + c];
    return mkc<R>((R)v.x, (R)v.y);
  }
  return (gi == C.S->src[c]) ? mkc<R>((R)C.S->bsc[c], (R)0) : mkc<R>((R)0, (R)0);
}

template <int Q>
__device__ __forceinline__ Pos<Q> make_pos(const Geo& g, int cw, int rad) {
  Pos<Q> ps;
  const int tid = threadIdx.x, T = blockDim.x;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int pos = tid + T * q;
    const int c = pos % cw;
    const int p = pos / cw;
    if (p < g.P) {
      const int ia = p % g.na, ib = p / g.na;
      ps.p[q] = p;
      ps.li[q] = ((ib + rad) * g.pa + (ia + rad)) * cw + c;
      ps.hal[q] = (ia < rad ? 1 : 0) | (ia >= g.na - rad ? 2 : 0) | (ib < rad ? 4 : 0) |
                  (ib >= g.nb - rad ? 8 : 0);
    } else {
      ps.p[q] = -1;
      ps.li[q] = 0;
      ps.hal[q] = 0;
    }
  }
  return ps;
}

// Load (and update) the sweep input at plane zl for one position.  The mode
// is uniform across the workgroup, so the switch is a scalar branch.
template <class R>
__device__ __forceinline__ cx<R> load_in(const SweepCtx<R>& C, int mode, int zl, int p, int c,
                                         const cx<R>& al, const cx<R>& om, const cx<R>& be,
                                         double& d0) {
  const size_t off = ((size_t)zl * C.g->P + p) * C.cw + c;
  const long long gi = (long long)zl * C.g->P + p;
  ColState* S = C.S;
  switch (mode) {
    case IN_INIT: {
      const cx<R> u = rhs_at<R>(C, gi, c);
      stv(&C.vec.x[off], mkc<R>((R)0, (R)0));
      stv(&C.vec.r[off], u);
      stv(&C.vec.p[off], u);
      return u;
    }
    case IN_A: {
      const cx<R> rv = ldv(&C.vec.r[off]);
      const cx<R> vv = ldv(&C.vec.v[off]);
      const cx<R> tv = ldv(&C.vec.t[off]);
      const cx<R> pv = ldv(&C.vec.p[off]);
      const cx<R> xv = ldv(&C.vec.x[off]);
      const cx<R> s = rv - cmul(al, vv);
      const cx<R> xn = xv + cmul(al, pv) + cmul(om, s);
      const cx<R> rn = s - cmul(om, tv);
      const cx<R> pn = rn + cmul(be, pv - cmul(om, vv));
      stv(&C.vec.x[off], xn);
      stv(&C.vec.r[off], rn);
      stv(&C.vec.p[off], pn);
      d0 += (double)cnorm2(rn);
      return pn;
    }
    case IN_RESTART: {
      const cx<R> rv = ldv(&C.vec.r[off]);
      stv(&C.vec.p[off], rv);
      if (gi == S->j0[c]) S->rj[c] = to64(rv);
      return rv;
    }
    case IN_B: {
      const cx<R> rv = ldv(&C.vec.r[off]);
      const cx<R> vv = ldv(&C.vec.v[off]);
      const cx<R> s = rv - cmul(al, vv);
      if (gi == S->j0[c]) S->sj[c] = to64(s);
      return s;
    }
    case IN_X:
      return ldv(&C.vec.x[off]);
    case IN_PC:
      return ldv(&C.pcsrc[off]);
    default: {  // IN_EXT
      if (C.ext_c0 + c < C.ext_ncol) {
        const double2 v = C.xext[(size_t)gi * C.ext_ld + C.ext_c0 + c];
        return mkc<R>((R)v.x, (R)v.y);
      }
      return mkc<R>((R)0, (R)0);
    }
  }
}

// Store the sweep output y = A u at grid point gi for one position.
template <class R>
__device__ __forceinline__ void store_out(const SweepCtx<R>& C, int mode, long long gi, int p, int c,
                                          const cx<R>& y, const cx<R>& u, long long j0, long long src,
                                          double bsc, bool do_gather, double (&dots)[4], double& rmax,
                                          long long& rmax_idx) {
  ColState* S = C.S;
  const int cw = C.cw;
  const size_t off = (size_t)gi * cw + c;
  switch (mode) {
    case OUT_V:
      stv(&C.vec.v[off], y);
      if (gi == j0) S->vj[c] = to64(y);
      if (do_gather) C.L.outpl[p * cw + c] = y;
      break;
    case OUT_T: {
      stv(&C.vec.t[off], y);
      const cx<double> y64 = to64(y), u64 = to64(u);
      const cx<double> ts = cmulc(y64, u64);
      dots[1] += ts.x;
      dots[2] += ts.y;
      dots[3] += cnorm2(y64);
      if (gi == j0) S->tj[c] = y64;
      if (do_gather) C.L.outpl[p * cw + c] = y;
      break;
    }
    case OUT_TS: {
      stv(&C.vec.t[off], y);
      const cx<double> y64 = to64(y), s64 = to64(ldv(&C.pcs[off]));
      const cx<double> ts = cmulc(y64, s64);
      dots[1] += ts.x;
      dots[2] += ts.y;
      dots[3] += cnorm2(y64);
      if (gi == j0) S->tj[c] = y64;
      break;
    }
    case OUT_RES: {
      const cx<R> rr = rhs_at<R>(C, gi, c) - y;
      stv(&C.vec.r[off], rr);
      const double n2 = (double)cnorm2(rr);
      dots[0] += n2;
      if (n2 > rmax || (n2 == rmax && gi < rmax_idx)) {
        rmax = n2;
        rmax_idx = gi;
      }
      if (do_gather) C.L.outpl[p * cw + c] = rr;
      break;
    }
    case OUT_RES32: {
      // r = b - A x in FP64, stored as the FP32 recursive residual of the
      // mixed-precision solver; r[j0] of the stored value and the FP64 gather
      cx<R> rr = mkc<R>(-y.x, -y.y);
      if (gi == src) rr.x += (R)bsc;
      const cx<float> r32 = mkc<float>((float)rr.x, (float)rr.y);
      stv(&C.r32[off], r32);
      if (gi == j0) S->rj[c] = to64(r32);
      const double n2 = (double)cnorm2(rr);
      dots[0] += n2;
      if (n2 > rmax || (n2 == rmax && gi < rmax_idx)) {
        rmax = n2;
        rmax_idx = gi;
      }
      if (do_gather) C.L.outpl[p * cw + c] = rr;
      break;
    }
    default:  // OUT_EXT
      if (C.ext_c0 + c < C.ext_ncol) {
        double2 o;
        o.x = (double)y.x;
        o.y = (double)y.y;
        C.yext[(size_t)gi * C.ext_ld + C.ext_c0 + c] = o;
      }
      break;
  }
}

// One sweep over all planes: input u per IN mode, y = A u, output per OUT mode.
// The register queue q[0..2M] holds planes z-M..z+M of this thread's
// positions; plane z+M+1 is loaded at the start of step z (one step of
// prefetch) and the queue rotates at the end of the step.
// dots[0..3] accumulate per-thread partial reductions (all positions of a thread
// belong to the same column because blockDim is a multiple of cw).
template <int RAD, int Q, class R>
__device__ __forceinline__ void sweep(SweepCtx<R>& C, const Pos<Q>& ps, int in_mode, int out_mode,
                                   double (&dots)[4], double& rmax, long long& rmax_idx) {
  constexpr int NQ = 2 * RAD + 1;
  const Geo& g = *C.g;
  const Proj& pj = *C.pj;
  const int cw = C.cw;
  const int P = g.P, nz = g.nz;
  const int c = threadIdx.x % cw;
  ColState* S = C.S;
  const cx<R> al = fromd<R>(S->alpha[c]);
  const cx<R> om = fromd<R>(S->omega[c]);
  const cx<R> be = fromd<R>(S->beta[c]);
  const double en = S->energy[c];
  const double bsc = S->bsc[c];
  const long long src = S->src[c];
  const long long j0 = S->j0[c];
  const cx<R> pha = mkc<R>((R)g.pha_x, (R)g.pha_y), phb = mkc<R>((R)g.phb_x, (R)g.phb_y);
  const cx<R> phac = mkc<R>((R)g.pha_x, (R)-g.pha_y), phbc = mkc<R>((R)g.phb_x, (R)-g.phb_y);
  const int sa = cw, sb = g.pa * cw;
  const bool do_gather = (pj.nproj > 0) && (C.acc != nullptr);
  R wz[RAD + 1], wa[RAD + 1], wb[RAD + 1];
#pragma unroll
  for (int j = 1; j <= RAD; ++j) {
    wz[j] = (R)g.cz[j];
    wa[j] = (R)g.ca[j];
    wb[j] = (R)g.cb[j];
  }
  double d0 = 0.0;  // input-side partial (IN_A: ||r'||^2), added to dots[0] at the end
  if (do_gather) pacc_zero<R>(pj, C.L, cw);

  cx<R> q[Q][NQ];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
#pragma unroll
    for (int s = 0; s < NQ; ++s) q[k][s] = mkc<R>((R)0, (R)0);
    // planes 0..RAD into slots RAD..2RAD
#pragma unroll
    for (int s = 0; s <= RAD; ++s)
      if (s < nz && ps.p[k] >= 0) q[k][RAD + s] = load_in<R>(C, in_mode, s, ps.p[k], c, al, om, be, d0);
  }

  for (int z = 0; z < nz; ++z) {
    // 1. prefetch plane z + RAD + 1
    const int zl = z + RAD + 1;
    cx<R> nxt[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      nxt[k] = mkc<R>((R)0, (R)0);
      if (zl < nz && ps.p[k] >= 0) nxt[k] = load_in<R>(C, in_mode, zl, ps.p[k], c, al, om, be, d0);
    }

    // 2. stage plane z (with phase-premultiplied halos) into LDS
    cx<R>* buf = (z & 1) ? C.L.inpl1 : C.L.inpl0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] >= 0) {
        const cx<R> u = q[k][RAD];
        const int li = ps.li[k];
        buf[li] = u;
        const unsigned h = ps.hal[k];
        if (h & 1) buf[li + g.na * sa] = cmul(u, pha);
        if (h & 2) buf[li - g.na * sa] = cmul(u, phac);
        if (h & 4) buf[li + g.nb * sb] = cmul(u, phb);
        if (h & 8) buf[li - g.nb * sb] = cmul(u, phbc);
      }
    }
    __syncthreads();
    // 3. y = A u at plane z
    const double gzz = C.gz[z];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] >= 0) {
        const int p = ps.p[k];
        const long long gi = (long long)z * P + p;
        const cx<R> u = q[k][RAD];
        const double dr = en - C.V[gi] + g.diag0;
        cx<R> y = mkc<R>((R)dr * u.x - (R)gzz * u.y, (R)dr * u.y + (R)gzz * u.x);
        const int li = ps.li[k];
#pragma unroll
        for (int j = 1; j <= RAD; ++j) {
          const cx<R> zz = q[k][RAD + j] + q[k][RAD - j];
          const cx<R> aa = buf[li + j * sa] + buf[li - j * sa];
          const cx<R> bb = buf[li + j * sb] + buf[li - j * sb];
          y.x += wz[j] * zz.x + wa[j] * aa.x + wb[j] * bb.x;
          y.y += wz[j] * zz.y + wa[j] * aa.y + wb[j] * bb.y;
        }
        if (pj.nproj) {
          const cx<double> sc2 = point_scatter<R>(gi, c, pj, C.L, cw);
          y.x -= (R)sc2.x;
          y.y -= (R)sc2.y;
        }
        store_out<R>(C, out_mode, gi, p, c, y, u, j0, src, bsc, do_gather, dots, rmax, rmax_idx);
      }
    }
    // 4. projector gathers of the output plane
    if (do_gather) {
      __syncthreads();
      plane_gather<R>(z, pj, C.L, cw);
    }
    // 5. rotate the queue
#pragma unroll
    for (int k = 0; k < Q; ++k) {
#pragma unroll
      for (int s = 0; s < NQ - 1; ++s) q[k][s] = q[k][s + 1];
      q[k][NQ - 1] = nxt[k];
    }
  }
  dots[0] += d0;
  __syncthreads();
  if (do_gather) {
    pacc_flush<R>(pj, C.L, cw, C.acc);
    __syncthreads();
  }
}

// Gather-only sweep over x (IN_X or IN_EXT source): projections into C.acc and
// the transmission accumulator sum_z gdst(z) |x|^2.
template <int Q, class R, bool EXT>
__device__ __forceinline__ void gather_sweep(SweepCtx<R>& C, const Pos<Q>& ps, const double* gdst, double& tacc) {
  const Geo& g = *C.g;
  const Proj& pj = *C.pj;
  const int cw = C.cw;
  const int c = threadIdx.x % cw;
  const bool any_g = pj.nproj > 0 && C.acc != nullptr;
  if (any_g) pacc_zero<R>(pj, C.L, cw);
  __syncthreads();
  for (int z = 0; z < g.nz; ++z) {
    const bool need_g = pj.nproj > 0 && C.acc != nullptr && pj.zc_offs[z + 1] > pj.zc_offs[z];
    const double gd = gdst ? gdst[z] : 0.0;
    if (!need_g && gd == 0.0) continue;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] >= 0) {
        const long long gi = (long long)z * g.P + ps.p[k];
        cx<R> xv;
        if constexpr (EXT) {
          if (C.ext_c0 + c < C.ext_ncol) {
            const double2 v = C.xext[(size_t)gi * C.ext_ld + C.ext_c0 + c];
            xv = mkc<R>((R)v.x, (R)v.y);
          } else {
            xv = mkc<R>((R)0, (R)0);
          }
        } else {
          xv = ldv(&C.vec.x[(size_t)gi * cw + c]);
        }
        tacc += gd * (double)cnorm2(xv);
        if (need_g) C.L.outpl[ps.p[k] * cw + c] = xv;
      }
    }
    if (need_g) {
      __syncthreads();
      plane_gather<R>(z, pj, C.L, cw);
      __syncthreads();
    }
  }
  __syncthreads();
  if (any_g) {
    pacc_flush<R>(pj, C.L, cw, C.acc);
    __syncthreads();
  }
}

}  // namespace rst
