// rst_mixed.hpp -- BiCGSTAB on FP32 vectors with FP64 reliable updates.
//
// The Krylov recurrences (plain or right-preconditioned: the same fused sweeps
// as the FP64 solvers) run on complex64 vectors with FP32 stencil, projector
// and preconditioner applies; inner products, scalars and projections stay
// FP64.  The solution is held as x64 + x32.  Whenever the recursive residual
// has fallen by the factor delta below the largest one seen since the last
// replacement (or has reached the tolerance, or the recurrence broke down),
// x32 is folded into x64 and the recursive residual is replaced by the FP64
// true residual b - A x64 (reliable updates: Sleijpen and van der Vorst,
// "Reliable updated residuals in hybrid Bi-CG methods", Computing 56, 1996).
// The direction p and v = A p are kept, so the Krylov process runs on across
// replacements; only a breakdown restarts it (p = r, shadow e_j0 moved to
// argmax |r|).  Convergence is decided on the FP64 true residual alone.  The
// drift between the recursive and the true residual grows like eps32 times
// the largest residual since the last replacement, which the replacement rule
// keeps within eps32 / delta of the current residual.  A column whose
// recursive residual norm has grown by more than 1e5 since the last
// replacement (a near-breakdown the FP32 recurrence cannot follow: x32 then has
// no correct digits) has x32 discarded instead of folded, and the block
// restarts from the FP64 residual of the unchanged x64.  Likewise a fold after
// which the true residual norm exceeds the recursive one tenfold is taken back
// (the FP32 increment was not reliable) and the block restarts.  A column
// whose best true residual norm has not fallen tenfold over STALL_UPDATES
// replacements is given up (status not converged): the library then solves it
// again with the FP64 kernel.  So is a column whose FP32 recursion has gone
// NOPROG_ITERS iterations without a replacement (it neither falls by delta nor
// diverges, so the replacement count alone would never stop it): it gets a
// replacement with its stall budget spent, and unless its true residual has
// fallen a hundredfold below its best, it goes to the FP64 kernel.
#pragma once
#include "rst_precond.hpp"

namespace rst {

constexpr double DIVERGE2 = 1e10;  // squared-norm growth that discards x32
constexpr double GAP2 = 100.0;     // ||r_true||^2 / ||r_rec||^2 that takes a fold back
constexpr int STALL_UPDATES = 30;  // replacements without a tenfold fall of the best residual
constexpr int NOPROG_ITERS = 1000; // FP32 iterations without a replacement (a column replaces every ~25)

// x64 += fold[c] * x32 (fold 1, 0 or -1) over all planes, with the gather of
// the new x64 into C.acc and the transmission accumulator sum_z gdst(z) |x64|^2.
template <int Q>
__device__ __forceinline__ void fold_gather_sweep(SweepCtx<double>& C, const Pos<Q>& ps, cx<float>* x32,
                                                  const double* gdst, double& tacc) {
  const Geo& g = *C.g;
  const Proj& pj = *C.pj;
  const int cw = C.cw;
  const int c = threadIdx.x % cw;
  const double fold = (double)C.S->fold[c];
  const bool any_g = pj.nproj > 0 && C.acc != nullptr;
  if (any_g) pacc_zero<double>(pj, C.L, cw);
  __syncthreads();
  for (int z = 0; z < g.nz; ++z) {
    const bool need_g = any_g && pj.zc_offs[z + 1] > pj.zc_offs[z];
    const double gd = gdst ? gdst[z] : 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] >= 0) {
        const size_t off = ((size_t)z * g.P + ps.p[k]) * cw + c;
        cx<double> xv = ldv(&C.vec.x[off]);
        if (fold != 0.0) {
          xv = xv + cscale(to64(ldv(&x32[off])), fold);
          stv(&C.vec.x[off], xv);
        }
        tacc += gd * cnorm2(xv);
        if (need_g) C.L.outpl[ps.p[k] * cw + c] = xv;
      }
    }
    if (need_g) {
      __syncthreads();
      plane_gather<double>(z, pj, C.L, cw);
      __syncthreads();
    }
  }
  __syncthreads();
  if (any_g) {
    pacc_flush<double>(pj, C.L, cw, C.acc);
    __syncthreads();
  }
}

// x32 = 0 over all planes.
template <int Q>
__device__ __forceinline__ void zero_sweep(const Geo& g, const Pos<Q>& ps, int cw, cx<float>* x32) {
  const int c = threadIdx.x % cw;
  for (int z = 0; z < g.nz; ++z) {
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (ps.p[k] >= 0) stv(&x32[((size_t)z * g.P + ps.p[k]) * cw + c], mkc<float>(0.0f, 0.0f));
  }
}

// r32 = b - A x64 (FP64 sweep; the plain recurrences take B^H r into Pr) after
// the fold sweep: S.rr, S.rmax_idx, S.tacc per column.
template <int RAD, int Q, bool PC>
__device__ __forceinline__ void fold_and_residual(const SolveArgs& A, SweepCtx<double>& C64, SweepCtx<float>& C32,
                                                  const Pos<Q>& ps, const ProjArrays& PA) {
  ColState& S = *C64.S;
  const int cw = A.cw;
  const int tid = threadIdx.x;
  double tacc = 0.0;
  C64.acc = PA.Px;
  fold_gather_sweep<Q>(C64, ps, C32.vec.x, A.gdst, tacc);
  {
    double v4[4] = {tacc, 0, 0, 0};
    __shared__ double red_out[4][CW_MAX];
    col_reduce4(C64.L.red, cw, v4, red_out);
    if (tid < cw) S.tacc[tid] = red_out[0][tid];
  }
  set_dco(A.pj, cw, C64.L.dco, PA.Px);
  __syncthreads();
  double dots[4] = {0, 0, 0, 0};
  double rmax = -1.0;
  long long rmax_idx = 0x7fffffffffffffffLL;
  C64.acc = PC ? nullptr : PA.Pr;
  C64.r32 = C32.vec.r;
  sweep<RAD, Q, double>(C64, ps, IN_X, OUT_RES32, dots, rmax, rmax_idx);
  {
    __shared__ double red_out[4][CW_MAX];
    col_reduce4(C64.L.red, cw, dots, red_out);
    double* bm = C64.L.red;
    long long* bi = reinterpret_cast<long long*>(C64.L.red + blockDim.x);
    bm[tid] = rmax;
    bi[tid] = rmax_idx;
    __syncthreads();
    if (tid < cw) {
      double m = -1.0;
      long long ix = 0x7fffffffffffffffLL;
      for (int i = tid; i < (int)blockDim.x; i += cw) {
        if (bm[i] > m || (bm[i] == m && bi[i] < ix)) {
          m = bm[i];
          ix = bi[i];
        }
      }
      S.rr[tid] = red_out[0][tid];
      S.rmax_idx[tid] = ix;
    }
    __syncthreads();
  }
}

// One reliable update of the block: fold x32 into x64, r32 = b - A x64
// (FP64 apply), decide every active column on its FP64 true residual, and
// restart the Krylov process of the block if `restart` (a breakdown or a
// discarded x32) asks.
template <int RAD, int Q, bool PC>
__device__ __forceinline__ void reliable_update(const SolveArgs& A, SweepCtx<double>& C64, SweepCtx<float>& C32,
                                                const PcVecs<float>& pv, const Pos<Q>& ps,
                                                const ProjArrays& PA, const DftSteps& dst_, bool final_check,
                                                bool restart, bool& all_done) {
  ColState& S = *C64.S;
  const int cw = A.cw;
  const int tid = threadIdx.x;
  // (1) x64 += x32 (or x32 discarded); r32 = b - A x64 in FP64
  fold_and_residual<RAD, Q, PC>(A, C64, C32, ps, PA);
  // (2) a fold whose true residual disagrees with the recursive one is taken back
  if (tid == 0) S.any_flag = 0;
  __syncthreads();
  if (tid < cw) {
    const int c = tid;
    const bool back = S.state[c] == 0 && S.fold[c] == 1 && !(S.rr[c] <= A.tol * A.tol * S.bb[c]) &&
                      !(S.rr[c] <= GAP2 * S.rr_rec[c]);
    S.fold[c] = back ? -1 : 0;
    if (back) atomicOr(&S.any_flag, 1);
  }
  __syncthreads();
  if (S.any_flag) {
    fold_and_residual<RAD, Q, PC>(A, C64, C32, ps, PA);
    restart = true;
  }
  zero_sweep<Q>(A.g, ps, cw, C32.vec.x);
  if (tid < cw) S.fold[tid] = 1;
  __syncthreads();
  // (3) decide: converged, failed, out of iterations, or go on from the true residual
  if (tid == 0) S.any_flag = 0;
  __syncthreads();
  if (tid < cw) {
    const int c = tid;
    if (S.state[c] == 0) {
      const double rr = S.rr[c];
      S.updates[c] += 1;
      if (!isfinite(rr)) {
        S.state[c] = 2;
      } else if (rr <= A.tol * A.tol * S.bb[c]) {
        S.state[c] = 1;
      } else if (final_check) {
        S.state[c] = 4;
      } else if (!(rr < 0.01 * S.best_rr[c]) && ++S.stall[c] >= STALL_UPDATES) {
        S.state[c] = 4;  // the FP32 recurrences make no progress on this column
      } else {
        if (rr < 0.01 * S.best_rr[c]) {
          S.best_rr[c] = rr;
          S.stall[c] = 0;
        }
        S.maxrr[c] = rr;
        S.rr_upd[c] = rr;
        S.it_upd[c] = S.iters[c];
        if (restart) {
          S.j0[c] = S.rmax_idx[c];
          S.restarts[c] += 1;
        } else {
          S.rho[c] = S.rj[c];  // (r^0, r) of the replaced residual
        }
        atomicOr(&S.any_flag, 1);
      }
    }
  }
  __syncthreads();
  all_done = (S.any_flag == 0);
  if (all_done || !restart) return;
  // (4) restart: p = r, v = A p (with the preconditioner: ph = M^-1 p, v = A ph)
  const int ncw = A.pj.nproj * cw;
  double d2[4] = {0, 0, 0, 0};
  if constexpr (PC) {
    pc_forward<Q, float>(C32, pv, ps, A.pc, dst_, PC_RESTART, d2);
    C32.acc = PA.Pr;
    pc_backward<Q, float>(C32, pv, ps, A.pc, dst_, pv.ph);
    set_dco(A.pj, cw, C32.L.dco, PA.Pr);
    __syncthreads();
    pc_apply<RAD, Q, float, false>(C32, pv, ps, d2);
  } else {
    for (int w = tid; w < ncw; w += blockDim.x) PA.Pp[w] = PA.Pr[w];
    set_dco(A.pj, cw, C32.L.dco, PA.Pr);
    __syncthreads();
    C32.acc = PA.Pv;
    double rm = 0;
    long long ri = 0;
    sweep<RAD, Q, float>(C32, ps, IN_RESTART, OUT_V, d2, rm, ri);
  }
  if (tid < cw) S.rho[tid] = S.rj[tid];
  __syncthreads();
}

template <int RAD, int Q, bool PC>
__device__ __forceinline__ void mixed_solve_item(const SolveArgs& A, SweepCtx<double>& C64,
                                                 SweepCtx<float>& C32, PcVecs<float>& pv, const Pos<Q>& ps,
                                                 const ProjArrays& PA, const DftSteps& dst_, int item) {
  ColState& S = *C64.S;
  const Geo& g = A.g;
  const int cw = A.cw;
  const int tid = threadIdx.x;
  const int ncw = A.pj.nproj * cw;
  const int e_idx = item / A.nblk;
  const int blk = item % A.nblk;
  if (tid < cw) {
    const int c = tid;
    const int col = blk * cw + c;
    S.energy[c] = A.energies[e_idx];
    S.alpha[c] = S.omega[c] = S.beta[c] = mkc(0.0, 0.0);
    S.iters[c] = 0;
    S.restarts[c] = 0;
    S.updates[c] = 0;
    S.fold[c] = 1;
    S.stall[c] = 0;
    S.it_upd[c] = 0;
    S.tacc[c] = 0.0;
    S.rr[c] = 0.0;
    if (col < A.ncols) {
      const long long src = A.cols[col];
      S.src[c] = src;
      S.j0[c] = src;
      const double gs = A.gsrc ? A.gsrc[src / g.P] : 1.0;
      S.bsc[c] = sqrt(gs);
      S.bb[c] = gs;
      S.maxrr[c] = gs;
      S.rr_upd[c] = gs;
      S.rr_rec[c] = gs;
      S.best_rr[c] = gs;
      S.state[c] = 0;
    } else {
      S.src[c] = -1;
      S.j0[c] = -1;
      S.bsc[c] = 0.0;
      S.bb[c] = 0.0;
      S.maxrr[c] = 0.0;
      S.rr_upd[c] = 0.0;
      S.rr_rec[c] = 0.0;
      S.best_rr[c] = 0.0;
      S.state[c] = 3;
    }
  }
  if constexpr (PC) pv.inv = reinterpret_cast<const cx<double>*>(A.pc.inv) + (size_t)e_idx * g.nz * g.P;
  __syncthreads();
  // x64 = 0, each element by the thread that owns it in every sweep
  {
    const int c = tid % cw;
    for (int z = 0; z < g.nz; ++z) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (ps.p[k] < 0) continue;
        stv(&C64.vec.x[((size_t)z * g.P + ps.p[k]) * cw + c], mkc(0.0, 0.0));
      }
    }
  }
  // x32 = 0, r32 = p32 = b, v = A p (preconditioned: ph = M^-1 p, v = A ph)
  double dots[4] = {0, 0, 0, 0};
  double rmax = 0;
  long long rmax_idx = 0;
  if constexpr (PC) {
    pc_forward<Q, float>(C32, pv, ps, A.pc, dst_, PC_INIT, dots);
    C32.acc = PA.Pr;
    pc_backward<Q, float>(C32, pv, ps, A.pc, dst_, pv.ph);
    set_dco(A.pj, cw, C32.L.dco, PA.Pr);
    __syncthreads();
    pc_apply<RAD, Q, float, false>(C32, pv, ps, dots);
  } else {
    // projections of b (entries at the source point only): Pr = Pp = B^H b
    zero_acc<double>(PA.Pr, ncw);
    __syncthreads();
    if (A.pj.nproj && tid < cw && S.state[tid] == 0) {
      const int c = tid;
      const long long src = S.src[c];
      for (int sl = 0; sl < SC_SLOTS; ++sl) {
        const size_t si = (size_t)src * SC_SLOTS + sl;
        const int pb = A.pj.sc_pb[si];
        if (pb < 0) continue;
        const double2 ph = A.pj.sc_eph[si];
        const cx<double> w = cscale(mkc(ph.x, -ph.y), S.bsc[c]);
        for (int m = 0; m < A.pj.nm && pb + m < A.pj.nproj; ++m) {
          const double b = A.pj.sc_beta[si * A.pj.nm + m];
          cx<double>* a = &PA.Pr[(size_t)(pb + m) * cw + c];
          *a = *a + cscale(w, b * A.pj.h3);
        }
      }
      for (int k = A.pj.pe_offs[src]; k < A.pj.pe_offs[src + 1]; ++k) {
        const int2 ge = A.pj.pe[k];
        const double2 ph = A.pj.eph[ge.y];
        const cx<double> w = cscale(mkc(ph.x, -ph.y), S.bsc[c]);
        for (int m = 0; m < A.pj.grp_nm[ge.x]; ++m) {
          const double b = A.pj.beta[(size_t)ge.y * A.pj.nm + m];
          cx<double>* a = &PA.Pr[(size_t)(A.pj.grp_pbase[ge.x] + m) * cw + c];
          *a = *a + cscale(w, b * A.pj.h3);
        }
      }
    }
    __syncthreads();
    for (int w = tid; w < ncw; w += blockDim.x) PA.Pp[w] = PA.Pr[w];
    set_dco(A.pj, cw, C32.L.dco, PA.Pr);
    __syncthreads();
    C32.acc = PA.Pv;
    sweep<RAD, Q, float>(C32, ps, IN_INIT, OUT_V, dots, rmax, rmax_idx);
  }
  if (tid < cw) S.rho[tid] = mkc(S.bsc[tid], 0.0);
  __syncthreads();

  const double d2max = A.delta * A.delta;
  bool all_done = false;
  int it = 0;
  while (!all_done) {
    if (!any_active(S, cw)) break;
    // every pass counts, breakdown passes included, so the loop is bounded
    if (it >= A.max_iter) {
      reliable_update<RAD, Q, PC>(A, C64, C32, pv, ps, PA, dst_, true, false, all_done);
      break;
    }
    ++it;
    // alpha = rho / (r^0, v)
    if (tid == 0) S.any_flag = 0;
    __syncthreads();
    if (tid < cw) {
      const int c = tid;
      S.alpha[c] = mkc(0.0, 0.0);
      if (S.state[c] == 0) {
        const cx<double> vj = S.vj[c];
        if (!(cnorm2(vj) > 0.0) || !finite2(vj) || !finite2(S.rho[c]))
          atomicOr(&S.any_flag, 1);
        else
          S.alpha[c] = cdiv(S.rho[c], vj);
      }
    }
    __syncthreads();
    if (S.any_flag) {
      reliable_update<RAD, Q, PC>(A, C64, C32, pv, ps, PA, dst_, false, true, all_done);
      continue;
    }
    // s = r - alpha v, t = A s (preconditioned: sh = M^-1 s, t = A sh); dots (t,s), (t,t)
    for (int k = 0; k < 4; ++k) dots[k] = 0;
    if constexpr (PC) {
      pc_forward<Q, float>(C32, pv, ps, A.pc, dst_, PC_S, dots);
      C32.acc = PA.Pp;
      pc_backward<Q, float>(C32, pv, ps, A.pc, dst_, pv.sh);
      set_dco(A.pj, cw, C32.L.dco, PA.Pp);
      __syncthreads();
      for (int k = 0; k < 4; ++k) dots[k] = 0;
      pc_apply<RAD, Q, float, true>(C32, pv, ps, dots);
    } else {
      for (int w = tid; w < ncw; w += blockDim.x) {
        const int c = w % cw;
        C32.L.dco[w] = cscale(PA.Pr[w] - cmul(S.alpha[c], PA.Pv[w]), A.pj.ekb[w / cw]);
      }
      __syncthreads();
      C32.acc = PA.Pt;
      sweep<RAD, Q, float>(C32, ps, IN_B, OUT_T, dots, rmax, rmax_idx);
    }
    {
      __shared__ double red_out[4][CW_MAX];
      col_reduce4(C32.L.red, cw, dots, red_out);
      if (tid == 0) S.any_flag = 0;
      __syncthreads();
      if (tid < cw) {
        const int c = tid;
        if (S.state[c] == 0) {
          const cx<double> ts = mkc(red_out[1][c], red_out[2][c]);
          const double tt = red_out[3][c];
          const cx<double> om = (tt > 0.0 && isfinite(tt)) ? cscale(ts, 1.0 / tt) : mkc(0.0, 0.0);
          const cx<double> rn = S.sj[c] - cmul(om, S.tj[c]);
          if (!(cnorm2(om) > 0.0) || !finite2(om) || !(cnorm2(rn) > 0.0) || !finite2(rn)) {
            atomicOr(&S.any_flag, 1);
            S.omega[c] = S.beta[c] = S.alpha[c] = mkc(0.0, 0.0);
          } else {
            S.omega[c] = om;
            S.rho_new[c] = rn;
            S.beta[c] = cmul(cdiv(rn, S.rho[c]), cdiv(S.alpha[c], om));
          }
        } else {
          S.omega[c] = S.beta[c] = S.alpha[c] = mkc(0.0, 0.0);
        }
      }
      __syncthreads();
    }
    if (S.any_flag) {
      reliable_update<RAD, Q, PC>(A, C64, C32, pv, ps, PA, dst_, false, true, all_done);
      continue;
    }
    // x += alpha p + omega s, r = s - omega t, p = r + beta (p - omega v), v = A p
    // (preconditioned: x += alpha ph + omega sh, v = A ph with ph = M^-1 p); ||r||^2
    for (int k = 0; k < 4; ++k) dots[k] = 0;
    if constexpr (PC) {
      pc_forward<Q, float>(C32, pv, ps, A.pc, dst_, PC_MERGED, dots);
      C32.acc = PA.Pr;
      pc_backward<Q, float>(C32, pv, ps, A.pc, dst_, pv.ph);
      set_dco(A.pj, cw, C32.L.dco, PA.Pr);
      __syncthreads();
      double d2[4] = {0, 0, 0, 0};
      pc_apply<RAD, Q, float, false>(C32, pv, ps, d2);
    } else {
      for (int w = tid; w < ncw; w += blockDim.x) {
        const int c = w % cw;
        const cx<double> al = S.alpha[c], om = S.omega[c], be = S.beta[c];
        const cx<double> Ps = PA.Pr[w] - cmul(al, PA.Pv[w]);
        const cx<double> Prn = Ps - cmul(om, PA.Pt[w]);
        const cx<double> Ppn = Prn + cmul(be, PA.Pp[w] - cmul(om, PA.Pv[w]));
        PA.Pr[w] = Prn;
        PA.Pp[w] = Ppn;
        C32.L.dco[w] = cscale(Ppn, A.pj.ekb[w / cw]);
      }
      __syncthreads();
      C32.acc = PA.Pv;
      sweep<RAD, Q, float>(C32, ps, IN_A, OUT_V, dots, rmax, rmax_idx);
    }
    {
      __shared__ double red_out[4][CW_MAX];
      col_reduce4(C32.L.red, cw, dots, red_out);
      if (tid == 0) S.any_flag = 0;
      __syncthreads();
      if (tid < cw) {
        const int c = tid;
        if (S.state[c] == 0) {
          S.iters[c] += 1;
          S.rho[c] = S.rho_new[c];
          const double rr = red_out[0][c];
          S.rr_rec[c] = rr;
          // replace the residual once it has fallen by delta below the largest
          // since the last replacement, or reached the tolerance; discard x32
          // and restart once it has diverged
          if (!isfinite(rr) || rr > DIVERGE2 * S.rr_upd[c]) {
            S.fold[c] = 0;
            atomicOr(&S.any_flag, 2);
          } else if (rr <= A.tol * A.tol * S.bb[c] || rr < d2max * S.maxrr[c]) {
            atomicOr(&S.any_flag, 1);
          } else if (S.iters[c] - S.it_upd[c] >= NOPROG_ITERS) {
            S.stall[c] = STALL_UPDATES - 1;  // the replacement below decides: FP64 unless it fell 100x
            atomicOr(&S.any_flag, 1);
          } else if (rr > S.maxrr[c]) {
            S.maxrr[c] = rr;
          }
        }
      }
      __syncthreads();
    }
    if (S.any_flag) {
      const bool rs = (S.any_flag & 2) != 0;
      reliable_update<RAD, Q, PC>(A, C64, C32, pv, ps, PA, dst_, false, rs, all_done);
    }
  }
  if (tid < cw) {
    const int c = tid;
    const int col = blk * cw + c;
    if (col < A.ncols) {
      const size_t o = (size_t)e_idx * A.ncols + col;
      A.T_col[o] = 4.0 * S.tacc[c];
      A.iters[o] = S.iters[c];
      A.restarts[o] = S.restarts[c];
      if (A.updates) A.updates[o] = S.updates[c];
      A.resid[o] = S.bb[c] > 0 ? sqrt(S.rr[c] / S.bb[c]) : 0.0;
      A.status[o] = S.state[c] == 1 ? 0 : (S.state[c] == 2 ? 2 : 1);
    }
  }
  if (A.xout) {
    __threadfence();  // x was stored by the position-owning threads; read here by another mapping
    __syncthreads();
    const size_t nall = (size_t)g.P * g.nz * cw;
    for (size_t w = tid; w < nall; w += blockDim.x) {
      const int c = (int)(w % cw);
      const size_t gi = w / cw;
      const int col = blk * cw + c;
      if (col < A.ncols) {
        const cx<double> xv = C64.vec.x[w];
        double2 o;
        o.x = xv.x;
        o.y = xv.y;
        A.xout[gi * ((size_t)A.ne * A.ncols) + (size_t)e_idx * A.ncols + col] = o;
      }
    }
  }
  __syncthreads();
}

template <int RAD, int Q, bool PC>
__global__ __launch_bounds__(MAX_T) RST_WAVES_ATTR void k_mixed(const SolveArgs* __restrict__ Ap) {
  const SolveArgs& A = *Ap;
  extern __shared__ __align__(16) char smem[];
  __shared__ ColState S;
  const int cw = A.cw;
  SweepCtx<double> C64;
  C64.g = &A.g;
  C64.pj = &A.pj;
  C64.V = A.V;
  C64.gz = A.gz;
  C64.cw = cw;
  C64.L = carve_lds<double>(smem, A.g, A.pj, cw, blockDim.x);
  C64.S = &S;
  C64.xext = nullptr;
  C64.yext = nullptr;
  C64.ext_ld = C64.ext_c0 = C64.ext_ncol = 0;
  C64.pcsrc = C64.pcs = nullptr;
  C64.r32 = nullptr;
  C64.rhs = nullptr;
  C64.rhs_ld = C64.rhs_c0 = 0;
  C64.rhs_nc = 0;
  SweepCtx<float> C32;
  C32.g = &A.g;
  C32.pj = &A.pj;
  C32.V = A.V;
  C32.gz = A.gz;
  C32.cw = cw;
  C32.L = carve_lds<float>(smem, A.g, A.pj, cw, blockDim.x);
  C32.S = &S;
  C32.xext = nullptr;
  C32.yext = nullptr;
  C32.ext_ld = C32.ext_c0 = C32.ext_ncol = 0;
  C32.pcsrc = C32.pcs = nullptr;
  C32.r32 = nullptr;
  C32.rhs = nullptr;
  C32.rhs_ld = C32.rhs_c0 = 0;
  C32.rhs_nc = 0;
  // workspace: FP64 x, then the FP32 vectors x r p v t (+ ph sh s w)
  const size_t nv = (size_t)A.g.P * A.g.nz * cw;
  cx<double>* b64 = reinterpret_cast<cx<double>*>(A.ws) + (size_t)blockIdx.x * A.ws_stride;
  C64.vec.x = b64;
  C64.vec.r = C64.vec.p = C64.vec.v = C64.vec.t = nullptr;
  cx<float>* b32 = reinterpret_cast<cx<float>*>(b64 + nv);
  C32.vec.x = b32;
  C32.vec.r = b32 + nv;
  C32.vec.p = b32 + 2 * nv;
  C32.vec.v = b32 + 3 * nv;
  C32.vec.t = b32 + 4 * nv;
  PcVecs<float> pv;
  pv.ph = b32 + 5 * nv;
  pv.sh = b32 + 6 * nv;
  pv.s = b32 + 7 * nv;
  pv.w = b32 + 8 * nv;
  pv.inv = nullptr;
  const size_t np = (size_t)A.pj.nproj * cw;
  cx<double>* pb = reinterpret_cast<cx<double>*>(A.pws) + (size_t)blockIdx.x * A.pws_stride;
  ProjArrays PA{pb, pb + np, pb + 2 * np, pb + 3 * np, pb + 4 * np};
  DftSteps dst_;
  dst_.fa = dst_.fb = dst_.ia = dst_.ib = dst_.pa = dst_.pb = nullptr;
  if constexpr (PC) {
    cx<double>* tab = reinterpret_cast<cx<double>*>(smem + A.pc_lds_off);
    const int ntab = 3 * (A.g.na + A.g.nb);
    for (int w = threadIdx.x; w < ntab; w += blockDim.x) {
      const double2 t = A.pc.steps[w];
      tab[w] = mkc(t.x, t.y);
    }
    dst_.fa = tab;
    dst_.fb = tab + A.g.na;
    dst_.ia = tab + A.g.na + A.g.nb;
    dst_.ib = tab + 2 * A.g.na + A.g.nb;
    dst_.pa = tab + 2 * A.g.na + 2 * A.g.nb;
    dst_.pb = tab + 3 * A.g.na + 2 * A.g.nb;
  }
  __syncthreads();
  const Pos<Q> ps = make_pos<Q>(A.g, cw, RAD);
  for (;;) {
    if (threadIdx.x == 0) S.item = atomicAdd(A.counter, 1);
    __syncthreads();
    const int item = S.item;
    if (item >= A.nitems) break;
    mixed_solve_item<RAD, Q, PC>(A, C64, C32, pv, ps, PA, dst_, item);
  }
}

}  // namespace rst
