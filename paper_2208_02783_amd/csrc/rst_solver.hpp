// rst_solver.hpp -- persistent BiCGSTAB kernel (one workgroup = one column
// block, start to finish) and the stand-alone apply kernel.
//
// BiCGSTAB (van der Vorst) with the shadow residual r^_0 = e_j0 (a unit vector,
// initially the column's source point), so (r^_0, w) = w[j0].  Each iteration
// is two sweeps:
//   sweep B: s = r - alpha v (formed on load), t = A s, dots (t,s), (t,t);
//   sweep A: x += alpha p + omega s, r = s - omega t, p = r + beta (p - omega v)
//            (all formed on load), v = A p, ||r||^2.
// beta needs rho' = r'[j0] = s[j0] - omega t[j0], which sweep B records, so the
// x/r/p updates of one iteration and the v = A p of the next share one sweep.
// Projections B^H w of the Krylov vectors are carried by the same recurrences;
// those of the apply outputs (v, t, r_true) are gathered from the output planes.
// Convergence is decided on the FP64 true residual b - A x (a fresh gather of x
// and a fresh apply); a column whose recursive residual reached tol but whose
// true residual did not, or a breakdown, restarts the block from the true
// residual with the shadow moved to argmax |r|.
#pragma once
#include "rst_sweep.hpp"

namespace rst {

template <class R>
__device__ __forceinline__ void zero_acc(cx<double>* a, int count) {
  for (int w = threadIdx.x; w < count; w += blockDim.x) a[w] = mkc(0.0, 0.0);
}

// dco = h3 * ekb * Pu  (per projector, per column)
__device__ __forceinline__ void set_dco(const Proj& pj, int cw, cx<double>* dco, const cx<double>* Pu) {
  for (int w = threadIdx.x; w < pj.nproj * cw; w += blockDim.x) {
    const int p = w / cw;
    dco[w] = cscale(Pu[w], pj.ekb[p]);
  }
}

// True while some column of the block still iterates (state 0); a block whose
// columns are all finished (e.g. every right-hand side zero) leaves its loop.
__device__ __forceinline__ bool any_active(ColState& S, int cw) {
  __syncthreads();
  if (threadIdx.x == 0) S.upd_flag = 0;
  __syncthreads();
  if ((int)threadIdx.x < cw && S.state[threadIdx.x] == 0) atomicOr(&S.upd_flag, 1);
  __syncthreads();
  return S.upd_flag != 0;
}

// Dense right-hand side of an item: point C at the item's columns, then one
// pass over b for ||b||^2, the shadow index j0 = argmax |b| (ties: smaller
// index), rho = b[j0] and, when `acc` is given, the projections B^H b.
template <int Q, class R>
__device__ __forceinline__ void rhs_scan(const SolveArgs& A, SweepCtx<R>& C, const Pos<Q>& ps, int e_idx, int blk,
                                         cx<double>* acc) {
  const Geo& g = *C.g;
  const Proj& pj = *C.pj;
  const int cw = C.cw;
  const int tid = threadIdx.x;
  const int c = tid % cw;
  ColState& S = *C.S;
  C.rhs = A.rhs;
  C.rhs_ld = A.rhs_ld;
  C.rhs_c0 = (long long)e_idx * A.rhs_estride + (long long)blk * cw;
  C.rhs_nc = min(cw, A.ncols - blk * cw);
  const bool any_g = pj.nproj > 0 && acc != nullptr;
  if (any_g) pacc_zero<R>(pj, C.L, cw);
  __syncthreads();
  double n2 = 0.0, bmax = -1.0;
  long long bidx = 0x7fffffffffffffffLL;
  for (int z = 0; z < g.nz; ++z) {
    const bool need_g = any_g && pj.zc_offs[z + 1] > pj.zc_offs[z];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] < 0) continue;
      const long long gi = (long long)z * g.P + ps.p[k];
      const cx<R> b = rhs_at<R>(C, gi, c);
      const double a2 = (double)cnorm2(b);
      n2 += a2;
      if (a2 > bmax || (a2 == bmax && gi < bidx)) {
        bmax = a2;
        bidx = gi;
      }
      if (need_g) C.L.outpl[ps.p[k] * cw + c] = b;
    }
    if (need_g) {
      __syncthreads();
      plane_gather<R>(z, pj, C.L, cw);
      __syncthreads();
    }
  }
  __syncthreads();
  if (any_g) {
    pacc_flush<R>(pj, C.L, cw, acc);
    __syncthreads();
  }
  double v4[4] = {n2, 0, 0, 0};
  __shared__ double red_out[4][CW_MAX];
  col_reduce4(C.L.red, cw, v4, red_out);
  double* bm = C.L.red;
  long long* bi = reinterpret_cast<long long*>(C.L.red + blockDim.x);
  bm[tid] = bmax;
  bi[tid] = bidx;
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
    S.src[tid] = -1;
    S.bb[tid] = red_out[0][tid];
    S.j0[tid] = ix;
    S.rj[tid] = (tid < C.rhs_nc && ix >= 0 && ix < (long long)g.P * g.nz) ? to64(rhs_at<R>(C, ix, tid))
                                                                          : mkc(0.0, 0.0);
    if (tid < C.rhs_nc && !(red_out[0][tid] > 0.0)) S.state[tid] = 1;  // b = 0: x = 0 is exact
  }
  __syncthreads();
}

template <int RAD, int Q, class R>
__device__ __forceinline__ void true_residual_and_restart(const SolveArgs& A, SweepCtx<R>& C, const Pos<Q>& ps,
                                          const ProjArrays& PA, bool final_check, bool& all_done) {
  ColState& S = *C.S;
  const int cw = A.cw;
  const int tid = threadIdx.x;
  const int ncw = A.pj.nproj * cw;
  // (1) gather x -> Px, T accumulator
  zero_acc<R>(PA.Px, ncw);
  __syncthreads();
  double tacc = 0.0;
  C.acc = PA.Px;
  gather_sweep<Q, R, false>(C, ps, A.gdst, tacc);
  {
    double v4[4] = {tacc, 0, 0, 0};
    __shared__ double red_out[4][CW_MAX];
    col_reduce4(C.L.red, cw, v4, red_out);
    if (tid < cw) S.tacc[tid] = red_out[0][tid];
  }
  // (2) r = b - A x, gathered into Pr
  set_dco(A.pj, cw, C.L.dco, PA.Px);
  zero_acc<R>(PA.Pr, ncw);
  __syncthreads();
  double dots[4] = {0, 0, 0, 0};
  double rmax = -1.0;
  long long rmax_idx = 0x7fffffffffffffffLL;
  C.acc = PA.Pr;
  sweep<RAD, Q, R>(C, ps, IN_X, OUT_RES, dots, rmax, rmax_idx);
  {
    __shared__ double red_out[4][CW_MAX];
    col_reduce4(C.L.red, cw, dots, red_out);
    // argmax |r| per column (ties: smaller index); scratch aliases the reduction buffer
    double* bm = C.L.red;
    long long* bi = reinterpret_cast<long long*>(C.L.red + blockDim.x);
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
      S.rmax[tid] = m;
      S.rmax_idx[tid] = ix;
    }
    __syncthreads();
  }
  // (3) decide
  if (tid == 0) S.any_flag = 0;
  __syncthreads();
  if (tid < cw) {
    const int c = tid;
    if (S.state[c] == 0) {
      const double rr = S.rr[c];
      if (!isfinite(rr)) {
        S.state[c] = 2;
      } else if (rr <= A.tol * A.tol * S.bb[c]) {
        S.state[c] = 1;
      } else if (final_check) {
        S.state[c] = 4;  // out of iterations
      } else {
        S.j0[c] = S.rmax_idx[c];
        S.restarts[c] += 1;
        atomicOr(&S.any_flag, 1);
      }
    }
  }
  __syncthreads();
  all_done = (S.any_flag == 0);
  if (all_done) return;
  // (4) restart: p = r, v = A p
  for (int w = tid; w < ncw; w += blockDim.x) PA.Pp[w] = PA.Pr[w];
  set_dco(A.pj, cw, C.L.dco, PA.Pr);
  zero_acc<R>(PA.Pv, ncw);
  __syncthreads();
  double d2[4] = {0, 0, 0, 0};
  C.acc = PA.Pv;
  sweep<RAD, Q, R>(C, ps, IN_RESTART, OUT_V, d2, rmax, rmax_idx);
  if (tid < cw) S.rho[tid] = S.rj[tid];
  __syncthreads();
}

template <int RAD, int Q, class R>
__device__ __forceinline__ void solve_item(const SolveArgs& A, SweepCtx<R>& C, const Pos<Q>& ps,
                           const ProjArrays& PA, int item) {
  ColState& S = *C.S;
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
    S.tacc[c] = 0.0;
    S.rr[c] = 0.0;
    if (col < A.ncols) {
      const long long src = A.cols[col];
      S.src[c] = src;
      S.j0[c] = src;
      const double gs = A.gsrc ? A.gsrc[src / A.g.P] : 1.0;
      S.bsc[c] = sqrt(gs);
      S.bb[c] = gs;
      S.state[c] = 0;
    } else {
      S.src[c] = -1;
      S.j0[c] = -1;
      S.bsc[c] = 0.0;
      S.bb[c] = 0.0;
      S.state[c] = 3;
    }
  }
  __syncthreads();
  // projections of b: Pr = Pp = h3-free B^H b (only entries at the source point)
  zero_acc<R>(PA.Pr, ncw);
  zero_acc<R>(PA.Pv, ncw);
  __syncthreads();
  if (A.rhs) rhs_scan<Q, R>(A, C, ps, e_idx, blk, PA.Pr);
  if (A.pj.nproj && tid < cw && S.state[tid] == 0 && !A.rhs) {
    const int c = tid;
    const long long src = S.src[c];
    // slot-table entries of the source point
    for (int sl = 0; sl < SC_SLOTS; ++sl) {
      const size_t si = (size_t)src * SC_SLOTS + sl;
      const int pb = A.pj.sc_pb[si];
      if (pb < 0) continue;
      const double2 ph = A.pj.sc_eph[si];
      const cx<double> w = cscale(mkc(ph.x, -ph.y), S.bsc[c]);
      for (int m = 0; m < A.pj.nm && pb + m < A.pj.nproj; ++m) {
        const double b = A.pj.sc_beta[si * A.pj.nm + m];  // zero past the group's projectors
        cx<double>* a = &PA.Pr[(size_t)(pb + m) * cw + c];
        *a = *a + cscale(w, b * A.pj.h3);
      }
    }
    // overflow entries
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
  set_dco(A.pj, cw, C.L.dco, PA.Pr);
  __syncthreads();
  double dots[4] = {0, 0, 0, 0};
  double rmax = 0;
  long long rmax_idx = 0;
  C.acc = PA.Pv;
  sweep<RAD, Q, R>(C, ps, IN_INIT, OUT_V, dots, rmax, rmax_idx);
  if (tid < cw) S.rho[tid] = A.rhs ? S.rj[tid] : mkc(S.bsc[tid], 0.0);
  __syncthreads();

  bool all_done = false;
  int it = 0;
  while (!all_done) {
    if (!any_active(S, cw)) break;
    // every pass counts, breakdown passes included, so the loop is bounded
    if (it >= A.max_iter) {
      true_residual_and_restart<RAD, Q, R>(A, C, ps, PA, true, all_done);
      break;
    }
    ++it;
    // alpha = rho / (r^0, v)
    if (tid == 0) S.any_flag = 0;
    __syncthreads();
    if (tid < cw) {
      const int c = tid;
      if (S.state[c] == 0) {
        const cx<double> vj = S.vj[c];
        if (!(cnorm2(vj) > 0.0) || !finite2(vj) || !finite2(S.rho[c])) {
          atomicOr(&S.any_flag, 1);
          S.alpha[c] = mkc(0.0, 0.0);
        } else {
          S.alpha[c] = cdiv(S.rho[c], vj);
        }
      } else {
        S.alpha[c] = mkc(0.0, 0.0);
      }
    }
    __syncthreads();
    if (S.any_flag) {
      true_residual_and_restart<RAD, Q, R>(A, C, ps, PA, false, all_done);
      continue;
    }
    // sweep B: s = r - alpha v, t = A s
    for (int w = tid; w < ncw; w += blockDim.x) {
      const int c = w % cw;
      const cx<double> ps_ = PA.Pr[w] - cmul(S.alpha[c], PA.Pv[w]);
      C.L.dco[w] = cscale(ps_, A.pj.ekb[w / cw]);
    }
    zero_acc<R>(PA.Pt, ncw);
    __syncthreads();
    for (int k = 0; k < 4; ++k) dots[k] = 0;
    C.acc = PA.Pt;
    sweep<RAD, Q, R>(C, ps, IN_B, OUT_T, dots, rmax, rmax_idx);
    {
      __shared__ double red_out[4][CW_MAX];
      col_reduce4(C.L.red, cw, dots, red_out);
      if (tid == 0) S.any_flag = 0;
      __syncthreads();
      if (tid < cw) {
        const int c = tid;
        S.ts[c] = mkc(red_out[1][c], red_out[2][c]);
        S.tt[c] = red_out[3][c];
        if (S.state[c] == 0) {
          const double tt = S.tt[c];
          const cx<double> om = (tt > 0.0 && isfinite(tt)) ? cscale(S.ts[c], 1.0 / tt) : mkc(0.0, 0.0);
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
      true_residual_and_restart<RAD, Q, R>(A, C, ps, PA, false, all_done);
      continue;
    }
    // projections of s, r', p'
    for (int w = tid; w < ncw; w += blockDim.x) {
      const int c = w % cw;
      const cx<double> al = S.alpha[c], om = S.omega[c], be = S.beta[c];
      const cx<double> Ps = PA.Pr[w] - cmul(al, PA.Pv[w]);
      const cx<double> Prn = Ps - cmul(om, PA.Pt[w]);
      const cx<double> Ppn = Prn + cmul(be, PA.Pp[w] - cmul(om, PA.Pv[w]));
      PA.Pr[w] = Prn;
      PA.Pp[w] = Ppn;
      C.L.dco[w] = cscale(Ppn, A.pj.ekb[w / cw]);
    }
    __syncthreads();
    zero_acc<R>(PA.Pv, ncw);
    __syncthreads();
    for (int k = 0; k < 4; ++k) dots[k] = 0;
    C.acc = PA.Pv;
    sweep<RAD, Q, R>(C, ps, IN_A, OUT_V, dots, rmax, rmax_idx);
    {
      __shared__ double red_out[4][CW_MAX];
      col_reduce4(C.L.red, cw, dots, red_out);
      if (tid == 0) S.any_flag = 0;
      __syncthreads();
      if (tid < cw) {
        const int c = tid;
        if (S.state[c] == 0) {
          S.iters[c] += 1;
          S.rho[c] = S.rho_new[c];
          const double rr = red_out[0][c];
          S.rr[c] = rr;
          if (!isfinite(rr) || rr <= A.tol * A.tol * S.bb[c]) atomicOr(&S.any_flag, 1);
        }
      }
      __syncthreads();
    }
    if (S.any_flag) true_residual_and_restart<RAD, Q, R>(A, C, ps, PA, false, all_done);
  }
  // outputs
  if (tid < cw) {
    const int c = tid;
    const int col = blk * cw + c;
    if (col < A.ncols) {
      const size_t o = (size_t)e_idx * A.ncols + col;
      A.T_col[o] = 4.0 * S.tacc[c];
      A.iters[o] = S.iters[c];
      A.restarts[o] = S.restarts[c];
      A.resid[o] = S.bb[c] > 0 ? sqrt(S.rr[c] / S.bb[c]) : 0.0;
      A.status[o] = S.state[c] == 1 ? 0 : (S.state[c] == 2 ? 2 : 1);
    }
  }
  if (A.xout) {
    __threadfence();  // x was stored by the position-owning threads; read here by another mapping
    __syncthreads();
    const Geo& g = A.g;
    const size_t nall = (size_t)g.P * g.nz * cw;
    for (size_t w = tid; w < nall; w += blockDim.x) {
      const int c = (int)(w % cw);
      const size_t gi = w / cw;
      const int col = blk * cw + c;
      if (col < A.ncols) {
        const cx<R> xv = C.vec.x[w];
        double2 o;
        o.x = (double)xv.x;
        o.y = (double)xv.y;
        A.xout[gi * ((size_t)A.ne * A.ncols) + (size_t)e_idx * A.ncols + col] = o;
      }
    }
  }
  __syncthreads();
}

// Arguments of one item of a batched launch: the structure that owns `item`
// (the last whose first item is <= item), its grid depth, Bloch phases,
// potential, CAPs, energies, columns and output slices (and, with PC, its
// preconditioner tables).  Returns the item's index within its structure.
template <bool PC>
__device__ inline int batch_item_args(const SolveArgs& A, int item, SolveArgs& Ai) {
  int lo = 0, hi = A.nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (A.batch[mid].item0 <= item) lo = mid; else hi = mid - 1;
  }
  const BatchProb bp = A.batch[lo];
  Ai = A;
  Ai.g.nz = bp.nz;
  Ai.g.pha_x = bp.pha_x;
  Ai.g.pha_y = bp.pha_y;
  Ai.g.phb_x = bp.phb_x;
  Ai.g.phb_y = bp.phb_y;
  Ai.V = A.V + bp.v_off;
  Ai.gz = A.gz + bp.gz_off;
  Ai.gdst = A.gdst + bp.gz_off;
  Ai.gsrc = A.gsrc + bp.gz_off;
  Ai.energies = A.energies + bp.e_off;
  Ai.cols = A.cols + bp.col_off;
  Ai.ncols = bp.ncols;
  Ai.nblk = bp.nblk;
  Ai.ne = bp.ne;
  Ai.T_col = A.T_col + bp.out_off;
  Ai.iters = A.iters + bp.out_off;
  Ai.restarts = A.restarts + bp.out_off;
  Ai.resid = A.resid + bp.out_off;
  Ai.status = A.status + bp.out_off;
  if constexpr (PC) {
    Ai.pc.vbar = bp.vbar;
    Ai.pc.eps = A.pc.eps + bp.eps_off;
    Ai.pc.steps = A.pc.steps + bp.steps_off;
    Ai.pc.inv = A.pc.inv + bp.inv_off;
  }
  return item - bp.item0;
}

// BATCH: items belong to the structures of A.batch (a separate instance, so
// the single-structure kernel carries one copy of the solve body).
template <int RAD, int Q, class R, bool BATCH>
__global__ __launch_bounds__(MAX_T) RST_WAVES_ATTR void k_bicgstab(const SolveArgs* __restrict__ Ap) {
  const SolveArgs& A = *Ap;
  extern __shared__ __align__(16) char smem[];
  __shared__ ColState S;
  const int cw = A.cw;
  SweepCtx<R> C;
  C.g = &A.g;
  C.pj = &A.pj;
  C.V = A.V;
  C.gz = A.gz;
  C.cw = cw;
  C.L = carve_lds<R>(smem, A.g, A.pj, cw, blockDim.x);
  C.S = &S;
  C.xext = nullptr;
  C.yext = nullptr;
  C.ext_ld = C.ext_c0 = C.ext_ncol = 0;
  C.pcsrc = C.pcs = nullptr;
  C.r32 = nullptr;
  C.rhs = nullptr;
  C.rhs_ld = C.rhs_c0 = 0;
  C.rhs_nc = 0;
  const size_t nv = (size_t)A.g.P * A.g.nz * cw;
  cx<R>* base = reinterpret_cast<cx<R>*>(A.ws) + (size_t)blockIdx.x * A.ws_stride;
  C.vec.x = base;
  C.vec.r = base + nv;
  C.vec.p = base + 2 * nv;
  C.vec.v = base + 3 * nv;
  C.vec.t = base + 4 * nv;
  const size_t np = (size_t)A.pj.nproj * cw;
  cx<double>* pb = reinterpret_cast<cx<double>*>(A.pws) + (size_t)blockIdx.x * A.pws_stride;
  ProjArrays PA{pb, pb + np, pb + 2 * np, pb + 3 * np, pb + 4 * np};
  const Pos<Q> ps = make_pos<Q>(A.g, cw, RAD);
  for (;;) {
    if (threadIdx.x == 0) S.item = atomicAdd(A.counter, 1);
    __syncthreads();
    const int item = S.item;
    if (item >= A.nitems) break;
    if constexpr (BATCH) {
      __shared__ SolveArgs Ai;  // per-item arguments of a batched launch
      __shared__ int local_item;
      if (threadIdx.x == 0) local_item = batch_item_args<false>(A, item, Ai);
      __syncthreads();
      C.g = &Ai.g;
      C.V = Ai.V;
      C.gz = Ai.gz;
      solve_item<RAD, Q, R>(Ai, C, ps, PA, local_item);
    } else {
      solve_item<RAD, Q, R>(A, C, ps, PA, item);
    }
  }
}

// y = (E - H_k + i Gamma) x on blocked vectors (the solvers' layout), one
// workgroup per column block: a gather sweep forms B^H x of the block (unless
// k_proj_mm has already put the projections in the block's pws array), then
// the stencil sweep applies the rest and scatters the projector part.
template <int RAD, int Q, class R>
__global__ __launch_bounds__(MAX_T) void k_apply(const ApplyArgs* __restrict__ Ap) {
  const ApplyArgs& A = *Ap;
  extern __shared__ __align__(16) char smem[];
  __shared__ ColState S;
  const int cw = A.cw;
  SweepCtx<R> C;
  C.g = &A.g;
  C.pj = &A.pj;
  C.V = A.V;
  C.gz = A.gz;
  C.cw = cw;
  C.L = carve_lds<R>(smem, A.g, A.pj, cw, blockDim.x);
  C.S = &S;
  const size_t boff = (size_t)blockIdx.x * A.g.P * A.g.nz * cw;
  C.xext = A.x + boff;
  C.yext = A.y + boff;
  C.ext_ld = cw;
  C.ext_c0 = 0;
  C.ext_ncol = cw;
  C.vec = Vecs<R>{nullptr, nullptr, nullptr, nullptr, nullptr};
  C.pcsrc = C.pcs = nullptr;
  C.r32 = nullptr;
  C.rhs = nullptr;
  C.rhs_ld = C.rhs_c0 = 0;
  C.rhs_nc = 0;
  const int tid = threadIdx.x;
  if (tid < cw) {
    S.energy[tid] = A.energy;
    S.alpha[tid] = S.omega[tid] = S.beta[tid] = mkc(0.0, 0.0);
    S.bsc[tid] = 0;
    S.src[tid] = -1;
    S.j0[tid] = -1;
  }
  const size_t np = (size_t)A.pj.nproj * cw;
  cx<double>* Px = reinterpret_cast<cx<double>*>(A.pws) + (size_t)blockIdx.x * A.pws_stride;
  if (!A.proj_pre) zero_acc<R>(Px, (int)np);
  __syncthreads();
  const Pos<Q> ps = make_pos<Q>(A.g, cw, RAD);
  double tacc = 0;
  if (A.pj.nproj && !A.proj_pre) {
    C.acc = Px;
    gather_sweep<Q, R, true>(C, ps, nullptr, tacc);
  }
  set_dco(A.pj, cw, C.L.dco, Px);
  __syncthreads();
  double dots[4] = {0, 0, 0, 0};
  double rmax = 0;
  long long ri = 0;
  C.acc = nullptr;
  sweep<RAD, Q, R>(C, ps, IN_EXT, OUT_EXT, dots, rmax, ri);
}

}  // namespace rst
