// rst_precond.hpp -- free-electron + CAP right preconditioner and the
// right-preconditioned BiCGSTAB workgroup solver.
//
// M = E - (-1/2 L_lat - 1/2 D2_z + Vbar) + i Gamma(z): the lateral part is the
// exact order-2M lateral Laplacian of the operator, diagonal in the twisted
// lateral Fourier basis exp(i (k + 2 pi m / L) x) (Bloch-form equation), the
// z part is the second-order three-point Laplacian with the CAP on its diagonal
// (Gaussian-CAP equation: Gamma depends on z only, so lateral modes never mix),
// and Vbar is the cell-mean potential.  M^-1 u is a lateral DFT of every plane,
// one tridiagonal solve along z per lateral mode (Thomas recursion; the CAP
// keeps every pivot away from zero), and the inverse DFT.  The forward
// elimination streams z upwards, the back substitution downwards, so each is
// one sweep of the plane-streaming workgroup.
#pragma once
#include "rst_solver.hpp"

namespace rst {

enum PcIn { PC_INIT, PC_MERGED, PC_RESTART, PC_S, PC_IN };

template <class R>
struct PcVecs {
  cx<R>* ph;   // M^-1 p
  cx<R>* sh;   // M^-1 s
  cx<R>* s;
  cx<R>* w;    // forward-eliminated values in mode space
  const cx<double>* inv;  // [nz*P] reciprocal Thomas pivots of the current item's energy
};

// Lateral DFT of the plane held in the positions' values u[k] -> modes out[k].
// Forward kernel exp(-2 pi i m a / N) exp(-i k a h): for the sum over a at
// fixed m it is the a-th power of w_m = exp(-i (2 pi m / N + k h)); the inverse
// sum over m at fixed a uses conj(exp(-2 pi i m a / N)) = v_a^m with
// v_a = exp(+2 pi i a / N), times exp(+i k a h).  Every sum therefore runs a
// register recurrence t <- t * step instead of reading twiddles.
// step tables (LDS): fa[ma] = w_ma, fb[mb] = w_mb, ia[a] = v_a, ib[b] = v_b,
// pa[a] = exp(+i k_a a h_a), pb[b] = exp(+i k_b b h_b).
// Forward: unnormalised; inverse: with 1/(Na Nb).
struct DftSteps {
  const cx<double>* fa;
  const cx<double>* fb;
  const cx<double>* ia;
  const cx<double>* ib;
  const cx<double>* pa;
  const cx<double>* pb;
};

template <int Q, class R>
__device__ __forceinline__ void lateral_dft(const Geo& g, const Pos<Q>& ps, int cw, cx<R>* b0, cx<R>* b1,
                                            const DftSteps& st, bool inverse, const cx<R> (&u)[Q],
                                            cx<R> (&out)[Q]) {
  const int na = g.na, nb = g.nb;
  const int c = threadIdx.x % cw;
  const size_t rs = (size_t)na * cw;  // row stride of the plane buffers
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (ps.p[k] >= 0) b0[ps.p[k] * cw + c] = u[k];
  __syncthreads();
  if (!inverse) {
    // pass A along a: g(ma, b) = sum_a w_ma^a f(a, b)
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] >= 0) {
        const int ma = ps.p[k] % na, b = ps.p[k] / na;
        const cx<double> w = st.fa[ma];
        cx<double> t = mkc(1.0, 0.0), s = mkc(0.0, 0.0);
        const cx<R>* row = b0 + b * rs + c;
        for (int a = 0; a < na; ++a) {
          s = s + cmul(t, to64(row[a * cw]));
          t = cmul(t, w);
        }
        b1[ps.p[k] * cw + c] = fromd<R>(s);
      }
    }
    __syncthreads();
    // pass B along b: F(ma, mb) = sum_b w_mb^b g(ma, b)
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] >= 0) {
        const int ma = ps.p[k] % na, mb = ps.p[k] / na;
        const cx<double> w = st.fb[mb];
        cx<double> t = mkc(1.0, 0.0), s = mkc(0.0, 0.0);
        const cx<R>* col = b1 + ma * cw + c;
        for (int b = 0; b < nb; ++b) {
          s = s + cmul(t, to64(col[b * rs]));
          t = cmul(t, w);
        }
        out[k] = fromd<R>(s);
      }
    }
  } else {
    // pass A' along ma: h(a, mb) = exp(i k_a a h) sum_ma v_a^ma F(ma, mb)
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] >= 0) {
        const int a = ps.p[k] % na, mb = ps.p[k] / na;
        const cx<double> v = st.ia[a];
        cx<double> t = mkc(1.0, 0.0), s = mkc(0.0, 0.0);
        const cx<R>* row = b0 + mb * rs + c;
        for (int ma = 0; ma < na; ++ma) {
          s = s + cmul(t, to64(row[ma * cw]));
          t = cmul(t, v);
        }
        b1[ps.p[k] * cw + c] = fromd<R>(cmul(st.pa[a], s));
      }
    }
    __syncthreads();
    // pass B' along mb: f(a, b) = exp(i k_b b h) / (Na Nb) sum_mb v_b^mb h(a, mb)
    const double inv_p = 1.0 / (double)(na * nb);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] >= 0) {
        const int a = ps.p[k] % na, b = ps.p[k] / na;
        const cx<double> v = st.ib[b];
        cx<double> t = mkc(1.0, 0.0), s = mkc(0.0, 0.0);
        const cx<R>* col = b1 + a * cw + c;
        for (int mb = 0; mb < nb; ++mb) {
          s = s + cmul(t, to64(col[mb * rs]));
          t = cmul(t, v);
        }
        out[k] = fromd<R>(cscale(cmul(st.pb[b], s), inv_p));
      }
    }
  }
  __syncthreads();
}

// Forward sweep: form the input plane by plane (per mode), lateral DFT, Thomas
// elimination into pv.w.
template <int Q, class R>
__device__ __forceinline__ void pc_forward(SweepCtx<R>& C, const PcVecs<R>& pv, const Pos<Q>& ps,
                                           const PcConst& K, const DftSteps& dst_,
                                           int IN, double (&dots)[4]) {
  const Geo& g = *C.g;
  const int cw = C.cw;
  const int c = threadIdx.x % cw;
  ColState* S = C.S;
  const cx<R> al = fromd<R>(S->alpha[c]);
  const cx<R> om = fromd<R>(S->omega[c]);
  const cx<R> be = fromd<R>(S->beta[c]);
  const long long j0 = S->j0[c];
  const R a = (R)K.a;
  cx<R> dprev[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) dprev[k] = mkc<R>((R)0, (R)0);
  for (int z = 0; z < g.nz; ++z) {
    cx<R> u[Q], f[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      u[k] = mkc<R>((R)0, (R)0);
      if (ps.p[k] < 0) continue;
      const long long gi = (long long)z * g.P + ps.p[k];
      const size_t off = (size_t)gi * cw + c;
      if (IN == PC_INIT) {
        const cx<R> bb = rhs_at<R>(C, gi, c);
        stv(&C.vec.x[off], mkc<R>((R)0, (R)0));
        stv(&C.vec.r[off], bb);
        stv(&C.vec.p[off], bb);
        u[k] = bb;
      } else if (IN == PC_MERGED) {
        const cx<R> xv = ldv(&C.vec.x[off]), phv = ldv(&pv.ph[off]), shv = ldv(&pv.sh[off]),
                    sv = ldv(&pv.s[off]);
        const cx<R> tv = ldv(&C.vec.t[off]), pvv = ldv(&C.vec.p[off]), vv = ldv(&C.vec.v[off]);
        const cx<R> xn = xv + cmul(al, phv) + cmul(om, shv);
        const cx<R> rn = sv - cmul(om, tv);
        const cx<R> pn = rn + cmul(be, pvv - cmul(om, vv));
        stv(&C.vec.x[off], xn);
        stv(&C.vec.r[off], rn);
        stv(&C.vec.p[off], pn);
        dots[0] += (double)cnorm2(rn);
        u[k] = pn;
      } else if (IN == PC_RESTART) {
        const cx<R> rv = ldv(&C.vec.r[off]);
        stv(&C.vec.p[off], rv);
        if (gi == j0) S->rj[c] = to64(rv);
        u[k] = rv;
      } else if (IN == PC_IN) {
        u[k] = ldv(&C.vec.r[off]);
      } else {  // PC_S
        const cx<R> sv = ldv(&C.vec.r[off]) - cmul(al, ldv(&C.vec.v[off]));
        stv(&pv.s[off], sv);
        if (gi == j0) S->sj[c] = to64(sv);
        u[k] = sv;
      }
    }
    lateral_dft<Q, R>(g, ps, cw, C.L.inpl0, C.L.inpl1, dst_, false, u, f);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] < 0) continue;
      const size_t mi = (size_t)z * g.P + ps.p[k];
      const cx<R> iv = fromd<R>(pv.inv[mi]);
      const cx<R> d = cmul(f[k] - cscale(dprev[k], a), iv);
      stv(&pv.w[mi * cw + c], d);
      dprev[k] = d;
    }
  }
  __syncthreads();
}

// Backward sweep: back substitution, inverse DFT, write dst, gather into acc.
template <int Q, class R>
__device__ __forceinline__ void pc_backward(SweepCtx<R>& C, const PcVecs<R>& pv, const Pos<Q>& ps,
                                            const PcConst& K, const DftSteps& dst_,
                                            cx<R>* dst) {
  const Geo& g = *C.g;
  const Proj& pj = *C.pj;
  const int cw = C.cw;
  const int c = threadIdx.x % cw;
  const R a = (R)K.a;
  const bool do_gather = pj.nproj > 0 && C.acc != nullptr;
  if (do_gather) pacc_zero<R>(pj, C.L, cw);
  cx<R> xnext[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) xnext[k] = mkc<R>((R)0, (R)0);
  for (int z = g.nz - 1; z >= 0; --z) {
    cx<R> m[Q], u[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      m[k] = mkc<R>((R)0, (R)0);
      if (ps.p[k] < 0) continue;
      const size_t mi = (size_t)z * g.P + ps.p[k];
      const cx<R> d = ldv(&pv.w[mi * cw + c]);
      const cx<R> iv = fromd<R>(pv.inv[mi]);
      const cx<R> xv = d - cscale(cmul(iv, xnext[k]), a);
      xnext[k] = xv;
      m[k] = xv;
    }
    lateral_dft<Q, R>(g, ps, cw, C.L.inpl0, C.L.inpl1, dst_, true, m, u);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ps.p[k] < 0) continue;
      const size_t off = ((size_t)z * g.P + ps.p[k]) * cw + c;
      stv(&dst[off], u[k]);
      if (do_gather) C.L.outpl[ps.p[k] * cw + c] = u[k];
    }
    if (do_gather) {
      __syncthreads();
      plane_gather<R>(z, pj, C.L, cw);
      __syncthreads();
    }
  }
  __syncthreads();
  if (do_gather) {
    pacc_flush<R>(pj, C.L, cw, C.acc);
    __syncthreads();
  }
}

// Apply sweep of the preconditioned path: y = A u with u = ph (-> v) or sh (-> t).
template <int RAD, int Q, class R, bool TS>
__device__ __forceinline__ void pc_apply(SweepCtx<R>& C, const PcVecs<R>& pv, const Pos<Q>& ps,
                                         double (&dots)[4]) {
  double rmax = 0;
  long long ri = 0;
  C.acc = nullptr;
  C.pcsrc = TS ? pv.sh : pv.ph;
  C.pcs = pv.s;
  if constexpr (TS)
    sweep<RAD, Q, R>(C, ps, IN_PC, OUT_TS, dots, rmax, ri);
  else
    sweep<RAD, Q, R>(C, ps, IN_PC, OUT_V, dots, rmax, ri);
}

template <int RAD, int Q, class R>
__device__ __forceinline__ void pc_true_residual_and_restart(const SolveArgs& A, SweepCtx<R>& C,
                                                             const PcVecs<R>& pv, const Pos<Q>& ps,
                                                             const ProjArrays& PA, const PcConst& K,
                                                             const DftSteps& dst_, bool final_check,
                                                             bool& all_done) {
  ColState& S = *C.S;
  const int cw = A.cw;
  const int tid = threadIdx.x;
  const int ncw = A.pj.nproj * cw;
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
  set_dco(A.pj, cw, C.L.dco, PA.Px);
  __syncthreads();
  double dots[4] = {0, 0, 0, 0};
  double rmax = -1.0;
  long long rmax_idx = 0x7fffffffffffffffLL;
  C.acc = nullptr;
  sweep<RAD, Q, R>(C, ps, IN_X, OUT_RES, dots, rmax, rmax_idx);
  {
    __shared__ double red_out[4][CW_MAX];
    col_reduce4(C.L.red, cw, dots, red_out);
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
      S.rmax_idx[tid] = ix;
    }
    __syncthreads();
  }
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
        S.state[c] = 4;
      } else {
        S.j0[c] = S.rmax_idx[c];
        S.restarts[c] += 1;
        S.rrmin[c] = rr;
        atomicOr(&S.any_flag, 1);
      }
    }
  }
  __syncthreads();
  all_done = (S.any_flag == 0);
  if (all_done) return;
  // restart: p = r, ph = M^-1 p, v = A ph
  double d2[4] = {0, 0, 0, 0};
  pc_forward<Q, R>(C, pv, ps, K, dst_, PC_RESTART, d2);
  zero_acc<R>(PA.Pr, ncw);
  __syncthreads();
  C.acc = PA.Pr;
  pc_backward<Q, R>(C, pv, ps, K, dst_, pv.ph);
  set_dco(A.pj, cw, C.L.dco, PA.Pr);
  __syncthreads();
  pc_apply<RAD, Q, R, false>(C, pv, ps, d2);
  if (tid < cw) S.rho[tid] = S.rj[tid];
  __syncthreads();
}

template <int RAD, int Q, class R>
__device__ __forceinline__ void pc_solve_item(const SolveArgs& A, SweepCtx<R>& C, PcVecs<R>& pv,
                                              const Pos<Q>& ps, const ProjArrays& PA, const PcConst& K,
                                              const DftSteps& dst_, int item) {
  ColState& S = *C.S;
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
    S.rrmin[c] = HUGE_VAL;
    S.tacc[c] = 0.0;
    S.rr[c] = 0.0;
    if (col < A.ncols) {
      const long long src = A.cols[col];
      S.src[c] = src;
      S.j0[c] = src;
      const double gs = A.gsrc ? A.gsrc[src / g.P] : 1.0;
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
  // this item's energy selects its slice of the shared Thomas pivots
  pv.inv = reinterpret_cast<const cx<double>*>(K.inv) + (size_t)e_idx * g.nz * g.P;
  __syncthreads();
  if (A.rhs) rhs_scan<Q, R>(A, C, ps, e_idx, blk, nullptr);
  double dots[4] = {0, 0, 0, 0};
  pc_forward<Q, R>(C, pv, ps, K, dst_, PC_INIT, dots);
  zero_acc<R>(PA.Pr, ncw);
  __syncthreads();
  C.acc = PA.Pr;
  pc_backward<Q, R>(C, pv, ps, K, dst_, pv.ph);
  set_dco(A.pj, cw, C.L.dco, PA.Pr);
  __syncthreads();
  pc_apply<RAD, Q, R, false>(C, pv, ps, dots);
  if (tid < cw) S.rho[tid] = A.rhs ? S.rj[tid] : mkc(S.bsc[tid], 0.0);
  __syncthreads();

  bool all_done = false;
  int it = 0;
  while (!all_done) {
    if (!any_active(S, cw)) break;
    if (it >= A.max_iter) {
      pc_true_residual_and_restart<RAD, Q, R>(A, C, pv, ps, PA, K, dst_, true, all_done);
      break;
    }
    ++it;
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
      pc_true_residual_and_restart<RAD, Q, R>(A, C, pv, ps, PA, K, dst_, false, all_done);
      continue;
    }
    // s = r - alpha v, sh = M^-1 s, t = A sh
    for (int k = 0; k < 4; ++k) dots[k] = 0;
    pc_forward<Q, R>(C, pv, ps, K, dst_, PC_S, dots);
    zero_acc<R>(PA.Pp, ncw);
    __syncthreads();
    C.acc = PA.Pp;
    pc_backward<Q, R>(C, pv, ps, K, dst_, pv.sh);
    set_dco(A.pj, cw, C.L.dco, PA.Pp);
    __syncthreads();
    for (int k = 0; k < 4; ++k) dots[k] = 0;
    pc_apply<RAD, Q, R, true>(C, pv, ps, dots);
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
      pc_true_residual_and_restart<RAD, Q, R>(A, C, pv, ps, PA, K, dst_, false, all_done);
      continue;
    }
    // x += alpha ph + omega sh, r = s - omega t, p = r + beta (p - omega v); ph = M^-1 p; v = A ph
    for (int k = 0; k < 4; ++k) dots[k] = 0;
    pc_forward<Q, R>(C, pv, ps, K, dst_, PC_MERGED, dots);
    zero_acc<R>(PA.Pr, ncw);
    __syncthreads();
    C.acc = PA.Pr;
    pc_backward<Q, R>(C, pv, ps, K, dst_, pv.ph);
    set_dco(A.pj, cw, C.L.dco, PA.Pr);
    __syncthreads();
    double d2[4] = {0, 0, 0, 0};
    pc_apply<RAD, Q, R, false>(C, pv, ps, d2);
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
          S.rrmin[c] = fmin(S.rrmin[c], rr);
          if (!isfinite(rr) || rr <= A.tol * A.tol * S.bb[c] || needs_restart(S, c, rr)) atomicOr(&S.any_flag, 1);
        }
      }
      __syncthreads();
    }
    if (S.any_flag)
      pc_true_residual_and_restart<RAD, Q, R>(A, C, pv, ps, PA, K, dst_, false, all_done);
  }
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

template <int RAD, int Q, class R, bool BATCH>
__global__ __launch_bounds__(MAX_T) RST_WAVES_ATTR void k_bicgstab_pc(const SolveArgs* __restrict__ Ap) {
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
  PcVecs<R> pv;
  pv.ph = base + 5 * nv;
  pv.sh = base + 6 * nv;
  pv.s = base + 7 * nv;
  pv.w = base + 8 * nv;
  pv.inv = nullptr;
  const size_t np = (size_t)A.pj.nproj * cw;
  cx<double>* pb = reinterpret_cast<cx<double>*>(A.pws) + (size_t)blockIdx.x * A.pws_stride;
  ProjArrays PA{pb, pb + np, pb + 2 * np, pb + 3 * np, pb + 4 * np};
  // DFT step tables in LDS after the solver's regions: fa[na] fb[nb] ia[na] ib[nb] pa[na] pb[nb]
  cx<double>* tab = reinterpret_cast<cx<double>*>(smem + A.pc_lds_off);
  const int ntab = 3 * (A.g.na + A.g.nb);
  for (int w = threadIdx.x; w < ntab; w += blockDim.x) {
    const double2 t = A.pc.steps[w];
    tab[w] = mkc(t.x, t.y);
  }
  DftSteps dst_;
  dst_.fa = tab;
  dst_.fb = tab + A.g.na;
  dst_.ia = tab + A.g.na + A.g.nb;
  dst_.ib = tab + 2 * A.g.na + A.g.nb;
  dst_.pa = tab + 2 * A.g.na + 2 * A.g.nb;
  dst_.pb = tab + 3 * A.g.na + 2 * A.g.nb;
  __syncthreads();
  const Pos<Q> ps = make_pos<Q>(A.g, cw, RAD);
  for (;;) {
    if (threadIdx.x == 0) S.item = atomicAdd(A.counter, 1);
    __syncthreads();
    const int item = S.item;
    if (item >= A.nitems) break;
    if constexpr (BATCH) {
      __shared__ SolveArgs Ai;  // per-item arguments of a batched launch
      __shared__ int local_item;
      if (threadIdx.x == 0) local_item = batch_item_args<true>(A, item, Ai);
      __syncthreads();
      for (int w = threadIdx.x; w < ntab; w += blockDim.x) {
        const double2 t = Ai.pc.steps[w];
        tab[w] = mkc(t.x, t.y);
      }
      __syncthreads();
      C.g = &Ai.g;
      C.V = Ai.V;
      C.gz = Ai.gz;
      pc_solve_item<RAD, Q, R>(Ai, C, pv, ps, PA, Ai.pc, dst_, local_item);
    } else {
      pc_solve_item<RAD, Q, R>(A, C, pv, ps, PA, A.pc, dst_, item);
    }
  }
}

// Stand-alone M^-1 on blocked vectors (the layout of the flexible-GMRES
// chunk): workgroup b maps block b of `in` (n x cw, column fastest) to block b
// of `out`, with `wbuf` as its mode-space scratch.  Energy: the pivots pc.inv.
struct PcApplyArgs {
  Geo g;
  PcConst pc;
  const double2* in;
  double2* out;
  double2* wbuf;
  int cw, nblk;
  size_t pc_lds_off;
};

template <int Q>
__global__ __launch_bounds__(MAX_T) void k_pc_apply(const PcApplyArgs* __restrict__ Ap) {
  const PcApplyArgs& A = *Ap;
  extern __shared__ __align__(16) char smem[];
  __shared__ ColState S;
  const int cw = A.cw;
  Proj pj0 = {};
  SweepCtx<double> C;
  C.g = &A.g;
  C.pj = &pj0;
  C.V = nullptr;
  C.gz = nullptr;
  C.cw = cw;
  C.L = carve_lds<double>(smem, A.g, pj0, cw, blockDim.x);
  C.S = &S;
  C.xext = nullptr;
  C.yext = nullptr;
  C.ext_ld = C.ext_c0 = C.ext_ncol = 0;
  C.pcsrc = C.pcs = nullptr;
  C.r32 = nullptr;
  C.rhs = nullptr;
  C.rhs_ld = C.rhs_c0 = 0;
  C.rhs_nc = 0;
  C.acc = nullptr;
  const size_t nv = (size_t)A.g.P * A.g.nz * cw;
  const size_t boff = (size_t)blockIdx.x * nv;
  C.vec = Vecs<double>{nullptr, reinterpret_cast<cx<double>*>(const_cast<double2*>(A.in)) + boff, nullptr,
                       nullptr, nullptr};
  PcVecs<double> pv;
  pv.ph = pv.sh = pv.s = nullptr;
  pv.w = reinterpret_cast<cx<double>*>(A.wbuf) + boff;
  pv.inv = reinterpret_cast<const cx<double>*>(A.pc.inv);
  if (threadIdx.x < CW_MAX) {
    const int c = threadIdx.x;
    S.alpha[c] = S.omega[c] = S.beta[c] = mkc(0.0, 0.0);
    S.j0[c] = -1;
    S.src[c] = -1;
    S.bsc[c] = 0.0;
  }
  cx<double>* tab = reinterpret_cast<cx<double>*>(smem + A.pc_lds_off);
  const int ntab = 3 * (A.g.na + A.g.nb);
  for (int w = threadIdx.x; w < ntab; w += blockDim.x) {
    const double2 t = A.pc.steps[w];
    tab[w] = mkc(t.x, t.y);
  }
  DftSteps dst_;
  dst_.fa = tab;
  dst_.fb = tab + A.g.na;
  dst_.ia = tab + A.g.na + A.g.nb;
  dst_.ib = tab + 2 * A.g.na + A.g.nb;
  dst_.pa = tab + 2 * A.g.na + 2 * A.g.nb;
  dst_.pb = tab + 3 * A.g.na + 2 * A.g.nb;
  __syncthreads();
  const Pos<Q> ps = make_pos<Q>(A.g, cw, 0);
  double dots[4] = {0, 0, 0, 0};
  pc_forward<Q, double>(C, pv, ps, A.pc, dst_, PC_IN, dots);
  pc_backward<Q, double>(C, pv, ps, A.pc, dst_, reinterpret_cast<cx<double>*>(A.out) + boff);
}

}  // namespace rst
