// rst_kernels.hpp -- gfx950 device code of librst.
//
// One workgroup owns a block of `cw` solve columns for the whole BiCGSTAB solve
// of A x = b, A = E - H_k + i Gamma (paper Sec. II.A), and streams the grid
// plane by plane along z:
//   * z-neighbours of the order-2M stencil come from a per-thread register
//     queue of 2M+1 planes (each input value is loaded from HBM once per sweep);
//   * lateral neighbours come from the current plane staged in LDS with a halo
//     of M points on each lateral face, written once with the Bloch phase
//     exp(+-i k_d L_d) already applied (Bloch-form equation: phi(r+R) = e^{ik.R} phi(r));
//   * the separable projectors use per-plane chunked gathers of the output plane
//     (deterministic fixed-order sums, no atomics) and a point-centric scatter
//     fused into the stencil epilogue;
//   * all BiCGSTAB vector updates are fused into the two stencil sweeps of an
//     iteration (12 vector streams per iteration), dot products are reduced
//     inside the workgroup, and the shadow residual is a unit vector so its
//     inner products are single elements.
// The column index is fastest in memory, so a wavefront's lanes read
// consecutive columns / points and every load is a contiguous 16-byte access.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rst {

constexpr int CW_MAX = 8;        // columns per workgroup
constexpr int NM_MAX = 16;       // projectors per group (atom)
constexpr int CHUNK = 8;         // entries per gather chunk
constexpr int SC_SLOTS = 1;      // scatter slots per grid point before the overflow list
constexpr int MAX_T = 512;       // workgroup size bound

// Minimum waves per SIMD requested for the solver kernels (caps VGPRs at 512/N).
#ifndef RST_WAVES_PER_EU
#define RST_WAVES_PER_EU 4
#endif
#if RST_WAVES_PER_EU > 0
#define RST_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(RST_WAVES_PER_EU)))
#else
#define RST_WAVES_ATTR
#endif

template <class R>
struct alignas(2 * sizeof(R)) cx {
  R x, y;
};

template <class R>
__device__ __forceinline__ cx<R> mkc(R a, R b) {
  cx<R> r;
  r.x = a;
  r.y = b;
  return r;
}
template <class R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return mkc(a.x + b.x, a.y + b.y); }
template <class R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return mkc(a.x - b.x, a.y - b.y); }
template <class R>
__device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return mkc(a.x * s, a.y * s); }
template <class R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <class R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return mkc(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <class R>
__device__ __forceinline__ R cnorm2(cx<R> a) { return a.x * a.x + a.y * a.y; }
template <class R>
__device__ __forceinline__ cx<double> to64(cx<R> a) { return mkc<double>((double)a.x, (double)a.y); }
template <class R>
__device__ __forceinline__ cx<R> fromd(cx<double> a) { return mkc<R>((R)a.x, (R)a.y); }
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  double d = b.x * b.x + b.y * b.y;
  return mkc((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ bool finite2(cx<double> a) { return isfinite(a.x) && isfinite(a.y); }

// Streaming (non-temporal) access to the Krylov vectors: they are touched once
// per sweep, so they should not evict the shared tables from L2.
#ifndef RST_NT
#define RST_NT 1
#endif
typedef double rst_d2 __attribute__((ext_vector_type(2)));
typedef float rst_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cx<double> ldv(const cx<double>* p) {
#if RST_NT
  const rst_d2 v = __builtin_nontemporal_load(reinterpret_cast<const rst_d2*>(p));
  return mkc(v.x, v.y);
#else
  return *p;
#endif
}
__device__ __forceinline__ cx<float> ldv(const cx<float>* p) {
#if RST_NT
  const rst_f2 v = __builtin_nontemporal_load(reinterpret_cast<const rst_f2*>(p));
  return mkc(v.x, v.y);
#else
  return *p;
#endif
}
__device__ __forceinline__ void stv(cx<double>* p, const cx<double>& v) {
#if RST_NT
  rst_d2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<rst_d2*>(p));
#else
  *p = v;
#endif
}
__device__ __forceinline__ void stv(cx<float>* p, const cx<float>& v) {
#if RST_NT
  rst_f2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<rst_f2*>(p));
#else
  *p = v;
#endif
}

// ---------------------------------------------------------------------------
// Kernel arguments
// ---------------------------------------------------------------------------

struct Geo {
  int na, nb, nz, P;     // P = na*nb points per plane
  int pa, pb;            // padded plane dims na+2M, nb+2M
  double cz[7], ca[7], cb[7];  // 1/2 c_j / h_d^2 for j = 1..M (index j)
  double diag0;          // 1/2 c_0 (1/ha^2 + 1/hb^2 + 1/hz^2)
  double pha_x, pha_y;   // exp(i k_a L_a)
  double phb_x, phb_y;   // exp(i k_b L_b)
};

struct Proj {
  int nproj, ngroup, nm;           // nm: stride of beta rows (max projectors per group)
  int max_chunks;                  // max gather chunks in one plane
  double h3;
  const int* grp_pbase;            // [ngroup] first projector of the group
  const int* grp_nm;               // [ngroup] projectors in the group
  const double* ekb;               // [nproj]
  const double* beta;              // [nent*nm] real projector values per entry
  const double2* eph;              // [nent] exp(+i k.R_e) of the entry's lateral image
  const int* ent_p;                // [nent] in-plane point index of the entry
  // gather order: chunk j (chunks numbered plane by plane) is entries
  // j*CHUNK..j*CHUNK+CHUNK-1, padding entries with zero beta and phase
  const int* g_ent_p;
  const double2* g_eph;
  const double* g_beta;
  const int* zc_offs;              // [nz+1] gather chunks per plane
  const int4* chunks;              // (group, first entry, count, -)
  const int* zg_offs;              // [nz+1] groups per plane
  const int4* zgroups;             // (group, first chunk, end chunk) relative to the plane
  // point-major scatter table: SC_SLOTS (group, entry) slots per grid point
  const int* sc_pb;                // [n*SC_SLOTS] first projector of the slot's group, -1 if empty
  const double2* sc_eph;           // [n*SC_SLOTS] exp(+i k.R) of the slot's entry
  const double* sc_beta;           // [n*SC_SLOTS*nm] projector values of the slot (zero-padded)
  const double* sc_w;              // [n*SC_SLOTS*(nm <= 9 ? 9 : 16)] beta_m E_{pb+m} of the slot, zero past
                                   // the group (rows as wide as the many-column apply's projector bound)
  int has_overflow;                // points touched by more than SC_SLOTS entries exist
  const int* pe_offs;              // [n+1] overflow entries of each grid point
  const int2* pe;                  // (group, entry)
};

// Constants of the free-electron + CAP preconditioner (see rst_precond.hpp).
struct PcConst {
  double vbar;           // shift of the reference operator (when vz is null)
  const double* vz;      // [nz] plane-dependent shift (the lateral mean of V per plane; nullable)
  double a;              // 1/2 / hz^2 (three-point z coupling)
  double shift;          // imaginary shift added to the CAP in the preconditioner (Ha)
  const double* eps;     // [P] lateral mode energies eps_perp(m)
  const double2* steps;  // [3(na+nb)] DFT recurrence steps fa, fb, ia, ib and phases pa, pb
  const double2* inv;    // [ne*nz*P] reciprocal Thomas pivots per energy, plane, lateral mode
};

// One structure of a batched launch (same lateral grid, order and spacings;
// own plane count, potential, CAPs, k, energies and columns).
struct BatchProb {
  long long item0;    // first work item of this structure
  long long v_off;    // offset of its potential in V
  long long col_off;  // offset of its columns in cols
  long long out_off;  // offset of its (energy x column) outputs
  int nz, ne, ncols, nblk;
  int gz_off;         // offset of its CAP profiles (gz, gdst, gsrc)
  int e_off;          // offset of its energies
  double pha_x, pha_y, phb_x, phb_y;
  // preconditioner: lateral mode energies, DFT steps and Thomas pivots of this structure
  long long eps_off, steps_off, inv_off;
  double vbar;
};

struct SolveArgs {
  const BatchProb* batch;  // nullptr: a single structure
  int nprob;
  Geo g;
  Proj pj;
  PcConst pc;
  double delta;             // mixed precision: reliable-update factor (see rst_mixed.hpp)
  int* updates;             // mixed precision: [ne*ncols] FP64 residual replacements per column
  size_t pc_lds_off;        // byte offset of the DFT tables in dynamic LDS
  const double* V;          // [n]
  const double* gz;         // [nz] Gamma_L + Gamma_R
  const double* gdst;       // [nz] Gamma on the side where T is accumulated (nullable)
  const double* gsrc;       // [nz] Gamma on the column side: rhs = sqrt(gsrc) e_i (null: rhs = e_i)
  const double* energies;   // [ne]
  const int64_t* cols;      // [ncols] source grid indices
  int ncols, ne, cw, nblk, nitems;
  double tol;
  int max_iter;
  void* ws;                 // per-workgroup vectors x, r, p, v, t (each n*cw complex of type R)
  size_t ws_stride;         // elements of cx<R> per workgroup
  double2* pws;             // per-workgroup projections: 5 arrays of nproj*cw
  size_t pws_stride;
  double* T_col;            // [ne*ncols] 4 sum_dst Gamma |x|^2 per column
  int* iters;               // [ne*ncols]
  int* restarts;            // [ne*ncols]
  double* resid;            // [ne*ncols] final FP64 true relative residual
  int* status;              // [ne*ncols] 0 converged, 1 not converged, 2 non-finite
  int* counter;             // work queue head
  double2* xout;            // optional export of x: element (gi, energy e, column j) at
                            // gi*(ne*ncols) + e*ncols + j
  const double2* rhs;       // optional dense right-hand sides: element (gi, e, j) at
                            // gi*rhs_ld + e*rhs_estride + j (null: point sources)
  long long rhs_ld, rhs_estride;
};

struct ApplyArgs {
  Geo g;
  Proj pj;
  const double* V;
  const double* gz;
  double energy;
  const double2* x;         // blocked layout: block b (columns b*cw ..) is n x cw column-fastest at b*n*cw
  double2* y;
  int ncol, cw, nblk;
  double2* pws;             // per-workgroup projection scratch (2 arrays nproj*cw)
  size_t pws_stride;
  int proj_pre;             // the projections of x are already in pws (k_proj_mm): no gather sweep
};

// ---------------------------------------------------------------------------
// Sweep modes
// ---------------------------------------------------------------------------

enum InMode { IN_INIT, IN_A, IN_RESTART, IN_B, IN_X, IN_EXT, IN_PC };
enum OutMode { OUT_V, OUT_T, OUT_RES, OUT_EXT, OUT_TS, OUT_RES32 };

// Per-column scalar state shared by the workgroup.
struct ColState {
  cx<double> alpha[CW_MAX], omega[CW_MAX], beta[CW_MAX], rho[CW_MAX], rho_new[CW_MAX];
  cx<double> vj[CW_MAX], sj[CW_MAX], tj[CW_MAX], rj[CW_MAX];
  cx<double> ts[CW_MAX];
  double tt[CW_MAX], rr[CW_MAX], bb[CW_MAX], tacc[CW_MAX], bsc[CW_MAX], energy[CW_MAX];
  double rmax[CW_MAX];
  long long src[CW_MAX], j0[CW_MAX], rmax_idx[CW_MAX];
  int state[CW_MAX];       // 0 active, 1 done, 2 failed, 3 padding
  int iters[CW_MAX], restarts[CW_MAX];
  // smallest recursive ||r||^2 since the last restart (divergence guard)
  double rrmin[CW_MAX];
  // mixed precision: largest recursive ||r||^2 since the last FP64 residual
  // replacement, ||r||^2 at it and the latest recursive ||r||^2, the
  // replacements so far, how the next replacement treats x32 (1 fold, 0
  // discard, -1 take a fold back), the best true ||r||^2 and the replacements
  // since it last fell tenfold, the block's request
  double maxrr[CW_MAX], rr_upd[CW_MAX], rr_rec[CW_MAX], best_rr[CW_MAX];
  int updates[CW_MAX], fold[CW_MAX], stall[CW_MAX];
  int it_upd[CW_MAX];  // mixed precision: iteration of the last FP64 residual replacement
  int upd_flag;
  int any_flag;
  int item;
};

// Restart guards of the preconditioned fused BiCGSTAB loop.  With the unit
// shadow vector e_j0, rho = r[j0] is one residual element: once it is tiny
// next to ||r|| the next alpha and beta carry no information (near-breakdown),
// and a recursion that has grown far above its best residual is diverging.
// Either sends the column to the FP64 true residual and a restart with
// j0 = argmax |r|.  (Measured: without them the preconditioned solver diverged
// on a few columns at the lateral zone boundary, k_a L_a = pi; the
// unpreconditioned solver, whose residual history spikes far more, converges
// there without them and is slowed down twofold by them, so it does not use them.)
constexpr double NEAR_BREAKDOWN2 = 1e-28;  // |rho|^2 <= this * ||r||^2
constexpr double DIVERGENCE2 = 1e10;       // ||r||^2 > this * min ||r||^2 since the restart

__device__ __forceinline__ bool needs_restart(const ColState& S, int c, double rr) {
  return rr > DIVERGENCE2 * S.rrmin[c] || (S.rho[c].x * S.rho[c].x + S.rho[c].y * S.rho[c].y) <= NEAR_BREAKDOWN2 * rr;
}

// Vectors of one workgroup.
template <class R>
struct Vecs {
  cx<R>* x;
  cx<R>* r;
  cx<R>* p;
  cx<R>* v;
  cx<R>* t;
};

struct ProjArrays {
  cx<double>* Pr;
  cx<double>* Pp;
  cx<double>* Pv;
  cx<double>* Pt;
  cx<double>* Px;
};

// LDS carve-up (dynamic shared memory)
template <class R>
struct Lds {
  cx<R>* inpl0;        // padded lateral plane, double-buffered
  cx<R>* inpl1;
  cx<R>* outpl;        // output plane for the gathers (P*cw)
  cx<double>* dco;     // scatter coefficients h^3 E_p (B^H u) (nproj*cw)
  cx<double>* pacc;    // gather accumulator of the current sweep (nproj*cw)
  cx<double>* slots;   // gather chunk partials (max_chunks*nm*cw)
  double* red;         // reduction scratch (blockDim*4)
};

// Dynamic LDS bytes: the reduction scratch (4 doubles per thread, used only
// between sweeps) aliases the two lateral plane buffers.
template <class R>
__host__ __device__ inline size_t lds_bytes(int pa, int pb, int P, int nproj, int max_chunks, int nm,
                                            int cw, int nthreads) {
  size_t planes = 2 * (size_t)pa * pb * cw * sizeof(cx<R>);
  size_t red = (size_t)nthreads * 4 * sizeof(double);
  size_t off = planes > red ? planes : red;
  off = (off + 15) & ~size_t(15);
  if (nproj) off += (size_t)P * cw * sizeof(cx<R>);
  off = (off + 15) & ~size_t(15);
  off += 2 * (size_t)nproj * cw * sizeof(cx<double>);
  off += (size_t)max_chunks * nm * cw * sizeof(cx<double>);
  return off;
}

template <class R>
__device__ __forceinline__ Lds<R> carve_lds(char* smem, const Geo& g, const Proj& pj, int cw,
                                            int nthreads) {
  Lds<R> L;
  size_t plane = (size_t)g.pa * g.pb * cw;
  L.inpl0 = reinterpret_cast<cx<R>*>(smem);
  L.inpl1 = reinterpret_cast<cx<R>*>(smem) + plane;
  L.red = reinterpret_cast<double*>(smem);
  size_t planes = 2 * plane * sizeof(cx<R>);
  size_t red = (size_t)nthreads * 4 * sizeof(double);
  size_t off = planes > red ? planes : red;
  off = (off + 15) & ~size_t(15);
  L.outpl = reinterpret_cast<cx<R>*>(smem + off);
  if (pj.nproj) off += (size_t)g.P * cw * sizeof(cx<R>);
  off = (off + 15) & ~size_t(15);
  L.dco = reinterpret_cast<cx<double>*>(smem + off);
  off += (size_t)pj.nproj * cw * sizeof(cx<double>);
  L.pacc = reinterpret_cast<cx<double>*>(smem + off);
  off += (size_t)pj.nproj * cw * sizeof(cx<double>);
  L.slots = reinterpret_cast<cx<double>*>(smem + off);
  return L;
}

// Per-thread positions in the plane.
template <int Q>
struct Pos {
  int p[Q];      // in-plane point, or -1
  int li[Q];     // LDS interior index in the padded plane
  unsigned char hal[Q];  // halo flags: 1 a-low, 2 a-high, 4 b-low, 8 b-high
};

// ---------------------------------------------------------------------------
// Gather of the plane staged in L.outpl into the LDS accumulator L.pacc.
// Chunks hold at most CHUNK entries of one group in one plane; the entry loop
// is unrolled so every chunk issues its loads at once.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void plane_gather(int z, const Proj& pj, const Lds<R>& L, int cw) {
  const int tid = threadIdx.x, T = blockDim.x;
  const int c0 = pj.zc_offs[z], c1 = pj.zc_offs[z + 1];
  const int nch = c1 - c0;
  const int nm = pj.nm;
  if (nch == 0) return;  // uniform across the workgroup
  // stage 1: chunk partial sums (fixed order inside a chunk); the chunk's
  // entries sit at a position known from the plane alone (no lookup chain)
  for (int w = tid; w < nch * nm * cw; w += T) {
    const int c = w % cw;
    const int m = (w / cw) % nm;
    const int ci = w / (cw * nm);
    const int e0 = (c0 + ci) * CHUNK;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int k = 0; k < CHUNK; ++k) {
      const int e = e0 + k;
      const cx<double> yv = to64(L.outpl[pj.g_ent_p[e] * cw + c]);
      const double2 ph = pj.g_eph[e];
      const cx<double> w2 = cmulc(mkc(ph.x, ph.y), yv);  // conj(phase) * y; zero for padding
      const double b = pj.g_beta[(size_t)e * nm + m];
      sx += b * w2.x;
      sy += b * w2.y;
    }
    L.slots[(ci * nm + m) * cw + c] = mkc(sx, sy);
  }
  __syncthreads();
  // stage 2: per (group, projector, column), add the plane's chunks in order
  const int g0 = pj.zg_offs[z], g1 = pj.zg_offs[z + 1];
  for (int w = tid; w < (g1 - g0) * nm * cw; w += T) {
    const int c = w % cw;
    const int m = (w / cw) % nm;
    const int gi = w / (cw * nm);
    const int4 zg = pj.zgroups[g0 + gi];  // (group, first chunk, end chunk, first projector)
    if (m < pj.grp_nm[zg.x]) {
      cx<double> s = mkc(0.0, 0.0);
      for (int ci = zg.y; ci < zg.z; ++ci) s = s + L.slots[(ci * nm + m) * cw + c];
      cx<double>* a = &L.pacc[(size_t)(zg.w + m) * cw + c];
      *a = *a + cscale(s, pj.h3);
    }
  }
}

// Scatter contribution sum_p beta_k,p(i) dco[p] at grid point i for column c.
template <class R>
__device__ __forceinline__ cx<double> point_scatter(long long i, int c, const Proj& pj,
                                                    const Lds<R>& L, int cw) {
  cx<double> acc = mkc(0.0, 0.0);
  const int nm = pj.nm;
  const int plast = pj.nproj - 1;
  // the slot's projector index, phase and values are loaded together (an empty
  // slot has zero values and phase, so it adds exactly zero): one memory
  // latency instead of a dependent chain
#pragma unroll
  for (int sl = 0; sl < SC_SLOTS; ++sl) {
    const size_t si = (size_t)i * SC_SLOTS + sl;
    const int pb = max(pj.sc_pb[si], 0);
    const double* bt = pj.sc_beta + si * nm;
    const double2 ph = pj.sc_eph[si];
    double tx = 0.0, ty = 0.0;
#pragma unroll
    for (int m = 0; m < NM_MAX; ++m) {
      if (m < nm) {
        const int pp = min(pb + m, plast);  // beta is zero past the group's projectors
        const cx<double> d = L.dco[pp * cw + c];
        tx += bt[m] * d.x;
        ty += bt[m] * d.y;
      }
    }
    acc = acc + cmul(mkc(ph.x, ph.y), mkc(tx, ty));
  }
  if (pj.has_overflow) {
    const int k0 = pj.pe_offs[i], k1 = pj.pe_offs[i + 1];
    for (int k = k0; k < k1; ++k) {
      const int2 ge = pj.pe[k];
      const int nmg = pj.grp_nm[ge.x];
      const int pb = pj.grp_pbase[ge.x];
      cx<double> t = mkc(0.0, 0.0);
      const double* bt = pj.beta + (size_t)ge.y * nm;
      for (int m = 0; m < nmg; ++m) {
        const cx<double> d = L.dco[(pb + m) * cw + c];
        t.x += bt[m] * d.x;
        t.y += bt[m] * d.y;
      }
      const double2 ph = pj.eph[ge.y];
      acc = acc + cmul(mkc(ph.x, ph.y), t);
    }
  }
  return acc;
}

// Start / end of a sweep that gathers into LDS: zero L.pacc; copy it to dst.
template <class R>
__device__ __forceinline__ void pacc_zero(const Proj& pj, const Lds<R>& L, int cw) {
  for (int w = threadIdx.x; w < pj.nproj * cw; w += blockDim.x) L.pacc[w] = mkc(0.0, 0.0);
}
template <class R>
__device__ __forceinline__ void pacc_flush(const Proj& pj, const Lds<R>& L, int cw, cx<double>* dst) {
  for (int w = threadIdx.x; w < pj.nproj * cw; w += blockDim.x) dst[w] = L.pacc[w];
}

// Workgroup reduction of four per-thread doubles per column into out[k][c]; thread t
// holds column t % cw.  Within a wavefront a shuffle butterfly over lane offsets
// 32, 16, ..., cw (each keeps the lane's column) leaves every lane with its
// column's wave sum; lanes 0..cw-1 write those to LDS and threads (k, c) add the
// waves in order (deterministic).  red: at least 4 * waves * cw doubles.
__device__ __forceinline__ void col_reduce4(double* red, int cw, const double (&v)[4],
                                            double (*out)[CW_MAX]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  double s[4] = {v[0], v[1], v[2], v[3]};
  for (int off = 32; off >= cw; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] += __shfl_xor(s[k], off, 64);
  }
  __syncthreads();
  if (lane < cw) {
#pragma unroll
    for (int k = 0; k < 4; ++k) red[(k * nw + wv) * cw + lane] = s[k];
  }
  __syncthreads();
  if (tid < 4 * cw) {
    const int k = tid / cw, c = tid % cw;
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[(k * nw + w) * cw + c];
    out[k][c] = t;
  }
  __syncthreads();
}

// The same for one complex value per thread over a 256-thread workgroup: returns the
// column sum (valid in threads 0..cw-1).  red: 4 * cw double2.
__device__ __forceinline__ double2 col_reduce_c(double2* red, int cw, double2 v) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  for (int off = 32; off >= cw; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  if (lane < cw) red[wv * cw + lane] = v;
  __syncthreads();
  double2 t = make_double2(0.0, 0.0);
  if (tid < cw)
    for (int w = 0; w < nw; ++w) {
      t.x += red[w * cw + tid].x;
      t.y += red[w * cw + tid].y;
    }
  return t;
}

}  // namespace rst
