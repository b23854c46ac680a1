// rst_lib.hip -- host runtime and C ABI of librst (see include/rst.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <array>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/rst.h"
#include "rst_cnn_api.hpp"
#include "rst_fgmres.hpp"
#include "rst_cocg.hpp"
#include "rst_lowrank.hpp"
#include "rst_projmm.hpp"
#include "rst_apply_cols.hpp"
#include "rst_mixed.hpp"
#include "rst_mk.hpp"
#include "rst_idr.hpp"
#include "rst_cocg2.hpp"
#include "rst_eig.hpp"
#include "rst_zeig.hpp"

using rst::cx;

// Scratch memory of rst_apply_h_noalloc: the projections h^3 B^H x of the applied
// columns (nproj*ncol complex128).  One copy per device, held until the process
// ends; its device address is looked up once per device by rst_create (with that
// device current) and kept in scratch_dev[].  Host code never passes `scratch`
// itself to a kernel: in host code the name is a host-side stand-in, not a device
// address.
constexpr size_t RST_SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) double2 scratch[RST_SCRATCH_BYTES / sizeof(double2)];
namespace {
constexpr int RST_MAX_DEVICES = 64;
double2* scratch_dev[RST_MAX_DEVICES] = {};
std::mutex scratch_mu;
}  // namespace

namespace rst {
// Fills n ints with v (used to reset the work-queue head without a memset node).
__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Reciprocal Thomas pivots of the preconditioner for every (energy, lateral
// mode): den_0 = b_0, den_z = b_z - a^2 / den_{z-1}, with
// b_z = E - Vref(z) - eps_perp(m) - 2a + i Gamma(z), Vref(z) the plane mean of V
// (pc.vz) or the cell mean (pc.vbar).  One thread per (E, m).
__global__ void k_pc_pivots(const SolveArgs* __restrict__ Ap) {
  const SolveArgs& A = *Ap;
  const int P = A.g.P, nz = A.g.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)A.ne * P) return;
  const int e = (int)(t / P), m = (int)(t % P);
  const double a = A.pc.a, a2 = a * a;
  const double re0 = A.energies[e] - A.pc.eps[m] - 2.0 * a;
  double2* inv = const_cast<double2*>(A.pc.inv) + (size_t)e * nz * P;
  cx<double> iv = mkc(0.0, 0.0);
  for (int z = 0; z < nz; ++z) {
    cx<double> den = mkc(re0 - (A.pc.vz ? A.pc.vz[z] : A.pc.vbar), A.gz[z] + A.pc.shift);
    if (z > 0) den = den - cscale(iv, a2);
    iv = cdiv(mkc(1.0, 0.0), den);
    double2 o;
    o.x = iv.x;
    o.y = iv.y;
    inv[(size_t)z * P + m] = o;
  }
}

}  // namespace rst

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

}  // namespace

struct rst_ctx {
  int device = 0;
  rst::cnn::Engine* cnn = nullptr;  // learned correction network (created on first use)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  hipEvent_t ev_apply[3] = {nullptr, nullptr, nullptr};  // apply timing (created on first use)
  double apply_ms[2] = {0.0, 0.0};                      // last apply: projector gather, stencil sweep

  // grid
  bool has_grid = false;
  int na = 0, nb = 0, nz = 0, order = 0, rad = 0;
  double ha = 0, hb = 0, hz = 0;
  std::vector<double> fdw;  // c_0..c_M
  // host copies
  std::vector<double> v, gl, gr;
  bool has_v = false, has_abc = false, has_k = false;
  double ka = 0, kb = 0;
  // projectors (host plan)
  int nproj = 0, ngroup = 0, nm = 0, max_chunks = 0;
  std::vector<int> grp_pbase, grp_nm;
  std::vector<double> ekb, beta;
  std::vector<int> ent_p, ent_gi;
  std::vector<int8_t> ent_img;  // 2 per entry
  std::vector<int> zc_offs, zg_offs, pe_offs;
  std::vector<int4> chunks, zgroups;
  std::vector<int2> pe;
  std::vector<int> sc_pb, sc_ent;  // scatter slots: first projector and entry (-1 empty)
  // gather order: plane-major, each (plane, group) run padded to whole chunks
  std::vector<int> g_ent_p, g_src;  // in-plane point and source entry (-1: padding)
  std::vector<double> g_beta;
  std::vector<double> sc_beta, sc_w;
  int has_overflow = 0;
  // device copies
  DevBuf d_v, d_gz, d_gl, d_gr, d_vz;  // d_vz: plane means of V (preconditioner reference)
  DevBuf d_pc_eps, d_pc_twa, d_pc_twb;
  DevBuf d_grp_pbase, d_grp_nm, d_ekb, d_beta, d_eph, d_ent_p, d_zc, d_chunks, d_zg, d_zgroups,
      d_pe_offs, d_pe, d_sc_pb, d_sc_eph, d_sc_beta, d_sc_w, d_g_ent_p, d_g_eph, d_g_beta;
  // batched projector gather (many-column apply): group entry ranges, entry grid indices, projections
  std::vector<int> grp_e0, grp_ne;
  DevBuf d_grp_e0, d_grp_ne, d_ent_gi, d_projP;
  // low-rank transmission buffers
  DevBuf d_lrB, d_lrX, d_lrY, d_lrQ, d_lrQ2, d_lrG, d_lrR, d_lrW, d_lrL, d_lrRc, d_lrT, d_lrYacc, d_lrYacc2, d_lrQf;
  // eigen route: subspace blocks, Ritz vectors, small matrices
  DevBuf d_egQ, d_egY, d_egW, d_egX, d_egKX, d_egS, d_egG, d_egR, d_egRm, d_egL, d_egTh, d_egRes, d_egMap, d_egSc;
  // many-column solvers, mixed mode: FP64 x and r; per-column right-hand-side offsets and budgets;
  // doubled COCG: per-column conjugation flags and per-pair state
  DevBuf d_mkv64, d_mkref, d_mkcfl, d_mkcd;
  // training of the network: its energies, solver pairs (x*, x_j) and their columns
  DevBuf d_tren, d_trX, d_trcols;
  // solver
  rst_solver_opts opts;
  // work buffers (grown on demand)
  DevBuf d_ws, d_pws, d_cols, d_en, d_T, d_it, d_rs, d_res, d_st, d_counter, d_args, d_pc_inv, d_up;
  std::vector<int> last_updates;  // mixed precision: FP64 residual replacements per column of the last solve
  long long last_fallbacks = 0;   // FGMRES: columns whose learned correction was switched off
  double last_cnn_flop = 0.0;     // FGMRES: network flops of the last solve
  double last_fg_bytes = 0.0;     // FGMRES: algorithmic vector bytes of the last solve
  double last_extra_bytes = 0.0;  // mixed precision: bytes of the FP64 re-solves
  bool last_mk = false;           // the last solve ran the many-column BiCGSTAB
  double last_mk_bytes = 0.0;     // its algorithmic bytes
  // many-column BiCGSTAB (planes of any size): vectors, per-column state, partial sums, column tables,
  // DFT matrices of the preconditioner
  DevBuf d_mkv, d_mkst, d_mkact, d_mkmark, d_mkpart, d_mkcol, d_mkF, d_mkT, d_mkvref, d_mkidr, d_mkshadow;
  // COCG chunk buffers: R, P, Q vectors; per-column scalars and flags
  DevBuf d_cgR, d_cgP, d_cgQ, d_cgs, d_cgi;
  // flexible GMRES chunk buffers
  DevBuf d_fgV, d_fgZ, d_fgX, d_fgW, d_fgM, d_fgwb, d_fgx0, d_fgf, d_fgH, d_fgcs, d_fgsn, d_fgg, d_fginv, d_fgest,
      d_fgact, d_fgit, d_fguse, d_fgh1, d_fgh2, d_fgn2, d_fgy, d_fgsrc, d_fgbsc, d_fgt, d_fgaa, d_fgpa, d_fgsa;
  // batch of structures (rst_batch_add)
  struct HostProb {
    long long grid_version;  // rst_set_grid calls made before the structure was added
    int nz;
    std::vector<double> v, gl, gr, en;
    double ka, kb;
  };
  std::vector<HostProb> batch;
  int batch_version = 0;
  long long grid_version = 0;
  // (lateral shape, order, preconditioner, direction, launch mode, caller's requests) -> tuned
  // (columns per workgroup, workgroup size) of the batched launch
  std::map<long long, std::pair<int, int>> tuned_shape;
  hipGraphExec_t gexec = nullptr;
  // what the captured launch depends on: batch contents, kernel, launch shape, LDS bytes and every
  // device pointer baked into the graph (argument block, work counter, workspace)
  std::array<long long, 9> gexec_key{};
  DevBuf d_bprob, d_bv, d_bgz, d_bgl, d_bgr, d_ben, d_bcols, d_bpc_eps, d_bpc_steps, d_bpargs;
  int last_cw = 0, last_threads = 0;
  // host copies of the last kernel-argument blocks (kept alive for async copies)
  rst::SolveArgs h_solve;
  rst::ApplyArgs h_apply;
};

namespace {

rst_status fail(rst_ctx* c, rst_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(ctx, call)                                                          \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, RST_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

rst_status ensure(rst_ctx* c, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return RST_OK;
  b.release();
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(c, RST_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return RST_OK;
}

template <class T>
rst_status upload(rst_ctx* c, DevBuf& b, const std::vector<T>& h) {
  rst_status s = ensure(c, b, std::max<size_t>(h.size() * sizeof(T), 16));
  if (s != RST_OK) return s;
  if (!h.empty()) HIPCHK(c, hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RST_OK;
}

// Finite-difference weights by Fornberg's recursion (B. Fornberg, Math. Comp.
// 51 (1988) 699) for the nodes -M..M, second derivative at 0.  Returns c_0..c_M.
std::vector<double> fornberg_second_derivative(int m) {
  const int npts = 2 * m + 1;
  std::vector<long double> x(npts);
  for (int i = 0; i < npts; ++i) x[i] = (long double)(i - m);
  const int md = 2;
  std::vector<std::vector<long double>> C(npts, std::vector<long double>(md + 1, 0.0L));
  long double c1 = 1.0L, c4 = x[0];
  C[0][0] = 1.0L;
  for (int i = 1; i < npts; ++i) {
    const int mn = std::min(i, md);
    long double c2 = 1.0L;
    const long double c5 = c4;
    c4 = x[i];
    for (int j = 0; j < i; ++j) {
      const long double c3 = x[i] - x[j];
      c2 *= c3;
      if (j == i - 1) {
        for (int k = mn; k >= 1; --k) C[i][k] = c1 * (k * C[i - 1][k - 1] - c5 * C[i - 1][k]) / c2;
        C[i][0] = -c1 * c5 * C[i - 1][0] / c2;
      }
      for (int k = mn; k >= 1; --k) C[j][k] = (c4 * C[j][k] - k * C[j][k - 1]) / c3;
      C[j][0] = c4 * C[j][0] / c3;
    }
    c1 = c2;
  }
  std::vector<double> w(m + 1);
  for (int j = 0; j <= m; ++j) w[j] = (double)C[m + j][2];
  return w;
}

rst::Geo make_geo(const rst_ctx* c) {
  rst::Geo g;
  std::memset(&g, 0, sizeof(g));
  g.na = c->na;
  g.nb = c->nb;
  g.nz = c->nz;
  g.P = c->na * c->nb;
  g.pa = c->na + 2 * c->rad;
  g.pb = c->nb + 2 * c->rad;
  for (int j = 1; j <= c->rad; ++j) {
    g.cz[j] = 0.5 * c->fdw[j] / (c->hz * c->hz);
    g.ca[j] = 0.5 * c->fdw[j] / (c->ha * c->ha);
    g.cb[j] = 0.5 * c->fdw[j] / (c->hb * c->hb);
  }
  g.diag0 = 0.5 * c->fdw[0] * (1.0 / (c->ha * c->ha) + 1.0 / (c->hb * c->hb) + 1.0 / (c->hz * c->hz));
  const double la = c->na * c->ha, lb = c->nb * c->hb;
  g.pha_x = std::cos(c->ka * la);
  g.pha_y = std::sin(c->ka * la);
  g.phb_x = std::cos(c->kb * lb);
  g.phb_y = std::sin(c->kb * lb);
  return g;
}

rst::Proj make_proj(const rst_ctx* c) {
  rst::Proj p;
  std::memset(&p, 0, sizeof(p));
  p.nproj = c->nproj;
  p.ngroup = c->ngroup;
  p.nm = std::max(1, c->nm);
  p.max_chunks = c->max_chunks;
  p.h3 = c->ha * c->hb * c->hz;
  p.grp_pbase = (const int*)c->d_grp_pbase.p;
  p.grp_nm = (const int*)c->d_grp_nm.p;
  p.ekb = (const double*)c->d_ekb.p;
  p.beta = (const double*)c->d_beta.p;
  p.eph = (const double2*)c->d_eph.p;
  p.ent_p = (const int*)c->d_ent_p.p;
  p.zc_offs = (const int*)c->d_zc.p;
  p.chunks = (const int4*)c->d_chunks.p;
  p.zg_offs = (const int*)c->d_zg.p;
  p.zgroups = (const int4*)c->d_zgroups.p;
  p.pe_offs = (const int*)c->d_pe_offs.p;
  p.pe = (const int2*)c->d_pe.p;
  p.sc_pb = (const int*)c->d_sc_pb.p;
  p.sc_eph = (const double2*)c->d_sc_eph.p;
  p.g_ent_p = (const int*)c->d_g_ent_p.p;
  p.g_eph = (const double2*)c->d_g_eph.p;
  p.g_beta = (const double*)c->d_g_beta.p;
  p.sc_beta = (const double*)c->d_sc_beta.p;
  p.sc_w = (const double*)c->d_sc_w.p;
  p.has_overflow = c->has_overflow;
  return p;
}

// Projections h^3 B^H x of a blocked apply's input (k_proj_mm on the FP64
// matrix cores, written into the per-block pws arrays), so that k_apply skips
// its gather sweep (proj_pre).  Nothing to do without projectors.
rst_status proj_blocked(rst_ctx* c, const rst::ApplyArgs& A) {
  if (c->nproj == 0 || !A.proj_pre) return RST_OK;
  rst::ProjMMArgs M;
  std::memset(&M, 0, sizeof(M));
  M.X = A.x;
  M.P = A.pws;
  M.grp_e0 = (const int*)c->d_grp_e0.p;
  M.grp_ne = (const int*)c->d_grp_ne.p;
  M.grp_pbase = (const int*)c->d_grp_pbase.p;
  M.grp_nm = (const int*)c->d_grp_nm.p;
  M.ent_gi = (const int*)c->d_ent_gi.p;
  M.eph = (const double2*)c->d_eph.p;
  M.beta = (const double*)c->d_beta.p;
  M.nm = c->nm;
  M.ngroup = c->ngroup;
  M.ncol = A.ncol;
  M.h3 = c->ha * c->hb * c->hz;
  M.cw = A.cw;
  M.n = (long long)c->na * c->nb * c->nz;
  M.p_stride = A.pws_stride;
  const long long tiles = (long long)c->ngroup * ((A.ncol + 63) / 64);
  hipLaunchKernelGGL(rst::k_proj_mm<double2>, dim3((unsigned)tiles), dim3(256), 0, c->stream, M);
  HIPCHK(c, hipGetLastError());
  return RST_OK;
}

// k_apply_cols instance for a stencil radius (FD order 2..12), projector group size and
// precision; wide: the 64-bit addressed kernel for planes or projection arrays past the
// buffer path's offsets.
void* apply_cols_kernel(int rad, bool nm9, bool f32, bool cj, bool wide) {
#define RST_APPLY_PICK(K, R)                                                                       \
  if (rad == R) {                                                                                  \
    if (cj && !f32) return nm9 ? (void*)rst::K<R, 9, double, true> : (void*)rst::K<R, 16, double, true>; \
    if (cj) return nullptr;                                                                        \
    if (f32) return nm9 ? (void*)rst::K<R, 9, float> : (void*)rst::K<R, 16, float>;                \
    return nm9 ? (void*)rst::K<R, 9, double> : (void*)rst::K<R, 16, double>;                       \
  }
  if (wide) {
    RST_APPLY_PICK(k_apply_cols_wide, 1)
    RST_APPLY_PICK(k_apply_cols_wide, 2)
    RST_APPLY_PICK(k_apply_cols_wide, 3)
    RST_APPLY_PICK(k_apply_cols_wide, 4)
    RST_APPLY_PICK(k_apply_cols_wide, 5)
    RST_APPLY_PICK(k_apply_cols_wide, 6)
    return nullptr;
  }
  RST_APPLY_PICK(k_apply_cols, 1)
  RST_APPLY_PICK(k_apply_cols, 2)
  RST_APPLY_PICK(k_apply_cols, 3)
  RST_APPLY_PICK(k_apply_cols, 4)
  RST_APPLY_PICK(k_apply_cols, 5)
  RST_APPLY_PICK(k_apply_cols, 6)
#undef RST_APPLY_PICK
  return nullptr;
}

// Strip width of k_apply_cols' point order.  A plane that the waves in flight on
// one XCD cover whole (about 32 CUs x 12 waves) keeps row-major order; on wider
// planes strips of APPLY_STRIP a-columns keep the b neighbours a few strips apart.
int apply_strip(int na, int P) { return P <= 512 ? na : std::min(na, rst::APPLY_STRIP); }

// y = (E - H_k + i Gamma) x on an n x ncol column-fastest block: the projections
// h^3 B^H x of every column on the FP64 matrix cores (k_proj_mm, into projP:
// nproj*ncol complex128), then one wave per (64 columns, z segment, grid point)
// (k_apply_cols).  ecol (nullable) gives each column its own energy, mask
// (nullable) the columns to apply.  ev (nullable): three events recorded before,
// between and after the two kernels.
rst_status apply_cols(rst_ctx* c, const void* x, void* y, int ncol, double energy, const double* ecol,
                      const int* mask, bool f32, double2* projP, hipEvent_t* ev, const int* cfl = nullptr) {
  const int P = c->na * c->nb;  // rst_set_grid guarantees na, nb > rad: one wrap at most
  // planes per wave: short segments keep the waves that share lateral rows close in z
  const int zseg = std::min(c->nz, rst::APPLY_ZSEG);
  const long long nseg = (c->nz + zseg - 1) / zseg;
  const long long nwg = (long long)((ncol + 63) / 64) * nseg * P;  // one wave per (64 columns, segment, point)
  if (nwg > 0x7fffffffLL) return fail(c, RST_EINVAL, "too many columns for one launch");
  rst::ColApplyArgs A;
  std::memset(&A, 0, sizeof(A));
  A.x = x;
  A.y = y;
  A.ncol = ncol;
  A.g = make_geo(c);
  A.V = (const double*)c->d_v.p;
  A.gz = (const double*)c->d_gz.p;
  A.energy = energy;
  A.pj = make_proj(c);
  A.zseg = zseg;
  A.strip = apply_strip(c->na, P);
  A.ecol = ecol;
  A.mask = mask;
  A.cfl = cfl;
  if (ev) HIPCHK(c, hipEventRecord(ev[0], c->stream));
  if (c->nproj > 0) {
    // all projections P = h^3 B^H x at once on the matrix cores; the apply kernel then scatters B E P
    rst::ProjMMArgs M;
    std::memset(&M, 0, sizeof(M));
    M.X = x;
    M.P = projP;
    M.grp_e0 = (const int*)c->d_grp_e0.p;
    M.grp_ne = (const int*)c->d_grp_ne.p;
    M.grp_pbase = (const int*)c->d_grp_pbase.p;
    M.grp_nm = (const int*)c->d_grp_nm.p;
    M.ent_gi = (const int*)c->d_ent_gi.p;
    M.eph = (const double2*)c->d_eph.p;
    M.beta = (const double*)c->d_beta.p;
    M.nm = c->nm;
    M.ngroup = c->ngroup;
    M.ncol = ncol;
    M.cfl = cfl;
    M.h3 = c->ha * c->hb * c->hz;
    const long long tiles = (long long)c->ngroup * ((ncol + 63) / 64);  // one workgroup per (group, 64 columns)
    if (f32)
      hipLaunchKernelGGL(rst::k_proj_mm<float2>, dim3((unsigned)tiles), dim3(256), 0, c->stream, M);
    else
      hipLaunchKernelGGL(rst::k_proj_mm<double2>, dim3((unsigned)tiles), dim3(256), 0, c->stream, M);
    HIPCHK(c, hipGetLastError());
    A.P = projP;
  }
  if (ev) HIPCHK(c, hipEventRecord(ev[1], c->stream));
  // the buffer path addresses a plane of rows and the projection array with 32-bit offsets
  const long long esz = f32 ? 8 : 16;
  const bool wide = (long long)P * ncol * esz > rst::APPLY_BUF_MAX ||
                    (long long)c->nproj * ncol * 16 > rst::APPLY_BUF_MAX;
  void* kern = apply_cols_kernel(c->rad, c->nm <= 9, f32, cfl != nullptr, wide);
  if (!kern) return fail(c, RST_EUNSUPPORTED, "no many-column apply for this FD order");
  {
    void* args[] = {&A};
    HIPCHK(c, hipLaunchKernel(kern, dim3((unsigned)nwg), dim3(64), args, 0, c->stream));
  }
  HIPCHK(c, hipGetLastError());
  if (ev) HIPCHK(c, hipEventRecord(ev[2], c->stream));
  return RST_OK;
}

// Builds the projector plan: groups of consecutive projectors with identical
// (point, image) entry lists, entries sorted by plane, per-plane gather chunks,
// and the point-centric scatter lists.
rst_status build_plan(rst_ctx* c, int nproj, const int32_t* offs, const int32_t* pt, const int8_t* img,
                      const double* beta, const double* ekb) {
  const long long n = (long long)c->na * c->nb * c->nz;
  const int P = c->na * c->nb;
  c->nproj = nproj;
  c->grp_pbase.clear();
  c->grp_nm.clear();
  c->grp_e0.clear();
  c->grp_ne.clear();
  c->ekb.assign(ekb, ekb + nproj);
  // group detection
  std::vector<std::pair<int, int>> groups;  // (first proj, count)
  for (int p = 0; p < nproj;) {
    int q = p + 1;
    const int len = offs[p + 1] - offs[p];
    while (q < nproj && q - p < rst::NM_MAX && offs[q + 1] - offs[q] == len) {
      bool same = true;
      for (int e = 0; e < len && same; ++e) {
        const int a = offs[p] + e, b = offs[q] + e;
        same = pt[a] == pt[b] && img[2 * a] == img[2 * b] && img[2 * a + 1] == img[2 * b + 1];
      }
      if (!same) break;
      ++q;
    }
    groups.push_back({p, q - p});
    p = q;
  }
  c->ngroup = (int)groups.size();
  int nm = 1;
  for (auto& g : groups) nm = std::max(nm, g.second);
  c->nm = nm;
  // entries per group sorted by (plane, in-plane point, image)
  c->ent_p.clear();
  c->ent_gi.clear();
  c->ent_img.clear();
  c->beta.clear();
  std::vector<int> grp_e0, grp_ne;
  for (int gi = 0; gi < c->ngroup; ++gi) {
    const int p0 = groups[gi].first, cnt = groups[gi].second;
    const int len = offs[p0 + 1] - offs[p0];
    std::vector<int> ord(len);
    for (int e = 0; e < len; ++e) ord[e] = e;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
      const int ia = pt[offs[p0] + a], ib = pt[offs[p0] + b];
      return ia < ib;
    });
    grp_e0.push_back((int)c->ent_p.size());
    grp_ne.push_back(len);
    c->grp_e0.push_back((int)c->ent_p.size());
    c->grp_ne.push_back(len);
    c->grp_pbase.push_back(p0);
    c->grp_nm.push_back(cnt);
    for (int e : ord) {
      const int a = offs[p0] + e;
      if (pt[a] < 0 || pt[a] >= n) return fail(c, RST_EINVAL, "projector point index out of range");
      c->ent_gi.push_back(pt[a]);
      c->ent_p.push_back(pt[a] % P);
      c->ent_img.push_back(img[2 * a]);
      c->ent_img.push_back(img[2 * a + 1]);
      for (int m = 0; m < nm; ++m)
        c->beta.push_back(m < cnt ? beta[offs[p0 + m] + e] : 0.0);
    }
  }
  const int nent = (int)c->ent_p.size();
  // per-plane chunks
  c->zc_offs.assign(c->nz + 1, 0);
  c->zg_offs.assign(c->nz + 1, 0);
  c->chunks.clear();
  c->zgroups.clear();
  std::vector<std::vector<int4>> zch(c->nz), zgr(c->nz);
  for (int gi = 0; gi < c->ngroup; ++gi) {
    int e = grp_e0[gi];
    const int eend = grp_e0[gi] + grp_ne[gi];
    while (e < eend) {
      const int z = c->ent_gi[e] / P;
      int f = e;
      while (f < eend && c->ent_gi[f] / P == z) ++f;
      int4 zg;
      zg.x = gi;
      zg.y = (int)zch[z].size();
      for (int s = e; s < f; s += rst::CHUNK) {
        int4 ch;
        ch.x = gi;
        ch.y = s;
        ch.z = std::min(rst::CHUNK, f - s);
        ch.w = 0;
        zch[z].push_back(ch);
      }
      zg.z = (int)zch[z].size();
      zg.w = groups[gi].first;
      zgr[z].push_back(zg);
      e = f;
    }
  }
  c->max_chunks = 0;
  for (int z = 0; z < c->nz; ++z) {
    c->zc_offs[z + 1] = c->zc_offs[z] + (int)zch[z].size();
    c->zg_offs[z + 1] = c->zg_offs[z] + (int)zgr[z].size();
    c->max_chunks = std::max(c->max_chunks, (int)zch[z].size());
    c->chunks.insert(c->chunks.end(), zch[z].begin(), zch[z].end());
    c->zgroups.insert(c->zgroups.end(), zgr[z].begin(), zgr[z].end());
  }
  // gather-order copies: chunk j (over all planes) holds entries j*CHUNK .. j*CHUNK+CHUNK-1
  c->g_ent_p.assign(c->chunks.size() * rst::CHUNK, 0);
  c->g_src.assign(c->chunks.size() * rst::CHUNK, -1);
  c->g_beta.assign(c->chunks.size() * rst::CHUNK * nm, 0.0);
  for (size_t j = 0; j < c->chunks.size(); ++j) {
    const int4 ch = c->chunks[j];
    for (int k = 0; k < ch.z; ++k) {
      const size_t g = j * rst::CHUNK + k;
      const int e = ch.y + k;
      c->g_ent_p[g] = c->ent_p[e];
      c->g_src[g] = e;
      for (int m = 0; m < nm; ++m) c->g_beta[g * nm + m] = c->beta[(size_t)e * nm + m];
    }
  }
  // point-centric scatter: the first SC_SLOTS entries of each point go to the
  // slot table (group order), further ones to the overflow lists
  const int K = rst::SC_SLOTS;
  c->sc_pb.assign((size_t)n * K, -1);
  c->sc_ent.assign((size_t)n * K, -1);
  c->sc_beta.assign((size_t)n * K * nm, 0.0);
  const int wn = nm <= 9 ? 9 : 16;  // the many-column apply's compile-time projector bound
  c->sc_w.assign((size_t)n * K * wn, 0.0);
  std::vector<int> used(n, 0);
  std::vector<int> cnt(n + 1, 0);
  std::vector<std::pair<long long, int2>> ovf;
  for (int gi = 0; gi < c->ngroup; ++gi)
    for (int e = grp_e0[gi]; e < grp_e0[gi] + grp_ne[gi]; ++e) {
      const long long i = c->ent_gi[e];
      if (used[i] < K) {
        const size_t si = (size_t)i * K + used[i];
        c->sc_pb[si] = c->grp_pbase[gi];
        c->sc_ent[si] = e;
        for (int m = 0; m < nm; ++m) c->sc_beta[si * nm + m] = c->beta[(size_t)e * nm + m];
        for (int m = 0; m < c->grp_nm[gi]; ++m)
          c->sc_w[si * wn + m] = c->beta[(size_t)e * nm + m] * c->ekb[c->grp_pbase[gi] + m];
        used[i]++;
      } else {
        int2 v;
        v.x = gi;
        v.y = e;
        ovf.push_back({i, v});
        cnt[i + 1]++;
      }
    }
  c->has_overflow = ovf.empty() ? 0 : 1;
  c->pe_offs.assign(n + 1, 0);
  for (long long i = 0; i < n; ++i) c->pe_offs[i + 1] = c->pe_offs[i] + cnt[i + 1];
  c->pe.assign(std::max<size_t>(1, c->pe_offs[n]), int2{0, 0});
  std::vector<int> fillp(c->pe_offs.begin(), c->pe_offs.end() - 1);
  for (auto& o : ovf) c->pe[fillp[o.first]++] = o.second;
  (void)nent;
  rst_status s;
  if ((s = upload(c, c->d_grp_pbase, c->grp_pbase)) != RST_OK) return s;
  if ((s = upload(c, c->d_grp_nm, c->grp_nm)) != RST_OK) return s;
  if ((s = upload(c, c->d_ekb, c->ekb)) != RST_OK) return s;
  if ((s = upload(c, c->d_beta, c->beta)) != RST_OK) return s;
  if ((s = upload(c, c->d_ent_p, c->ent_p)) != RST_OK) return s;
  if ((s = upload(c, c->d_g_ent_p, c->g_ent_p)) != RST_OK) return s;
  if ((s = upload(c, c->d_grp_e0, c->grp_e0)) != RST_OK) return s;
  if ((s = upload(c, c->d_grp_ne, c->grp_ne)) != RST_OK) return s;
  if ((s = upload(c, c->d_ent_gi, c->ent_gi)) != RST_OK) return s;
  if ((s = upload(c, c->d_g_beta, c->g_beta)) != RST_OK) return s;
  if ((s = upload(c, c->d_zc, c->zc_offs)) != RST_OK) return s;
  if ((s = upload(c, c->d_chunks, c->chunks)) != RST_OK) return s;
  if ((s = upload(c, c->d_zg, c->zg_offs)) != RST_OK) return s;
  if ((s = upload(c, c->d_zgroups, c->zgroups)) != RST_OK) return s;
  if ((s = upload(c, c->d_pe_offs, c->pe_offs)) != RST_OK) return s;
  if ((s = upload(c, c->d_pe, c->pe)) != RST_OK) return s;
  if ((s = upload(c, c->d_sc_pb, c->sc_pb)) != RST_OK) return s;
  if ((s = upload(c, c->d_sc_beta, c->sc_beta)) != RST_OK) return s;
  if ((s = upload(c, c->d_sc_w, c->sc_w)) != RST_OK) return s;
  return RST_OK;
}

void pc_tables(const rst_ctx* c, double ka, double kb, std::vector<double>& eps, std::vector<double2>& steps) {
  const int na = c->na, nb = c->nb;
  const double la = na * c->ha, lb = nb * c->hb;
  const double pi = 3.14159265358979323846;
  auto symbol = [&](double th) {
    double s = -c->fdw[0];
    for (int j = 1; j <= c->rad; ++j) s -= 2.0 * c->fdw[j] * std::cos(j * th);
    return s;
  };
  eps.assign((size_t)na * nb, 0.0);
  for (int mb = 0; mb < nb; ++mb)
    for (int ma = 0; ma < na; ++ma) {
      const double ta = (ka + 2 * pi * ma / la) * c->ha;
      const double tb = (kb + 2 * pi * mb / lb) * c->hb;
      eps[(size_t)mb * na + ma] = 0.5 * (symbol(ta) / (c->ha * c->ha) + symbol(tb) / (c->hb * c->hb));
    }
  // DFT recurrence steps: fa[m] = exp(-i(2 pi m/na + k_a h_a)), ia[a] = exp(+2 pi i a/na),
  // pa[a] = exp(+i k_a a h_a) (same for b)
  steps.clear();
  auto push = [&](double ph) { steps.push_back(double2{std::cos(ph), std::sin(ph)}); };
  for (int m = 0; m < na; ++m) push(-(2 * pi * m / na + ka * c->ha));
  for (int m = 0; m < nb; ++m) push(-(2 * pi * m / nb + kb * c->hb));
  for (int a = 0; a < na; ++a) push(2 * pi * a / na);
  for (int b = 0; b < nb; ++b) push(2 * pi * b / nb);
  for (int a = 0; a < na; ++a) push(ka * a * c->ha);
  for (int b = 0; b < nb; ++b) push(kb * b * c->hb);
}

// Reference potential of the preconditioner: the plane means of V (the default, pc_vref
// RST_VREF_PLANE) or, with RST_VREF_CELL, none (the kernels then use the cell mean pc.vbar).
const double* pc_vz(const rst_ctx* c) {
  return c->opts.pc_vref == RST_VREF_CELL ? nullptr : (const double*)c->d_vz.p;
}

// Lateral mode energies and DFT steps of the free-electron + CAP
// preconditioner for the current grid and k.
rst_status upload_pc(rst_ctx* c) {
  std::vector<double> eps;
  std::vector<double2> steps;
  pc_tables(c, c->ka, c->kb, eps, steps);
  rst_status s;
  if ((s = upload(c, c->d_pc_eps, eps)) != RST_OK) return s;
  return upload(c, c->d_pc_twa, steps);
}

rst_status upload_k(rst_ctx* c) {
  const double la = c->na * c->ha, lb = c->nb * c->hb;
  std::vector<double2> eph(c->ent_p.size());
  for (size_t e = 0; e < eph.size(); ++e) {
    const double ph = c->ka * la * c->ent_img[2 * e] + c->kb * lb * c->ent_img[2 * e + 1];
    eph[e].x = std::cos(ph);
    eph[e].y = std::sin(ph);
  }
  rst_status s = upload(c, c->d_eph, eph);
  if (s != RST_OK) return s;
  std::vector<double2> gph(c->g_src.size());
  for (size_t g = 0; g < gph.size(); ++g) {
    const int e = c->g_src[g];
    gph[g] = e >= 0 ? eph[e] : double2{0.0, 0.0};
  }
  if ((s = upload(c, c->d_g_eph, gph)) != RST_OK) return s;
  std::vector<double2> sce(c->sc_ent.size());
  for (size_t i = 0; i < sce.size(); ++i) {
    const int e = c->sc_ent[i];
    sce[i] = e >= 0 ? eph[e] : double2{0.0, 0.0};
  }
  return upload(c, c->d_sc_eph, sce);
}

// kernel dispatch ------------------------------------------------------------
// Instances live in kern_inst.hip (one translation unit per radius / positions).
// Kinds: 0 plain solver, 1 apply, 2 preconditioned solver, 3/4 mixed-precision
// plain/preconditioned solvers, 5/6 batched plain/preconditioned solvers.
#define RST_KINST(K)                       \
  extern "C" void* rst_kptr_k##K##_r2_q1(); \
  extern "C" void* rst_kptr_k##K##_r2_q2(); \
  extern "C" void* rst_kptr_k##K##_r6_q1(); \
  extern "C" void* rst_kptr_k##K##_r6_q2();
RST_KINST(0)
RST_KINST(1)
RST_KINST(2)
RST_KINST(3)
RST_KINST(4)
RST_KINST(5)
RST_KINST(6)
RST_KINST(7)
#undef RST_KINST

// The persistent kernels are built for FD orders 4 and 12; the other even orders 2..12 run on
// the many-column solvers.
bool persistent_order(int rad) { return rad == 2 || rad == 6; }

void* pick_kernel(int rad, int q, int w) {
#define RST_KPICK(K)                                                \
  if (w == K) {                                                     \
    if (rad == 2) return q == 1 ? rst_kptr_k##K##_r2_q1() : rst_kptr_k##K##_r2_q2(); \
    if (rad == 6) return q == 1 ? rst_kptr_k##K##_r6_q1() : rst_kptr_k##K##_r6_q2(); \
    return nullptr;                                                 \
  }
  if (q != 1 && q != 2) return nullptr;
  RST_KPICK(0)
  RST_KPICK(1)
  RST_KPICK(2)
  RST_KPICK(3)
  RST_KPICK(4)
  RST_KPICK(5)
  RST_KPICK(6)
  RST_KPICK(7)
#undef RST_KPICK
  return nullptr;
}

struct LaunchShape {
  int cw, threads, q;
};

rst_status choose_shape(rst_ctx* c, int cw_req, int t_req, LaunchShape& ls) {
  const int P = c->na * c->nb;
  int cw = cw_req > 0 ? cw_req : 1;
  if (cw > rst::CW_MAX || (cw & (cw - 1))) return fail(c, RST_EINVAL, "col_block must be a power of two <= 8");
  const int pos = P * cw;
  for (int q : {1, 2}) {
    int t = t_req > 0 ? t_req : ((pos + q - 1) / q + 63) / 64 * 64;
    if (t < 64) t = 64;
    if (t > rst::MAX_T || t % 64 || t % cw) continue;
    if ((long long)t * q < pos) continue;
    ls.cw = cw;
    ls.threads = t;
    ls.q = q;
    return RST_OK;
  }
  return fail(c, RST_EUNSUPPORTED, "plane of " + std::to_string(P) + " points x " + std::to_string(cw) +
                                       " columns does not fit one workgroup (max 2 per thread at 512 threads)");
}

rst_status check_ready(rst_ctx* c) {
  if (!c) return RST_EINVAL;
  if (!c->has_grid) return fail(c, RST_ESTATE, "rst_set_grid not called");
  if (!c->has_v) return fail(c, RST_ESTATE, "rst_set_potential not called");
  if (!c->has_abc) return fail(c, RST_ESTATE, "rst_set_abc not called");
  if (!c->has_k) return fail(c, RST_ESTATE, "rst_set_k not called");
  return RST_OK;
}

// Runs the persistent solver over ncols columns x ne energies.
rst_status run_fgmres(rst_ctx* c, int ne, const double* energies, const std::vector<int64_t>& cols,
                      const double* d_gdst, const std::vector<double>* hsrc, double2* xout,
                      std::vector<double>& Tcol, std::vector<int>& its, std::vector<int>& rss,
                      std::vector<double>& res, std::vector<int>& st, double& ms);

rst_status run_cocg(rst_ctx* c, int ne, const double* energies, const std::vector<int64_t>& cols,
                    const double* d_gdst, const std::vector<double>* hsrc, double2* xout,
                    std::vector<double>& Tcol, std::vector<int>& its, std::vector<int>& rss,
                    std::vector<double>& res, std::vector<int>& st, double& ms);

rst_status run_bicgstab_mk(rst_ctx* c, int ne, const double* energies, const std::vector<int64_t>& cols,
                           const double* d_gsrc, const double* d_gdst, double2* xout, std::vector<double>& Tcol,
                           std::vector<int>& its, std::vector<int>& rss, std::vector<double>& res,
                           std::vector<int>& st, double& ms, const double2* rhs, long long rhs_ld,
                           long long rhs_estride);

rst_status run_solver(rst_ctx* c, int ne, const double* energies, const std::vector<int64_t>& cols,
                      const double* d_gsrc, const double* d_gdst, double2* xout,
                      std::vector<double>& Tcol, std::vector<int>& its, std::vector<int>& rss,
                      std::vector<double>& res, std::vector<int>& st, double& ms,
                      const double2* rhs = nullptr, long long rhs_ld = 0, long long rhs_estride = 0) {
  c->last_mk = false;
  if (c->opts.method == RST_FGMRES) {
    const std::vector<double>* hsrc = d_gsrc == nullptr ? nullptr : (d_gsrc == c->d_gr.p ? &c->gr : &c->gl);
    return run_fgmres(c, ne, energies, cols, d_gdst, hsrc, xout, Tcol, its, rss, res, st, ms);
  }
  if (c->opts.method == RST_COCG) {
    // a real H_k (A complex symmetric) on a plane the persistent kernels hold: the blocked COCG;
    // otherwise COCG on the doubled k / -k system over many columns
    const rst::Geo g0 = make_geo(c);
    const bool real_hk = std::fabs(g0.pha_y) <= 1e-12 && std::fabs(g0.phb_y) <= 1e-12;
    if (real_hk && c->na * c->nb <= 2 * rst::MAX_T && persistent_order(c->rad) && rhs == nullptr) {
      const std::vector<double>* hsrc = d_gsrc == nullptr ? nullptr : (d_gsrc == c->d_gr.p ? &c->gr : &c->gl);
      return run_cocg(c, ne, energies, cols, d_gdst, hsrc, xout, Tcol, its, rss, res, st, ms);
    }
    if (c->opts.col_block > 0 || c->opts.threads > 0)
      return fail(c, RST_EUNSUPPORTED, "col_block and threads apply to the blocked COCG (a real H_k)");
    return run_bicgstab_mk(c, ne, energies, cols, d_gsrc, d_gdst, xout, Tcol, its, rss, res, st, ms, rhs, rhs_ld,
                           rhs_estride);
  }
  // the persistent kernels hold a whole lateral plane per workgroup; wider planes go to the
  // many-column BiCGSTAB, one kernel per step
  if (c->opts.method == RST_BICGSTAB_MC || c->opts.method == RST_IDRS || c->na * c->nb > 2 * rst::MAX_T ||
      !persistent_order(c->rad)) {
    if (c->opts.col_block > 0 || c->opts.threads > 0)
      return fail(c, RST_EUNSUPPORTED, "col_block and threads apply to the persistent kernels (planes of at most " +
                                           std::to_string(2 * rst::MAX_T) + " points)");
    return run_bicgstab_mk(c, ne, energies, cols, d_gsrc, d_gdst, xout, Tcol, its, rss, res, st, ms, rhs, rhs_ld,
                           rhs_estride);
  }
  LaunchShape ls;
  rst_status s = choose_shape(c, c->opts.col_block, c->opts.threads, ls);
  if (s != RST_OK) return s;
  const int ncols = (int)cols.size();
  const int nblk = (ncols + ls.cw - 1) / ls.cw;
  c->last_cw = ls.cw;
  c->last_threads = ls.threads;
  const long long nitems = (long long)nblk * ne;
  if (nitems > 0x7fffffff) return fail(c, RST_EINVAL, "too many column blocks");
  const size_t n = (size_t)c->na * c->nb * c->nz;
  const bool pc = c->opts.precond == RST_PRECOND_FREE_CAP;
  const bool mixed = c->opts.precision == RST_FP32_REFINE;
  void* kern = pick_kernel(c->rad, ls.q, mixed ? (pc ? 4 : 3) : (pc ? 2 : 0));
  if (!kern) return fail(c, RST_EUNSUPPORTED, "no kernel instance");
  rst::Geo g = make_geo(c);
  rst::Proj pj = make_proj(c);
  size_t lds = rst::lds_bytes<double>(g.pa, g.pb, g.P, pj.nproj, pj.max_chunks, pj.nm, ls.cw, ls.threads);
  const size_t pc_off = (lds + 15) & ~size_t(15);
  if (pc) lds = pc_off + (size_t)3 * (c->na + c->nb) * 16;
  int dev_lds = 0;
  HIPCHK(c, hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
  if (lds + sizeof(rst::ColState) + 1024 > (size_t)dev_lds)
    return fail(c, RST_EUNSUPPORTED, "LDS requirement " + std::to_string(lds) + " exceeds the device limit");
  if (lds > 64 * 1024) HIPCHK(c, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = 0;
  HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, ls.threads, lds));
  if (per_cu < 1) return fail(c, RST_EUNSUPPORTED, "kernel does not fit on a compute unit");
  int ncu = 0;
  HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  long long nwg = std::min<long long>(nitems, (long long)per_cu * ncu);
  // bound the workspace to a quarter of free memory
  // x r p v t (+ ph sh s w with the preconditioner); mixed: FP64 x and the FP32 vectors
  const size_t nfv = pc ? 9 : 5;
  const size_t ws_stride = mixed ? n * ls.cw + (nfv * n * ls.cw + 1) / 2
                                 : nfv * n * ls.cw;  // elements of cx<double>
  size_t free_b = 0, total_b = 0;
  HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
  const size_t per_wg = ws_stride * sizeof(cx<double>) + 5 * (size_t)c->nproj * ls.cw * 16;
  const long long cap = std::max<long long>(1, (long long)(free_b / 4 / per_wg));
  nwg = std::min(nwg, cap);
  if ((s = ensure(c, c->d_ws, nwg * ws_stride * sizeof(cx<double>))) != RST_OK) return s;
  const size_t pws_stride = std::max<size_t>(1, 5 * (size_t)c->nproj * ls.cw);
  if ((s = ensure(c, c->d_pws, nwg * pws_stride * 16)) != RST_OK) return s;
  std::vector<double> en(energies, energies + ne);
  if ((s = upload(c, c->d_en, en)) != RST_OK) return s;
  if ((s = upload(c, c->d_cols, cols)) != RST_OK) return s;
  const size_t nout = (size_t)ne * ncols;
  if ((s = ensure(c, c->d_T, nout * 8)) != RST_OK) return s;
  if ((s = ensure(c, c->d_it, nout * 4)) != RST_OK) return s;
  if ((s = ensure(c, c->d_rs, nout * 4)) != RST_OK) return s;
  if ((s = ensure(c, c->d_res, nout * 8)) != RST_OK) return s;
  if ((s = ensure(c, c->d_st, nout * 4)) != RST_OK) return s;
  if ((s = ensure(c, c->d_counter, 64)) != RST_OK) return s;
  if (mixed && (s = ensure(c, c->d_up, nout * 4)) != RST_OK) return s;
  rst::SolveArgs A;
  std::memset(&A, 0, sizeof(A));
  A.g = g;
  A.pj = pj;
  A.pc_lds_off = pc_off;
  if (pc) {
    double vbar = 0;
    for (double x : c->v) vbar += x;
    A.pc.vbar = vbar / (double)c->v.size();
    A.pc.a = 0.5 / (c->hz * c->hz);
    A.pc.eps = (const double*)c->d_pc_eps.p;
    A.pc.vz = pc_vz(c);
    A.pc.shift = c->opts.pc_shift;
    A.pc.steps = (const double2*)c->d_pc_twa.p;
    if ((s = ensure(c, c->d_pc_inv, (size_t)ne * n * 16)) != RST_OK) return s;
    A.pc.inv = (const double2*)c->d_pc_inv.p;
  }
  A.V = (const double*)c->d_v.p;
  A.gz = (const double*)c->d_gz.p;
  A.gdst = d_gdst;
  A.gsrc = d_gsrc;
  A.energies = (const double*)c->d_en.p;
  A.cols = (const int64_t*)c->d_cols.p;
  A.ncols = ncols;
  A.ne = ne;
  A.cw = ls.cw;
  A.nblk = nblk;
  A.nitems = (int)nitems;
  A.tol = c->opts.tol;
  A.max_iter = c->opts.max_iter;
  A.delta = c->opts.update_delta;
  A.updates = mixed ? (int*)c->d_up.p : nullptr;
  A.ws = c->d_ws.p;
  A.ws_stride = ws_stride;
  A.pws = (double2*)c->d_pws.p;
  A.pws_stride = pws_stride;
  A.T_col = (double*)c->d_T.p;
  A.iters = (int*)c->d_it.p;
  A.restarts = (int*)c->d_rs.p;
  A.resid = (double*)c->d_res.p;
  A.status = (int*)c->d_st.p;
  A.counter = (int*)c->d_counter.p;
  A.xout = xout;
  A.rhs = rhs;
  A.rhs_ld = rhs_ld;
  A.rhs_estride = rhs_estride;
  hipLaunchKernelGGL(rst::k_fill_int, dim3(1), dim3(64), 0, c->stream, (int*)c->d_counter.p, 16, 0);
  HIPCHK(c, hipGetLastError());
  if ((s = ensure(c, c->d_args, sizeof(A))) != RST_OK) return s;
  c->h_solve = A;
  HIPCHK(c, hipMemcpyAsync(c->d_args.p, &c->h_solve, sizeof(A), hipMemcpyHostToDevice, c->stream));
  if (pc) {
    const long long nt = (long long)ne * c->na * c->nb;
    hipLaunchKernelGGL(rst::k_pc_pivots, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream,
                       (const rst::SolveArgs*)c->d_args.p);
    HIPCHK(c, hipGetLastError());
  }
  void* dargs = c->d_args.p;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, hipEventRecord(e0, c->stream));
  void* args[] = {&dargs};
  HIPCHK(c, hipLaunchKernel(kern, dim3((unsigned)nwg), dim3(ls.threads), args, lds, c->stream));
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float fms = 0;
  HIPCHK(c, hipEventElapsedTime(&fms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  ms = fms;
  Tcol.resize(nout);
  its.resize(nout);
  rss.resize(nout);
  res.resize(nout);
  st.resize(nout);
  HIPCHK(c, hipMemcpy(Tcol.data(), c->d_T.p, nout * 8, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(its.data(), c->d_it.p, nout * 4, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(rss.data(), c->d_rs.p, nout * 4, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(res.data(), c->d_res.p, nout * 8, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(st.data(), c->d_st.p, nout * 4, hipMemcpyDeviceToHost));
  c->last_updates.assign(mixed ? nout : 0, 0);
  if (mixed) HIPCHK(c, hipMemcpy(c->last_updates.data(), c->d_up.p, nout * 4, hipMemcpyDeviceToHost));
  return RST_OK;
}

// Mixed precision: columns the FP32 recurrences did not converge are solved
// again with the FP64 kernel (per energy, only those columns); their results
// replace the mixed ones.  With an x export the whole set is solved again.
rst_status mixed_fp64_fallback(rst_ctx* c, int ne, const double* energies, const std::vector<int64_t>& cols,
                               const double* d_gsrc, const double* d_gdst, double2* xout, std::vector<double>& Tcol,
                               std::vector<int>& its, std::vector<int>& rss, std::vector<double>& res,
                               std::vector<int>& stv, double& ms) {
  if (c->opts.precision != RST_FP32_REFINE) return RST_OK;
  c->last_fallbacks = 0;
  c->last_extra_bytes = 0.0;
  const size_t ncols = cols.size();
  bool any = false;
  for (int v : stv) any = any || v != 0;
  if (!any) return RST_OK;
  const int saved = c->opts.precision;
  const std::vector<int> ups = c->last_updates;
  c->opts.precision = RST_FP64;
  const double streams = c->opts.precond == RST_PRECOND_FREE_CAP ? 24.0 : 12.0;
  const double n = (double)c->na * c->nb * c->nz;
  rst_status s = RST_OK;
  for (int ie = 0; ie < ne && s == RST_OK; ++ie) {
    std::vector<int64_t> sub;
    std::vector<size_t> where;
    for (size_t j = 0; j < ncols; ++j)
      if (xout || stv[(size_t)ie * ncols + j] != 0) {
        sub.push_back(cols[j]);
        where.push_back((size_t)ie * ncols + j);
      }
    if (sub.empty()) continue;
    std::vector<double> T2, r2;
    std::vector<int> i2, s2, st2;
    double ms2 = 0;
    s = run_solver(c, 1, energies + ie, sub, d_gsrc, d_gdst, xout, T2, i2, s2, r2, st2, ms2);
    if (s != RST_OK) break;
    ms += ms2;
    for (size_t q = 0; q < sub.size(); ++q) {
      const size_t o = where[q];
      if (stv[o] != 0) c->last_fallbacks += 1;
      Tcol[o] = T2[q];
      its[o] += i2[q];
      c->last_extra_bytes += (double)i2[q] * streams * 16.0 * n;
      rss[o] = s2[q];
      res[o] = r2[q];
      stv[o] = st2[q];
    }
  }
  c->opts.precision = saved;
  c->last_updates = ups;
  return s;
}

void fill_stats(rst_ctx* c, rst_stats* st, const std::vector<int>& its, const std::vector<int>& rss,
                const std::vector<double>& res, const std::vector<int>& stv, double ms, int& nbad,
                int cw = 0, int threads = 0, double n_override = 0.0) {
  nbad = 0;
  rst_stats s;
  std::memset(&s, 0, sizeof(s));
  s.columns = (int64_t)its.size();
  for (size_t i = 0; i < its.size(); ++i) {
    s.iterations_total += its[i];
    s.iterations_max = std::max(s.iterations_max, its[i]);
    s.restarts_total += rss[i];
    s.max_rel_residual = std::max(s.max_rel_residual, res[i]);
    if (stv[i] != 0) ++nbad;
  }
  s.columns_unconverged = nbad;
  const bool mixed = c->opts.precision == RST_FP32_REFINE && c->last_updates.size() == its.size();
  if (mixed)
    for (int u : c->last_updates) s.updates_total += u;
  const bool fgm = (c->opts.method == RST_FGMRES || c->opts.method == RST_COCG) && n_override == 0.0;
  if (fgm) {
    s.fallback_columns = c->last_fallbacks;
    s.cnn_flop = c->last_cnn_flop;
  }
  if (mixed) s.fallback_columns = c->last_fallbacks;
  s.kernel_ms = ms;
  s.col_block = cw;
  s.threads = threads;
  const double n = n_override > 0 ? n_override : (double)c->na * c->nb * c->nz;
  const double streams = c->opts.precond == RST_PRECOND_FREE_CAP ? 24.0 : 12.0;
  if (mixed)
    // iterations on FP32 vectors; per reliable update: the fold (read x64 and x32,
    // write x64 and x32 = 0: 48 B) and the FP64 residual (read x64, write r32: 24 B)
    s.bytes_algorithmic = (double)s.iterations_total * streams * 8.0 * n +
                          (double)s.updates_total * 72.0 * n + c->last_extra_bytes;
  else if (fgm)
    s.bytes_algorithmic = c->last_fg_bytes;
  else if (c->last_mk)
    s.bytes_algorithmic = c->last_mk_bytes;
  else
    s.bytes_algorithmic = (double)s.iterations_total * streams * 16.0 * n;
  if (st) *st = s;
}


// Launch shape of the blocked apply and M^-1 kernels: the widest column block
// (<= 8, at most two positions per thread) whose LDS fits the device.
struct BlockedShape {
  LaunchShape ls;
  size_t lds_apply = 0, lds_pc = 0, pc_off = 0;
};

rst_status blocked_shape(rst_ctx* c, int cw_max, int threads_req, BlockedShape& bs) {
  const int P = c->na * c->nb;
  int dev_lds = 0;
  HIPCHK(c, hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
  rst::Geo g = make_geo(c);
  rst::Proj pj = make_proj(c);
  for (int cw = std::min(cw_max, rst::CW_MAX); cw >= 1; cw /= 2) {
    if ((long long)P * cw > 2LL * rst::MAX_T && cw > 1) continue;
    LaunchShape ls;
    if (choose_shape(c, cw, threads_req, ls) != RST_OK) continue;
    const size_t la = rst::lds_bytes<double>(g.pa, g.pb, g.P, pj.nproj, pj.max_chunks, pj.nm, ls.cw, ls.threads);
    size_t lp = rst::lds_bytes<double>(g.pa, g.pb, g.P, 0, 0, pj.nm, ls.cw, ls.threads);
    const size_t po = (lp + 15) & ~size_t(15);
    lp = po + (size_t)3 * (c->na + c->nb) * 16;
    if (std::max(la, lp) + sizeof(rst::ColState) + 1024 <= (size_t)dev_lds) {
      bs.ls = ls;
      bs.lds_apply = la;
      bs.lds_pc = lp;
      bs.pc_off = po;
      c->err.clear();
      return RST_OK;
    }
  }
  return fail(c, RST_EUNSUPPORTED, "no column block fits the device LDS");
}

// Flexible GMRES(m) over chunks of columns (host-driven; every vector
// operation is one of the fg kernels, the stencil apply or the preconditioner
// kernel).  Preconditioner per column: z = v (NONE), z = M^-1 v (FREE_CAP) or
// z = M^-1 v + f(v, M^-1 v) (LEARNED).  A column whose true residual did not
// fall below fallback_ratio times its previous cycle's value while the
// learned correction was on continues with M^-1 alone.
rst_status run_fgmres(rst_ctx* c, int ne, const double* energies, const std::vector<int64_t>& cols,
                      const double* d_gdst, const std::vector<double>* hsrc, double2* xout,
                      std::vector<double>& Tcol, std::vector<int>& its, std::vector<int>& rss,
                      std::vector<double>& res, std::vector<int>& st, double& ms) {
  const bool learned = c->opts.precond == RST_PRECOND_LEARNED;
  const bool usepc = c->opts.precond != RST_PRECOND_NONE;
  if (learned && (!c->cnn || !rst::cnn::engine_has_weights(c->cnn)))
    return fail(c, RST_ESTATE, "the learned preconditioner has no network weights");
  const int m = c->opts.restart;
  const int P = c->na * c->nb;
  const long long n = (long long)P * c->nz;
  const int ncols = (int)cols.size();
  // launch shape shared by the apply and preconditioner kernels
  BlockedShape bs;
  // automatic: one column per workgroup (config 2: 5.7 s against 6.0 s with the widest block on 512
  // columns)
  rst_status s = blocked_shape(c, c->opts.col_block > 0 ? c->opts.col_block : 1, c->opts.threads, bs);
  if (s != RST_OK) return s;
  const LaunchShape ls = bs.ls;
  const int cw = ls.cw;
  c->last_cw = cw;
  c->last_threads = ls.threads;
  void* kapply = pick_kernel(c->rad, ls.q, 1);
  void* kpc = pick_kernel(c->rad, ls.q, 7);
  if (!kapply || !kpc) return fail(c, RST_EUNSUPPORTED, "no kernel instance");
  // chunk of columns: bounded by a quarter of free memory
  const size_t per_col = (size_t)(2 * m + 6) * n * 16 + (size_t)(learned ? 11 * 64 + 24 : 0) * n;
  size_t free_b = 0, total_b = 0;
  HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
  long long chunk = std::min<long long>(512, std::max<long long>(cw, (long long)(free_b / 4 / per_col)));
  chunk = std::max<long long>(cw, chunk / cw * cw);
  chunk = std::min<long long>(chunk, ((long long)ncols + cw - 1) / cw * cw);
  const int ncolp = (int)chunk;
  const int nblk = ncolp / cw;
  const size_t vlen = (size_t)nblk * n * cw;  // elements of one chunk vector
  rst_status e;
  if ((e = ensure(c, c->d_fgV, (size_t)(m + 1) * vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgZ, (size_t)m * vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgX, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgW, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgM, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgwb, vlen * 16)) != RST_OK) return e;
  if (learned) {
    if ((e = ensure(c, c->d_fgx0, (size_t)ncolp * n * 16)) != RST_OK) return e;
    if ((e = ensure(c, c->d_fgf, (size_t)ncolp * n * 8)) != RST_OK) return e;
  }
  const size_t m1 = (size_t)m + 1;
  if ((e = ensure(c, c->d_fgH, (size_t)ncolp * m1 * m * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgcs, (size_t)ncolp * m * 8)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgsn, (size_t)ncolp * m * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgg, (size_t)ncolp * m1 * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fginv, (size_t)ncolp * 8)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgest, (size_t)ncolp * 8)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgact, (size_t)ncolp * 4)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgit, (size_t)ncolp * 4)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fguse, (size_t)ncolp * 4)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgh1, m1 * ncolp * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgh2, m1 * ncolp * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgn2, (size_t)ncolp * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgy, (size_t)m * ncolp * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgsrc, (size_t)ncolp * 8)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgbsc, (size_t)ncolp * 8)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgt, (size_t)ncolp * 8)) != RST_OK) return e;
  // kernel arguments: apply slots j < m (Z_j -> W) and m (X -> W); preconditioner slots j <= m (V_j -> M or Z_j)
  rst::Geo g = make_geo(c);
  rst::Proj pj = make_proj(c);
  const size_t pws_stride = std::max<size_t>(1, (size_t)c->nproj * cw);
  if ((e = ensure(c, c->d_pws, (size_t)nblk * pws_stride * 16)) != RST_OK) return e;
  const size_t lds_apply = bs.lds_apply, lds_pc = bs.lds_pc, pc_off = bs.pc_off;
  if (lds_apply > 64 * 1024)
    HIPCHK(c, hipFuncSetAttribute(kapply, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_apply));
  if (lds_pc > 64 * 1024) HIPCHK(c, hipFuncSetAttribute(kpc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_pc));
  double2* V = (double2*)c->d_fgV.p;
  double2* Z = (double2*)c->d_fgZ.p;
  double2* X = (double2*)c->d_fgX.p;
  double2* W = (double2*)c->d_fgW.p;
  double2* Mb = (double2*)c->d_fgM.p;
  rst::fg::Shape S{n, cw, nblk, 0, m};
  rst::fg::Hess Hs{(double2*)c->d_fgH.p, (double*)c->d_fgcs.p, (double2*)c->d_fgsn.p, (double2*)c->d_fgg.p,
                   (double*)c->d_fginv.p, (double*)c->d_fgest.p, (const int*)c->d_fgact.p, (int*)c->d_fgit.p};
  std::vector<double> en(energies, energies + ne);
  if ((e = upload(c, c->d_en, en)) != RST_OK) return e;
  double vbar = 0;
  for (double x : c->v) vbar += x;
  vbar /= (double)c->v.size();
  if (usepc && (e = ensure(c, c->d_pc_inv, (size_t)n * 16)) != RST_OK) return e;
  const size_t nout = (size_t)ne * ncols;
  Tcol.assign(nout, 0.0);
  its.assign(nout, 0);
  rss.assign(nout, 0);
  res.assign(nout, 0.0);
  st.assign(nout, 1);
  c->last_fallbacks = 0;
  c->last_cnn_flop = 0.0;
  c->last_updates.clear();
  double bytes = 0.0;
  const double cnn_flop_col = [&]() {
    // 2 * 27 * cin * cout flops per point and layer, at the level of the layer
    const double n0 = (double)n;
    const double n1 = (double)((c->nz + 1) / 2) * ((c->nb + 1) / 2) * ((c->na + 1) / 2);
    const double n2 = (double)((c->nz + 3) / 4) * ((c->nb + 3) / 4) * ((c->na + 3) / 4);
    const double k16 = 2.0 * 27 * 16 * 16;
    return n0 * (2.0 * 27 * 4 * 16 + k16 + k16 + 2.0 * 27 * 16 * 2) + n1 * 3 * k16 + n2 * 2 * k16;
  }();
  const unsigned gv = (unsigned)((vlen + 255) / 256);
  const unsigned gc = (unsigned)((ncolp + 63) / 64);
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, hipEventRecord(e0, c->stream));
  const int max_cycles = std::max(1, (c->opts.max_iter + m - 1) / m);
  double export_ms = 0.0;
  for (int ie = 0; ie < ne; ++ie) {
    const double energy = energies[ie];
    // kernel arguments of this energy
    std::vector<rst::ApplyArgs> aa(m + 1);
    for (int j = 0; j <= m; ++j) {
      rst::ApplyArgs& A = aa[j];
      std::memset(&A, 0, sizeof(A));
      A.g = g;
      A.pj = pj;
      A.V = (const double*)c->d_v.p;
      A.gz = (const double*)c->d_gz.p;
      A.energy = energy;
      A.x = j < m ? Z + (size_t)j * vlen : X;
      A.y = W;
      A.ncol = ncolp;
      A.cw = cw;
      A.nblk = nblk;
      A.pws = (double2*)c->d_pws.p;
      A.pws_stride = pws_stride;
      A.proj_pre = c->nproj > 0;
    }
    if ((e = upload(c, c->d_fgaa, aa)) != RST_OK) return e;
    if (usepc) {
      // Thomas pivots of this energy
      rst::SolveArgs A;
      std::memset(&A, 0, sizeof(A));
      A.g = g;
      A.gz = (const double*)c->d_gz.p;
      A.energies = (const double*)c->d_en.p + ie;
      A.ne = 1;
      A.pc.vbar = vbar;
      A.pc.a = 0.5 / (c->hz * c->hz);
      A.pc.eps = (const double*)c->d_pc_eps.p;
      A.pc.vz = pc_vz(c);
      A.pc.shift = c->opts.pc_shift;
      A.pc.steps = (const double2*)c->d_pc_twa.p;
      A.pc.inv = (const double2*)c->d_pc_inv.p;
      std::vector<rst::SolveArgs> sa(1, A);
      if ((e = upload(c, c->d_fgsa, sa)) != RST_OK) return e;
      hipLaunchKernelGGL(rst::k_pc_pivots, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, c->stream,
                         (const rst::SolveArgs*)c->d_fgsa.p);
      HIPCHK(c, hipGetLastError());
      std::vector<rst::PcApplyArgs> pa(m + 1);
      for (int j = 0; j <= m; ++j) {
        rst::PcApplyArgs& B = pa[j];
        std::memset(&B, 0, sizeof(B));
        B.g = g;
        B.pc = A.pc;
        B.in = V + (size_t)j * vlen;
        B.out = (learned || j == m) ? Mb : Z + (size_t)j * vlen;
        B.wbuf = (double2*)c->d_fgwb.p;
        B.cw = cw;
        B.nblk = nblk;
        B.pc_lds_off = pc_off;
      }
      if ((e = upload(c, c->d_fgpa, pa)) != RST_OK) return e;
    }
    for (int c0 = 0; c0 < ncols; c0 += ncolp) {
      const int nc = std::min(ncolp, ncols - c0);
      S.ncol = nc;
      std::vector<long long> src(ncolp, -1);
      std::vector<double> bsc(ncolp, 0.0), bnorm(ncolp, 0.0), prev(ncolp, 1.0);
      std::vector<int> act(ncolp, 0), use(ncolp, 0), cyc(ncolp, 0), fb(ncolp, 0);
      for (int j = 0; j < nc; ++j) {
        src[j] = cols[c0 + j];
        const double gs = hsrc ? (*hsrc)[cols[c0 + j] / P] : 1.0;
        bsc[j] = std::sqrt(gs);
        bnorm[j] = bsc[j];
        act[j] = 1;
        use[j] = learned ? 1 : 0;
      }
      std::vector<int> zero(ncolp, 0);
      if ((e = upload(c, c->d_fgsrc, src)) != RST_OK) return e;
      if ((e = upload(c, c->d_fgbsc, bsc)) != RST_OK) return e;
      if ((e = upload(c, c->d_fgact, act)) != RST_OK) return e;
      if ((e = upload(c, c->d_fguse, use)) != RST_OK) return e;
      if ((e = upload(c, c->d_fgit, zero)) != RST_OK) return e;
      hipLaunchKernelGGL(rst::fg::k_fg_init, dim3(gv), dim3(256), 0, c->stream, S, (const long long*)c->d_fgsrc.p,
                         (const double*)c->d_fgbsc.p, X, W);
      HIPCHK(c, hipGetLastError());
      std::vector<double2> n2(ncolp);
      std::vector<double> est(ncolp);
      for (int cy = 0; cy < max_cycles; ++cy) {
        // start: V0 = R / ||R|| (R is in W)
        hipLaunchKernelGGL(rst::fg::k_fg_dots, dim3(nblk, 1), dim3(256), 0, c->stream, S, (const double2*)W,
                           (long long)vlen, 1, (const double2*)W, (double2*)c->d_fgn2.p, ncolp);
        hipLaunchKernelGGL(rst::fg::k_fg_start, dim3(gc), dim3(64), 0, c->stream, S, (const double2*)c->d_fgn2.p,
                           Hs, ncolp);
        hipLaunchKernelGGL(rst::fg::k_fg_scale, dim3(gv), dim3(256), 0, c->stream, S, V, (const double2*)W,
                           (const double*)c->d_fginv.p);
        HIPCHK(c, hipGetLastError());
        int k = 0;
        int nact = 0;
        for (int j = 0; j < nc; ++j) nact += act[j];
        for (int j = 0; j < m; ++j) {
          double2* Vj = V + (size_t)j * vlen;
          double2* Zj = Z + (size_t)j * vlen;
          // Z_j = precondition(V_j)
          if (usepc) {
            void* pargs = (char*)c->d_fgpa.p + (size_t)j * sizeof(rst::PcApplyArgs);
            void* args[] = {&pargs};
            HIPCHK(c, hipLaunchKernel(kpc, dim3(nblk), dim3(ls.threads), args, lds_pc, c->stream));
            bytes += (double)nact * n * 16.0 * 4;
            if (learned) {
              const long long tot = (long long)nc * n;
              hipLaunchKernelGGL(rst::fg::k_fg_features, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                                 c->stream, S, (const double2*)Vj, (const double2*)Mb, (float*)c->d_fgx0.p);
              HIPCHK(c, hipGetLastError());
              hipError_t he = rst::cnn::engine_forward(c->cnn, (const float*)c->d_fgx0.p, (float*)c->d_fgf.p, nc,
                                                       c->nz, c->nb, c->na, false);
              if (he != hipSuccess) return fail(c, RST_EDEVICE, std::string("network: ") + hipGetErrorString(he));
              hipLaunchKernelGGL(rst::fg::k_fg_combine, dim3(gv), dim3(256), 0, c->stream, S, (const double2*)Mb,
                                 (const float*)c->d_fgf.p, (const int*)c->d_fguse.p, Zj);
              HIPCHK(c, hipGetLastError());
              c->last_cnn_flop += cnn_flop_col * nc;
            }
          } else {
            HIPCHK(c, hipMemcpyAsync(Zj, Vj, vlen * 16, hipMemcpyDeviceToDevice, c->stream));
          }
          // W = A Z_j
          {
            void* aargs = (char*)c->d_fgaa.p + (size_t)j * sizeof(rst::ApplyArgs);
            void* args[] = {&aargs};
            if ((e = proj_blocked(c, aa[j])) != RST_OK) return e;
            HIPCHK(c, hipLaunchKernel(kapply, dim3(nblk), dim3(ls.threads), args, lds_apply, c->stream));
          }
          // CGS2 against V_0..V_j, then ||W||, the Hessenberg column and V_{j+1}
          double2* h1 = (double2*)c->d_fgh1.p;
          double2* h2 = (double2*)c->d_fgh2.p;
          hipLaunchKernelGGL(rst::fg::k_fg_dots, dim3(nblk, j + 1), dim3(256), 0, c->stream, S, (const double2*)V,
                             (long long)vlen, j + 1, (const double2*)W, h1, ncolp);
          hipLaunchKernelGGL(rst::fg::k_fg_update, dim3(gv), dim3(256), 0, c->stream, S, W, (const double2*)V,
                             (long long)vlen, j + 1, (const double2*)h1, ncolp, -1.0);
          hipLaunchKernelGGL(rst::fg::k_fg_dots, dim3(nblk, j + 1), dim3(256), 0, c->stream, S, (const double2*)V,
                             (long long)vlen, j + 1, (const double2*)W, h2, ncolp);
          hipLaunchKernelGGL(rst::fg::k_fg_update, dim3(gv), dim3(256), 0, c->stream, S, W, (const double2*)V,
                             (long long)vlen, j + 1, (const double2*)h2, ncolp, -1.0);
          hipLaunchKernelGGL(rst::fg::k_fg_dots, dim3(nblk, 1), dim3(256), 0, c->stream, S, (const double2*)W,
                             (long long)vlen, 1, (const double2*)W, (double2*)c->d_fgn2.p, ncolp);
          hipLaunchKernelGGL(rst::fg::k_fg_arnoldi, dim3(gc), dim3(64), 0, c->stream, S, j, (const double2*)h1,
                             (const double2*)h2, (const double2*)c->d_fgn2.p, Hs, ncolp);
          hipLaunchKernelGGL(rst::fg::k_fg_scale, dim3(gv), dim3(256), 0, c->stream, S, V + (size_t)(j + 1) * vlen,
                             (const double2*)W, (const double*)c->d_fginv.p);
          HIPCHK(c, hipGetLastError());
          bytes += (double)nact * n * 16.0 * (4.0 * (j + 1) + 10.0);
          k = j + 1;
          HIPCHK(c, hipMemcpyAsync(est.data(), c->d_fgest.p, (size_t)ncolp * 8, hipMemcpyDeviceToHost, c->stream));
          HIPCHK(c, hipStreamSynchronize(c->stream));
          bool all = true;
          for (int q = 0; q < nc; ++q)
            if (act[q] && !(est[q] <= 0.5 * c->opts.tol * bnorm[q])) all = false;
          if (all) break;
        }
        // X += sum_{i<k} Z_i y_i
        hipLaunchKernelGGL(rst::fg::k_fg_trisolve, dim3(gc), dim3(64), 0, c->stream, S, k, Hs, (double2*)c->d_fgy.p,
                           ncolp);
        hipLaunchKernelGGL(rst::fg::k_fg_update, dim3(gv), dim3(256), 0, c->stream, S, X, (const double2*)Z,
                           (long long)vlen, k, (const double2*)c->d_fgy.p, ncolp, 1.0);
        HIPCHK(c, hipGetLastError());
        // true residual R = b - A X (into W)
        {
          void* aargs = (char*)c->d_fgaa.p + (size_t)m * sizeof(rst::ApplyArgs);
          void* args[] = {&aargs};
          if ((e = proj_blocked(c, aa[m])) != RST_OK) return e;
          HIPCHK(c, hipLaunchKernel(kapply, dim3(nblk), dim3(ls.threads), args, lds_apply, c->stream));
        }
        hipLaunchKernelGGL(rst::fg::k_fg_resid, dim3(gv), dim3(256), 0, c->stream, S, (const long long*)c->d_fgsrc.p,
                           (const double*)c->d_fgbsc.p, (const double2*)W, W);
        hipLaunchKernelGGL(rst::fg::k_fg_dots, dim3(nblk, 1), dim3(256), 0, c->stream, S, (const double2*)W,
                           (long long)vlen, 1, (const double2*)W, (double2*)c->d_fgn2.p, ncolp);
        HIPCHK(c, hipGetLastError());
        bytes += (double)nact * n * 16.0 * (k + 6.0);
        HIPCHK(c, hipMemcpyAsync(n2.data(), c->d_fgn2.p, (size_t)ncolp * 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        bool any = false, use_changed = false;
        for (int q = 0; q < nc; ++q) {
          if (!act[q]) continue;
          cyc[q] += 1;
          const double rel = std::sqrt(n2[q].x) / bnorm[q];
          res[(size_t)ie * ncols + c0 + q] = rel;
          if (!std::isfinite(rel)) {
            act[q] = 0;
            st[(size_t)ie * ncols + c0 + q] = 2;
          } else if (rel <= c->opts.tol) {
            act[q] = 0;
            st[(size_t)ie * ncols + c0 + q] = 0;
          } else {
            if (use[q] && rel > c->opts.fallback_ratio * prev[q]) {
              use[q] = 0;
              fb[q] = 1;
              use_changed = true;
            }
            any = true;
          }
          prev[q] = rel;
        }
        if (!any) break;
        if ((e = upload(c, c->d_fgact, act)) != RST_OK) return e;
        if (use_changed && (e = upload(c, c->d_fguse, use)) != RST_OK) return e;
      }
      // T accumulation, per-column results, optional export of x
      if (d_gdst) {
        hipLaunchKernelGGL(rst::fg::k_fg_tacc, dim3(nblk), dim3(256), 0, c->stream, S, (const double2*)X, d_gdst,
                           (long long)P, (double*)c->d_fgt.p);
        HIPCHK(c, hipGetLastError());
        std::vector<double> ta(ncolp);
        HIPCHK(c, hipMemcpyAsync(ta.data(), c->d_fgt.p, (size_t)ncolp * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int q = 0; q < nc; ++q) Tcol[(size_t)ie * ncols + c0 + q] = 4.0 * ta[q];
      }
      std::vector<int> itv(ncolp);
      HIPCHK(c, hipMemcpyAsync(itv.data(), c->d_fgit.p, (size_t)ncolp * 4, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      for (int q = 0; q < nc; ++q) {
        its[(size_t)ie * ncols + c0 + q] = itv[q];
        rss[(size_t)ie * ncols + c0 + q] = cyc[q];
        c->last_fallbacks += fb[q];
        if (st[(size_t)ie * ncols + c0 + q] != 0 && st[(size_t)ie * ncols + c0 + q] != 2)
          st[(size_t)ie * ncols + c0 + q] = 1;
      }
      if (xout) {
        // x (n x ncols, column fastest) from the blocked X (a test-sized export through the
        // host, kept out of the reported time)
        const auto t_exp = std::chrono::steady_clock::now();
        std::vector<double2> hx(vlen), rows((size_t)n * nc);
        HIPCHK(c, hipMemcpyAsync(hx.data(), X, vlen * 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int q = 0; q < nc; ++q)
          for (long long p = 0; p < n; ++p) rows[(size_t)p * nc + q] = hx[((size_t)(q / cw) * n + p) * cw + q % cw];
        HIPCHK(c, hipMemcpy2D(xout + c0, (size_t)ncols * 16, rows.data(), (size_t)nc * 16, (size_t)nc * 16, (size_t)n,
                              hipMemcpyHostToDevice));
        export_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_exp).count();
      }
    }
  }
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float fms = 0;
  HIPCHK(c, hipEventElapsedTime(&fms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  ms = std::max(0.0, (double)fms - export_ms);
  c->last_fg_bytes = bytes;
  return RST_OK;
}

// Preconditioned COCG over chunks of columns (host-driven like FGMRES; every
// vector operation is a kernel of rst_cocg.hpp, the blocked stencil apply or
// the M^-1 kernel).  Needs a real H_k: complex symmetric A and M.  The
// recursive residual norm is read every CHECK steps; a column whose estimate
// fell below tol, or whose recurrence broke down (p^T A p or rho zero), has
// its FP64 true residual computed: below tol it is done, otherwise the
// chunk's residual is replaced by the true one and that column restarts with
// p = M^-1 r.  Columns still running at max_iter end unconverged.
// Algorithmic bytes per grid point, iteration and column of the many-column BiCGSTAB: p update
// 64, M^-1 p 192 (four DFT passes and the Thomas sweeps, each reading and writing the block),
// apply 32, (r0h, v) 32, s update 48, M^-1 s 192, apply 32, (t, s) and (t, t) 32, x/r update and
// dots 128; without the preconditioner the two M^-1 passes drop out.  Plus 16 B per projector
// sphere entry per apply (the projections read x at the entries).
double mk_bytes_per_point(bool pc) { return pc ? 752.0 : 368.0; }

// Algorithmic bytes per grid point, operator apply and column of the many-column IDR(s), averaged over
// a cycle of s + 1 applies: step k reads r and g_k..g_{s-1} and writes v (s - k + 2 streams), forms
// u_k from u_k..u_{s-1} and M^-1 v (s - k + 2), applies M^-1 (12) and A (2), the dots read g_k (1),
// the update reads and writes g_k, u_k, r, x and reads g_0..g_{k-1}, u_0..u_{k-1} (2k + 8); the
// dimension-reduction step costs M^-1, A, the two dots (2) and the r/x update with the dots with P (5).
// 16 B per stream.
double idr_bytes_per_matvec(int s, bool pc) {
  const double mpc = pc ? 12.0 : 0.0;
  double streams = 0.0;
  for (int k = 0; k < s; ++k) streams += (s - k + 2) + (s - k + 2) + mpc + 2 + 1 + (2 * k + 8);
  streams += mpc + 2 + 2 + 5;
  return 16.0 * streams / (s + 1);
}

// Banded z solve instance for a stencil radius (the band's half width) and vector storage.
const void* band_solve_kernel(int rad, bool f32) {
#define RST_BAND_PICK(R)                                                                        \
  if (rad == R) return f32 ? (const void*)rst::mk::k_mk_band_solve<R, float2>                   \
                           : (const void*)rst::mk::k_mk_band_solve<R, double2>;
  RST_BAND_PICK(1)
  RST_BAND_PICK(2)
  RST_BAND_PICK(3)
  RST_BAND_PICK(4)
  RST_BAND_PICK(5)
  RST_BAND_PICK(6)
#undef RST_BAND_PICK
  return nullptr;
}

// Factored lateral DFT instances (k_mk_fft<N1, N2, NW>, N = N1 N2); other N use the direct
// evaluation (k_mk_dft).
struct FftInstance {
  const void* kern;
  int nw;
};
FftInstance fft_instance(int N, bool f32, bool cj = false) {
  if (cj) {  // conjugate-space columns (the doubled COCG, FP64)
    switch (N) {
      case 8: return {(const void*)rst::mk::k_mk_fft<2, 4, 2, 1, double2, true>, 2};
      case 16: return {(const void*)rst::mk::k_mk_fft<4, 4, 4, 1, double2, true>, 4};
      case 54: return {(const void*)rst::mk::k_mk_fft<6, 9, 3, 1, double2, true>, 3};
      default: return {nullptr, 0};
    }
  }
  if (f32) {
    switch (N) {
      case 8: return {(const void*)rst::mk::k_mk_fft<2, 4, 2, 1, float2>, 2};
      case 16: return {(const void*)rst::mk::k_mk_fft<4, 4, 4, 1, float2>, 4};
      case 54: return {(const void*)rst::mk::k_mk_fft<6, 9, 3, 1, float2>, 3};
      default: return {nullptr, 0};
    }
  }
  switch (N) {
    case 8: return {(const void*)rst::mk::k_mk_fft<2, 4, 2, 1>, 2};
    case 12: return {(const void*)rst::mk::k_mk_fft<3, 4, 2, 1>, 2};
    case 16: return {(const void*)rst::mk::k_mk_fft<4, 4, 4, 1>, 4};
    case 18: return {(const void*)rst::mk::k_mk_fft<3, 6, 3, 1>, 3};
    case 24: return {(const void*)rst::mk::k_mk_fft<4, 6, 2, 1>, 2};
    case 27: return {(const void*)rst::mk::k_mk_fft<3, 9, 3, 1>, 3};
    case 32: return {(const void*)rst::mk::k_mk_fft<4, 8, 4, 1>, 4};
    case 36: return {(const void*)rst::mk::k_mk_fft<6, 6, 3, 1>, 3};
    case 48: return {(const void*)rst::mk::k_mk_fft<6, 8, 2, 1>, 2};
    case 54: return {(const void*)rst::mk::k_mk_fft<6, 9, 3, 1>, 3};
    case 64: return {(const void*)rst::mk::k_mk_fft<8, 8, 4, 1>, 4};
    default: return {nullptr, 0};
  }
}

// Many-column right-preconditioned BiCGSTAB and IDR(s) (rst_mk.hpp, rst_idr.hpp) over the (energy,
// column) items, in blocks of up to `ld` columns with one kernel per step; same inputs and outputs as
// the persistent solver.  RST_FP32_REFINE (IDR(s) only): FP64 iterative refinement, x += d with d
// from an IDR(s) run on complex64 vectors (FP64 arithmetic, the complex64 operator apply) for the
// current FP64 residual r = b - A x, until the FP64 true residual meets the tolerance.
rst_status run_bicgstab_mk(rst_ctx* c, int ne, const double* energies, const std::vector<int64_t>& cols,
                           const double* d_gsrc, const double* d_gdst, double2* xout, std::vector<double>& Tcol,
                           std::vector<int>& its, std::vector<int>& rss, std::vector<double>& res,
                           std::vector<int>& st, double& ms, const double2* rhs, long long rhs_ld,
                           long long rhs_estride) {
  const bool pc = c->opts.precond == RST_PRECOND_FREE_CAP;
  const int na = c->na, nb = c->nb, nz = c->nz, P = na * nb;
  const long long n = (long long)P * nz;
  const int ncols = (int)cols.size();
  const long long nitems = (long long)ne * ncols;
  const std::vector<double>* hsrc = d_gsrc == nullptr ? nullptr : (d_gsrc == c->d_gr.p ? &c->gr : &c->gl);
  c->last_cw = 0;
  c->last_threads = 256;
  // IDR(s) for RST_IDRS and for wide planes under RST_BICGSTAB (the method that converges on them)
  const bool idr = c->opts.method == RST_IDRS || (c->opts.method == RST_BICGSTAB && P > 2 * rst::MAX_T);
  const int sdim = idr ? c->opts.idr_s : 0;
  const bool mixed = c->opts.precision == RST_FP32_REFINE;
  // COCG on the doubled k / -k system (generic k; run_solver sends the real-H_k points to the
  // persistent COCG): a block of ld columns holds ld/2 (energy, column) pairs
  const bool cocg2 = c->opts.method == RST_COCG;
  if (mixed && !idr)
    return fail(c, RST_EUNSUPPORTED, "the many-column BiCGSTAB runs in FP64 only (mixed precision: RST_IDRS)");
  // block width: vectors X R R0 P V T (+ PH SH W with the preconditioner); IDR(s): X R V T G_0..G_{s-1}
  // U_0..U_{s-1} (+ VH W), complex64 in the mixed mode, which adds the FP64 x and r; at most a quarter
  // of free memory
  const int nvec = cocg2 ? (pc ? 6 : 5) : idr ? (4 + 2 * sdim + (pc ? 2 : 0)) : (pc ? 9 : 6);
  const size_t esz = mixed ? 8 : 16;
  size_t free_b = 0, total_b = 0;
  HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
  const size_t per_col = (size_t)nvec * n * esz + (mixed ? (size_t)2 * n * 16 : 0) + (size_t)c->nproj * 16;
  long long ldmax = std::max<long long>(64, (long long)(free_b / 4 / per_col) / 64 * 64);
  ldmax = std::min<long long>(ldmax, 1024);
  const int ld = (int)std::min<long long>(ldmax, ((cocg2 ? 2 : 1) * nitems + 63) / 64 * 64);
  const int per_blk = cocg2 ? ld / 2 : ld;  // items per block
  rst::mk::Shape S;
  S.n = n;
  S.ld = ld;
  int ncu = 0;
  HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  // row ranges: about eight reducing workgroups per compute unit in all
  S.nsplit = (int)std::max<long long>(1, std::min<long long>(n / 64, 8LL * ncu / (ld / 64)));
  S.rows = (n + S.nsplit - 1) / S.nsplit;
  const size_t vlen = (size_t)n * ld;
  rst_status e;
  if ((e = ensure(c, c->d_mkv, (size_t)nvec * vlen * esz)) != RST_OK) return e;
  if (mixed && (e = ensure(c, c->d_mkv64, (size_t)2 * vlen * 16)) != RST_OK) return e;
  double2* X = (double2*)c->d_mkv.p;  // the FP64 vectors (BiCGSTAB; IDR(s) in FP64 lays them out itself)
  double2* X64 = mixed ? (double2*)c->d_mkv64.p : nullptr;  // mixed mode: FP64 x and r
  double2* R64 = mixed ? X64 + vlen : nullptr;
  const double2* Xres = mixed ? X64 : X;  // the block's solutions
  double2* R = X + vlen;
  double2* R0 = R + vlen;  // BiCGSTAB: shadow residual; IDR(s): v
  double2* Pv = R0 + vlen; // BiCGSTAB: p; IDR(s): t
  double2 *V, *T, *PH, *SH, *W, *Gb = nullptr, *Ub = nullptr;
  if (!idr) {
    V = Pv + vlen;
    T = V + vlen;
    PH = pc ? T + vlen : Pv;
    SH = pc ? PH + vlen : R;
    W = pc ? SH + vlen : nullptr;
  } else {
    V = R0;
    T = Pv;
    Gb = Pv + vlen;
    Ub = Gb + (size_t)sdim * vlen;
    PH = pc ? Ub + (size_t)sdim * vlen : V;  // M^-1 v
    W = pc ? PH + vlen : nullptr;
    SH = nullptr;
  }
  double2* Wres = idr ? T : V;  // the true residual's A x reuses a vector the next step rebuilds
  if ((e = ensure(c, c->d_mkst, (size_t)ld * sizeof(rst::mk::ColSt))) != RST_OK) return e;
  if ((e = ensure(c, c->d_mkact, (size_t)ld * 4)) != RST_OK) return e;
  if ((e = ensure(c, c->d_mkmark, (size_t)ld * 4)) != RST_OK) return e;
  if ((e = ensure(c, c->d_mkpart, (size_t)(idr ? sdim + 1 : 2) * S.nsplit * ld * 16)) != RST_OK) return e;
  if (idr) {
    if ((e = ensure(c, c->d_mkidr, (size_t)ld * sizeof(rst::idr::IdrSt))) != RST_OK) return e;
    if ((e = ensure(c, c->d_mkshadow, (size_t)n * sdim * 16)) != RST_OK) return e;
    const long long ns = n * sdim;
    hipLaunchKernelGGL(rst::idr::k_idr_shadow, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, c->stream, n, sdim,
                       (unsigned long long)0x5EED1D25ULL, (double2*)c->d_mkshadow.p);
    HIPCHK(c, hipGetLastError());
  }
  if ((e = ensure(c, c->d_mkT, (size_t)ld * 8)) != RST_OK) return e;
  if (c->nproj > 0 && (e = ensure(c, c->d_projP, (size_t)c->nproj * ld * 16)) != RST_OK) return e;
  rst::mk::ColSt* dst_ = (rst::mk::ColSt*)c->d_mkst.p;
  int* act = (int*)c->d_mkact.p;
  int* mark = (int*)c->d_mkmark.p;
  double2* part = (double2*)c->d_mkpart.p;
  // column tables: energy, pivot slice, point source, its value, dense offset
  const size_t tab_bytes = (size_t)ld * (8 + 4 + 8 + 8 + 8);
  if ((e = ensure(c, c->d_mkcol, tab_bytes)) != RST_OK) return e;
  double* d_ecol = (double*)c->d_mkcol.p;
  long long* d_src = (long long*)(d_ecol + ld);
  double* d_bsc = (double*)(d_src + ld);
  long long* d_doff = (long long*)(d_bsc + ld);
  int* d_eidx = (int*)(d_doff + ld);
  rst::mk::Rhs B;
  B.src = d_src;
  B.bsc = d_bsc;
  B.dense = rhs;
  B.dld = rhs_ld;
  B.doff = d_doff;
  // preconditioner: DFT passes: (w, post) tables of forward a, inverse a, forward b, inverse b; band factors
  const double2 *band_L = nullptr, *band_dinv = nullptr;
  struct DftTabs {
    const double2 *w = nullptr, *post = nullptr, *pre = nullptr, *root = nullptr;
  } FA, IA, FB, IB;
  if (pc) {
    const double pi = 3.14159265358979323846;
    // per axis (N points, Bloch phase kh per point): w and post of the forward and inverse
    // passes, then the factored form's tables: the forward twist pre[i] = exp(-i kh i), ones
    // (no twist on the inverse), and the roots exp(-+2 pi i m/N)
    std::vector<double2> F((size_t)8 * na + (size_t)8 * nb);
    auto put = [](double2& d, double ph, double sc) { d = double2{sc * std::cos(ph), sc * std::sin(ph)}; };
    auto axis = [&](double2* t, int N, double kh) {
      for (int j = 0; j < N; ++j) {
        put(t[j], -(2 * pi * j / N + kh), 1.0);  // forward: w
        put(t[N + j], 0.0, 1.0);                 // forward: post
        put(t[2 * N + j], 2 * pi * j / N, 1.0);  // inverse: w
        put(t[3 * N + j], kh * j, 1.0 / N);      // inverse: post
        put(t[4 * N + j], -kh * j, 1.0);         // forward: pre
        put(t[5 * N + j], 0.0, 1.0);             // inverse: pre
        put(t[6 * N + j], -2 * pi * j / N, 1.0); // forward: root^j
        put(t[7 * N + j], 2 * pi * j / N, 1.0);  // inverse: root^j
      }
    };
    axis(F.data(), na, c->ka * c->ha);
    axis(F.data() + 8 * na, nb, c->kb * c->hb);
    if ((e = upload(c, c->d_mkF, F)) != RST_OK) return e;
    const double2* d = (const double2*)c->d_mkF.p;
    auto tabs = [](const double2* t, int N, bool inv, DftTabs& o) {
      o.w = t + (inv ? 2 : 0) * N;
      o.post = t + (inv ? 3 : 1) * N;
      o.pre = t + (inv ? 5 : 4) * N;
      o.root = t + (inv ? 7 : 6) * N;
    };
    tabs(d, na, false, FA);
    tabs(d, na, true, IA);
    tabs(d + 8 * na, nb, false, FB);
    tabs(d + 8 * na, nb, true, IB);
    // banded L D L^T of the z operator per (energy, lateral mode)
    // (the doubled COCG adds the conjugate-space factors of every energy as entries ne..2ne-1)
    const int nef = cocg2 ? 2 * ne : ne;
    std::vector<double> en(energies, energies + ne);
    if (cocg2) en.insert(en.end(), energies, energies + ne);
    if ((e = upload(c, c->d_en, en)) != RST_OK) return e;
    if ((e = ensure(c, c->d_pc_inv, (size_t)nef * n * 16 * (1 + c->rad))) != RST_OK) return e;
    rst::mk::Band Bd;
    std::memset(&Bd, 0, sizeof(Bd));
    Bd.dinv = (double2*)c->d_pc_inv.p;
    Bd.L = Bd.dinv + (size_t)nef * n;
    Bd.energies = (const double*)c->d_en.p;
    Bd.eps = (const double*)c->d_pc_eps.p;
    Bd.gz = (const double*)c->d_gz.p;
    // the reference potential per plane: the plane means, or the cell mean on every plane
    std::vector<double> vref(nz, 0.0);
    {
      double vbar = 0.0;
      for (double x : c->v) vbar += x;
      vbar /= (double)c->v.size();
      for (int z = 0; z < nz; ++z) {
        double acc = 0.0;
        for (int q = 0; q < P; ++q) acc += c->v[(size_t)z * P + q];
        vref[z] = c->opts.pc_vref == RST_VREF_CELL ? vbar : acc / P;
      }
    }
    if ((e = upload(c, c->d_mkvref, vref)) != RST_OK) return e;
    Bd.vz = (const double*)c->d_mkvref.p;
    for (int j = 0; j <= c->rad; ++j) Bd.cz[j] = 0.5 * c->fdw[j] / (c->hz * c->hz);
    Bd.M = c->rad;
    Bd.shift = c->opts.pc_shift;
    Bd.P = P;
    Bd.nz = nz;
    Bd.ne = nef;
    Bd.neg_from = ne;
    const long long nt = (long long)nef * P;
    hipLaunchKernelGGL(rst::mk::k_mk_band_factor, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream, Bd);
    HIPCHK(c, hipGetLastError());
    band_L = Bd.L;
    band_dinv = Bd.dinv;
  }
  // direct evaluation: the smallest instance with 4*RW >= N (N > 64 takes several rounds of 64)
  auto dft_kernel = [](int N, bool f32, bool cj) -> const void* {
    if (cj) {
      if (N <= 8) return (const void*)rst::mk::k_mk_dft<2, double2, true>;
      if (N <= 16) return (const void*)rst::mk::k_mk_dft<4, double2, true>;
      if (N <= 32) return (const void*)rst::mk::k_mk_dft<8, double2, true>;
      return (const void*)rst::mk::k_mk_dft<16, double2, true>;
    }
    if (f32) {
      if (N <= 8) return (const void*)rst::mk::k_mk_dft<2, float2>;
      if (N <= 16) return (const void*)rst::mk::k_mk_dft<4, float2>;
      if (N <= 32) return (const void*)rst::mk::k_mk_dft<8, float2>;
      return (const void*)rst::mk::k_mk_dft<16, float2>;
    }
    if (N <= 8) return (const void*)rst::mk::k_mk_dft<2>;
    if (N <= 16) return (const void*)rst::mk::k_mk_dft<4>;
    if (N <= 32) return (const void*)rst::mk::k_mk_dft<8>;
    return (const void*)rst::mk::k_mk_dft<16>;
  };
  auto dft_lds = [](int N) -> size_t { return ((size_t)N * 64 + 2 * (size_t)N) * 16; };
  for (int N : {na, nb})
    for (int v = 0; v < 3; ++v)  // complex128, complex64, conjugate-space complex128
      if (!fft_instance(N, v == 1, v == 2).kern && dft_lds(N) > 64 * 1024)
        HIPCHK(c, hipFuncSetAttribute(dft_kernel(N, v == 1, v == 2), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)dft_lds(N)));
  // out = the DFT pass of `in` for the columns of `mask` (factored where N has an instance); f32:
  // complex64 vectors
  const int* pc_cfl = nullptr;  // columns preconditioned in the conjugate space (doubled COCG)
  auto dft = [&](const void* in, void* out, const DftTabs& tb, bool axis_a, const int* mask, bool f32, int cin,
                 int cout) -> rst_status {
    rst::mk::DftPass D;
    D.cfl = pc_cfl;
    D.cin = cin;
    D.cout = cout;
    D.in = in;
    D.out = out;
    D.w = tb.w;
    D.post = tb.post;
    D.pre = tb.pre;
    D.root = tb.root;
    D.act = mask;
    D.N = axis_a ? na : nb;
    D.stride = axis_a ? 1 : na;
    D.nline_inner = axis_a ? nb : na;
    D.inner_mul = axis_a ? na : 1;
    D.P = P;
    D.nz = nz;
    D.ld = ld;
    const long long nwg = (long long)nz * D.nline_inner * (ld / 64);
    void* args[] = {&D};
    const bool cj = pc_cfl != nullptr && (cin || cout);
    const FftInstance fi = fft_instance(D.N, f32, cj);
    if (fi.kern)
      HIPCHK(c, hipLaunchKernel(fi.kern, dim3((unsigned)nwg), dim3(64 * fi.nw), args, 0, c->stream));
    else
      HIPCHK(c, hipLaunchKernel(dft_kernel(D.N, f32, cj), dim3((unsigned)nwg), dim3(256), args, dft_lds(D.N),
                                c->stream));
    return RST_OK;
  };
  // out = M^-1 in (Wp: a work vector of the same type)
  auto precondition = [&](const void* in, void* out, void* Wp, const int* mask, bool f32) -> rst_status {
    rst_status ps;
    if ((ps = dft(in, Wp, FA, true, mask, f32, 1, 0)) != RST_OK) return ps;
    if ((ps = dft(Wp, out, FB, false, mask, f32, 0, 0)) != RST_OK) return ps;
    const long long nt = (long long)P * ld;
    const dim3 gb((unsigned)((nt + 255) / 256));
    {
      const void* kb = band_solve_kernel(c->rad, f32);
      const int* eix = d_eidx;
      void* args[] = {&out, &Wp, (void*)&band_L, (void*)&band_dinv, (void*)&eix, (void*)&mask, (void*)&P,
                      (void*)&nz, (void*)&ld};
      HIPCHK(c, hipLaunchKernel(kb, gb, dim3(256), args, 0, c->stream));
    }
    if ((ps = dft(out, Wp, IB, false, mask, f32, 0, 0)) != RST_OK) return ps;
    return dft(Wp, out, IA, true, mask, f32, 0, 1);
  };
  // y = A x on the block (f32: complex64 vectors, the FP32 stencil)
  auto apply = [&](const void* x, void* y, const int* mask, bool f32, const int* cfl = nullptr) -> rst_status {
    return apply_cols(c, x, y, ld, 0.0, d_ecol, mask, f32, (double2*)c->d_projP.p, nullptr, cfl);
  };
  const dim3 gred((unsigned)(ld / 64), (unsigned)S.nsplit);
  const unsigned gsc = (unsigned)ld;  // one wavefront per column in the scalar and sum kernels
  const unsigned gel = (unsigned)((vlen + 255) / 256);
  auto scalar = [&](int step) -> rst_status {
    hipLaunchKernelGGL(rst::mk::k_mk_scalar, dim3(gsc), dim3(64), 0, c->stream, S, step, dst_, act,
                       (const double2*)part, c->opts.tol, c->opts.max_iter);
    HIPCHK(c, hipGetLastError());
    return RST_OK;
  };
  const size_t nout = (size_t)nitems;
  Tcol.assign(nout, 0.0);
  its.assign(nout, 0);
  rss.assign(nout, 0);
  res.assign(nout, 0.0);
  st.assign(nout, 1);
  c->last_updates.clear();
  if (mixed) c->last_updates.assign((size_t)nitems, 0);  // refinement cycles per item
  c->last_fallbacks = 0;
  c->last_cnn_flop = 0.0;
  long long nent = 0;
  for (int g = 0; g < c->ngroup; ++g) nent += c->grp_ne[g];
  double bytes = 0.0;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, hipEventRecord(e0, c->stream));
  std::vector<rst::mk::ColSt> hst(ld);
  std::vector<rst::idr::IdrSt> hid(idr ? ld : 0);
  rst::idr::IdrSt* did = (rst::idr::IdrSt*)c->d_mkidr.p;
  const double2* Psh = (const double2*)c->d_mkshadow.p;
  std::vector<int> hact(ld), hmark(ld);
  std::vector<double2> hpart;
  // doubled COCG on one block of m = ld/2 pairs (rst_cocg2.hpp): X, R, P, Q, Z (+ W) in d_mkv;
  // columns cc < m run the operator as A_-k (conjugated), columns cc >= m the preconditioner as
  // M_-k^-1 (conjugated, the factor entries ne..2ne-1)
  auto run_cocg2 = [&](int nc) -> rst_status {
    const int m = per_blk;
    double2* Xc = (double2*)c->d_mkv.p;
    double2* Rc = Xc + vlen;
    double2* Pc = Rc + vlen;
    double2* Qc = Pc + vlen;
    double2* Zc = pc ? Qc + vlen : Rc;  // M^-1 r (swapped halves), or r itself without M^-1
    double2* Wc = pc ? Zc + vlen : nullptr;
    const int zsw = pc ? 1 : 0;
    rst_status rs;
    if ((rs = ensure(c, c->d_mkcfl, (size_t)2 * ld * 4)) != RST_OK) return rs;
    if ((rs = ensure(c, c->d_mkcd, (size_t)m * sizeof(rst::cd::CdSt))) != RST_OK) return rs;
    int* cfl_ap = (int*)c->d_mkcfl.p;
    int* cfl_pc = cfl_ap + ld;
    {
      std::vector<int> fl(2 * (size_t)ld, 0);
      for (int cc = 0; cc < ld; ++cc) {
        fl[cc] = cc < m ? 1 : 0;
        fl[ld + cc] = cc >= m ? 1 : 0;
      }
      HIPCHK(c, hipMemcpyAsync(cfl_ap, fl.data(), fl.size() * 4, hipMemcpyHostToDevice, c->stream));
    }
    rst::cd::CdSt* dcd = (rst::cd::CdSt*)c->d_mkcd.p;
    std::vector<rst::cd::CdSt> hcd(m);
    auto cscal = [&](int step, int* actp, const int* mk_) -> rst_status {
      hipLaunchKernelGGL(rst::cd::k_cd_scalar, dim3((unsigned)m), dim3(64), 0, c->stream, S, m, step, dcd, actp, mk_,
                         (const double2*)part, c->opts.tol, c->opts.max_iter);
      HIPCHK(c, hipGetLastError());
      return RST_OK;
    };
    auto zstep = [&](const int* msk) -> rst_status {  // Z = K r (swapped), or r itself
      if (!pc) return RST_OK;
      pc_cfl = cfl_pc;
      rst_status r2 = precondition(Rc, Zc, Wc, msk, false);
      pc_cfl = nullptr;
      return r2;
    };
    // start: x = p = 0, r = b, z = K r, rho = r^T z, p = z
    hipLaunchKernelGGL(rst::cd::k_cd_init, gred, dim3(256), 0, c->stream, S, B, Xc, Rc, Pc, part);
    if ((rs = cscal(rst::cd::CD_INIT, act, nullptr)) != RST_OK) return rs;
    if ((rs = zstep(act)) != RST_OK) return rs;
    hipLaunchKernelGGL(rst::cd::k_cd_dot, gred, dim3(256), 0, c->stream, S, m, (const int*)act, (const double2*)Rc,
                       (const double2*)Zc, zsw, part);
    if ((rs = cscal(rst::cd::CD_RHO, act, nullptr)) != RST_OK) return rs;
    hipLaunchKernelGGL(rst::cd::k_cd_p, gred, dim3(256), 0, c->stream, S, m, (const rst::cd::CdSt*)dcd,
                       (const int*)act, Pc, (const double2*)Zc, zsw);
    HIPCHK(c, hipGetLastError());
    for (;;) {
      // q = B p (Q holds its halves swapped), alpha = rho / p^T q, x += alpha p, r -= alpha q
      if ((rs = apply(Pc, Qc, act, false, cfl_ap)) != RST_OK) return rs;
      hipLaunchKernelGGL(rst::cd::k_cd_dot, gred, dim3(256), 0, c->stream, S, m, (const int*)act,
                         (const double2*)Pc, (const double2*)Qc, 1, part);
      if ((rs = cscal(rst::cd::CD_ALPHA, act, nullptr)) != RST_OK) return rs;
      hipLaunchKernelGGL(rst::cd::k_cd_xr, gred, dim3(256), 0, c->stream, S, m, (const rst::cd::CdSt*)dcd,
                         (const int*)act, Xc, Rc, (const double2*)Pc, (const double2*)Qc, part);
      if ((rs = cscal(rst::cd::CD_CONV, act, nullptr)) != RST_OK) return rs;
      // z = K r, beta = r^T z / rho, p = z + beta p
      if ((rs = zstep(act)) != RST_OK) return rs;
      hipLaunchKernelGGL(rst::cd::k_cd_dot, gred, dim3(256), 0, c->stream, S, m, (const int*)act,
                         (const double2*)Rc, (const double2*)Zc, zsw, part);
      if ((rs = cscal(rst::cd::CD_BETA, act, nullptr)) != RST_OK) return rs;
      hipLaunchKernelGGL(rst::cd::k_cd_p, gred, dim3(256), 0, c->stream, S, m, (const rst::cd::CdSt*)dcd,
                         (const int*)act, Pc, (const double2*)Zc, zsw);
      HIPCHK(c, hipGetLastError());
      HIPCHK(c, hipMemcpyAsync(hcd.data(), dcd, m * sizeof(rst::cd::CdSt), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(hact.data(), act, ld * 4, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      int nmark = 0, nact = 0;
      for (int j = 0; j < ld; ++j) hmark[j] = 0;
      for (int j = 0; j < m; ++j) {
        const bool stop = hcd[j].done == 0 && !hact[j] && (hcd[j].check || hcd[j].brk);
        hmark[j] = hmark[j + m] = stop ? 1 : 0;
        nmark += stop;
        nact += hact[j];
      }
      if (nmark > 0) {
        // stopped pairs: the true residual b - B x decides between done and a restart from it
        HIPCHK(c, hipMemcpyAsync(mark, hmark.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
        if ((rs = apply(Xc, Qc, mark, false, cfl_ap)) != RST_OK) return rs;
        hipLaunchKernelGGL(rst::cd::k_cd_resid, gred, dim3(256), 0, c->stream, S, m, B, (const int*)mark,
                           (const double2*)Qc, Rc, part);
        HIPCHK(c, hipGetLastError());
        hpart.resize((size_t)S.nsplit * ld);
        HIPCHK(c, hipMemcpyAsync(hpart.data(), part, hpart.size() * 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        std::vector<int> rmark(ld, 0);
        int nrestart = 0;
        for (int j = 0; j < m; ++j) {
          if (!hmark[j]) continue;
          double rr = 0.0;
          for (int r = 0; r < S.nsplit; ++r) rr += hpart[(size_t)r * ld + j].x + hpart[(size_t)r * ld + j + m].x;
          rst::cd::CdSt& q = hcd[j];
          const double rel = q.bb > 0 ? std::sqrt(rr / q.bb) : 0.0;
          q.check = q.brk = 0;
          if (rel <= c->opts.tol) {
            q.done = 1;
            q.rr = rel;
          } else if (q.its >= c->opts.max_iter || !std::isfinite(rel) || q.restarts >= 1000) {
            q.done = 2;
            q.rr = rel;
          } else {
            q.restarts += 1;
            q.rr = q.rrmin = rr;
            rmark[j] = rmark[j + m] = 1;
            hact[j] = hact[j + m] = 1;
            ++nrestart;
          }
        }
        HIPCHK(c, hipMemcpyAsync(dcd, hcd.data(), m * sizeof(rst::cd::CdSt), hipMemcpyHostToDevice, c->stream));
        if (nrestart > 0) {
          // restart the marked pairs from their true residual (now in R): z = K r, rho, p = z
          HIPCHK(c, hipMemcpyAsync(mark, rmark.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
          if ((rs = zstep(mark)) != RST_OK) return rs;
          hipLaunchKernelGGL(rst::cd::k_cd_dot, gred, dim3(256), 0, c->stream, S, m, (const int*)mark,
                             (const double2*)Rc, (const double2*)Zc, zsw, part);
          if ((rs = cscal(rst::cd::CD_RHO, mark, nullptr)) != RST_OK) return rs;
          hipLaunchKernelGGL(rst::cd::k_cd_p, gred, dim3(256), 0, c->stream, S, m, (const rst::cd::CdSt*)dcd,
                             (const int*)mark, Pc, (const double2*)Zc, zsw);
          HIPCHK(c, hipGetLastError());
          HIPCHK(c, hipMemcpyAsync(act, hact.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
          nact += nrestart;
        }
      }
      if (nact == 0) break;
    }
    for (int j = 0; j < nc; ++j) {
      hst[j].its = hcd[j].its;
      hst[j].restarts = hcd[j].restarts;
      hst[j].rr = hcd[j].rr;
      hst[j].done = hcd[j].done;
    }
    return RST_OK;
  };
  for (long long it0 = 0; it0 < nitems; it0 += per_blk) {
    const int nc = (int)std::min<long long>(per_blk, nitems - it0);
    std::vector<double> ecol(ld, energies[0]);
    std::vector<long long> src(ld, -1), doff(ld, -1);
    std::vector<double> bsc(ld, 0.0);
    std::vector<int> eidx(ld, 0);
    // column cc of the block holds item it0 + cc (doubled COCG: item it0 + cc mod m in both halves,
    // the second half's preconditioner factors at entries ne + e)
    for (int cc = 0; cc < ld; ++cc) {
      const int j = cocg2 ? cc % per_blk : cc;
      if (j >= nc) continue;
      const long long it = it0 + j;
      const int ie = (int)(it / ncols), jc = (int)(it % ncols);
      ecol[cc] = energies[ie];
      eidx[cc] = cocg2 && cc >= per_blk ? ne + ie : ie;
      if (rhs) {
        doff[cc] = (long long)ie * rhs_estride + jc;
      } else {
        src[cc] = cols[jc];
        bsc[cc] = hsrc ? std::sqrt((*hsrc)[cols[jc] / P]) : 1.0;
      }
    }
    HIPCHK(c, hipMemcpyAsync(d_ecol, ecol.data(), ld * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d_src, src.data(), ld * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d_bsc, bsc.data(), ld * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d_doff, doff.data(), ld * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d_eidx, eidx.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
    rst_status ps;
    long long col_its = 0, col_cyc = 0;
    if (cocg2) {
      if ((ps = run_cocg2(nc)) != RST_OK) return ps;
    } else if (!idr) {
      hipLaunchKernelGGL(rst::mk::k_mk_init, gred, dim3(256), 0, c->stream, S, B, X, R, R0, Pv, part);
      HIPCHK(c, hipGetLastError());
      if ((ps = scalar(rst::mk::SC_INIT)) != RST_OK) return ps;
      for (int iter = 0;; ++iter) {
        // one BiCGSTAB step of every iterating column
        if (iter > 0)
          hipLaunchKernelGGL(rst::mk::k_mk_p, gred, dim3(256), 0, c->stream, S, (const rst::mk::ColSt*)dst_,
                             (const int*)act, Pv, (const double2*)R, (const double2*)V);
        if (pc && (ps = precondition(Pv, PH, W, act, false)) != RST_OK) return ps;
        if ((ps = apply(PH, V, act, false)) != RST_OK) return ps;
        hipLaunchKernelGGL(rst::mk::k_mk_dots<1>, gred, dim3(256), 0, c->stream, S, (const int*)act,
                           (const double2*)R0, (const double2*)V, (const double2*)nullptr, (const double2*)nullptr,
                           part);
        if ((ps = scalar(rst::mk::SC_ALPHA)) != RST_OK) return ps;
        hipLaunchKernelGGL(rst::mk::k_mk_s, gred, dim3(256), 0, c->stream, S, (const rst::mk::ColSt*)dst_,
                           (const int*)act, R, (const double2*)V);
        if (pc && (ps = precondition(R, SH, W, act, false)) != RST_OK) return ps;
        if ((ps = apply(SH, T, act, false)) != RST_OK) return ps;
        hipLaunchKernelGGL(rst::mk::k_mk_dots<2>, gred, dim3(256), 0, c->stream, S, (const int*)act,
                           (const double2*)T, (const double2*)R, (const double2*)T, (const double2*)T, part);
        if ((ps = scalar(rst::mk::SC_OMEGA)) != RST_OK) return ps;
        hipLaunchKernelGGL(rst::mk::k_mk_xr, gred, dim3(256), 0, c->stream, S, (const rst::mk::ColSt*)dst_,
                           (const int*)act, X, R, (const double2*)R0, (const double2*)PH, (const double2*)SH,
                           (const double2*)T, part);
        if ((ps = scalar(rst::mk::SC_BETA)) != RST_OK) return ps;
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(hst.data(), dst_, ld * sizeof(rst::mk::ColSt), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(hact.data(), act, ld * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        // columns that stopped this step: true residual b - A x decides between done and restart
        int nmark = 0, nact = 0;
        for (int j = 0; j < ld; ++j) {
          hmark[j] = (hst[j].done == 0 && !hact[j] && (hst[j].check || hst[j].brk)) ? 1 : 0;
          nmark += hmark[j];
          nact += hact[j];
        }
        if (nmark > 0) {
          HIPCHK(c, hipMemcpyAsync(mark, hmark.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
          if ((ps = apply(X, Wres, mark, false)) != RST_OK) return ps;
          hipLaunchKernelGGL(rst::mk::k_mk_resid, gred, dim3(256), 0, c->stream, S, B, (const int*)mark,
                             (const double2*)Wres, R, part);
          HIPCHK(c, hipGetLastError());
          hpart.resize((size_t)S.nsplit * ld);
          HIPCHK(c, hipMemcpyAsync(hpart.data(), part, hpart.size() * 16, hipMemcpyDeviceToHost, c->stream));
          HIPCHK(c, hipStreamSynchronize(c->stream));
          std::vector<int> rmark(ld, 0);
          int nrestart = 0;
          for (int j = 0; j < ld; ++j) {
            if (!hmark[j]) continue;
            double rr = 0.0;
            for (int r = 0; r < S.nsplit; ++r) rr += hpart[(size_t)r * ld + j].x;
            rst::mk::ColSt& q = hst[j];
            const double rel = q.bb > 0 ? std::sqrt(rr / q.bb) : 0.0;
            q.check = q.brk = 0;
            if (rel <= c->opts.tol) {
              q.done = 1;
              q.rr = rel;
            } else if (q.its >= c->opts.max_iter || !std::isfinite(rel) || q.restarts >= 1000) {
              q.done = 2;
              q.rr = rel;
            } else {
              // restart from the true residual (now in R): r0h = p = r, rho = ||r||^2
              q.rho = double2{rr, 0.0};
              q.r0n = rr;
              q.rrmin = rr;
              q.rr = rr;
              q.alpha = q.omega = q.beta = double2{0.0, 0.0};
              q.restarts += 1;
              rmark[j] = 1;
              hact[j] = 1;
              ++nrestart;
            }
          }
          HIPCHK(c, hipMemcpyAsync(dst_, hst.data(), ld * sizeof(rst::mk::ColSt), hipMemcpyHostToDevice, c->stream));
          if (nrestart > 0) {
            HIPCHK(c, hipMemcpyAsync(mark, rmark.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(act, hact.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(rst::mk::k_mk_restart, dim3(gel), dim3(256), 0, c->stream, S, (const int*)mark,
                               (const double2*)R, R0, Pv);
            HIPCHK(c, hipGetLastError());
            nact += nrestart;
          }
          // a restarted column starts with p = r (no p update on its first step): the p kernel sees
          // beta = 0, omega = 0 and recomputes p = r, which is the same
        }
        if (nact == 0) break;
      }
    } else {
      // IDR(s) cycles: s steps of one apply each, then the dimension-reduction step.  `run_idr` runs
      // them on vectors of storage type VT (complex128, or complex64 for the corrections of the mixed
      // mode) from the right-hand sides Bv to the relative tolerance tol.  inner: a column that stops
      // (tolerance, iteration budget cap[c], breakdown) is finished for this run; the FP64 refinement
      // around it checks the true residual.  Otherwise a stopped column's true residual b - A x decides
      // between done and a restart from it.
      auto run_idr = [&](auto tag, const rst::mk::Rhs& Bv, double tol, bool inner, const int* capd) -> rst_status {
        using VT = typename std::remove_pointer<decltype(tag)>::type;
        constexpr bool f32 = std::is_same<VT, float2>::value;
        VT* Xv = (VT*)c->d_mkv.p;
        VT* Rv = Xv + vlen;
        VT* Vv = Rv + vlen;
        VT* Tv = Vv + vlen;
        VT* Gv = Tv + vlen;
        VT* Uv = Gv + (size_t)sdim * vlen;
        VT* PHv = pc ? Uv + (size_t)sdim * vlen : Vv;  // M^-1 v
        VT* Wv = pc ? PHv + vlen : nullptr;
        VT* VH = pc ? PHv : Vv;
        rst_status rs;
        auto iscal = [&](int step, int k, const int* mk_) -> rst_status {
          hipLaunchKernelGGL(rst::idr::k_idr_scalar, dim3((unsigned)ld), dim3(64), 0, c->stream, S, step, sdim, k,
                             did, act, mk_, (const double2*)part, tol, c->opts.max_iter, capd);
          HIPCHK(c, hipGetLastError());
          return RST_OK;
        };
        hipLaunchKernelGGL(rst::idr::k_idr_init<VT>, dim3(gel), dim3(256), 0, c->stream, S, sdim, Bv, Xv, Rv, Gv,
                           Uv);
        hipLaunchKernelGGL((rst::idr::k_idr_pdots<true, VT>), gred, dim3(256), 0, c->stream, S, sdim,
                           (const int*)nullptr, Psh, (const VT*)Rv, part);
        if ((rs = iscal(rst::idr::ID_INIT, 0, nullptr)) != RST_OK) return rs;
        for (;;) {
          for (int k = 0; k < sdim; ++k) {
            VT* Gk = Gv + (size_t)k * vlen;
            VT* Uk = Uv + (size_t)k * vlen;
            if ((rs = iscal(rst::idr::ID_C, k, nullptr)) != RST_OK) return rs;
            hipLaunchKernelGGL(rst::idr::k_idr_v<VT>, gred, dim3(256), 0, c->stream, S, sdim, k,
                               (const rst::idr::IdrSt*)did, (const int*)act, (const VT*)Rv, (const VT*)Gv, Vv);
            if (pc && (rs = precondition(Vv, PHv, Wv, act, f32)) != RST_OK) return rs;
            hipLaunchKernelGGL(rst::idr::k_idr_u<VT>, gred, dim3(256), 0, c->stream, S, sdim, k,
                               (const rst::idr::IdrSt*)did, (const int*)act, (const VT*)VH, Uv);
            if ((rs = apply(Uk, Gk, act, f32)) != RST_OK) return rs;
            hipLaunchKernelGGL((rst::idr::k_idr_pdots<false, VT>), gred, dim3(256), 0, c->stream, S, sdim,
                               (const int*)act, Psh, (const VT*)Gk, part);
            if ((rs = iscal(rst::idr::ID_D, k, nullptr)) != RST_OK) return rs;
            hipLaunchKernelGGL(rst::idr::k_idr_upd<VT>, gred, dim3(256), 0, c->stream, S, k,
                               (const rst::idr::IdrSt*)did, (const int*)act, Gv, Uv, Rv, Xv, part);
            if ((rs = iscal(rst::idr::ID_CONV, k, nullptr)) != RST_OK) return rs;
          }
          // dimension reduction: v = M^-1 r, t = A v, omega from (t, r) and (t, t)
          VT* vr = Rv;
          if (pc) {
            if ((rs = precondition(Rv, PHv, Wv, act, f32)) != RST_OK) return rs;
            vr = PHv;
          }
          if ((rs = apply(vr, Tv, act, f32)) != RST_OK) return rs;
          hipLaunchKernelGGL((rst::mk::k_mk_dots<2, VT>), gred, dim3(256), 0, c->stream, S, (const int*)act,
                             (const VT*)Tv, (const VT*)Rv, (const VT*)Tv, (const VT*)Tv, part);
          if ((rs = iscal(rst::idr::ID_OMEGA, 0, nullptr)) != RST_OK) return rs;
          hipLaunchKernelGGL(rst::idr::k_idr_rx<VT>, gred, dim3(256), 0, c->stream, S, sdim,
                             (const rst::idr::IdrSt*)did, (const int*)act, Rv, Xv, (const VT*)Tv, (const VT*)vr,
                             Psh, part);
          if ((rs = iscal(rst::idr::ID_END, 0, nullptr)) != RST_OK) return rs;
          HIPCHK(c, hipGetLastError());
          HIPCHK(c, hipMemcpyAsync(hid.data(), did, ld * sizeof(rst::idr::IdrSt), hipMemcpyDeviceToHost, c->stream));
          HIPCHK(c, hipMemcpyAsync(hact.data(), act, ld * 4, hipMemcpyDeviceToHost, c->stream));
          HIPCHK(c, hipStreamSynchronize(c->stream));
          int nmark = 0, nact = 0;
          for (int j = 0; j < ld; ++j) {
            hmark[j] = (hid[j].done == 0 && !hact[j] && (hid[j].check || hid[j].brk)) ? 1 : 0;
            nmark += hmark[j];
            nact += hact[j];
          }
          if (inner) {
            for (int j = 0; j < ld; ++j)
              if (hmark[j]) hid[j].done = hid[j].check ? 1 : 2;
            if (nmark > 0)
              HIPCHK(c, hipMemcpyAsync(did, hid.data(), ld * sizeof(rst::idr::IdrSt), hipMemcpyHostToDevice,
                                       c->stream));
          } else if constexpr (!f32) {
            if (nmark > 0) {
              HIPCHK(c, hipMemcpyAsync(mark, hmark.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
              if ((rs = apply(Xv, Tv, mark, false)) != RST_OK) return rs;  // t is rebuilt by the next cycle
              hipLaunchKernelGGL(rst::mk::k_mk_resid, gred, dim3(256), 0, c->stream, S, Bv, (const int*)mark,
                                 (const double2*)Tv, Rv, part);
              HIPCHK(c, hipGetLastError());
              hpart.resize((size_t)S.nsplit * ld);
              HIPCHK(c, hipMemcpyAsync(hpart.data(), part, hpart.size() * 16, hipMemcpyDeviceToHost, c->stream));
              HIPCHK(c, hipStreamSynchronize(c->stream));
              std::vector<int> rmark(ld, 0);
              int nrestart = 0;
              for (int j = 0; j < ld; ++j) {
                if (!hmark[j]) continue;
                double rr = 0.0;
                for (int r = 0; r < S.nsplit; ++r) rr += hpart[(size_t)r * ld + j].x;
                rst::idr::IdrSt& q = hid[j];
                const double rel = q.bb > 0 ? std::sqrt(rr / q.bb) : 0.0;
                q.check = q.brk = 0;
                if (rel <= tol) {
                  q.done = 1;
                  q.rr = rel;
                } else if (q.its >= c->opts.max_iter || !std::isfinite(rel) || q.restarts >= 1000) {
                  q.done = 2;
                  q.rr = rel;
                } else {
                  q.restarts += 1;  // restart from the true residual (now in R)
                  rmark[j] = 1;
                  hact[j] = 1;
                  ++nrestart;
                }
              }
              HIPCHK(c, hipMemcpyAsync(did, hid.data(), ld * sizeof(rst::idr::IdrSt), hipMemcpyHostToDevice,
                                       c->stream));
              if (nrestart > 0) {
                HIPCHK(c, hipMemcpyAsync(mark, rmark.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
                hipLaunchKernelGGL(rst::idr::k_idr_zero<VT>, dim3(gel), dim3(256), 0, c->stream, S, sdim,
                                   (const int*)mark, Gv, Uv);
                hipLaunchKernelGGL((rst::idr::k_idr_pdots<true, VT>), gred, dim3(256), 0, c->stream, S, sdim,
                                   (const int*)mark, Psh, (const VT*)Rv, part);
                if ((rs = iscal(rst::idr::ID_RESTART, 0, mark)) != RST_OK) return rs;
                HIPCHK(c, hipMemcpyAsync(act, hact.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
                nact += nrestart;
              }
            }
          }
          if (nact == 0) break;
        }
        return RST_OK;
      };
      if (!mixed) {
        if ((ps = run_idr((double2*)nullptr, B, c->opts.tol, false, nullptr)) != RST_OK) return ps;
        for (int j = 0; j < ld; ++j) {
          hst[j].its = hid[j].its;
          hst[j].restarts = hid[j].restarts;
          hst[j].rr = hid[j].rr;
          hst[j].done = hid[j].done;
        }
      } else {
        // FP64 refinement: x = 0, r = b; each cycle solves A d = r in complex64 to the relative
        // tolerance update_delta for the columns not yet done, x += d, r = b - A x in FP64
        hipLaunchKernelGGL(rst::mk::k_mk_rhs, gred, dim3(256), 0, c->stream, S, B, X64, R64, part);
        HIPCHK(c, hipGetLastError());
        hpart.resize((size_t)S.nsplit * ld);
        HIPCHK(c, hipMemcpyAsync(hpart.data(), part, hpart.size() * 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        std::vector<double> bb(ld, 0.0), rel(ld, 0.0);
        std::vector<int> cum(ld, 0), cyc(ld, 0), fin(ld, 0), stall(ld, 0), cap(ld, 0), open(ld, 0);
        std::vector<long long> doff2(ld, -1);
        for (int j = 0; j < ld; ++j) {
          for (int r = 0; r < S.nsplit; ++r) bb[j] += hpart[(size_t)r * ld + j].x;
          fin[j] = bb[j] > 0.0 ? 0 : 1;  // a zero right-hand side (or a padding column) is solved by x = 0
          rel[j] = bb[j] > 0.0 ? 1.0 : 0.0;
        }
        if ((e = ensure(c, c->d_mkref, (size_t)ld * (8 + 4))) != RST_OK) return e;
        long long* d_doff2 = (long long*)c->d_mkref.p;
        int* d_cap = (int*)(d_doff2 + ld);
        rst::mk::Rhs Bi;
        Bi.src = d_src;
        Bi.bsc = d_bsc;
        Bi.dense = R64;
        Bi.dld = ld;
        Bi.doff = d_doff2;
        for (;;) {
          int nopen = 0;
          for (int j = 0; j < ld; ++j) {
            open[j] = fin[j] == 0 ? 1 : 0;
            doff2[j] = open[j] ? j : -1;
            cap[j] = open[j] ? c->opts.max_iter - cum[j] : 0;
            nopen += open[j];
          }
          if (nopen == 0) break;
          HIPCHK(c, hipMemcpyAsync(d_doff2, doff2.data(), ld * 8, hipMemcpyHostToDevice, c->stream));
          HIPCHK(c, hipMemcpyAsync(d_cap, cap.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
          HIPCHK(c, hipMemcpyAsync(mark, open.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
          if ((ps = run_idr((float2*)nullptr, Bi, c->opts.update_delta, true, d_cap)) != RST_OK) return ps;
          hipLaunchKernelGGL(rst::mk::k_mk_addx, gred, dim3(256), 0, c->stream, S, (const int*)mark, X64,
                             (const float2*)c->d_mkv.p);
          if ((ps = apply(X64, R64, mark, false)) != RST_OK) return ps;
          hipLaunchKernelGGL(rst::mk::k_mk_resid, gred, dim3(256), 0, c->stream, S, B, (const int*)mark,
                             (const double2*)R64, R64, part);
          HIPCHK(c, hipGetLastError());
          HIPCHK(c, hipMemcpyAsync(hpart.data(), part, hpart.size() * 16, hipMemcpyDeviceToHost, c->stream));
          HIPCHK(c, hipStreamSynchronize(c->stream));
          for (int j = 0; j < ld; ++j) {
            if (!open[j]) continue;
            double rr = 0.0;
            for (int r = 0; r < S.nsplit; ++r) rr += hpart[(size_t)r * ld + j].x;
            const double rn = std::sqrt(rr / bb[j]);
            cum[j] += hid[j].its;
            cyc[j] += 1;
            // a cycle that does not halve the residual counts as a stall; three in a row end the column
            stall[j] = rn > 0.5 * rel[j] ? stall[j] + 1 : 0;
            rel[j] = rn;
            if (rn <= c->opts.tol)
              fin[j] = 1;
            else if (cum[j] >= c->opts.max_iter || !std::isfinite(rn) || stall[j] >= 3)
              fin[j] = 2;
          }
        }
        for (int j = 0; j < ld; ++j) {
          hst[j].its = cum[j];
          hst[j].restarts = std::max(0, cyc[j] - 1);
          hst[j].rr = rel[j];
          hst[j].done = fin[j];
          if (j < nc) c->last_updates[(size_t)(it0 + j)] = cyc[j];
        }
      }
    }
    // outputs of the block: T over the destination CAP, the exported solutions, per-column records
    std::vector<double> tb(ld, 0.0);
    const int xc0 = cocg2 ? per_blk : 0;  // the +k solutions of the doubled COCG
    if (d_gdst) {
      hipLaunchKernelGGL(rst::mk::k_mk_tacc, gred, dim3(256), 0, c->stream, S, P, d_gdst, Xres, part);
      hipLaunchKernelGGL(rst::mk::k_mk_sum, dim3(gsc), dim3(64), 0, c->stream, S, (const double2*)part,
                         (double*)c->d_mkT.p);
      HIPCHK(c, hipGetLastError());
      HIPCHK(c, hipMemcpyAsync(tb.data(), c->d_mkT.p, ld * 8, hipMemcpyDeviceToHost, c->stream));
    }
    if (xout) {
      hipLaunchKernelGGL(rst::mk::k_mk_export, dim3(gel), dim3(256), 0, c->stream, S, nc, Xres, xout, nitems,
                         it0, xc0);
      HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int j = 0; j < nc; ++j) {
      const rst::mk::ColSt& q = hst[j];
      const size_t o = (size_t)(it0 + j);
      Tcol[o] = tb[xc0 + j];
      its[o] = q.its;
      rss[o] = q.restarts;
      res[o] = q.done == 0 ? 0.0 : q.rr;
      st[o] = q.done == 1 ? 0 : 1;
      col_its += q.its;
      col_cyc += mixed && q.its > 0 ? q.restarts + 1 : 0;
    }
    // mixed: complex64 vectors in the inner solves (half the bytes), and per cycle the FP64 apply,
    // residual and correction (x, r: 104 B per point)
    // doubled COCG: per step one apply and one M^-1 over both halves and the vector work (x, r, p
    // updates, two dots): 2 x (apply 32 + M^-1 192 + 160) B per point
    if (cocg2)
      bytes += (double)col_its * (2.0 * ((pc ? 224.0 : 32.0) + 160.0) * (double)n + 2.0 * 16.0 * (double)nent);
    else
      bytes += idr ? (double)col_its * ((mixed ? 0.5 : 1.0) * idr_bytes_per_matvec(sdim, pc) * (double)n +
                                      16.0 * (double)nent) +
                       (double)col_cyc * (104.0 * (double)n + 16.0 * (double)nent)
                 : (double)col_its * (mk_bytes_per_point(pc) * (double)n + 2.0 * 16.0 * (double)nent);
  }
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float fms = 0;
  HIPCHK(c, hipEventElapsedTime(&fms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  ms = fms;
  c->last_mk = true;
  c->last_mk_bytes = bytes;
  c->last_cw = ld;
  return RST_OK;
}

rst_status run_cocg(rst_ctx* c, int ne, const double* energies, const std::vector<int64_t>& cols,
                    const double* d_gdst, const std::vector<double>* hsrc, double2* xout,
                    std::vector<double>& Tcol, std::vector<int>& its, std::vector<int>& rss,
                    std::vector<double>& res, std::vector<int>& st, double& ms) {
  constexpr int CHECK = 4;
  const bool usepc = c->opts.precond == RST_PRECOND_FREE_CAP;
  {
    const rst::Geo g0 = make_geo(c);
    if (std::fabs(g0.pha_y) > 1e-12 || std::fabs(g0.phb_y) > 1e-12)
      return fail(c, RST_EUNSUPPORTED, "COCG needs a real H_k: k_a L_a and k_b L_b must be multiples of pi");
  }
  const int P = c->na * c->nb;
  const long long n = (long long)P * c->nz;
  const int ncols = (int)cols.size();
  BlockedShape bs;
  // automatic: one column per workgroup (config 2 at the Gamma point: 9.2 s against 11.2 s with two)
  rst_status s = blocked_shape(c, c->opts.col_block > 0 ? c->opts.col_block : 1, c->opts.threads, bs);
  if (s != RST_OK) return s;
  const LaunchShape ls = bs.ls;
  const int cw = ls.cw;
  c->last_cw = cw;
  c->last_threads = ls.threads;
  void* kapply = pick_kernel(c->rad, ls.q, 1);
  void* kpc = pick_kernel(c->rad, ls.q, 7);
  if (!kapply || !kpc) return fail(c, RST_EUNSUPPORTED, "no kernel instance");
  // chunk of columns: X, R, Z, P, Q, W and the M^-1 work buffer, bounded by a quarter of free memory;
  // wide chunks give the blocked kernels enough workgroups (4096 columns of config 2: 22 GB)
  const size_t per_col = (size_t)7 * n * 16;
  size_t free_b = 0, total_b = 0;
  HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
  long long chunk = std::min<long long>(4096, std::max<long long>(cw, (long long)(free_b / 4 / per_col)));
  chunk = std::max<long long>(cw, chunk / cw * cw);
  chunk = std::min<long long>(chunk, ((long long)ncols + cw - 1) / cw * cw);
  const int ncolp = (int)chunk;
  const int nblk = ncolp / cw;
  const size_t vlen = (size_t)nblk * n * cw;
  rst_status e;
  if ((e = ensure(c, c->d_fgX, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgW, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgM, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgwb, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_cgR, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_cgP, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_cgQ, vlen * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_cgs, (size_t)6 * ncolp * 16)) != RST_OK) return e;
  if ((e = ensure(c, c->d_cgi, (size_t)3 * ncolp * 4)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgsrc, (size_t)ncolp * 8)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgbsc, (size_t)ncolp * 8)) != RST_OK) return e;
  if ((e = ensure(c, c->d_fgt, (size_t)ncolp * 8)) != RST_OK) return e;
  double2* X = (double2*)c->d_fgX.p;
  double2* W = (double2*)c->d_fgW.p;
  double2* Z = (double2*)c->d_fgM.p;
  double2* R = (double2*)c->d_cgR.p;
  double2* Pv = (double2*)c->d_cgP.p;
  double2* Q = (double2*)c->d_cgQ.p;
  double2* rho = (double2*)c->d_cgs.p;
  double2* pq = rho + ncolp;
  double2* rhon = pq + ncolp;
  double2* n2 = rhon + ncolp;
  double2* alpha = n2 + ncolp;
  double2* beta = alpha + ncolp;
  int* actd = (int*)c->d_cgi.p;
  int* brkd = actd + ncolp;
  int* markd = brkd + ncolp;
  rst::Geo g = make_geo(c);
  rst::Proj pj = make_proj(c);
  const size_t pws_stride = std::max<size_t>(1, (size_t)c->nproj * cw);
  if ((e = ensure(c, c->d_pws, (size_t)nblk * pws_stride * 16)) != RST_OK) return e;
  if (bs.lds_apply > 64 * 1024)
    HIPCHK(c, hipFuncSetAttribute(kapply, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bs.lds_apply));
  if (bs.lds_pc > 64 * 1024)
    HIPCHK(c, hipFuncSetAttribute(kpc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bs.lds_pc));
  rst::fg::Shape S{n, cw, nblk, 0, 0};
  std::vector<double> en(energies, energies + ne);
  if ((e = upload(c, c->d_en, en)) != RST_OK) return e;
  double vbar = 0;
  for (double x : c->v) vbar += x;
  vbar /= (double)c->v.size();
  if (usepc && (e = ensure(c, c->d_pc_inv, (size_t)n * 16)) != RST_OK) return e;
  const size_t nout = (size_t)ne * ncols;
  Tcol.assign(nout, 0.0);
  its.assign(nout, 0);
  rss.assign(nout, 0);
  res.assign(nout, 0.0);
  st.assign(nout, 1);
  c->last_fallbacks = 0;
  c->last_cnn_flop = 0.0;
  c->last_updates.clear();
  double bytes = 0.0;
  const unsigned gv = (unsigned)((vlen + 255) / 256);
  const unsigned gc = (unsigned)((ncolp + 63) / 64);
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, hipEventRecord(e0, c->stream));
  double export_ms = 0.0;
  for (int ie = 0; ie < ne; ++ie) {
    // operator slots: 0 applies P -> Q, 1 applies X -> W (true residual)
    std::vector<rst::ApplyArgs> aa(2);
    for (int j = 0; j < 2; ++j) {
      rst::ApplyArgs& A = aa[j];
      std::memset(&A, 0, sizeof(A));
      A.g = g;
      A.pj = pj;
      A.V = (const double*)c->d_v.p;
      A.gz = (const double*)c->d_gz.p;
      A.energy = energies[ie];
      A.x = j == 0 ? Pv : X;
      A.y = j == 0 ? Q : W;
      A.ncol = ncolp;
      A.cw = cw;
      A.nblk = nblk;
      A.pws = (double2*)c->d_pws.p;
      A.pws_stride = pws_stride;
      A.proj_pre = c->nproj > 0;
    }
    if ((e = upload(c, c->d_fgaa, aa)) != RST_OK) return e;
    if (usepc) {
      rst::SolveArgs A;
      std::memset(&A, 0, sizeof(A));
      A.g = g;
      A.gz = (const double*)c->d_gz.p;
      A.energies = (const double*)c->d_en.p + ie;
      A.ne = 1;
      A.pc.vbar = vbar;
      A.pc.a = 0.5 / (c->hz * c->hz);
      A.pc.eps = (const double*)c->d_pc_eps.p;
      A.pc.vz = pc_vz(c);
      A.pc.shift = c->opts.pc_shift;
      A.pc.steps = (const double2*)c->d_pc_twa.p;
      A.pc.inv = (const double2*)c->d_pc_inv.p;
      std::vector<rst::SolveArgs> sa(1, A);
      if ((e = upload(c, c->d_fgsa, sa)) != RST_OK) return e;
      hipLaunchKernelGGL(rst::k_pc_pivots, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, c->stream,
                         (const rst::SolveArgs*)c->d_fgsa.p);
      HIPCHK(c, hipGetLastError());
      std::vector<rst::PcApplyArgs> pa(1);
      std::memset(&pa[0], 0, sizeof(pa[0]));
      pa[0].g = g;
      pa[0].pc = A.pc;
      pa[0].in = R;
      pa[0].out = Z;
      pa[0].wbuf = (double2*)c->d_fgwb.p;
      pa[0].cw = cw;
      pa[0].nblk = nblk;
      pa[0].pc_lds_off = bs.pc_off;
      if ((e = upload(c, c->d_fgpa, pa)) != RST_OK) return e;
    }
    void* aarg0 = c->d_fgaa.p;
    void* aarg1 = (char*)c->d_fgaa.p + sizeof(rst::ApplyArgs);
    void* parg = c->d_fgpa.p;
    auto apply_pq = [&]() -> rst_status {
      rst_status ps = proj_blocked(c, aa[0]);
      if (ps != RST_OK) return ps;
      void* args[] = {&aarg0};
      HIPCHK(c, hipLaunchKernel(kapply, dim3(nblk), dim3(ls.threads), args, bs.lds_apply, c->stream));
      return RST_OK;
    };
    auto precondition = [&]() -> rst_status {  // Z = M^-1 R (or R)
      if (usepc) {
        void* args[] = {&parg};
        HIPCHK(c, hipLaunchKernel(kpc, dim3(nblk), dim3(ls.threads), args, bs.lds_pc, c->stream));
      } else {
        HIPCHK(c, hipMemcpyAsync(Z, R, vlen * 16, hipMemcpyDeviceToDevice, c->stream));
      }
      return RST_OK;
    };
    // true residual W = b - A X and its squared norms into n2
    auto true_residual = [&]() -> rst_status {
      rst_status ps = proj_blocked(c, aa[1]);
      if (ps != RST_OK) return ps;
      void* args[] = {&aarg1};
      HIPCHK(c, hipLaunchKernel(kapply, dim3(nblk), dim3(ls.threads), args, bs.lds_apply, c->stream));
      hipLaunchKernelGGL(rst::fg::k_fg_resid, dim3(gv), dim3(256), 0, c->stream, S, (const long long*)c->d_fgsrc.p,
                         (const double*)c->d_fgbsc.p, (const double2*)W, W);
      hipLaunchKernelGGL(rst::cg::k_cg_dot, dim3(nblk), dim3(256), 0, c->stream, S, (const double2*)W,
                         (const double2*)W, 1, n2, ncolp);
      HIPCHK(c, hipGetLastError());
      return RST_OK;
    };
    for (int c0 = 0; c0 < ncols; c0 += ncolp) {
      const int nc = std::min(ncolp, ncols - c0);
      S.ncol = nc;
      std::vector<long long> src(ncolp, -1);
      std::vector<double> bsc(ncolp, 0.0), bnorm(ncolp, 1.0);
      std::vector<int> act(ncolp, 0), itc(ncolp, 0), rst_n(ncolp, 0), mark(ncolp, 0), need(ncolp, 0);
      for (int j = 0; j < nc; ++j) {
        src[j] = cols[c0 + j];
        const double gs = hsrc ? (*hsrc)[cols[c0 + j] / P] : 1.0;
        bsc[j] = std::sqrt(gs);
        bnorm[j] = bsc[j];
        act[j] = bsc[j] > 0 ? 1 : 0;
        if (!act[j]) st[(size_t)ie * ncols + c0 + j] = 0;  // zero right-hand side: x = 0
      }
      if ((e = upload(c, c->d_fgsrc, src)) != RST_OK) return e;
      if ((e = upload(c, c->d_fgbsc, bsc)) != RST_OK) return e;
      HIPCHK(c, hipMemcpyAsync(actd, act.data(), (size_t)ncolp * 4, hipMemcpyHostToDevice, c->stream));
      std::vector<int> zeros(ncolp, 0), ones(ncolp, 1);
      HIPCHK(c, hipMemcpyAsync(brkd, zeros.data(), (size_t)ncolp * 4, hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(markd, ones.data(), (size_t)ncolp * 4, hipMemcpyHostToDevice, c->stream));
      // x = 0, r = b, z = M^-1 r, p = z, rho = r^T z
      hipLaunchKernelGGL(rst::fg::k_fg_init, dim3(gv), dim3(256), 0, c->stream, S, (const long long*)c->d_fgsrc.p,
                         (const double*)c->d_fgbsc.p, X, R);
      HIPCHK(c, hipGetLastError());
      if ((e = precondition()) != RST_OK) return e;
      hipLaunchKernelGGL(rst::cg::k_cg_copy_marked, dim3(gv), dim3(256), 0, c->stream, S, Pv, (const double2*)Z,
                         (const int*)markd);
      hipLaunchKernelGGL(rst::cg::k_cg_dot, dim3(nblk), dim3(256), 0, c->stream, S, (const double2*)R,
                         (const double2*)Z, 0, rhon, ncolp);
      hipLaunchKernelGGL(rst::cg::k_cg_rho_set, dim3(gc), dim3(64), 0, c->stream, ncolp, rho, (const double2*)rhon,
                         (const int*)markd);
      HIPCHK(c, hipGetLastError());
      std::vector<double2> hn2(ncolp);
      std::vector<int> hbrk(ncolp);
      int nact = 0;
      for (int q = 0; q < nc; ++q) nact += act[q];
      for (int it = 0; it < c->opts.max_iter && nact > 0; ++it) {
        if ((e = apply_pq()) != RST_OK) return e;
        hipLaunchKernelGGL(rst::cg::k_cg_dot, dim3(nblk), dim3(256), 0, c->stream, S, (const double2*)Pv,
                           (const double2*)Q, 0, pq, ncolp);
        hipLaunchKernelGGL(rst::cg::k_cg_alpha, dim3(gc), dim3(64), 0, c->stream, ncolp, (const double2*)rho,
                           (const double2*)pq, (const int*)actd, alpha, brkd);
        hipLaunchKernelGGL(rst::cg::k_cg_xr, dim3(gv), dim3(256), 0, c->stream, S, X, R, (const double2*)Pv,
                           (const double2*)Q, (const double2*)alpha);
        HIPCHK(c, hipGetLastError());
        if ((e = precondition()) != RST_OK) return e;
        hipLaunchKernelGGL(rst::cg::k_cg_dot, dim3(nblk), dim3(256), 0, c->stream, S, (const double2*)R,
                           (const double2*)Z, 0, rhon, ncolp);
        hipLaunchKernelGGL(rst::cg::k_cg_dot, dim3(nblk), dim3(256), 0, c->stream, S, (const double2*)R,
                           (const double2*)R, 1, n2, ncolp);
        hipLaunchKernelGGL(rst::cg::k_cg_beta, dim3(gc), dim3(64), 0, c->stream, ncolp, rho, (const double2*)rhon,
                           (const int*)actd, beta, brkd);
        hipLaunchKernelGGL(rst::cg::k_cg_p, dim3(gv), dim3(256), 0, c->stream, S, Pv, (const double2*)Z,
                           (const double2*)beta);
        HIPCHK(c, hipGetLastError());
        for (int q = 0; q < nc; ++q) itc[q] += act[q];
        // apply 48, pq 32, x/r update 96, M^-1 64 (or copy 32), two dots 48, p update 48 B per point
        bytes += (double)nact * n * (48.0 + 32.0 + 96.0 + (usepc ? 64.0 : 32.0) + 48.0 + 48.0);
        const bool last = it + 1 == c->opts.max_iter;
        if ((it + 1) % CHECK != 0 && !last) continue;
        HIPCHK(c, hipMemcpyAsync(hn2.data(), n2, (size_t)ncolp * 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(hbrk.data(), brkd, (size_t)ncolp * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        bool check = last;
        for (int q = 0; q < nc; ++q) {
          need[q] = 0;
          if (!act[q]) continue;
          const double est = std::sqrt(hn2[q].x) / bnorm[q];
          if (hbrk[q] || !std::isfinite(est) || est <= c->opts.tol) need[q] = 1;
          check = check || need[q];
        }
        if (!check) continue;
        // FP64 true residual of the chunk
        if ((e = true_residual()) != RST_OK) return e;
        bytes += (double)nact * n * (48.0 + 32.0 + 16.0);
        HIPCHK(c, hipMemcpyAsync(hn2.data(), n2, (size_t)ncolp * 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        bool restart = false;
        for (int q = 0; q < nc; ++q) {
          mark[q] = 0;
          if (!act[q]) continue;
          const double rel = std::sqrt(hn2[q].x) / bnorm[q];
          res[(size_t)ie * ncols + c0 + q] = rel;
          if (rel <= c->opts.tol) {
            act[q] = 0;
            st[(size_t)ie * ncols + c0 + q] = 0;
          } else if (!std::isfinite(rel)) {
            act[q] = 0;
            st[(size_t)ie * ncols + c0 + q] = 2;
          } else if (last) {
            act[q] = 0;  // iteration cap: unconverged (status 1)
          } else if (need[q]) {
            // the estimate fell below tol but the true residual did not, or a breakdown: restart
            mark[q] = 1;
            ++rst_n[q];
            restart = true;
          }
        }
        nact = 0;
        for (int q = 0; q < nc; ++q) nact += act[q];
        HIPCHK(c, hipMemcpyAsync(actd, act.data(), (size_t)ncolp * 4, hipMemcpyHostToDevice, c->stream));
        if (restart && nact > 0) {
          // marked columns: r = b - A x, z = M^-1 r, p = z, rho = r^T z (the others keep their recurrences)
          HIPCHK(c, hipMemcpyAsync(markd, mark.data(), (size_t)ncolp * 4, hipMemcpyHostToDevice, c->stream));
          hipLaunchKernelGGL(rst::cg::k_cg_copy_marked, dim3(gv), dim3(256), 0, c->stream, S, R, (const double2*)W,
                             (const int*)markd);
          HIPCHK(c, hipMemcpyAsync(brkd, zeros.data(), (size_t)ncolp * 4, hipMemcpyHostToDevice, c->stream));
          if ((e = precondition()) != RST_OK) return e;
          hipLaunchKernelGGL(rst::cg::k_cg_dot, dim3(nblk), dim3(256), 0, c->stream, S, (const double2*)R,
                             (const double2*)Z, 0, rhon, ncolp);
          hipLaunchKernelGGL(rst::cg::k_cg_copy_marked, dim3(gv), dim3(256), 0, c->stream, S, Pv, (const double2*)Z,
                             (const int*)markd);
          hipLaunchKernelGGL(rst::cg::k_cg_rho_set, dim3(gc), dim3(64), 0, c->stream, ncolp, rho,
                             (const double2*)rhon, (const int*)markd);
          HIPCHK(c, hipGetLastError());
        }
      }
      if (d_gdst) {
        hipLaunchKernelGGL(rst::fg::k_fg_tacc, dim3(nblk), dim3(256), 0, c->stream, S, (const double2*)X, d_gdst,
                           (long long)P, (double*)c->d_fgt.p);
        HIPCHK(c, hipGetLastError());
        std::vector<double> ta(ncolp);
        HIPCHK(c, hipMemcpyAsync(ta.data(), c->d_fgt.p, (size_t)ncolp * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int q = 0; q < nc; ++q) Tcol[(size_t)ie * ncols + c0 + q] = 4.0 * ta[q];
      }
      for (int q = 0; q < nc; ++q) {
        its[(size_t)ie * ncols + c0 + q] = itc[q];
        rss[(size_t)ie * ncols + c0 + q] = rst_n[q];
      }
      if (xout) {
        // x (n x ncols, column fastest) from the blocked X (a test-sized export through the
        // host, kept out of the reported time)
        const auto t_exp = std::chrono::steady_clock::now();
        std::vector<double2> hx(vlen), rows((size_t)n * nc);
        HIPCHK(c, hipMemcpyAsync(hx.data(), X, vlen * 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int q = 0; q < nc; ++q)
          for (long long p = 0; p < n; ++p) rows[(size_t)p * nc + q] = hx[((size_t)(q / cw) * n + p) * cw + q % cw];
        HIPCHK(c, hipMemcpy2D(xout + c0, (size_t)ncols * 16, rows.data(), (size_t)nc * 16, (size_t)nc * 16, (size_t)n,
                              hipMemcpyHostToDevice));
        export_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_exp).count();
      }
    }
  }
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float fms = 0;
  HIPCHK(c, hipEventElapsedTime(&fms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  ms = std::max(0.0, (double)fms - export_ms);
  c->last_fg_bytes = bytes;
  return RST_OK;
}

// Launches the batched solver over the structures `sel` of the batch (all
// energies of each, or the first `ne_cap` if > 0) with cw columns per
// workgroup.  Returns per-structure, per-energy T and the per-column stats.
struct BatchOut {
  std::vector<std::vector<double>> T;  // [structure in sel order][energy]
  std::vector<int> its, rss, stv;
  std::vector<double> res;
  double ms = 0;
  double points_n = 0;  // sum over columns of the structure's grid size (bytes bookkeeping)
  int cw = 0, threads = 0;
};

rst_status batch_collect(rst_ctx* c, const std::vector<int>& sel, const std::vector<std::vector<int64_t>>& pcols,
                         const std::vector<long long>& out_off, const std::vector<int>& ne_of, long long outs,
                         int P, BatchOut& out);

rst_status run_batch(rst_ctx* c, const std::vector<int>& sel, int ne_cap, int cw, bool use_graph,
                     BatchOut& out, bool per_structure = false, int threads = -1) {
  LaunchShape ls;
  rst_status s = choose_shape(c, cw, threads >= 0 ? threads : c->opts.threads, ls);
  if (s != RST_OK) return s;
  const int P = c->na * c->nb;
  const bool lr = c->opts.direction == RST_DIR_LR;
  // order the work by decreasing cost so the long structures start first
  std::vector<int> order(sel.size());
  std::vector<double> cost(sel.size());
  std::vector<std::vector<int64_t>> pcols(sel.size());
  for (size_t i = 0; i < sel.size(); ++i) {
    const auto& hp = c->batch[sel[i]];
    const std::vector<double>& gs = lr ? hp.gr : hp.gl;
    for (int z = 0; z < hp.nz; ++z)
      if (gs[z] > 0)
        for (int p = 0; p < P; ++p) pcols[i].push_back((int64_t)z * P + p);
    const int ne = ne_cap > 0 ? std::min<int>(ne_cap, (int)hp.en.size()) : (int)hp.en.size();
    cost[i] = (double)hp.nz * pcols[i].size() * ne;
    order[i] = (int)i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  const bool pc = c->opts.precond == RST_PRECOND_FREE_CAP;
  std::vector<double> pc_eps;
  std::vector<double2> pc_steps;
  long long inv_total = 0;
  std::vector<rst::BatchProb> bp(sel.size());
  std::vector<double> v, gz, gl, gr, en;
  std::vector<int64_t> cols;
  long long items = 0, outs = 0;
  int nz_max = 1;
  std::vector<long long> out_off(sel.size());
  std::vector<int> ne_of(sel.size());
  for (int oi : order) {
    const auto& hp = c->batch[sel[oi]];
    const int ne = ne_cap > 0 ? std::min<int>(ne_cap, (int)hp.en.size()) : (int)hp.en.size();
    const int ncols = (int)pcols[oi].size();
    rst::BatchProb& b = bp[oi];
    std::memset(&b, 0, sizeof(b));
    b.nz = hp.nz;
    b.ne = ne;
    b.ncols = ncols;
    b.nblk = (ncols + ls.cw - 1) / ls.cw;
    b.item0 = items;
    b.v_off = (long long)v.size();
    b.gz_off = (int)gz.size();
    b.e_off = (int)en.size();
    b.col_off = (long long)cols.size();
    b.out_off = outs;
    const double la = c->na * c->ha, lb = c->nb * c->hb;
    b.pha_x = std::cos(hp.ka * la);
    b.pha_y = std::sin(hp.ka * la);
    b.phb_x = std::cos(hp.kb * lb);
    b.phb_y = std::sin(hp.kb * lb);
    if (pc) {
      std::vector<double> eps;
      std::vector<double2> steps;
      pc_tables(c, hp.ka, hp.kb, eps, steps);
      b.eps_off = (long long)pc_eps.size();
      b.steps_off = (long long)pc_steps.size();
      b.inv_off = inv_total;
      double vb = 0;
      for (double x : hp.v) vb += x;
      b.vbar = vb / (double)hp.v.size();
      pc_eps.insert(pc_eps.end(), eps.begin(), eps.end());
      pc_steps.insert(pc_steps.end(), steps.begin(), steps.end());
      inv_total += (long long)ne * hp.nz * P;
    }
    items += ncols > 0 ? (long long)b.nblk * ne : 0;
    outs += (long long)ne * ncols;
    out_off[oi] = b.out_off;
    ne_of[oi] = ne;
    nz_max = std::max(nz_max, hp.nz);
    v.insert(v.end(), hp.v.begin(), hp.v.end());
    for (int z = 0; z < hp.nz; ++z) gz.push_back(hp.gl[z] + hp.gr[z]);
    gl.insert(gl.end(), hp.gl.begin(), hp.gl.end());
    gr.insert(gr.end(), hp.gr.begin(), hp.gr.end());
    en.insert(en.end(), hp.en.begin(), hp.en.begin() + ne);
    cols.insert(cols.end(), pcols[oi].begin(), pcols[oi].end());
  }
  // the structures in item order (binary search by item0)
  std::vector<rst::BatchProb> bsorted;
  for (int oi : order) bsorted.push_back(bp[oi]);
  out.T.assign(sel.size(), {});
  for (size_t i = 0; i < sel.size(); ++i) out.T[i].assign(ne_of[i], 0.0);
  out.cw = ls.cw;
  out.threads = ls.threads;
  if (items == 0) return RST_OK;
  if (items > 0x7fffffff) return fail(c, RST_EINVAL, "too many work items in the batch");
  if ((s = upload(c, c->d_bprob, bsorted)) != RST_OK) return s;
  if ((s = upload(c, c->d_bv, v)) != RST_OK) return s;
  if ((s = upload(c, c->d_bgz, gz)) != RST_OK) return s;
  if ((s = upload(c, c->d_bgl, gl)) != RST_OK) return s;
  if ((s = upload(c, c->d_bgr, gr)) != RST_OK) return s;
  if ((s = upload(c, c->d_ben, en)) != RST_OK) return s;
  if ((s = upload(c, c->d_bcols, cols)) != RST_OK) return s;
  // per_structure: the single-structure kernel once per structure, back to back
  void* kern = pick_kernel(c->rad, ls.q, per_structure ? (pc ? 2 : 0) : (pc ? 6 : 5));
  if (!kern) return fail(c, RST_EUNSUPPORTED, "no kernel instance");
  rst::Geo g = make_geo(c);
  g.nz = nz_max;
  rst::Proj pj = make_proj(c);
  pj.nproj = 0;
  size_t lds = rst::lds_bytes<double>(g.pa, g.pb, g.P, 0, 0, pj.nm, ls.cw, ls.threads);
  const size_t pc_off = (lds + 15) & ~size_t(15);
  if (pc) lds = pc_off + (size_t)3 * (c->na + c->nb) * 16;
  int per_cu = 0, ncu = 0;
  HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, ls.threads, lds));
  HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  if (per_cu < 1) return fail(c, RST_EUNSUPPORTED, "kernel does not fit on a compute unit");
  const size_t n_max = (size_t)P * nz_max;
  const size_t ws_stride = (pc ? 9 : 5) * n_max * ls.cw;
  size_t free_b = 0, total_b = 0;
  HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
  long long nwg = std::min<long long>(items, (long long)per_cu * ncu);
  nwg = std::min<long long>(nwg, std::max<long long>(1, (long long)(free_b / 4 / (ws_stride * 16))));
  if ((s = ensure(c, c->d_ws, nwg * ws_stride * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_pws, 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_T, outs * 8)) != RST_OK) return s;
  if ((s = ensure(c, c->d_it, outs * 4)) != RST_OK) return s;
  if ((s = ensure(c, c->d_rs, outs * 4)) != RST_OK) return s;
  if ((s = ensure(c, c->d_res, outs * 8)) != RST_OK) return s;
  if ((s = ensure(c, c->d_st, outs * 4)) != RST_OK) return s;
  if ((s = ensure(c, c->d_counter, 64)) != RST_OK) return s;
  rst::SolveArgs A;
  std::memset(&A, 0, sizeof(A));
  A.batch = (const rst::BatchProb*)c->d_bprob.p;
  A.nprob = (int)bsorted.size();
  A.g = g;
  A.pj = pj;
  A.V = (const double*)c->d_bv.p;
  A.gz = (const double*)c->d_bgz.p;
  A.gdst = lr ? (const double*)c->d_bgl.p : (const double*)c->d_bgr.p;
  A.gsrc = lr ? (const double*)c->d_bgr.p : (const double*)c->d_bgl.p;
  A.energies = (const double*)c->d_ben.p;
  A.cols = (const int64_t*)c->d_bcols.p;
  A.cw = ls.cw;
  A.nitems = (int)items;
  A.tol = c->opts.tol;
  A.max_iter = c->opts.max_iter;
  A.ws = c->d_ws.p;
  A.ws_stride = ws_stride;
  A.pws = (double2*)c->d_pws.p;
  A.pws_stride = 1;
  A.T_col = (double*)c->d_T.p;
  A.iters = (int*)c->d_it.p;
  A.restarts = (int*)c->d_rs.p;
  A.resid = (double*)c->d_res.p;
  A.status = (int*)c->d_st.p;
  A.counter = (int*)c->d_counter.p;
  A.pc_lds_off = pc_off;
  if (pc) {
    if ((s = upload(c, c->d_bpc_eps, pc_eps)) != RST_OK) return s;
    if ((s = upload(c, c->d_bpc_steps, pc_steps)) != RST_OK) return s;
    if ((s = ensure(c, c->d_pc_inv, (size_t)inv_total * 16)) != RST_OK) return s;
    A.pc.a = 0.5 / (c->hz * c->hz);
    A.pc.eps = (const double*)c->d_bpc_eps.p;
    A.pc.shift = c->opts.pc_shift;
    A.pc.steps = (const double2*)c->d_bpc_steps.p;
    A.pc.inv = (const double2*)c->d_pc_inv.p;
    // Thomas pivots of every (structure, energy): one pivot launch per structure
    std::vector<rst::SolveArgs> pargs(bsorted.size(), A);
    for (size_t i = 0; i < bsorted.size(); ++i) {
      const rst::BatchProb& b = bsorted[i];
      rst::SolveArgs& q = pargs[i];
      q.batch = nullptr;
      q.nprob = 0;
      q.g.nz = b.nz;
      q.ne = b.ne;
      q.energies = A.energies + b.e_off;
      q.gz = A.gz + b.gz_off;
      q.pc.vbar = b.vbar;
      q.pc.eps = A.pc.eps + b.eps_off;
      q.pc.inv = A.pc.inv + b.inv_off;
    }
    if ((s = upload(c, c->d_bpargs, pargs)) != RST_OK) return s;
    for (size_t i = 0; i < bsorted.size(); ++i) {
      const long long nt = (long long)bsorted[i].ne * P;
      if (nt == 0) continue;
      hipLaunchKernelGGL(rst::k_pc_pivots, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream,
                         (const rst::SolveArgs*)c->d_bpargs.p + i);
    }
    HIPCHK(c, hipGetLastError());
  }
  if (per_structure) {
    // each structure's own arguments; every launch resets the work counter first
    std::vector<rst::SolveArgs> qs(bsorted.size(), A);
    std::vector<long long> nit(bsorted.size());
    for (size_t i = 0; i < bsorted.size(); ++i) {
      const rst::BatchProb& b = bsorted[i];
      rst::SolveArgs& q = qs[i];
      q.batch = nullptr;
      q.nprob = 0;
      q.g.nz = b.nz;
      q.g.pha_x = b.pha_x;
      q.g.pha_y = b.pha_y;
      q.g.phb_x = b.phb_x;
      q.g.phb_y = b.phb_y;
      q.V = A.V + b.v_off;
      q.gz = A.gz + b.gz_off;
      q.gdst = A.gdst + b.gz_off;
      q.gsrc = A.gsrc + b.gz_off;
      q.energies = A.energies + b.e_off;
      q.cols = A.cols + b.col_off;
      q.ncols = b.ncols;
      q.nblk = b.nblk;
      q.ne = b.ne;
      q.nitems = b.ncols > 0 ? b.nblk * b.ne : 0;
      q.T_col = A.T_col + b.out_off;
      q.iters = A.iters + b.out_off;
      q.restarts = A.restarts + b.out_off;
      q.resid = A.resid + b.out_off;
      q.status = A.status + b.out_off;
      if (pc) {
        q.pc.vbar = b.vbar;
        q.pc.eps = A.pc.eps + b.eps_off;
        q.pc.steps = A.pc.steps + b.steps_off;
        q.pc.inv = A.pc.inv + b.inv_off;
      }
      nit[i] = q.nitems;
    }
    if ((s = upload(c, c->d_args, qs)) != RST_OK) return s;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // the launches, back to back (captured once into a HIP graph and replayed with use_graph)
    auto launch_all = [&]() -> rst_status {
      for (size_t i = 0; i < qs.size(); ++i) {
        if (nit[i] == 0) continue;
        void* qarg = (char*)c->d_args.p + i * sizeof(rst::SolveArgs);
        void* qargs[] = {&qarg};
        hipLaunchKernelGGL(rst::k_fill_int, dim3(1), dim3(64), 0, c->stream, (int*)c->d_counter.p, 16, 0);
        HIPCHK(c, hipLaunchKernel(kern, dim3((unsigned)std::min<long long>(nwg, nit[i])), dim3(ls.threads), qargs,
                                  lds, c->stream));
      }
      return RST_OK;
    };
    const std::array<long long, 9> key = {(long long)c->batch_version, (long long)(uintptr_t)kern,
                                          (long long)ls.cw, (long long)ls.threads, -(long long)qs.size(),
                                          (long long)lds, (long long)(uintptr_t)c->d_args.p,
                                          (long long)(uintptr_t)c->d_counter.p, (long long)(uintptr_t)c->d_ws.p};
    if (use_graph && (c->gexec == nullptr || c->gexec_key != key)) {
      if (c->gexec) {
        HIPCHK(c, hipGraphExecDestroy(c->gexec));
        c->gexec = nullptr;
      }
      hipGraph_t graph;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      rst_status ls_ = launch_all();
      HIPCHK(c, hipStreamEndCapture(c->stream, &graph));
      if (ls_ != RST_OK) {
        hipGraphDestroy(graph);
        return ls_;
      }
      HIPCHK(c, hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0));
      HIPCHK(c, hipGraphDestroy(graph));
      c->gexec_key = key;
    }
    HIPCHK(c, hipEventRecord(e0, c->stream));
    if (use_graph) {
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    } else if ((s = launch_all()) != RST_OK) {
      return s;
    }
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float fq = 0;
    HIPCHK(c, hipEventElapsedTime(&fq, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    out.ms = fq;
    return batch_collect(c, sel, pcols, out_off, ne_of, outs, P, out);
  }
  if ((s = ensure(c, c->d_args, sizeof(A))) != RST_OK) return s;
  c->h_solve = A;
  HIPCHK(c, hipMemcpyAsync(c->d_args.p, &c->h_solve, sizeof(A), hipMemcpyHostToDevice, c->stream));
  void* dargs = c->d_args.p;
  void* args[] = {&dargs};
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  // graph key: batch contents, kernel, launch shape and the device buffers the graph refers to
  const std::array<long long, 9> key = {(long long)c->batch_version, (long long)(uintptr_t)kern,
                                        (long long)ls.cw, (long long)ls.threads, nwg, (long long)lds,
                                        (long long)(uintptr_t)c->d_args.p, (long long)(uintptr_t)c->d_counter.p,
                                        (long long)(uintptr_t)c->d_ws.p};
  if (use_graph && (c->gexec == nullptr || c->gexec_key != key)) {
    if (c->gexec) {
      HIPCHK(c, hipGraphExecDestroy(c->gexec));
      c->gexec = nullptr;
    }
    hipGraph_t graph;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(rst::k_fill_int, dim3(1), dim3(64), 0, c->stream, (int*)c->d_counter.p, 16, 0);
    hipLaunchKernel(kern, dim3((unsigned)nwg), dim3(ls.threads), args, lds, c->stream);
    HIPCHK(c, hipStreamEndCapture(c->stream, &graph));
    HIPCHK(c, hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0));
    HIPCHK(c, hipGraphDestroy(graph));
    c->gexec_key = key;
  }
  HIPCHK(c, hipEventRecord(e0, c->stream));
  if (use_graph) {
    HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  } else {
    hipLaunchKernelGGL(rst::k_fill_int, dim3(1), dim3(64), 0, c->stream, (int*)c->d_counter.p, 16, 0);
    HIPCHK(c, hipLaunchKernel(kern, dim3((unsigned)nwg), dim3(ls.threads), args, lds, c->stream));
  }
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float fms = 0;
  HIPCHK(c, hipEventElapsedTime(&fms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  out.ms = fms;
  return batch_collect(c, sel, pcols, out_off, ne_of, outs, P, out);
}

// Per-column results of a batched solve and the per-structure, per-energy T.
rst_status batch_collect(rst_ctx* c, const std::vector<int>& sel, const std::vector<std::vector<int64_t>>& pcols,
                         const std::vector<long long>& out_off, const std::vector<int>& ne_of, long long outs,
                         int P, BatchOut& out) {
  std::vector<double> Tcol(outs);
  out.its.resize(outs);
  out.rss.resize(outs);
  out.res.resize(outs);
  out.stv.resize(outs);
  HIPCHK(c, hipMemcpy(Tcol.data(), c->d_T.p, outs * 8, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(out.its.data(), c->d_it.p, outs * 4, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(out.rss.data(), c->d_rs.p, outs * 4, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(out.res.data(), c->d_res.p, outs * 8, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(out.stv.data(), c->d_st.p, outs * 4, hipMemcpyDeviceToHost));
  out.points_n = 0;
  for (size_t i = 0; i < sel.size(); ++i) {
    const int ncols = (int)pcols[i].size();
    const double n_i = (double)P * c->batch[sel[i]].nz;
    for (int e = 0; e < ne_of[i]; ++e) {
      double t = 0;
      for (int j = 0; j < ncols; ++j) {
        const size_t o = out_off[i] + (size_t)e * ncols + j;
        t += Tcol[o];
        out.points_n += n_i * out.its[o];
      }
      out.T[i][e] = t;
    }
  }
  return RST_OK;
}

}  // namespace

extern "C" {

rst_status rst_batch_clear(rst_ctx* c) {
  if (!c) return RST_EINVAL;
  c->batch.clear();
  c->batch_version++;
  return RST_OK;
}

rst_status rst_batch_add(rst_ctx* c, const rst_problem* p) {
  if (!c || !p) return RST_EINVAL;
  if (!c->has_grid) return fail(c, RST_ESTATE, "rst_set_grid not called");
  if (c->nproj > 0) return fail(c, RST_EUNSUPPORTED, "batched structures carry local potentials only");
  if (p->nz < 1 || !p->v || !p->gamma_l || !p->gamma_r || p->n_e < 0 || (p->n_e > 0 && !p->energies))
    return fail(c, RST_EINVAL, "bad rst_problem");
  if (!std::isfinite(p->ka) || !std::isfinite(p->kb)) return fail(c, RST_EINVAL, "non-finite k");
  const size_t n = (size_t)c->na * c->nb * p->nz;
  rst_ctx::HostProb hp;
  hp.grid_version = c->grid_version;
  hp.nz = p->nz;
  hp.v.assign(p->v, p->v + n);
  hp.gl.assign(p->gamma_l, p->gamma_l + p->nz);
  hp.gr.assign(p->gamma_r, p->gamma_r + p->nz);
  hp.en.assign(p->energies, p->energies + p->n_e);
  hp.ka = p->ka;
  hp.kb = p->kb;
  for (double x : hp.v)
    if (!std::isfinite(x)) return fail(c, RST_EINVAL, "non-finite potential value");
  for (int z = 0; z < p->nz; ++z)
    if (!(hp.gl[z] >= 0) || !(hp.gr[z] >= 0) || !std::isfinite(hp.gl[z]) || !std::isfinite(hp.gr[z]))
      return fail(c, RST_EINVAL, "CAP values must be finite and >= 0");
  for (double e : hp.en)
    if (!std::isfinite(e)) return fail(c, RST_EINVAL, "non-finite energy");
  c->batch.push_back(std::move(hp));
  c->batch_version++;
  return RST_OK;
}

rst_status rst_batch_run(rst_ctx* c, double* T_out, rst_stats* stats) {
  if (!c) return RST_EINVAL;
  if (!c->has_grid) return fail(c, RST_ESTATE, "rst_set_grid not called");
  if (c->rad != 2 && c->rad != 6) return fail(c, RST_EUNSUPPORTED, "GPU kernels are built for FD orders 4 and 12");
  if (c->opts.precision != RST_FP64 || c->opts.method != RST_BICGSTAB)
    return fail(c, RST_EUNSUPPORTED, "the batched launch runs FP64 BiCGSTAB");
  if (c->batch.empty()) return RST_OK;
  if (!T_out) return fail(c, RST_EINVAL, "null T_out");
  for (const auto& hp : c->batch)
    if (hp.grid_version != c->grid_version)
      return fail(c, RST_ESTATE, "rst_set_grid was called after rst_batch_add (rst_batch_clear, then add again)");
  hipSetDevice(c->device);
  std::vector<int> all(c->batch.size());
  for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
  int cw = c->opts.col_block;
  rst_status s;
  // When every structure alone has enough column items to fill the device many times over (four
  // times the most workgroups it can hold: 16 per CU), the single-structure kernel runs once per
  // structure, back to back: measured faster than the one batched launch in that regime.
  int ncu = 0;
  HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  const int P = c->na * c->nb;
  long long min_items = -1;
  for (const auto& hp : c->batch) {
    const std::vector<double>& gs = c->opts.direction == RST_DIR_LR ? hp.gr : hp.gl;
    long long ncols = 0;
    for (int z = 0; z < hp.nz; ++z)
      if (gs[z] > 0) ncols += P;
    const long long it = ncols * (long long)hp.en.size();
    if (it > 0) min_items = min_items < 0 ? it : std::min(min_items, it);
  }
  const bool per_structure = min_items >= 4LL * 16 * ncu;
  if (per_structure && cw == 0) cw = 1;  // measured best for launches that each fill the device
  int threads = c->opts.threads;
  if (cw == 0 || threads == 0) {
    // autotune the launch shape: columns per workgroup (1, 2, 4, 8, or the caller's) times the
    // positions per thread (one or two, i.e. the workgroup size), each candidate timed on every
    // structure at its first energy in the launch mode the full batch uses: a sample large
    // enough to fill the device like the full launch does (timed on one structure alone, the
    // half-empty device favoured wide column blocks that lose on the full batch)
    const long long key = ((long long)c->na << 40) ^ ((long long)c->nb << 24) ^ ((long long)c->rad << 8) ^
                          ((long long)c->opts.precond << 4) ^ ((long long)c->opts.direction << 2) ^
                          ((long long)per_structure << 1) ^ ((long long)cw << 48) ^ ((long long)threads << 52);
    auto it = c->tuned_shape.find(key);
    if (it != c->tuned_shape.end()) {
      cw = it->second.first;
      threads = it->second.second;
    } else {
      std::vector<int> cws = cw > 0 ? std::vector<int>{cw} : std::vector<int>{1, 2, 4, 8};
      int best_cw = cws[0], best_t = threads;
      double best_ms = 1e300;
      for (int cand : cws) {
        std::vector<int> tcands;
        if (threads > 0) {
          tcands.push_back(threads);
        } else {
          const int pos = P * cand;
          for (int q : {1, 2}) {
            const int t = std::max(64, ((pos + q - 1) / q + 63) / 64 * 64);
            if (t <= rst::MAX_T && t % cand == 0 && (long long)t * 2 >= pos &&
                std::find(tcands.begin(), tcands.end(), t) == tcands.end())
              tcands.push_back(t);
          }
        }
        for (int t : tcands) {
          LaunchShape ls;
          if (choose_shape(c, cand, t, ls) != RST_OK) continue;
          BatchOut o;
          if ((s = run_batch(c, all, 1, cand, false, o, per_structure, t)) != RST_OK) return s;
          const double per = o.ms / std::max<size_t>(1, o.its.size());
          if (per < best_ms) {
            best_ms = per;
            best_cw = cand;
            best_t = t;
          }
        }
      }
      c->tuned_shape[key] = {best_cw, best_t};
      cw = best_cw;
      threads = best_t;
    }
  }
  BatchOut o;
  if ((s = run_batch(c, all, 0, cw, true, o, per_structure, threads)) != RST_OK) return s;
  size_t k = 0;
  for (size_t i = 0; i < all.size(); ++i)
    for (double t : o.T[i]) T_out[k++] = t;
  int nbad = 0;
  fill_stats(c, stats, o.its, o.rss, o.res, o.stv, o.ms, nbad, o.cw, o.threads, 0.0);
  if (stats)
    stats->bytes_algorithmic = o.points_n * (c->opts.precond == RST_PRECOND_FREE_CAP ? 24.0 : 12.0) * 16.0;
  return nbad ? RST_ENOCONV : RST_OK;
}

void rst_default_solver(rst_solver_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = RST_BICGSTAB;
  o->precision = RST_FP64;
  o->tol = 1e-10;
  o->max_iter = 20000;
  o->col_block = 0;
  o->threads = 0;
  o->direction = RST_DIR_LR;
  o->update_delta = 0.1;
  o->restart = 30;
  o->fallback_ratio = 0.5;
  o->precond = RST_PRECOND_NONE;
  o->pc_vref = RST_VREF_PLANE;
  o->idr_s = 4;
}

rst_status rst_create(rst_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return RST_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return RST_EDEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return RST_EDEVICE;
  if (hip_device < RST_MAX_DEVICES) {
    // this device's copy of the no-allocation scratch array (looked up once, with the device current)
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[hip_device]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RST_EDEVICE;
      scratch_dev[hip_device] = (double2*)ptr;
    }
  }
  rst_ctx* c = new rst_ctx();
  c->device = hip_device;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return RST_EDEVICE;
    }
    c->own_stream = true;
  }
  rst_default_solver(&c->opts);
  *out = c;
  return RST_OK;
}

void rst_destroy(rst_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  for (hipEvent_t& e : c->ev_apply)
    if (e) hipEventDestroy(e);
  rst::cnn::engine_destroy(c->cnn);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  delete c;
}

const char* rst_last_error(const rst_ctx* c) { return c ? c->err.c_str() : "null context"; }

rst_status rst_set_grid(rst_ctx* c, int na, int nb, int nz, double ha, double hb, double hz, int order) {
  if (!c) return RST_EINVAL;
  if (na < 1 || nb < 1 || nz < 1 || !(ha > 0) || !(hb > 0) || !(hz > 0))
    return fail(c, RST_EINVAL, "grid dimensions and spacings must be positive");
  if (order < 2 || order > 12 || order % 2) return fail(c, RST_EINVAL, "fd_order must be even in 2..12");
  const int rad = order / 2;
  if (na <= rad || nb <= rad)
    return fail(c, RST_EUNSUPPORTED, "lateral grid must exceed the stencil radius (na, nb > fd_order/2)");
  if ((long long)na * nb * nz > 0x7fffffffLL) return fail(c, RST_EINVAL, "grid too large");
  hipSetDevice(c->device);
  c->na = na;
  c->nb = nb;
  c->nz = nz;
  c->ha = ha;
  c->hb = hb;
  c->hz = hz;
  c->order = order;
  c->rad = rad;
  c->fdw = fornberg_second_derivative(rad);
  c->has_grid = true;
  c->has_v = c->has_abc = c->has_k = false;
  // structures added before this call carry potentials of the previous grid: rst_batch_run refuses
  // them (RST_ESTATE) until the batch is rebuilt, and the launch captured for them is dropped
  c->grid_version++;
  c->batch_version++;
  if (c->gexec) {
    hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  c->nproj = c->ngroup = 0;
  c->nm = 1;
  c->max_chunks = 0;
  c->has_overflow = 0;
  c->ent_p.clear();
  c->ent_img.clear();
  c->sc_ent.clear();
  c->g_ent_p.clear();
  c->g_src.clear();
  c->g_beta.clear();
  // empty projector plan
  const long long n = (long long)na * nb * nz;
  c->zc_offs.assign(nz + 1, 0);
  c->zg_offs.assign(nz + 1, 0);
  c->pe_offs.assign(n + 1, 0);
  rst_status s;
  if ((s = upload(c, c->d_zc, c->zc_offs)) != RST_OK) return s;
  if ((s = upload(c, c->d_zg, c->zg_offs)) != RST_OK) return s;
  if ((s = upload(c, c->d_pe_offs, c->pe_offs)) != RST_OK) return s;
  return RST_OK;
}

rst_status rst_set_potential(rst_ctx* c, const double* v) {
  if (!c) return RST_EINVAL;
  if (!c->has_grid) return fail(c, RST_ESTATE, "rst_set_grid not called");
  if (!v) return fail(c, RST_EINVAL, "null potential");
  const size_t n = (size_t)c->na * c->nb * c->nz;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return fail(c, RST_EINVAL, "non-finite potential value");
  hipSetDevice(c->device);
  c->v.assign(v, v + n);
  rst_status s = upload(c, c->d_v, c->v);
  if (s != RST_OK) return s;
  // plane means: the preconditioner's default reference potential
  const size_t P = (size_t)c->na * c->nb;
  std::vector<double> vz(c->nz, 0.0);
  for (int z = 0; z < c->nz; ++z) {
    double acc = 0.0;
    for (size_t p = 0; p < P; ++p) acc += c->v[(size_t)z * P + p];
    vz[z] = acc / (double)P;
  }
  if ((s = upload(c, c->d_vz, vz)) != RST_OK) return s;
  c->has_v = true;
  return RST_OK;
}

rst_status rst_set_projectors(rst_ctx* c, int nproj, const int32_t* offs, const int32_t* pt, const int8_t* img,
                              const double* beta, const double* e_kb) {
  if (!c) return RST_EINVAL;
  if (!c->has_grid) return fail(c, RST_ESTATE, "rst_set_grid not called");
  if (nproj < 0) return fail(c, RST_EINVAL, "nproj < 0");
  hipSetDevice(c->device);
  if (nproj == 0) {
    c->nproj = c->ngroup = 0;
    c->nm = 1;
    c->max_chunks = 0;
    c->has_overflow = 0;
    c->ent_p.clear();
    c->ent_img.clear();
    c->sc_ent.clear();
    c->g_ent_p.clear();
    c->g_src.clear();
    c->g_beta.clear();
    return RST_OK;
  }
  if (!offs || !pt || !img || !beta || !e_kb) return fail(c, RST_EINVAL, "null projector array");
  if (offs[0] != 0) return fail(c, RST_EINVAL, "offs[0] must be 0");
  for (int p = 0; p < nproj; ++p) {
    if (offs[p + 1] < offs[p]) return fail(c, RST_EINVAL, "offs must be non-decreasing");
    if (!std::isfinite(e_kb[p])) return fail(c, RST_EINVAL, "non-finite projector energy");
  }
  for (int e = 0; e < offs[nproj]; ++e)
    if (!std::isfinite(beta[e])) return fail(c, RST_EINVAL, "non-finite projector value");
  rst_status s = build_plan(c, nproj, offs, pt, img, beta, e_kb);
  if (s != RST_OK) return s;
  if (c->has_k) return upload_k(c);
  return RST_OK;
}

rst_status rst_set_abc(rst_ctx* c, const double* gl, const double* gr) {
  if (!c) return RST_EINVAL;
  if (!c->has_grid) return fail(c, RST_ESTATE, "rst_set_grid not called");
  if (!gl || !gr) return fail(c, RST_EINVAL, "null CAP profile");
  for (int z = 0; z < c->nz; ++z)
    if (!(gl[z] >= 0) || !(gr[z] >= 0) || !std::isfinite(gl[z]) || !std::isfinite(gr[z]))
      return fail(c, RST_EINVAL, "CAP values must be finite and >= 0");
  hipSetDevice(c->device);
  c->gl.assign(gl, gl + c->nz);
  c->gr.assign(gr, gr + c->nz);
  std::vector<double> gz(c->nz);
  for (int z = 0; z < c->nz; ++z) gz[z] = gl[z] + gr[z];
  rst_status s;
  if ((s = upload(c, c->d_gz, gz)) != RST_OK) return s;
  if ((s = upload(c, c->d_gl, c->gl)) != RST_OK) return s;
  if ((s = upload(c, c->d_gr, c->gr)) != RST_OK) return s;
  c->has_abc = true;
  return RST_OK;
}

rst_status rst_set_k(rst_ctx* c, double ka, double kb) {
  if (!c) return RST_EINVAL;
  if (!c->has_grid) return fail(c, RST_ESTATE, "rst_set_grid not called");
  if (!std::isfinite(ka) || !std::isfinite(kb)) return fail(c, RST_EINVAL, "non-finite k");
  hipSetDevice(c->device);
  c->ka = ka;
  c->kb = kb;
  rst_status s = upload_k(c);
  if (s != RST_OK) return s;
  if ((s = upload_pc(c)) != RST_OK) return s;
  c->has_k = true;
  return RST_OK;
}

rst_status rst_set_solver(rst_ctx* c, const rst_solver_opts* o) {
  if (!c || !o) return RST_EINVAL;
  if (o->method != RST_BICGSTAB && o->method != RST_FGMRES && o->method != RST_COCG && o->method != RST_BICGSTAB_MC &&
      o->method != RST_IDRS)
    return fail(c, RST_EINVAL, "unknown method");
  if (o->method == RST_BICGSTAB_MC && o->precision != RST_FP64)
    return fail(c, RST_EUNSUPPORTED, "the many-column BiCGSTAB runs in FP64 only (mixed precision: RST_IDRS)");
  if (o->idr_s < 1 || o->idr_s > rst::idr::SMAX) return fail(c, RST_EINVAL, "idr_s must be in 1..8");
  if (!(o->pc_shift >= 0) || !std::isfinite(o->pc_shift)) return fail(c, RST_EINVAL, "pc_shift must be finite and >= 0");
  if (o->method == RST_COCG && o->precision != RST_FP64) return fail(c, RST_EUNSUPPORTED, "COCG runs in FP64 only");
  if (o->method == RST_FGMRES) {
    if (o->restart < 1 || o->restart > 200) return fail(c, RST_EINVAL, "restart must be in 1..200");
    if (o->precision != RST_FP64) return fail(c, RST_EUNSUPPORTED, "FGMRES runs in FP64 only");
  }
  if (o->precond == RST_PRECOND_LEARNED) {
    if (o->method != RST_FGMRES)
      return fail(c, RST_EINVAL, "the learned preconditioner needs method RST_FGMRES");
    if (!(o->fallback_ratio > 0) || o->fallback_ratio > 1) return fail(c, RST_EINVAL, "fallback_ratio must be in (0, 1]");
  }
  if (o->precision != RST_FP64 && o->precision != RST_FP32_REFINE) return fail(c, RST_EINVAL, "unknown precision");
  if (o->precision == RST_FP32_REFINE && (!(o->update_delta > 0) || o->update_delta >= 1))
    return fail(c, RST_EINVAL, "update_delta must be in (0, 1)");
  if (!(o->tol > 0) || o->max_iter < 1) return fail(c, RST_EINVAL, "tol must be > 0 and max_iter >= 1");
  if (o->col_block < 0 || o->col_block > rst::CW_MAX || (o->col_block & (o->col_block - 1)))
    return fail(c, RST_EINVAL, "col_block must be 0 or a power of two <= 8");
  if (o->threads < 0 || o->threads > rst::MAX_T || o->threads % 64)
    return fail(c, RST_EINVAL, "threads must be 0 or a multiple of 64 <= 512");
  if (o->direction != RST_DIR_LR && o->direction != RST_DIR_RL) return fail(c, RST_EINVAL, "bad direction");
  if (o->precond != RST_PRECOND_NONE && o->precond != RST_PRECOND_FREE_CAP && o->precond != RST_PRECOND_LEARNED)
    return fail(c, RST_EINVAL, "unknown preconditioner");
  if (o->pc_vref != RST_VREF_PLANE && o->pc_vref != RST_VREF_CELL)
    return fail(c, RST_EINVAL, "unknown preconditioner reference potential");
  c->opts = *o;
  return RST_OK;
}

rst_status rst_transmission(rst_ctx* c, int n_e, const double* E, double* T_out, rst_stats* stats) {
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  if (n_e < 0 || (n_e > 0 && (!E || !T_out))) return fail(c, RST_EINVAL, "bad energy arguments");
  for (int i = 0; i < n_e; ++i)
    if (!std::isfinite(E[i])) return fail(c, RST_EINVAL, "non-finite energy");
  hipSetDevice(c->device);
  const bool lr = c->opts.direction == RST_DIR_LR;
  const std::vector<double>& gsrc = lr ? c->gr : c->gl;
  const int P = c->na * c->nb;
  std::vector<int64_t> cols;
  for (int z = 0; z < c->nz; ++z)
    if (gsrc[z] > 0)
      for (int p = 0; p < P; ++p) cols.push_back((int64_t)z * P + p);
  if (n_e == 0) return RST_OK;
  if (cols.empty()) {
    for (int i = 0; i < n_e; ++i) T_out[i] = 0.0;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    return RST_OK;
  }
  std::vector<double> Tcol, res;
  std::vector<int> its, rss, stv;
  double ms = 0;
  s = run_solver(c, n_e, E, cols, lr ? (const double*)c->d_gr.p : (const double*)c->d_gl.p,
                 lr ? (const double*)c->d_gl.p : (const double*)c->d_gr.p, nullptr, Tcol, its, rss, res, stv,
                 ms);
  if (s != RST_OK) return s;
  s = mixed_fp64_fallback(c, n_e, E, cols, lr ? (const double*)c->d_gr.p : (const double*)c->d_gl.p,
                          lr ? (const double*)c->d_gl.p : (const double*)c->d_gr.p, nullptr, Tcol, its, rss, res,
                          stv, ms);
  if (s != RST_OK) return s;
  const size_t nc = cols.size();
  for (int i = 0; i < n_e; ++i) {
    double t = 0;
    for (size_t j = 0; j < nc; ++j) t += Tcol[(size_t)i * nc + j];
    T_out[i] = t;
  }
  int nbad = 0;
  fill_stats(c, stats, its, rss, res, stv, ms, nbad, c->last_cw, c->last_threads);
  return nbad ? RST_ENOCONV : RST_OK;
}

rst_status rst_solve_columns(rst_ctx* c, double energy, int ncol, const int64_t* col, void* x_dev,
                             rst_stats* stats) {
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  const long long n = (long long)c->na * c->nb * c->nz;
  if (ncol < 0 || (ncol > 0 && (!col || !x_dev))) return fail(c, RST_EINVAL, "bad column arguments");
  if (!std::isfinite(energy)) return fail(c, RST_EINVAL, "non-finite energy");
  for (int j = 0; j < ncol; ++j)
    if (col[j] < 0 || col[j] >= n) return fail(c, RST_EINVAL, "column index out of range");
  if (ncol == 0) return RST_OK;
  hipSetDevice(c->device);
  std::vector<int64_t> cols(col, col + ncol);
  std::vector<double> Tcol, res;
  std::vector<int> its, rss, stv;
  double ms = 0;
  s = run_solver(c, 1, &energy, cols, nullptr, nullptr, (double2*)x_dev, Tcol, its, rss, res, stv, ms);
  if (s != RST_OK) return s;
  s = mixed_fp64_fallback(c, 1, &energy, cols, nullptr, nullptr, (double2*)x_dev, Tcol, its, rss, res, stv, ms);
  if (s != RST_OK) return s;
  int nbad = 0;
  fill_stats(c, stats, its, rss, res, stv, ms, nbad, c->last_cw, c->last_threads);
  return nbad ? RST_ENOCONV : RST_OK;
}

rst_status rst_solve_rhs(rst_ctx* c, int n_e, const double* energies, int ncol, const void* rhs_dev,
                         int64_t rhs_estride, void* x_dev, rst_stats* stats) {
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  if (n_e < 0 || ncol < 0 || ((n_e > 0 && ncol > 0) && (!energies || !rhs_dev || !x_dev)))
    return fail(c, RST_EINVAL, "bad right-hand-side arguments");
  if (rhs_estride != 0 && rhs_estride != ncol) return fail(c, RST_EINVAL, "rhs_estride must be 0 or ncol");
  for (int i = 0; i < n_e; ++i)
    if (!std::isfinite(energies[i])) return fail(c, RST_EINVAL, "non-finite energy");
  if ((c->opts.method != RST_BICGSTAB && c->opts.method != RST_BICGSTAB_MC && c->opts.method != RST_IDRS) ||
      c->opts.precision != RST_FP64)
    return fail(c, RST_EUNSUPPORTED, "dense right-hand sides are solved by FP64 BiCGSTAB or IDR(s)");
  if (n_e == 0 || ncol == 0) return RST_OK;
  hipSetDevice(c->device);
  std::vector<int64_t> cols(ncol, 0);
  std::vector<double> Tcol, res;
  std::vector<int> its, rss, stv;
  double ms = 0;
  const long long ld = rhs_estride ? (long long)n_e * ncol : ncol;
  s = run_solver(c, n_e, energies, cols, nullptr, nullptr, (double2*)x_dev, Tcol, its, rss, res, stv, ms,
                 (const double2*)rhs_dev, ld, rhs_estride);
  if (s != RST_OK) return s;
  int nbad = 0;
  fill_stats(c, stats, its, rss, res, stv, ms, nbad, c->last_cw, c->last_threads);
  return nbad ? RST_ENOCONV : RST_OK;
}

rst_status rst_transmission_kavg(rst_ctx* c, int n_k, const double* kpts, int fold, int n_e, const double* E,
                                 double* T_out, double* T_k, int* n_solved, rst_stats* stats) {
  if (!c) return RST_EINVAL;
  if (!c->has_grid) return fail(c, RST_ESTATE, "rst_set_grid not called");
  if (!c->has_v) return fail(c, RST_ESTATE, "rst_set_potential not called");
  if (!c->has_abc) return fail(c, RST_ESTATE, "rst_set_abc not called");
  if (n_k < 1 || !kpts) return fail(c, RST_EINVAL, "at least one k-point is needed");
  if (n_e < 0 || (n_e > 0 && (!E || !T_out))) return fail(c, RST_EINVAL, "bad energy arguments");
  for (int i = 0; i < 2 * n_k; ++i)
    if (!std::isfinite(kpts[i])) return fail(c, RST_EINVAL, "non-finite k");
  for (int i = 0; i < n_e; ++i)
    if (!std::isfinite(E[i])) return fail(c, RST_EINVAL, "non-finite energy");
  // representative of each k: itself, or an earlier k equal to it or to its
  // negative modulo a reciprocal lattice vector (T(k + G) = T(k) = T(-k))
  const double two_pi = 6.283185307179586;
  const double ga = two_pi / (c->na * c->ha), gb = two_pi / (c->nb * c->hb);
  auto integral = [](double x) { return std::fabs(x - std::nearbyint(x)) <= 1e-9; };
  std::vector<int> rep(n_k);
  for (int i = 0; i < n_k; ++i) {
    rep[i] = i;
    if (!fold) continue;
    for (int j = 0; j < i; ++j) {
      if (rep[j] != j) continue;
      const double ka = kpts[2 * i], kb = kpts[2 * i + 1], ja = kpts[2 * j], jb = kpts[2 * j + 1];
      const bool same = integral((ka - ja) / ga) && integral((kb - jb) / gb);
      const bool neg = integral((ka + ja) / ga) && integral((kb + jb) / gb);
      if (same || neg) {
        rep[i] = j;
        break;
      }
    }
  }
  const bool had_k = c->has_k;
  const double ka0 = c->ka, kb0 = c->kb;
  std::vector<double> tk((size_t)n_k * n_e, 0.0);
  rst_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  rst_status worst = RST_OK;
  int solved = 0;
  rst_status s = RST_OK;
  for (int i = 0; i < n_k && s >= 0; ++i) {
    if (rep[i] != i) continue;
    if ((s = rst_set_k(c, kpts[2 * i], kpts[2 * i + 1])) != RST_OK) break;
    rst_stats st;
    std::memset(&st, 0, sizeof(st));
    s = rst_transmission(c, n_e, E, tk.data() + (size_t)i * n_e, &st);
    if (s < 0) break;
    if (s == RST_ENOCONV) worst = RST_ENOCONV;
    ++solved;
    acc.columns += st.columns;
    acc.columns_unconverged += st.columns_unconverged;
    acc.iterations_total += st.iterations_total;
    acc.iterations_max = std::max(acc.iterations_max, st.iterations_max);
    acc.restarts_total += st.restarts_total;
    acc.max_rel_residual = std::max(acc.max_rel_residual, st.max_rel_residual);
    acc.kernel_ms += st.kernel_ms;
    acc.bytes_algorithmic += st.bytes_algorithmic;
    acc.updates_total += st.updates_total;
    acc.fallback_columns += st.fallback_columns;
    acc.cnn_flop += st.cnn_flop;
    acc.col_block = st.col_block;
    acc.threads = st.threads;
  }
  // put the caller's k back (or leave none set if there was none)
  if (had_k) {
    const std::string err = c->err;
    const rst_status r = rst_set_k(c, ka0, kb0);
    if (s >= 0 && r != RST_OK) s = r;
    if (s < 0 && r == RST_OK) c->err = err;
  } else {
    c->has_k = false;
  }
  if (s < 0) return s;
  for (int i = 0; i < n_k; ++i)
    if (rep[i] != i)
      std::copy(tk.begin() + (size_t)rep[i] * n_e, tk.begin() + (size_t)(rep[i] + 1) * n_e,
                tk.begin() + (size_t)i * n_e);
  for (int e = 0; e < n_e; ++e) {
    double t = 0.0;
    for (int i = 0; i < n_k; ++i) t += tk[(size_t)i * n_e + e];
    T_out[e] = t / n_k;
  }
  if (T_k) std::copy(tk.begin(), tk.end(), T_k);
  if (n_solved) *n_solved = solved;
  if (stats) *stats = acc;
  return worst;
}

rst_status rst_apply_h(rst_ctx* c, double energy, const void* x_dev, void* y_dev, int ncol, int precision) {
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  if (ncol < 0 || (ncol > 0 && (!x_dev || !y_dev))) return fail(c, RST_EINVAL, "bad apply arguments");
  if (precision != RST_FP64 && precision != RST_FP32_REFINE)
    return fail(c, RST_EINVAL, "precision must be RST_FP64 or RST_FP32_REFINE");
  const bool f32 = precision == RST_FP32_REFINE;
  if (x_dev == y_dev) return fail(c, RST_EINVAL, "x and y must be distinct buffers");
  if (!std::isfinite(energy)) return fail(c, RST_EINVAL, "non-finite energy");
  if (ncol == 0) return RST_OK;
  hipSetDevice(c->device);
  for (hipEvent_t& e : c->ev_apply)
    if (!e) HIPCHK(c, hipEventCreate(&e));
  if (c->nproj > 0 && (s = ensure(c, c->d_projP, (size_t)c->nproj * ncol * 16)) != RST_OK) return s;
  if ((s = apply_cols(c, x_dev, y_dev, ncol, energy, nullptr, nullptr, f32, (double2*)c->d_projP.p,
                      c->ev_apply)) != RST_OK)
    return s;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float f0 = 0.f, f1 = 0.f;
  HIPCHK(c, hipEventElapsedTime(&f0, c->ev_apply[0], c->ev_apply[1]));
  HIPCHK(c, hipEventElapsedTime(&f1, c->ev_apply[1], c->ev_apply[2]));
  c->apply_ms[0] = f0;
  c->apply_ms[1] = f1;
  return RST_OK;
}

rst_status rst_apply_h_noalloc(rst_ctx* c, double energy, const void* x_dev, void* y_dev, int ncol, int precision) {
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  if (ncol < 0 || (ncol > 0 && (!x_dev || !y_dev))) return fail(c, RST_EINVAL, "bad apply arguments");
  if (precision != RST_FP64 && precision != RST_FP32_REFINE)
    return fail(c, RST_EINVAL, "precision must be RST_FP64 or RST_FP32_REFINE");
  if (x_dev == y_dev) return fail(c, RST_EINVAL, "x and y must be distinct buffers");
  if (!std::isfinite(energy)) return fail(c, RST_EINVAL, "non-finite energy");
  if (ncol == 0) return RST_OK;
  if ((size_t)c->nproj * (size_t)ncol * sizeof(double2) > RST_SCRATCH_BYTES)
    return fail(c, RST_EINVAL, "nproj x ncol projections exceed the " + std::to_string(RST_SCRATCH_BYTES >> 20) +
                                   " MiB scratch of the no-allocation apply (at most " +
                                   std::to_string(RST_SCRATCH_BYTES / sizeof(double2) / std::max(1, c->nproj)) +
                                   " columns with these projectors)");
  double2* sp = c->device < RST_MAX_DEVICES ? scratch_dev[c->device] : nullptr;
  if (!sp) return fail(c, RST_EDEVICE, "no scratch address for this device");
  hipSetDevice(c->device);
  // the projections k_proj_mm writes cover every (projector, column) entry: nothing to clear
  if ((s = apply_cols(c, x_dev, y_dev, ncol, energy, nullptr, nullptr, precision == RST_FP32_REFINE, sp, nullptr)) !=
      RST_OK)
    return s;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RST_OK;
}

rst_status rst_apply_block_width(rst_ctx* c, int* col_block) {
  if (!col_block) return RST_EINVAL;
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  hipSetDevice(c->device);
  BlockedShape bs;
  if ((s = blocked_shape(c, rst::CW_MAX, c->opts.threads, bs)) != RST_OK) return s;
  *col_block = bs.ls.cw;
  return RST_OK;
}

rst_status rst_apply_h_blocked(rst_ctx* c, double energy, const void* x_dev, void* y_dev, int ncol,
                               int col_block) {
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  if (ncol < 0 || (ncol > 0 && (!x_dev || !y_dev))) return fail(c, RST_EINVAL, "bad apply arguments");
  if (col_block < 1 || col_block > rst::CW_MAX || (col_block & (col_block - 1)))
    return fail(c, RST_EINVAL, "col_block must be a power of two <= 8");
  if (ncol % col_block) return fail(c, RST_EINVAL, "ncol must be a multiple of col_block");
  if (x_dev == y_dev) return fail(c, RST_EINVAL, "x and y must be distinct buffers");
  if (!std::isfinite(energy)) return fail(c, RST_EINVAL, "non-finite energy");
  if (ncol == 0) return RST_OK;
  hipSetDevice(c->device);
  BlockedShape bs;
  if ((s = blocked_shape(c, col_block, c->opts.threads, bs)) != RST_OK) return s;
  if (bs.ls.cw != col_block)
    return fail(c, RST_EUNSUPPORTED, "column block of " + std::to_string(col_block) +
                                         " does not fit one workgroup on this grid (widest: " +
                                         std::to_string(bs.ls.cw) + ")");
  void* kern = pick_kernel(c->rad, bs.ls.q, 1);
  if (!kern) return fail(c, RST_EUNSUPPORTED, "no kernel instance");
  rst::ApplyArgs A;
  std::memset(&A, 0, sizeof(A));
  A.g = make_geo(c);
  A.pj = make_proj(c);
  A.V = (const double*)c->d_v.p;
  A.gz = (const double*)c->d_gz.p;
  A.energy = energy;
  A.x = (const double2*)x_dev;
  A.y = (double2*)y_dev;
  A.ncol = ncol;
  A.cw = col_block;
  A.nblk = ncol / col_block;
  const size_t pws_stride = std::max<size_t>(1, (size_t)c->nproj * col_block);
  if ((s = ensure(c, c->d_pws, (size_t)A.nblk * pws_stride * 16)) != RST_OK) return s;
  A.pws = (double2*)c->d_pws.p;
  A.pws_stride = pws_stride;
  A.proj_pre = c->nproj > 0;
  if (bs.lds_apply > 64 * 1024)
    HIPCHK(c, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bs.lds_apply));
  if ((s = ensure(c, c->d_args, sizeof(A))) != RST_OK) return s;
  c->h_apply = A;
  HIPCHK(c, hipMemcpyAsync(c->d_args.p, &c->h_apply, sizeof(A), hipMemcpyHostToDevice, c->stream));
  for (hipEvent_t& e : c->ev_apply)
    if (!e) HIPCHK(c, hipEventCreate(&e));
  void* dargs = c->d_args.p;
  void* args[] = {&dargs};
  HIPCHK(c, hipEventRecord(c->ev_apply[0], c->stream));
  if ((s = proj_blocked(c, A)) != RST_OK) return s;
  HIPCHK(c, hipEventRecord(c->ev_apply[1], c->stream));
  HIPCHK(c, hipLaunchKernel(kern, dim3(A.nblk), dim3(bs.ls.threads), args, bs.lds_apply, c->stream));
  HIPCHK(c, hipEventRecord(c->ev_apply[2], c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float f0 = 0.f, f1 = 0.f;
  HIPCHK(c, hipEventElapsedTime(&f0, c->ev_apply[0], c->ev_apply[1]));
  HIPCHK(c, hipEventElapsedTime(&f1, c->ev_apply[1], c->ev_apply[2]));
  c->apply_ms[0] = f0;
  c->apply_ms[1] = f1;
  return RST_OK;
}

rst_status rst_apply_timing(const rst_ctx* c, double* proj_ms, double* stencil_ms) {
  if (!c || !proj_ms || !stencil_ms) return RST_EINVAL;
  *proj_ms = c->apply_ms[0];
  *stencil_ms = c->apply_ms[1];
  return RST_OK;
}

}  // extern "C"

// learned correction network ---------------------------------------------------

// ---- eigen route -------------------------------------------------------------------------------

// Cholesky of the m x m Hermitian Gram matrix g (column-major) and W = R^-1 with g = R^H R; a pivot
// below 1e-24 of the largest diagonal drops its column (zero row of W).  Host, O(m^3).
static void chol_inv(int m, const std::vector<double2>& g, std::vector<double2>& w) {
  using cd = std::complex<double>;
  std::vector<cd> R((size_t)m * m, cd(0.0)), W((size_t)m * m, cd(0.0));
  auto G = [&](int i, int j) { return cd(g[i + (size_t)j * m].x, g[i + (size_t)j * m].y); };
  double dmax = 0.0;
  for (int i = 0; i < m; ++i) dmax = std::max(dmax, G(i, i).real());
  for (int j = 0; j < m; ++j) {
    double d = G(j, j).real();
    for (int k = 0; k < j; ++k) d -= std::norm(R[k + (size_t)j * m]);
    if (!(d > 1e-24 * dmax)) continue;
    const double rjj = std::sqrt(d);
    R[j + (size_t)j * m] = rjj;
    for (int c2 = j + 1; c2 < m; ++c2) {
      cd t = G(j, c2);
      for (int k = 0; k < j; ++k) t -= std::conj(R[k + (size_t)j * m]) * R[k + (size_t)c2 * m];
      R[j + (size_t)c2 * m] = t / rjj;
    }
  }
  for (int b = 0; b < m; ++b)
    for (int a = b; a >= 0; --a) {
      const cd raa = R[a + (size_t)a * m];
      if (raa == cd(0.0)) continue;
      cd t = a == b ? cd(1.0) : cd(0.0);
      for (int c2 = a + 1; c2 <= b; ++c2) t -= R[a + (size_t)c2 * m] * W[c2 + (size_t)b * m];
      W[a + (size_t)b * m] = t / raa;
    }
  w.resize((size_t)m * m);
  for (size_t i = 0; i < w.size(); ++i) w[i] = double2{W[i].real(), W[i].imag()};
}

// Right eigenpairs of K_k = H_k - i Gamma nearest sigma at the context's current k: shift-invert
// subspace iteration (Y = G(sigma) Q, Q = orth(Y) by Cholesky QR twice) with Rayleigh-Ritz
// (B = Q^H K Q from one apply, eigenpairs of B on the host, X = Q S).  Leaves the m Ritz vectors,
// nearest sigma first, in c->d_egX (n x m) and their values in theta; resid gets the relative residuals
// ||K x - theta x|| / max(1, |theta|) of the first p.
static rst_status eig_right(rst_ctx* c, const rst_eig_opts* o, int m, int p, uint64_t seed,
                            std::vector<std::complex<double>>& theta, std::vector<double>& resid, int& iters,
                            rst_stats& acc) {
  using cd = std::complex<double>;
  const int P = c->na * c->nb;
  const long long n = (long long)P * c->nz;
  rst_status s;
  if ((s = ensure(c, c->d_egQ, (size_t)n * m * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egY, (size_t)n * m * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egW, (size_t)n * m * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egX, (size_t)n * m * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egKX, (size_t)n * m * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egS, (size_t)m * m * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egG, (size_t)m * m * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egTh, (size_t)m * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egRes, (size_t)m * 8)) != RST_OK) return s;
  if (c->nproj > 0 && (s = ensure(c, c->d_projP, (size_t)c->nproj * m * 16)) != RST_OK) return s;
  double2* Q = (double2*)c->d_egQ.p;
  double2* Y = (double2*)c->d_egY.p;
  double2* W = (double2*)c->d_egW.p;
  double2* X = (double2*)c->d_egX.p;
  double2* KX = (double2*)c->d_egKX.p;
  const unsigned gnm = (unsigned)((n * m + 255) / 256);
  hipLaunchKernelGGL(rst::eig::k_eig_randn, dim3(gnm), dim3(256), 0, c->stream, n, m, (unsigned long long)seed, X);
  HIPCHK(c, hipGetLastError());
  std::vector<double2> hg((size_t)m * m), hw;
  auto gram = [&](const double2* A, const double2* B, int cj) -> rst_status {
    hipLaunchKernelGGL(rst::eig::k_eig_gram, dim3((unsigned)m * m), dim3(256), 0, c->stream, A, m, B, m, n, m, m, cj,
                       (const double*)nullptr, P, (double2*)c->d_egG.p);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(hg.data(), c->d_egG.p, hg.size() * 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RST_OK;
  };
  auto rmul = [&](const double2* A, const std::vector<double2>& S, double alpha, double2* Z) -> rst_status {
    HIPCHK(c, hipMemcpyAsync(c->d_egS.p, S.data(), S.size() * 16, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(rst::eig::k_eig_rmul, dim3(gnm), dim3(256), 0, c->stream, A, m, n, m,
                       (const double2*)c->d_egS.p, m, alpha, Z, m);
    HIPCHK(c, hipGetLastError());
    return RST_OK;
  };
  std::vector<int64_t> zcols(m, 0);
  theta.assign(m, cd(0.0));
  resid.assign(p, 1e300);
  iters = 0;
  for (int it = 0; it < o->max_iter; ++it) {
    iters = it + 1;
    // Y = G(sigma) X  (dense right-hand sides, the context's solver)
    std::vector<double> Tcol, res;
    std::vector<int> its, rss, stv;
    double ms = 0.0;
    if (m == n) {
      // the subspace is the whole space: Rayleigh-Ritz on any basis is exact, so the random block
      // itself is orthonormalised (no solves, and no conditioning lost to G(sigma))
      HIPCHK(c, hipMemcpyAsync(Y, X, (size_t)n * m * 16, hipMemcpyDeviceToDevice, c->stream));
    } else {
      HIPCHK(c, hipMemsetAsync(Y, 0, (size_t)n * m * 16, c->stream));
      if ((s = run_solver(c, 1, &o->sigma, zcols, nullptr, nullptr, Y, Tcol, its, rss, res, stv, ms, X, m, 0)) !=
          RST_OK)
        return s;
    }
    int nbad = 0;
    rst_stats st;
    fill_stats(c, &st, its, rss, res, stv, ms, nbad, c->last_cw, c->last_threads);
    acc.columns += st.columns;
    acc.columns_unconverged += st.columns_unconverged;
    acc.iterations_total += st.iterations_total;
    acc.iterations_max = std::max(acc.iterations_max, st.iterations_max);
    acc.kernel_ms += st.kernel_ms;
    acc.bytes_algorithmic += st.bytes_algorithmic;
    acc.max_rel_residual = std::max(acc.max_rel_residual, st.max_rel_residual);
    // Q = orth(Y): Cholesky QR twice
    if ((s = gram(Y, Y, 1)) != RST_OK) return s;
    chol_inv(m, hg, hw);
    if ((s = rmul(Y, hw, 1.0, Q)) != RST_OK) return s;
    if ((s = gram(Q, Q, 1)) != RST_OK) return s;
    chol_inv(m, hg, hw);
    if ((s = rmul(Q, hw, 1.0, Y)) != RST_OK) return s;
    std::swap(Q, Y);
    // B = Q^H K Q with K Q = -A(0) Q
    if ((s = apply_cols(c, Q, W, m, 0.0, nullptr, nullptr, false, (double2*)c->d_projP.p, nullptr)) != RST_OK)
      return s;
    if ((s = gram(Q, W, 1)) != RST_OK) return s;
    std::vector<cd> B((size_t)m * m), w, v;
    for (size_t i = 0; i < B.size(); ++i) B[i] = -cd(hg[i].x, hg[i].y);
    if (!rst::zeig::eig(m, B, w, v)) return fail(c, RST_ENOCONV, "Rayleigh-Ritz eigensolver did not converge");
    // Ritz pairs sorted by distance to sigma
    std::vector<int> ord(m);
    for (int i = 0; i < m; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int a, int b) { return std::abs(w[a] - o->sigma) < std::abs(w[b] - o->sigma); });
    std::vector<double2> S((size_t)m * m);
    std::vector<double2> th(m);
    for (int b = 0; b < m; ++b) {
      theta[b] = w[ord[b]];
      th[b] = double2{w[ord[b]].real(), w[ord[b]].imag()};
      for (int a = 0; a < m; ++a) {
        const cd x = v[a + (size_t)ord[b] * m];
        S[a + (size_t)b * m] = double2{x.real(), x.imag()};
      }
    }
    if ((s = rmul(Q, S, 1.0, X)) != RST_OK) return s;    // Ritz vectors (unit 2-norm: Q orthonormal)
    if ((s = rmul(W, S, -1.0, KX)) != RST_OK) return s;  // K X
    HIPCHK(c, hipMemcpyAsync(c->d_egTh.p, th.data(), m * 16, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(rst::eig::k_eig_resid, dim3((unsigned)p), dim3(256), 0, c->stream, (const double2*)KX,
                       (const double2*)X, m, n, (const double2*)c->d_egTh.p, (double*)c->d_egRes.p);
    HIPCHK(c, hipGetLastError());
    std::vector<double> r2(p);
    HIPCHK(c, hipMemcpyAsync(r2.data(), c->d_egRes.p, p * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool conv = true;
    for (int i = 0; i < p; ++i) {
      resid[i] = std::sqrt(r2[i]) / std::max(1.0, std::abs(theta[i]));
      conv = conv && resid[i] <= o->tol;
    }
    if (conv || m == n) break;
  }
  return RST_OK;
}

extern "C" {

void rst_default_eig(rst_eig_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->n_eig = 32;
  o->subspace = 0;
  o->max_iter = 40;
  o->sigma = 0.0;
  o->tol = 1e-8;
  o->seed = 1;
}

rst_status rst_transmission_eigen(rst_ctx* c, int n_e, const double* E, const rst_eig_opts* o, double* T_out,
                                  double* eig_out, rst_stats* stats) {
  using cd = std::complex<double>;
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  if (!o || n_e < 0 || (n_e > 0 && (!E || !T_out))) return fail(c, RST_EINVAL, "bad eigen-route arguments");
  for (int i = 0; i < n_e; ++i)
    if (!std::isfinite(E[i])) return fail(c, RST_EINVAL, "non-finite energy");
  const int P = c->na * c->nb;
  const long long n = (long long)P * c->nz;
  if (o->n_eig < 1 || o->n_eig > 512 || o->n_eig > n || o->max_iter < 1 || !(o->tol > 0) || !std::isfinite(o->sigma) ||
      o->subspace < 0 || o->subspace > 1024)
    return fail(c, RST_EINVAL, "bad eigen-route options (1 <= n_eig <= min(512, n), subspace <= 1024)");
  if ((c->opts.method != RST_BICGSTAB && c->opts.method != RST_BICGSTAB_MC && c->opts.method != RST_IDRS) ||
      c->opts.precision != RST_FP64)
    return fail(c, RST_EUNSUPPORTED, "the eigen route solves with FP64 BiCGSTAB or IDR(s)");
  hipSetDevice(c->device);
  const int p = o->n_eig;
  int m = o->subspace > 0 ? o->subspace : std::min<long long>(n, 2 * p + 16);
  m = (int)std::min<long long>(std::max(m, p), n);
  rst_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  // right eigenvectors at +k (kept in d_egR) and at -k (in d_egX after the second run)
  std::vector<cd> th_p, th_m;
  std::vector<double> res_p, res_m;
  int it_p = 0, it_m = 0;
  if ((s = eig_right(c, o, m, p, o->seed, th_p, res_p, it_p, acc)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egR, (size_t)n * p * 16)) != RST_OK) return s;
  // R = the first p Ritz vectors (n x p, column fastest)
  {
    std::vector<double2> sel((size_t)m * p, double2{0.0, 0.0});
    for (int i = 0; i < p; ++i) sel[i + (size_t)i * m] = double2{1.0, 0.0};
    HIPCHK(c, hipMemcpyAsync(c->d_egS.p, sel.data(), sel.size() * 16, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(rst::eig::k_eig_rmul, dim3((unsigned)((n * p + 255) / 256)), dim3(256), 0, c->stream,
                       (const double2*)c->d_egX.p, m, n, m, (const double2*)c->d_egS.p, p, 1.0,
                       (double2*)c->d_egR.p, p);
    HIPCHK(c, hipGetLastError());
  }
  const double ka0 = c->ka, kb0 = c->kb;
  const bool self = std::fabs(std::remainder(2 * ka0 * c->na * c->ha, 2 * M_PI)) < 1e-12 &&
                    std::fabs(std::remainder(2 * kb0 * c->nb * c->hb, 2 * M_PI)) < 1e-12;
  if (!self) {
    c->ka = -ka0;
    c->kb = -kb0;
    if ((s = upload_k(c)) == RST_OK && (s = upload_pc(c)) == RST_OK)
      s = eig_right(c, o, m, p, o->seed + 7919, th_m, res_m, it_m, acc);
    c->ka = ka0;
    c->kb = kb0;
    rst_status s2 = upload_k(c);
    if (s2 == RST_OK) s2 = upload_pc(c);
    if (s != RST_OK) return s;
    if (s2 != RST_OK) return s2;
  }
  // the -k Ritz vector of each +k eigenvalue (nearest eigenvalue; at a k equal to -k modulo a
  // reciprocal vector the right vectors themselves), then L_i = conj(R'_j / d_i), d_i = R'_j . R_i
  const double2* Rm = self ? (const double2*)c->d_egR.p : (const double2*)c->d_egX.p;
  const int ldm = self ? p : m;
  std::vector<int> map(p);
  double mism = 0.0;
  for (int i = 0; i < p; ++i) {
    if (self) {
      map[i] = i;
      continue;
    }
    int best = 0;
    for (int j = 1; j < m; ++j)
      if (std::abs(th_m[j] - th_p[i]) < std::abs(th_m[best] - th_p[i])) best = j;
    map[i] = best;
    mism = std::max(mism, std::abs(th_m[best] - th_p[i]) / std::max(1.0, std::abs(th_p[i])));
  }
  if ((s = ensure(c, c->d_egL, (size_t)n * p * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egMap, (size_t)p * 4)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egSc, (size_t)p * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_egG, (size_t)std::max(m, p) * std::max(m, p) * 16)) != RST_OK) return s;
  // d_i = sum_g R'_map(i)[g] R_i[g] (bilinear): the diagonal of a Gram block, one entry per workgroup
  std::vector<double2> scale(p);
  {
    std::vector<double2> dv(1);
    for (int i = 0; i < p; ++i) {
      hipLaunchKernelGGL(rst::eig::k_eig_gram, dim3(1), dim3(256), 0, c->stream, Rm + map[i], ldm,
                         (const double2*)c->d_egR.p + i, p, n, 1, 1, 0, (const double*)nullptr, P,
                         (double2*)c->d_egG.p + i);
    }
    HIPCHK(c, hipGetLastError());
    std::vector<double2> d(p);
    HIPCHK(c, hipMemcpyAsync(d.data(), c->d_egG.p, p * 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < p; ++i) {
      const cd inv = 1.0 / cd(d[i].x, d[i].y);
      scale[i] = double2{inv.real(), inv.imag()};
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->d_egMap.p, map.data(), p * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_egSc.p, scale.data(), p * 16, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(rst::eig::k_eig_left, dim3((unsigned)((n * p + 255) / 256)), dim3(256), 0, c->stream, Rm, ldm, n,
                     p, (const int*)c->d_egMap.p, (const double2*)c->d_egSc.p, (double2*)c->d_egL.p);
  HIPCHK(c, hipGetLastError());
  // transformed CAPs GtL = R^H Gamma_L R, GtR = L^H Gamma_R L (p x p, column-major)
  std::vector<double2> gtl((size_t)p * p), gtr((size_t)p * p);
  hipLaunchKernelGGL(rst::eig::k_eig_gram, dim3((unsigned)p * p), dim3(256), 0, c->stream,
                     (const double2*)c->d_egR.p, p, (const double2*)c->d_egR.p, p, n, p, p, 1,
                     (const double*)c->d_gl.p, P, (double2*)c->d_egG.p);
  HIPCHK(c, hipMemcpyAsync(gtl.data(), c->d_egG.p, gtl.size() * 16, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  hipLaunchKernelGGL(rst::eig::k_eig_gram, dim3((unsigned)p * p), dim3(256), 0, c->stream,
                     (const double2*)c->d_egL.p, p, (const double2*)c->d_egL.p, p, n, p, p, 1,
                     (const double*)c->d_gr.p, P, (double2*)c->d_egG.p);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(gtr.data(), c->d_egG.p, gtr.size() * 16, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // T(E) = 4 sum_{m,n} GtL[m,n] GtR[n,m] / ((E - lam_n)(E - lam_m)^*)
  for (int ie = 0; ie < n_e; ++ie) {
    std::vector<cd> dd(p);
    for (int i = 0; i < p; ++i) dd[i] = 1.0 / (E[ie] - th_p[i]);
    cd t = 0.0;
    for (int b = 0; b < p; ++b)
      for (int a = 0; a < p; ++a) {
        const cd l(gtl[a + (size_t)b * p].x, gtl[a + (size_t)b * p].y);   // GtL[a, b]
        const cd r(gtr[b + (size_t)a * p].x, gtr[b + (size_t)a * p].y);   // GtR[b, a]
        t += l * r * dd[b] * std::conj(dd[a]);
      }
    T_out[ie] = 4.0 * t.real();
  }
  if (eig_out)
    for (int i = 0; i < p; ++i) {
      eig_out[2 * i] = th_p[i].real();
      eig_out[2 * i + 1] = th_p[i].imag();
    }
  double rmax = 0.0;
  for (int i = 0; i < p; ++i) rmax = std::max(rmax, res_p[i]);
  for (double r : res_m) rmax = std::max(rmax, r);
  acc.restarts_total = it_p + it_m;  // subspace iterations (both Bloch vectors)
  if (stats) {
    *stats = acc;
    stats->max_rel_residual = std::max(acc.max_rel_residual, rmax);
  }
  const bool ok = rmax <= o->tol && mism <= 1e3 * o->tol && acc.columns_unconverged == 0;
  if (!ok && rmax > o->tol)
    c->err = "eigenpairs not converged to tol: largest relative residual " + std::to_string(rmax) +
             ", +k/-k eigenvalue mismatch " + std::to_string(mism);
  return ok ? RST_OK : RST_ENOCONV;
}

}  // extern "C"

static rst_status cnn_engine(rst_ctx* c, bool need_weights) {
  if (!c->cnn) c->cnn = rst::cnn::engine_create(c->stream);
  if (need_weights && !rst::cnn::engine_has_weights(c->cnn))
    return fail(c, RST_ESTATE, "the network has no weights (rst_cnn_seed or rst_cnn_set_weights)");
  return RST_OK;
}

#define CNN_HIP(c, x)                                                             \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      if (e_ == hipErrorOutOfMemory) return fail(c, RST_ENOMEM, "network buffers"); \
      return fail(c, RST_EDEVICE, std::string("network: ") + hipGetErrorString(e_)); \
    }                                                                             \
  } while (0)

static rst_status cnn_shape(rst_ctx* c, int ncol, int nz, int nb, int na) {
  if (ncol < 1 || nz < 1 || nb < 1 || na < 1 || (long long)ncol * nz * nb * na > (1LL << 31))
    return fail(c, RST_EINVAL, "network shape must be positive and ncol*nz*nb*na <= 2^31");
  return RST_OK;
}

extern "C" {

int64_t rst_cnn_weight_count(void) { return (int64_t)rst::cnn::natural_count(); }

rst_status rst_cnn_seed(rst_ctx* c, uint64_t seed) {
  if (!c) return RST_EINVAL;
  hipSetDevice(c->device);
  rst_status s = cnn_engine(c, false);
  if (s != RST_OK) return s;
  CNN_HIP(c, rst::cnn::engine_seed(c->cnn, seed));
  return RST_OK;
}

rst_status rst_cnn_set_weights(rst_ctx* c, const float* w, int64_t count) {
  if (!c || !w) return RST_EINVAL;
  if (count != rst_cnn_weight_count()) return fail(c, RST_EINVAL, "weight count mismatch");
  for (int64_t i = 0; i < count; ++i)
    if (!std::isfinite(w[i])) return fail(c, RST_EINVAL, "non-finite weight");
  hipSetDevice(c->device);
  rst_status s = cnn_engine(c, false);
  if (s != RST_OK) return s;
  CNN_HIP(c, rst::cnn::engine_set_weights(c->cnn, w));
  return RST_OK;
}

rst_status rst_cnn_get_weights(rst_ctx* c, float* w, int64_t count) {
  if (!c || !w) return RST_EINVAL;
  if (count != rst_cnn_weight_count()) return fail(c, RST_EINVAL, "weight count mismatch");
  hipSetDevice(c->device);
  rst_status s = cnn_engine(c, true);
  if (s != RST_OK) return s;
  CNN_HIP(c, rst::cnn::engine_get_weights(c->cnn, w));
  return RST_OK;
}

rst_status rst_cnn_forward(rst_ctx* c, int ncol, int nz, int nb, int na, const float* x_dev, float* out_dev) {
  if (!c || !x_dev || !out_dev) return RST_EINVAL;
  rst_status s = cnn_shape(c, ncol, nz, nb, na);
  if (s != RST_OK) return s;
  hipSetDevice(c->device);
  if ((s = cnn_engine(c, true)) != RST_OK) return s;
  CNN_HIP(c, rst::cnn::engine_forward(c->cnn, x_dev, out_dev, ncol, nz, nb, na, false));
  CNN_HIP(c, hipStreamSynchronize(c->stream));
  return RST_OK;
}

rst_status rst_cnn_gradient(rst_ctx* c, int ncol, int nz, int nb, int na, const float* x_dev,
                            const float* gout_dev, float* grad) {
  if (!c || !x_dev || !gout_dev || !grad) return RST_EINVAL;
  rst_status s = cnn_shape(c, ncol, nz, nb, na);
  if (s != RST_OK) return s;
  hipSetDevice(c->device);
  if ((s = cnn_engine(c, true)) != RST_OK) return s;
  CNN_HIP(c, rst::cnn::engine_gradient(c->cnn, x_dev, gout_dev, ncol, nz, nb, na));
  CNN_HIP(c, rst::cnn::engine_get_grad(c->cnn, grad));
  return RST_OK;
}

rst_status rst_cnn_train_step(rst_ctx* c, int ncol, int nz, int nb, int na, const float* x_dev,
                              const float* target_dev, float lr, double* loss) {
  if (!c || !x_dev || !target_dev || !loss) return RST_EINVAL;
  if (!(lr > 0.f)) return fail(c, RST_EINVAL, "lr must be > 0");
  rst_status s = cnn_shape(c, ncol, nz, nb, na);
  if (s != RST_OK) return s;
  hipSetDevice(c->device);
  if ((s = cnn_engine(c, true)) != RST_OK) return s;
  CNN_HIP(c, rst::cnn::engine_train_step(c->cnn, x_dev, target_dev, ncol, nz, nb, na, lr, loss));
  CNN_HIP(c, hipStreamSynchronize(c->stream));
  return RST_OK;
}

rst_status rst_precond_train(rst_ctx* c, const rst_train_opts* o, rst_train_stats* ts) {
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  if (!o || o->pairs < 1 || o->batch < 1 || o->batch > 64 || !(o->lr > 0.f) || o->n_e < 1 || !o->energies ||
      o->n_k < 1 || !o->kpts || (o->source != 0 && o->source != 1))
    return fail(c, RST_EINVAL, "bad training options");
  const bool from_solver = o->source == 1;
  for (int i = 0; i < o->n_e; ++i)
    if (!std::isfinite(o->energies[i])) return fail(c, RST_EINVAL, "non-finite energy");
  for (int i = 0; i < 2 * o->n_k; ++i)
    if (!std::isfinite(o->kpts[i])) return fail(c, RST_EINVAL, "non-finite k");
  hipSetDevice(c->device);
  if ((s = cnn_engine(c, false)) != RST_OK) return s;
  if (!rst::cnn::engine_has_weights(c->cnn)) CNN_HIP(c, rst::cnn::engine_seed(c->cnn, o->seed));
  const int P = c->na * c->nb;
  const long long n = (long long)P * c->nz;
  BlockedShape bs;
  if ((s = blocked_shape(c, 8, 0, bs)) != RST_OK) return s;
  const LaunchShape ls = bs.ls;
  const int cw = ls.cw, B = o->batch;
  const int ncolp = (B + cw - 1) / cw * cw, nblk = ncolp / cw;
  const size_t vlen = (size_t)nblk * n * cw;
  void* kapply = pick_kernel(c->rad, ls.q, 1);
  void* kpc = pick_kernel(c->rad, ls.q, 7);
  if (!kapply || !kpc) return fail(c, RST_EUNSUPPORTED, "no kernel instance");
  if ((s = ensure(c, c->d_fgV, 3 * vlen * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_fgM, vlen * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_fgwb, vlen * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_fgx0, (size_t)B * n * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_fgf, (size_t)B * n * 8)) != RST_OK) return s;
  if ((s = ensure(c, c->d_fginv, (size_t)ncolp * 8)) != RST_OK) return s;
  if ((s = ensure(c, c->d_fgn2, (size_t)ncolp * 16)) != RST_OK) return s;
  double2* Xi = (double2*)c->d_fgV.p;
  double2* Ev = Xi + vlen;
  double2* Rv = Ev + vlen;
  double2* Mv = (double2*)c->d_fgM.p;
  rst::Proj pj = make_proj(c);
  const size_t pws_stride = std::max<size_t>(1, (size_t)c->nproj * cw);
  if ((s = ensure(c, c->d_pws, (size_t)nblk * pws_stride * 16)) != RST_OK) return s;
  const double ka0 = c->ka, kb0 = c->kb;
  std::vector<double> en(o->energies, o->energies + o->n_e);
  if ((s = upload(c, c->d_tren, en)) != RST_OK) return s;
  // solver pairs: the right-CAP columns to draw from, x* and x_j (column-fastest n x B), the columns
  std::vector<int64_t> rcols;
  const rst_solver_opts opts0 = c->opts;
  if (from_solver) {
    for (int z = 0; z < c->nz; ++z)
      if (c->gr[z] > 0)
        for (int q = 0; q < P; ++q) rcols.push_back((int64_t)z * P + q);
    if (rcols.empty()) return fail(c, RST_EINVAL, "solver pairs need a right CAP");
    if ((s = ensure(c, c->d_trX, (size_t)2 * n * B * 16)) != RST_OK) return s;
    if ((s = ensure(c, c->d_trcols, (size_t)B * 8)) != RST_OK) return s;
  }
  if ((s = ensure(c, c->d_pc_inv, (size_t)n * 16)) != RST_OK) return s;
  double vbar = 0;
  for (double x : c->v) vbar += x;
  vbar /= (double)c->v.size();
  std::mt19937_64 gen(o->seed);
  const int steps = (o->pairs + B - 1) / B;
  std::vector<double> losses;
  losses.reserve(steps);
  rst::fg::Shape S{n, cw, nblk, B, 1};
  const unsigned gv = (unsigned)((vlen + 255) / 256);
  const unsigned gf = (unsigned)(((long long)B * n + 255) / 256);
  int cur_k = -1;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, hipEventRecord(e0, c->stream));
  int jcheck = 0;  // solver pairs: the next iterate of the current draw (iterations 2^jcheck)
  std::vector<int64_t> dcols(B);
  int ie = 0, ik = 0;
  for (int st = 0; st < steps; ++st) {
    if (!from_solver || jcheck == 0) {
      ie = (int)(gen() % (uint64_t)o->n_e);
      ik = (int)(gen() % (uint64_t)o->n_k);
    }
    if (ik != cur_k) {
      c->ka = o->kpts[2 * ik];
      c->kb = o->kpts[2 * ik + 1];
      if ((s = upload_k(c)) != RST_OK) return s;
      if ((s = upload_pc(c)) != RST_OK) return s;
      cur_k = ik;
    }
    rst::Geo g = make_geo(c);
    const size_t lds_apply = bs.lds_apply, lds_pc = bs.lds_pc, pc_off = bs.pc_off;
    if (lds_apply > 64 * 1024)
      HIPCHK(c, hipFuncSetAttribute(kapply, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_apply));
    if (lds_pc > 64 * 1024)
      HIPCHK(c, hipFuncSetAttribute(kpc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_pc));
    rst::SolveArgs A;
    std::memset(&A, 0, sizeof(A));
    A.g = g;
    A.gz = (const double*)c->d_gz.p;
    A.energies = (const double*)c->d_tren.p + ie;
    A.ne = 1;
    A.pc.vbar = vbar;
    A.pc.a = 0.5 / (c->hz * c->hz);
    A.pc.eps = (const double*)c->d_pc_eps.p;
    A.pc.vz = pc_vz(c);
    A.pc.shift = c->opts.pc_shift;
    A.pc.steps = (const double2*)c->d_pc_twa.p;
    A.pc.inv = (const double2*)c->d_pc_inv.p;
    std::vector<rst::SolveArgs> sa(1, A);
    if ((s = upload(c, c->d_fgsa, sa)) != RST_OK) return s;
    hipLaunchKernelGGL(rst::k_pc_pivots, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, c->stream,
                       (const rst::SolveArgs*)c->d_fgsa.p);
    std::vector<rst::PcApplyArgs> pa(2);
    for (int j = 0; j < 2; ++j) {
      std::memset(&pa[j], 0, sizeof(pa[j]));
      pa[j].g = g;
      pa[j].pc = A.pc;
      pa[j].in = j == 0 ? Xi : Rv;
      pa[j].out = j == 0 ? Ev : Mv;
      pa[j].wbuf = (double2*)c->d_fgwb.p;
      pa[j].cw = cw;
      pa[j].nblk = nblk;
      pa[j].pc_lds_off = pc_off;
    }
    if ((s = upload(c, c->d_fgpa, pa)) != RST_OK) return s;
    std::vector<rst::ApplyArgs> aa(1);
    std::memset(&aa[0], 0, sizeof(aa[0]));
    aa[0].g = g;
    aa[0].pj = pj;
    aa[0].V = (const double*)c->d_v.p;
    aa[0].gz = (const double*)c->d_gz.p;
    aa[0].energy = o->energies[ie];
    aa[0].x = from_solver ? Xi : Ev;
    aa[0].y = Rv;
    aa[0].ncol = ncolp;
    aa[0].cw = cw;
    aa[0].nblk = nblk;
    aa[0].pws = (double2*)c->d_pws.p;
    aa[0].pws_stride = pws_stride;
    aa[0].proj_pre = c->nproj > 0;
    if ((s = upload(c, c->d_fgaa, aa)) != RST_OK) return s;
    void* p0 = c->d_fgpa.p;
    void* p1 = (char*)c->d_fgpa.p + sizeof(rst::PcApplyArgs);
    void* a0 = c->d_fgaa.p;
    void* argsa[] = {&a0};
    if (!from_solver) {
      // xi -> e = M^-1 xi -> r = A e; scale to ||r|| = 1; m = M^-1 r; (features, target)
      hipLaunchKernelGGL(rst::fg::k_fg_randn, dim3(gv), dim3(256), 0, c->stream, S,
                         (unsigned long long)(o->seed * 0x9E3779B97F4A7C15ULL + (uint64_t)st), Xi);
      void* args0[] = {&p0};
      HIPCHK(c, hipLaunchKernel(kpc, dim3(nblk), dim3(ls.threads), args0, lds_pc, c->stream));
      if ((s = proj_blocked(c, aa[0])) != RST_OK) return s;
      HIPCHK(c, hipLaunchKernel(kapply, dim3(nblk), dim3(ls.threads), argsa, lds_apply, c->stream));
    } else {
      // x* (on a new draw), then the iterate x_j of the same solver after 2^(jcheck+1) iterations:
      // e = x* - x_j, r = b - A x_j; scale to ||r|| = 1; m = M^-1 r; (features, target)
      double2* Xs = (double2*)c->d_trX.p;
      double2* Xj = Xs + (size_t)n * B;
      std::vector<double> Tc, rs_;
      std::vector<int> itc, rsc, stc;
      double msc = 0;
      c->opts = opts0;
      c->opts.method = RST_BICGSTAB;
      c->opts.precond = RST_PRECOND_FREE_CAP;
      c->opts.precision = RST_FP64;
      c->opts.col_block = 0;
      c->opts.threads = 0;
      c->opts.tol = 1e-10;
      rst_status sv = RST_OK;
      if (jcheck == 0) {
        for (int b = 0; b < B; ++b) dcols[b] = rcols[gen() % (uint64_t)rcols.size()];
        c->opts.max_iter = 20000;
        sv = run_solver(c, 1, o->energies + ie, dcols, nullptr, nullptr, Xs, Tc, itc, rsc, rs_, stc, msc);
      }
      if (sv == RST_OK) {
        c->opts.max_iter = 2 << jcheck;
        sv = run_solver(c, 1, o->energies + ie, dcols, nullptr, nullptr, Xj, Tc, itc, rsc, rs_, stc, msc);
      }
      c->opts = opts0;
      if (sv != RST_OK) return sv;
      jcheck = jcheck + 1 < 6 ? jcheck + 1 : 0;  // iterates after 2, 4, ..., 64 iterations per draw
      HIPCHK(c, hipMemcpyAsync(c->d_trcols.p, dcols.data(), (size_t)B * 8, hipMemcpyHostToDevice, c->stream));
      hipLaunchKernelGGL(rst::fg::k_fg_pairs, dim3(gv), dim3(256), 0, c->stream, S, B, (const double2*)Xs,
                         (const double2*)Xj, Xi, Ev);
      // the solves above may have regrown the projection scratch: the apply's arguments again
      aa[0].pws = (double2*)c->d_pws.p;
      if ((s = upload(c, c->d_fgaa, aa)) != RST_OK) return s;
      a0 = c->d_fgaa.p;
      if ((s = proj_blocked(c, aa[0])) != RST_OK) return s;
      HIPCHK(c, hipLaunchKernel(kapply, dim3(nblk), dim3(ls.threads), argsa, lds_apply, c->stream));
      hipLaunchKernelGGL(rst::fg::k_fg_bsub, dim3(gv), dim3(256), 0, c->stream, S, B,
                         (const long long*)c->d_trcols.p, Rv);
    }
    // pair scale: 1/||r|| (synthetic pairs), 1/||e|| (solver pairs, whose errors exceed their residuals
    // by up to the condition number: every pair then weighs the same in the loss; the bias-free ReLU
    // network is positively homogeneous, so a common scale of input and target changes nothing else)
    const double2* Sv = from_solver ? (const double2*)Ev : (const double2*)Rv;
    hipLaunchKernelGGL(rst::fg::k_fg_dots, dim3(nblk, 1), dim3(256), 0, c->stream, S, Sv, (long long)vlen, 1, Sv,
                       (double2*)c->d_fgn2.p, ncolp);
    hipLaunchKernelGGL(rst::fg::k_fg_rsqrt, dim3((ncolp + 63) / 64), dim3(64), 0, c->stream,
                       (const double2*)c->d_fgn2.p, (double*)c->d_fginv.p, ncolp);
    hipLaunchKernelGGL(rst::fg::k_fg_scale, dim3(gv), dim3(256), 0, c->stream, S, Rv, (const double2*)Rv,
                       (const double*)c->d_fginv.p);
    void* args1[] = {&p1};
    HIPCHK(c, hipLaunchKernel(kpc, dim3(nblk), dim3(ls.threads), args1, lds_pc, c->stream));
    hipLaunchKernelGGL(rst::fg::k_fg_features, dim3(gf), dim3(256), 0, c->stream, S, (const double2*)Rv,
                       (const double2*)Mv, (float*)c->d_fgx0.p);
    hipLaunchKernelGGL(rst::fg::k_fg_target, dim3(gf), dim3(256), 0, c->stream, S, (const double2*)Ev,
                       (const double2*)Mv, (const double*)c->d_fginv.p, (float*)c->d_fgf.p);
    HIPCHK(c, hipGetLastError());
    double loss = 0;
    CNN_HIP(c, rst::cnn::engine_train_step(c->cnn, (const float*)c->d_fgx0.p, (const float*)c->d_fgf.p, B, c->nz,
                                           c->nb, c->na, o->lr, &loss));
    losses.push_back(loss);
  }
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float fms = 0;
  HIPCHK(c, hipEventElapsedTime(&fms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  // restore the context's k (and options)
  c->opts = opts0;
  c->ka = ka0;
  c->kb = kb0;
  if ((s = upload_k(c)) != RST_OK) return s;
  if ((s = upload_pc(c)) != RST_OK) return s;
  if (ts) {
    const int w = std::max(1, std::min<int>(10, (int)losses.size() / 4));
    double f = 0, l = 0;
    for (int i = 0; i < w; ++i) {
      f += losses[i];
      l += losses[losses.size() - 1 - i];
    }
    ts->steps = steps;
    ts->loss_first = f / w;
    ts->loss_last = l / w;
    ts->ms = fms;
  }
  return RST_OK;
}

static rst_status lr_solve(rst_ctx* c, int ne, const double* E, int ncol, const double2* rhs, long long estride,
                           double2* x, rst_stats& acc) {
  std::vector<int64_t> cols(ncol, 0);
  std::vector<double> Tcol, res;
  std::vector<int> its, rss, stv;
  double ms = 0;
  const long long ld = estride ? (long long)ne * ncol : ncol;
  rst_status s = run_solver(c, ne, E, cols, nullptr, nullptr, x, Tcol, its, rss, res, stv, ms, rhs, ld, estride);
  if (s != RST_OK) return s;
  int nbad = 0;
  rst_stats st;
  fill_stats(c, &st, its, rss, res, stv, ms, nbad, c->last_cw, c->last_threads);
  acc.columns += st.columns;
  acc.columns_unconverged += st.columns_unconverged;
  acc.iterations_total += st.iterations_total;
  acc.iterations_max = std::max(acc.iterations_max, st.iterations_max);
  acc.restarts_total += st.restarts_total;
  acc.max_rel_residual = std::max(acc.max_rel_residual, st.max_rel_residual);
  acc.kernel_ms += st.kernel_ms;
  acc.bytes_algorithmic += st.bytes_algorithmic;
  acc.col_block = st.col_block;
  acc.threads = st.threads;
  return RST_OK;
}

void rst_default_lowrank(rst_lowrank_opts* o) {
  if (!o) return;
  o->probes = 32;
  o->heldout = 8;
  o->max_probes = 256;
  o->tail_tol = 1e-7;
  o->seed = 0x5eed;
}

rst_status rst_transmission_lowrank(rst_ctx* c, int n_e, const double* E, const rst_lowrank_opts* o, double* T_out,
                                    double* T_err, rst_stats* stats) {
  rst_status s = check_ready(c);
  if (s != RST_OK) return s;
  if (!o || n_e < 0 || (n_e > 0 && (!E || !T_out))) return fail(c, RST_EINVAL, "bad low-rank arguments");
  if (o->probes < 1 || o->heldout < 1 || o->max_probes < o->probes || !(o->tail_tol > 0))
    return fail(c, RST_EINVAL, "bad low-rank options");
  for (int i = 0; i < n_e; ++i)
    if (!std::isfinite(E[i])) return fail(c, RST_EINVAL, "non-finite energy");
  if ((c->opts.method != RST_BICGSTAB && c->opts.method != RST_BICGSTAB_MC && c->opts.method != RST_IDRS) ||
      c->opts.precision != RST_FP64)
    return fail(c, RST_EUNSUPPORTED, "the low-rank transmission uses FP64 BiCGSTAB or IDR(s)");
  // direction RL exchanges the roles of the two CAPs (T_RL = 4 ||Gamma_R^1/2 G Gamma_L^1/2||_F^2)
  const bool rl = c->opts.direction == RST_DIR_RL;
  const std::vector<double>& g_dst = rl ? c->gr : c->gl;
  const std::vector<double>& g_src = rl ? c->gl : c->gr;
  if (n_e == 0) return RST_OK;
  hipSetDevice(c->device);
  const int P = c->na * c->nb;
  const long long n = (long long)P * c->nz;
  std::vector<long long> Lh, Rh;
  for (int z = 0; z < c->nz; ++z)
    for (int p = 0; p < P; ++p) {
      if (g_dst[z] > 0) Lh.push_back((long long)z * P + p);
      if (g_src[z] > 0) Rh.push_back((long long)z * P + p);
    }
  rst_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  if (Lh.empty() || Rh.empty()) {
    for (int i = 0; i < n_e; ++i) {
      T_out[i] = 0.0;
      if (T_err) T_err[i] = 0.0;
    }
    if (stats) *stats = acc;
    return RST_OK;
  }
  const int nL = (int)Lh.size(), nR = (int)Rh.size();
  if ((s = upload(c, c->d_lrL, Lh)) != RST_OK) return s;
  if ((s = upload(c, c->d_lrRc, Rh)) != RST_OK) return s;
  const double* d_gl = (const double*)(rl ? c->d_gr.p : c->d_gl.p);
  const double* d_gr = (const double*)(rl ? c->d_gl.p : c->d_gr.p);
  const long long* dL = (const long long*)c->d_lrL.p;
  const long long* dR = (const long long*)c->d_lrRc.p;
  std::vector<int> done(n_e, 0);
  std::vector<double> Tq(n_e, 0.0), tail(n_e, 0.0);
  const int smax = std::min(o->max_probes, nR);
  int sprobe = std::min(o->probes, nR);  // probes in the basis after this doubling step
  const int hp = o->heldout;
  uint64_t seed = o->seed;
  const double ka0 = c->ka, kb0 = c->kb;
  // Y of the probes of earlier rounds, per open energy (compact over the open energies, in their
  // order): Yacc[j][col][i], columns 0..s_prev-1, stride smax*nL per energy
  const size_t ystride = (size_t)smax * nL;
  if ((s = ensure(c, c->d_lrYacc, (size_t)n_e * ystride * 16)) != RST_OK) return s;
  if ((s = ensure(c, c->d_lrYacc2, (size_t)n_e * ystride * 16)) != RST_OK) return s;
  double2* Yacc = (double2*)c->d_lrYacc.p;
  double2* Ynext = (double2*)c->d_lrYacc2.p;
  std::vector<int> open_prev;  // open energies of the previous round, in Yacc order
  int s_prev = 0;
  for (;;) {
    // energies still open
    std::vector<double> Eo;
    std::vector<int> idx;
    for (int i = 0; i < n_e; ++i)
      if (!done[i]) {
        Eo.push_back(E[i]);
        idx.push_back(i);
      }
    const int ne = (int)Eo.size();
    const int snew = sprobe - s_prev;  // probes added by this doubling step
    const int sc = snew + hp;
    // (1) new probes and held-out probes, forward solves
    if ((s = ensure(c, c->d_lrB, (size_t)n * sc * 16)) != RST_OK) return s;
    if ((s = ensure(c, c->d_lrX, (size_t)n * ne * sc * 16)) != RST_OK) return s;
    hipLaunchKernelGGL(rst::lr::k_lr_probes, dim3((unsigned)((n * sc + 255) / 256)), dim3(256), 0, c->stream, n, P, sc,
                       d_gr, (unsigned long long)seed, (double2*)c->d_lrB.p);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemsetAsync(c->d_lrX.p, 0, (size_t)n * ne * sc * 16, c->stream));
    if ((s = lr_solve(c, ne, Eo.data(), sc, (const double2*)c->d_lrB.p, 0, (double2*)c->d_lrX.p, acc)) != RST_OK)
      return s;
    // (2) Y = Gamma_L^1/2 X on the left CAP for the new columns; the basis columns of every open
    // energy are its earlier ones followed by the new ones
    const size_t ylen = (size_t)ne * sc * nL;
    if ((s = ensure(c, c->d_lrY, ylen * 16)) != RST_OK) return s;
    hipLaunchKernelGGL(rst::lr::k_lr_gather_left, dim3((unsigned)((ylen + 255) / 256)), dim3(256), 0, c->stream,
                       (const double2*)c->d_lrX.p, ne, sc, dL, nL, P, d_gl, (double2*)c->d_lrY.p);
    HIPCHK(c, hipGetLastError());
    const double2* Ynew = (const double2*)c->d_lrY.p;
    for (int j = 0; j < ne; ++j) {
      double2* dstj = Ynext + (size_t)j * ystride;
      if (s_prev > 0) {
        const int jp = (int)(std::find(open_prev.begin(), open_prev.end(), idx[j]) - open_prev.begin());
        HIPCHK(c, hipMemcpyAsync(dstj, Yacc + (size_t)jp * ystride, (size_t)s_prev * nL * 16,
                                 hipMemcpyDeviceToDevice, c->stream));
      }
      HIPCHK(c, hipMemcpyAsync(dstj + (size_t)s_prev * nL, Ynew + (size_t)j * sc * nL, (size_t)snew * nL * 16,
                               hipMemcpyDeviceToDevice, c->stream));
    }
    std::swap(Yacc, Ynext);
    open_prev = idx;
    s_prev = sprobe;
    // Q = orth(Yacc[:, :sprobe]) by Cholesky QR twice
    if ((s = ensure(c, c->d_lrQ, (size_t)ne * sprobe * nL * 16)) != RST_OK) return s;
    if ((s = ensure(c, c->d_lrQ2, (size_t)ne * sprobe * nL * 16)) != RST_OK) return s;
    if ((s = ensure(c, c->d_lrG, (size_t)ne * std::max(sprobe, hp) * std::max(sprobe, hp) * 16)) != RST_OK) return s;
    if ((s = ensure(c, c->d_lrR, (size_t)ne * sprobe * sprobe * 16)) != RST_OK) return s;
    if ((s = ensure(c, c->d_lrW, (size_t)ne * sprobe * sprobe * 16)) != RST_OK) return s;
    double2* Q = (double2*)c->d_lrQ.p;
    double2* Q2 = (double2*)c->d_lrQ2.p;
    const long long sq = (long long)sprobe * nL;
    const unsigned gq = (unsigned)(((size_t)ne * sprobe * nL + 255) / 256);
    for (int pass = 0; pass < 2; ++pass) {
      const double2* src = pass == 0 ? Yacc : Q;
      const long long ss = pass == 0 ? (long long)ystride : sq;
      double2* dst = pass == 0 ? Q : Q2;
      hipLaunchKernelGGL(rst::lr::k_lr_gram, dim3(sprobe, sprobe, ne), dim3(256), 0, c->stream, src, ss, src, ss, nL,
                         sprobe, sprobe, (double2*)c->d_lrG.p);
      hipLaunchKernelGGL(rst::lr::k_lr_chol_inv, dim3((ne + 63) / 64), dim3(64), 0, c->stream,
                         (const double2*)c->d_lrG.p, sprobe, ne, (double2*)c->d_lrR.p, (double2*)c->d_lrW.p);
      hipLaunchKernelGGL(rst::lr::k_lr_right_mul, dim3(gq), dim3(256), 0, c->stream, src, ss,
                         (const double2*)c->d_lrW.p, sprobe, nL, ne, dst);
      HIPCHK(c, hipGetLastError());
    }
    // (3) tail of the held-out probes (the last hp columns of this doubling step): ||y||^2 - ||Q^H y||^2
    const double2* Yh = Ynew + (long long)snew * nL;
    const long long sy = (long long)sc * nL;
    std::vector<double2> cq((size_t)ne * sprobe * hp), yy((size_t)ne * hp * hp);
    hipLaunchKernelGGL(rst::lr::k_lr_gram, dim3(sprobe, hp, ne), dim3(256), 0, c->stream, (const double2*)Q2, sq, Yh,
                       sy, nL, sprobe, hp, (double2*)c->d_lrG.p);
    HIPCHK(c, hipMemcpyAsync(cq.data(), c->d_lrG.p, cq.size() * 16, hipMemcpyDeviceToHost, c->stream));
    hipLaunchKernelGGL(rst::lr::k_lr_gram, dim3(hp, hp, ne), dim3(256), 0, c->stream, Yh, sy, Yh, sy, nL, hp, hp,
                       (double2*)c->d_lrG.p);
    HIPCHK(c, hipMemcpyAsync(yy.data(), c->d_lrG.p, yy.size() * 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<int> fin;  // positions (in this doubling step's order) of the energies that end in this doubling step
    for (int e = 0; e < ne; ++e) {
      double t = 0.0;
      for (int b = 0; b < hp; ++b) {
        double r = yy[((size_t)e * hp + b) * hp + b].x;
        for (int a = 0; a < sprobe; ++a) {
          const double2 v = cq[((size_t)e * sprobe + a) * hp + b];
          r -= v.x * v.x + v.y * v.y;
        }
        t += std::max(r, 0.0);
      }
      tail[idx[e]] = 4.0 * t / hp;
      if (tail[idx[e]] <= o->tail_tol || sprobe >= smax) fin.push_back(e);
    }
    // (4) for the energies that end here: adjoint solves at -k, Z = G_{-k} Gamma_L^1/2 conj(Q),
    // T_Q = 4 ||Gamma_R^1/2 Z|_R||_F^2
    if (!fin.empty()) {
      const int nf = (int)fin.size();
      std::vector<double> Ef(nf);
      for (int f = 0; f < nf; ++f) Ef[f] = Eo[fin[f]];
      if ((s = ensure(c, c->d_lrQf, (size_t)nf * sprobe * nL * 16)) != RST_OK) return s;
      for (int f = 0; f < nf; ++f)
        HIPCHK(c, hipMemcpyAsync((double2*)c->d_lrQf.p + (size_t)f * sq, Q2 + (size_t)fin[f] * sq, (size_t)sq * 16,
                                 hipMemcpyDeviceToDevice, c->stream));
      if ((s = ensure(c, c->d_lrB, (size_t)n * nf * sprobe * 16)) != RST_OK) return s;
      if ((s = ensure(c, c->d_lrX, (size_t)n * nf * sprobe * 16)) != RST_OK) return s;
      HIPCHK(c, hipMemsetAsync(c->d_lrB.p, 0, (size_t)n * nf * sprobe * 16, c->stream));
      HIPCHK(c, hipMemsetAsync(c->d_lrX.p, 0, (size_t)n * nf * sprobe * 16, c->stream));
      const unsigned gf = (unsigned)(((size_t)nf * sprobe * nL + 255) / 256);
      hipLaunchKernelGGL(rst::lr::k_lr_adjoint_rhs, dim3(gf), dim3(256), 0, c->stream, (const double2*)c->d_lrQf.p, nf,
                         sprobe, dL, nL, P, d_gl, n, (double2*)c->d_lrB.p);
      HIPCHK(c, hipGetLastError());
      c->ka = -ka0;
      c->kb = -kb0;
      if ((s = upload_k(c)) != RST_OK) return s;
      if ((s = upload_pc(c)) != RST_OK) return s;
      s = lr_solve(c, nf, Ef.data(), sprobe, (const double2*)c->d_lrB.p, sprobe, (double2*)c->d_lrX.p, acc);
      c->ka = ka0;
      c->kb = kb0;
      rst_status s2 = upload_k(c);
      if (s2 == RST_OK) s2 = upload_pc(c);
      if (s != RST_OK) return s;
      if (s2 != RST_OK) return s2;
      if ((s = ensure(c, c->d_lrT, (size_t)nf * 8)) != RST_OK) return s;
      hipLaunchKernelGGL(rst::lr::k_lr_tq, dim3(nf), dim3(256), 0, c->stream, (const double2*)c->d_lrX.p, nf, sprobe,
                         dR, nR, P, d_gr, (double*)c->d_lrT.p);
      HIPCHK(c, hipGetLastError());
      std::vector<double> tq(nf);
      HIPCHK(c, hipMemcpyAsync(tq.data(), c->d_lrT.p, (size_t)nf * 8, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      for (int f = 0; f < nf; ++f) {
        Tq[idx[fin[f]]] = tq[f];
        done[idx[fin[f]]] = 1;
      }
    }
    if ((int)fin.size() == ne) break;
    // the energies left open double their basis with new probes
    sprobe = std::min(2 * sprobe, smax);
    seed = seed * 0x9E3779B97F4A7C15ULL + 1;
  }
  bool within = true;
  for (int i = 0; i < n_e; ++i) {
    T_out[i] = Tq[i];
    if (T_err) T_err[i] = tail[i];
    within = within && tail[i] <= o->tail_tol;
  }
  if (stats) *stats = acc;
  return (acc.columns_unconverged || !within) ? RST_ENOCONV : RST_OK;
}

}  // extern "C"
