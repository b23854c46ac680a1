/*
 * rst.h -- C ABI of librst, the MI355X (gfx950) Bloch-CAP transmission library.
 *
 * Computes the per-spin transmission of a lateral-periodic real-space structure,
 *
 *     T(E, k) = 4 Tr[ Gamma_L G Gamma_R G^+ ],   G = (E - H_k + i(Gamma_L + Gamma_R))^-1,
 *
 * (paper Sec. II.A: transmission equation, retarded Green's function and the
 * Gaussian-CAP equation; the factor 4 makes one open channel count as 1) by
 * Krylov solves of A x = sqrt(Gamma_R,i) e_i over the grid points i of the
 * right absorbing region, one solve per column, for one lateral Bloch vector k
 * (Bloch-form equation) at a time.  The k-average of T (end of Sec. II.A) is
 * left to the caller.
 *
 * Hamiltonian (Hartree atomic units):
 *     H_k = -1/2 L_k + diag(V) + h^3 sum_p E_p |beta_k,p><beta_k,p|
 *   L_k : central finite-difference Laplacian of even order 2M (2..12) on an
 *         orthorhombic grid; a lateral neighbour that leaves the cell across the
 *         +a face (resp. -a) is the wrapped point times exp(+i k_a L_a)
 *         (resp. exp(-i k_a L_a)), same for b: phi(r + R) = exp(i k.R) phi(r);
 *         psi = 0 outside the planes 0..Nz-1 along z (transport axis).
 *   beta_k,p(r) = sum over table entries e of projector p at r of
 *         beta_e exp(+i k.R_e), R_e the lateral image the entry comes from.
 *   Gamma_L, Gamma_R : functions of z only (constant in the lateral plane).
 *
 * Grid index i = ia + Na*(ib + Nb*iz) (a fastest, z slowest).  Vectors passed
 * as device pointers are complex, interleaved (re, im), with the column index
 * fastest: element (i, c) of an (n x ncol) block is at [2*(i*ncol + c)].
 *
 * Conventions
 *  - Host arrays given to rst_set_* are copied; the caller keeps ownership.
 *  - Device pointers (names ending in _dev) are borrowed for the duration of
 *    the call and used on the context's stream; the call returns after the
 *    stream has finished with them.
 *  - Outputs are caller-allocated.
 *  - Status < 0: the call failed and wrote no output.  Status > 0: the call
 *    completed and wrote its outputs, with the condition recorded in rst_stats.
 *  - Setters invalidate dependent state: rst_set_grid clears potential,
 *    projectors, CAPs and k, and makes a batch built before it stale
 *    (rst_batch_run then returns RST_ESTATE until rst_batch_clear).  Calling
 *    out of order returns RST_ESTATE.
 *  - A context is not thread-safe.  rst_last_error() describes the last failure.
 */
#ifndef RST_H
#define RST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rst_ctx rst_ctx;

typedef enum {
  RST_OK = 0,
  RST_ENOCONV = 1,        /* completed; some columns did not reach the tolerance */
  RST_EINVAL = -1,        /* invalid argument */
  RST_ESTATE = -2,        /* call out of order (e.g. no grid yet) */
  RST_ENOMEM = -3,        /* device allocation failed */
  RST_EDEVICE = -4,       /* HIP runtime error */
  RST_EUNSUPPORTED = -5   /* valid but not supported by the GPU kernels */
} rst_status;

typedef enum { RST_BICGSTAB = 0, RST_FGMRES = 1, RST_COCG = 2, RST_BICGSTAB_MC = 3, RST_IDRS = 4 } rst_method;
typedef enum { RST_FP64 = 0, RST_FP32_REFINE = 1 } rst_precision;
typedef enum { RST_DIR_LR = 0, RST_DIR_RL = 1 } rst_direction;
typedef enum { RST_PRECOND_NONE = 0, RST_PRECOND_FREE_CAP = 1, RST_PRECOND_LEARNED = 2 } rst_precond;
typedef enum { RST_VREF_PLANE = 0, RST_VREF_CELL = 1 } rst_vref;

/* Solver options.  rst_default_solver() fills the defaults. */
typedef struct {
  int method;        /* rst_method.  RST_BICGSTAB: the persistent fused BiCGSTAB kernels (every precision
                        and preconditioner except RST_PRECOND_LEARNED) for lateral planes of up to 1024
                        points; wider planes (na*nb > 1024) are solved by RST_IDRS instead (FP64 only;
                        col_block and threads must then be 0): BiCGSTAB stalls on long point-contact slabs.
                        RST_BICGSTAB_MC: the same right-preconditioned BiCGSTAB over blocks of up to 1024
                        columns in the column-fastest layout, one kernel per step (the many-column apply with
                        per-column energies; the preconditioner as lateral DFT passes and one banded L D L^T
                        solve of the operator's own order-2M z Laplacian per lateral mode and column), any
                        plane size, FP64, preconditioner NONE or FREE_CAP, convergence on the FP64 true
                        residual with restarts from it after a breakdown.  RST_IDRS: IDR(idr_s) with
                        biorthogonalisation (Sonneveld and van Gijzen 2008; van Gijzen and Sonneveld 2011) on
                        the same kernels and layout, right-preconditioned, a random shadow space shared by
                        all columns; iterations_total then counts operator applies.  RST_FGMRES: restarted flexible
                        GMRES(restart) in FP64 over chunks of columns (classical Gram-Schmidt twice),
                        convergence on the FP64 true residual after each cycle; precision FP64 only.
                        RST_COCG: conjugate orthogonal conjugate gradients (van der Vorst and Melissen
                        1990), FP64, preconditioner NONE or FREE_CAP, convergence on the FP64 true
                        residual.  For a real H_k (k_a L_a and k_b L_b multiples of pi, e.g. the Gamma
                        point: A = E - H_k + i Gamma is then complex symmetric) on planes of up to 1024
                        points: the blocked COCG, one operator apply per step.  At any other k (and on
                        wider planes or other FD orders): COCG on the doubled system
                        B = [[0, A_k], [A_-k, 0]], complex symmetric because A_k^T = A_-k (paper
                        Sec. II.B: the doubled operator of k and -k), with the preconditioner
                        [[0, M_k], [M_-k, 0]]^-1; it solves each column at k and at -k together (one
                        step: one apply at k and one at -k; iterations_total counts steps) and
                        reports the k solution.  col_block and threads are refused there, and dense
                        right-hand sides stay BiCGSTAB / IDR(s) */
  int precision;     /* rst_precision; RST_FP32_REFINE: BiCGSTAB on complex64 vectors with FP32 stencil,
                        projector and preconditioner applies (inner products, scalars and projections
                        FP64), the solution kept as x64 + x32 and the recursive residual replaced by the
                        FP64 true residual b - A x64 whenever it has fallen by update_delta (reliable
                        updates, Sleijpen and van der Vorst 1996); convergence is decided on the FP64
                        true residual.  A column whose best FP64 residual has not fallen tenfold over
                        30 replacements, or that ran 1000 FP32 iterations without a replacement, is
                        solved again in FP64 (stats.fallback_columns).  With RST_IDRS (and wide planes
                        under RST_BICGSTAB): FP64 iterative refinement, x += d where d comes from an
                        IDR(s) run on complex64 vectors (FP64 arithmetic, FP32 stencil) for the current
                        FP64 residual r = b - A x to the relative tolerance update_delta; stats
                        updates_total counts the cycles, iterations_total all inner applies.  A column
                        ends unconverged when three cycles in a row fail to halve its FP64 residual.
                        RST_BICGSTAB_MC refuses it (RST_EUNSUPPORTED) */
  double tol;        /* stop when the FP64 true residual ||b - A x|| <= tol ||b|| per column (default 1e-10) */
  int max_iter;      /* BiCGSTAB iterations per column (default 20000) */
  int col_block;     /* columns solved together by one workgroup; 0 = automatic (FGMRES and COCG: 1) */
  int threads;       /* workgroup size (multiple of 64, <= 512); 0 = automatic */
  int direction;     /* RST_DIR_LR: columns in the right CAP, T accumulated on the left (default);
                        RST_DIR_RL: the reverse.  Both give the same T (exact identity). */
  double update_delta; /* RST_FP32_REFINE: the residual is replaced once its norm is below update_delta
                          times the largest since the last replacement (default 0.1, in (0, 1)); under
                          RST_IDRS the relative tolerance of each complex64 correction solve (values
                          near 1e-4 to 1e-5 take the fewest cycles) */
  int precond;       /* rst_precond.  RST_PRECOND_FREE_CAP: right preconditioner
                        M = E - (-1/2 L_lat - 1/2 D2_z + Vref(z)) + i Gamma(z) with the exact
                        lateral FD Laplacian (diagonal in the twisted lateral Fourier basis),
                        the three-point z Laplacian and the reference potential Vref (pc_vref);
                        applied by lateral DFTs and one tridiagonal solve per lateral mode.  RST_PRECOND_LEARNED (RST_FGMRES
                        only): z = M^-1 r + f(r, M^-1 r) with the context's network f (rst_cnn_*).
                        Default NONE. */
  int restart;       /* RST_FGMRES: Krylov steps per cycle (default 30, 1..200) */
  double fallback_ratio; /* RST_PRECOND_LEARNED: a column whose true residual after a cycle is above
                            fallback_ratio times the previous cycle's continues with M^-1 alone
                            (default 0.5, in (0, 1]) */
  int pc_vref;       /* rst_vref, the preconditioner's reference potential.  RST_VREF_PLANE (default):
                        Vref(z) = the mean of V over plane z, which keeps M separable (lateral modes
                        still do not mix) and follows a potential that changes along the transport
                        axis (a constriction, vacuum padding); RST_VREF_CELL: Vref = the mean of V
                        over the cell. */
  int idr_s;         /* RST_IDRS: dimension s of the shadow space (default 4, 1..8) */
  double pc_shift;   /* imaginary shift eta >= 0 (Ha) added to the CAP inside the preconditioner only,
                        M(eta) = M + i eta: damps the reference operator's standing waves between the
                        CAPs of a long slab (a shifted-Laplacian preconditioner); default 0 */
} rst_solver_opts;

/* Statistics of the last rst_transmission / rst_solve_columns call. */
typedef struct {
  int64_t columns;          /* column solves performed */
  int64_t columns_unconverged;
  int64_t iterations_total; /* BiCGSTAB iterations summed over columns */
  int32_t iterations_max;   /* RST_FGMRES: Arnoldi steps; restarts_total then counts cycles */
  int32_t restarts_total;   /* breakdown restarts */
  double max_rel_residual;  /* largest FP64 true relative residual */
  double kernel_ms;         /* device time of the solver kernel(s) */
  double bytes_algorithmic; /* algorithmic HBM bytes of the Krylov sweeps: FP64 BiCGSTAB 12 (plain) or
                               24 (preconditioned) complex128 streams per grid point, iteration and
                               column; RST_FP32_REFINE the same counts of complex64 streams plus
                               72 B per grid point and reliable update */
  int64_t updates_total;     /* RST_FP32_REFINE: FP64 residual replacements summed over columns */
  int32_t col_block;         /* columns per workgroup used by the launch */
  int32_t threads;           /* workgroup size used by the launch */
  int64_t fallback_columns;  /* RST_PRECOND_LEARNED: columns switched to M^-1 alone;
                                RST_FP32_REFINE: columns solved again by the FP64 kernel because the
                                FP32 recurrences stopped making progress */
  double cnn_flop;           /* RST_PRECOND_LEARNED: network flops (2 per multiply-add) */
} rst_stats;

/* One structure of a batch (rst_batch_add).  The lateral grid, spacings and
 * FD order are the context's (rst_set_grid; its nz is ignored here); each
 * structure has its own plane count, potential, CAPs, lateral k and energies.
 * Host arrays are copied by rst_batch_add. */
typedef struct {
  int nz;                  /* planes of this structure (>= 1) */
  const double *v;         /* na*nb*nz potential (Ha) */
  const double *gamma_l;   /* nz left CAP (Ha, >= 0) */
  const double *gamma_r;   /* nz right CAP (Ha, >= 0) */
  double ka, kb;           /* lateral Bloch vector (bohr^-1) */
  int n_e;                 /* energies of this structure */
  const double *energies;  /* n_e (Ha) */
} rst_problem;

void rst_default_solver(rst_solver_opts *opts);

/* Creates a context on HIP device `hip_device` into *out.  `hip_stream` (a
 * hipStream_t) may be NULL, in which case the context creates and owns a
 * stream; a caller's stream stays the caller's.  RST_EINVAL for a null out,
 * RST_EDEVICE for a device that does not exist or a failed stream creation
 * (*out is then NULL). */
rst_status rst_create(rst_ctx **out, int hip_device, void *hip_stream);
/* Frees the context and every device buffer it allocated (NULL is ignored). */
void rst_destroy(rst_ctx *ctx);
/* Message of the last failed call on ctx, owned by the context and valid until
 * its next call. */
const char *rst_last_error(const rst_ctx *ctx);

/* Grid of na x nb x nz points with spacings ha, hb, hz (bohr); fd_order even
 * in 2..12 (the order-2M central Laplacian of the Bloch-form equation).
 * RST_EINVAL for non-positive sizes or spacings, another order, or more than
 * 2^31 - 1 points.  The GPU kernels require na > fd_order/2 and
 * nb > fd_order/2 (RST_EUNSUPPORTED otherwise).  Every order runs on the
 * many-column apply and solvers (rst_apply_h, rst_transmission and the calls
 * built on it route orders other than 4 and 12 there); the persistent
 * kernels (the blocked apply, FGMRES, COCG, the batched launch) are built for
 * orders 4 and 12 and return RST_EUNSUPPORTED for the others. */
rst_status rst_set_grid(rst_ctx *ctx, int na, int nb, int nz, double ha, double hb, double hz,
                        int fd_order);

/* Local potential V, n = na*nb*nz doubles (Ha), host memory, copied: the
 * local part of the Kohn-Sham effective potential V_KS(x, y, z), periodic in
 * the lateral plane (Sec. II.A, preliminaries), sampled on the grid and added
 * to the diagonal of H_KS in G(E) = [E - H_KS + i Gamma]^-1 (ibid.).
 * RST_ESTATE before rst_set_grid; RST_EINVAL for NULL or a non-finite value. */
rst_status rst_set_potential(rst_ctx *ctx, const double *v);

/* The nonlocal part of the norm-conserving pseudopotentials (s, p and d
 * channels inside per-channel cutoff radii, Sec. IV.A bulk Cu and Sec. V.A
 * bulk Rh), in separable Kleinman-Bylander form h^3 sum_p E_p |beta_p><beta_p|;
 * the lateral images carry the Bloch phase exp(+i k.R) of the Bloch-form
 * equation (Sec. II.A).  Compressed rows over projectors: entries
 * offs[p]..offs[p+1]-1 of projector p.  pt[e] is a grid index, img[2e],
 * img[2e+1] the lateral image (ia, ib) the entry comes from, beta[e] its real
 * value; e_kb[p] the projector energy (Ha).  nproj may be 0.  Host arrays,
 * copied.  RST_ESTATE before rst_set_grid; RST_EINVAL for nproj < 0, a null
 * array with nproj > 0, offs not non-decreasing from 0, a grid index outside
 * 0..n-1, or a non-finite beta or e_kb. */
rst_status rst_set_projectors(rst_ctx *ctx, int nproj, const int32_t *offs, const int32_t *pt,
                              const int8_t *img, const double *beta, const double *e_kb);

/* CAP strengths Gamma_L(iz), Gamma_R(iz) >= 0 (nz doubles each, Ha), copied
 * (the absorbing terms of the retarded Green's function, Sec. II.A).  The
 * solve columns of RST_DIR_LR are all grid points of the planes with
 * Gamma_R > 0 (RST_DIR_RL: Gamma_L > 0).  RST_ESTATE before rst_set_grid;
 * RST_EINVAL for NULL, a negative or a non-finite value. */
rst_status rst_set_abc(rst_ctx *ctx, const double *gamma_l_z, const double *gamma_r_z);

/* Lateral Bloch vector (bohr^-1) along a and b (the phases exp(i k_a L_a),
 * exp(i k_b L_b) of the Bloch-form equation).  RST_ESTATE before
 * rst_set_grid; RST_EINVAL for a non-finite component. */
rst_status rst_set_k(rst_ctx *ctx, double ka, double kb);

/* Copies the solver options (rst_solver_opts above).  RST_EINVAL for NULL, an
 * unknown method, precision, direction or preconditioner, tol <= 0,
 * max_iter < 1, a col_block other than 0 or a power of two <= 8, threads not 0
 * or a multiple of 64 <= 512, update_delta outside (0, 1), restart outside
 * 1..200 (FGMRES), fallback_ratio outside (0, 1] or the learned
 * preconditioner with another method than FGMRES; RST_EUNSUPPORTED for
 * FGMRES or COCG with RST_FP32_REFINE. */
rst_status rst_set_solver(rst_ctx *ctx, const rst_solver_opts *opts);

/* T(E_j, k) for j < n_e into T_out (host, caller-allocated, n_e doubles).
 * Returns RST_ENOCONV if any column missed the tolerance (T is still written). */
rst_status rst_transmission(rst_ctx *ctx, int n_e, const double *energies, double *T_out,
                            rst_stats *stats);

/* k-averaged transmission T(E) = (1/n_k) sum_k T(E, k) over the lateral k-points
 * kpts (host, n_k pairs (ka, kb) in bohr^-1), each T(E, k) by rst_transmission
 * (the k-point average of the paper's transmission over the lateral Brillouin
 * zone).  With fold != 0 a k-point equal to an earlier one, or to its negative,
 * modulo a reciprocal lattice vector 2 pi / L is not solved again: T(k + G) =
 * T(k) (Bloch periodicity) and T(-k) = T(k) (H_-k = conj(H_k) for real V,
 * beta and E_KB, so G_-k = G_k^T and the trace is unchanged) make this exact.
 * T_out (n_e) gets the average; T_k (nullable, n_k x n_e, row per k-point) the
 * per-k values; n_solved (nullable) the number of k-points actually solved;
 * stats (nullable) sums columns, iterations, kernel time and bytes over them.
 * The caller's k is restored.  Grid, potential and CAPs must be set; k need
 * not be.  RST_EINVAL for n_k < 1, a null or non-finite input; RST_ENOCONV if
 * any column hit the iteration cap (all outputs written). */
rst_status rst_transmission_kavg(rst_ctx *ctx, int n_k, const double *kpts, int fold, int n_e,
                                 const double *E, double *T_out, double *T_k, int *n_solved,
                                 rst_stats *stats);

/* y = (E - H_k + i Gamma) x for an (n x ncol) block, column fastest (element
 * (gi, c) at gi*ncol + c): the FD Laplacian with Bloch-phase lateral wraps, V,
 * the CAPs and the KB projectors (Bloch-form and transmission equations).
 * precision RST_FP64: complex128 x and y (n*ncol*16 bytes each), FP64
 * arithmetic.  RST_FP32_REFINE: complex64 x and y (n*ncol*8 bytes each), the
 * stencil in FP32; the projections h^3 B^H x are formed in FP64 from the
 * widened x, and the projector term is summed in FP64 and rounded once.
 * x_dev and y_dev are distinct device buffers; a projection buffer of
 * nproj*ncol*16 bytes is grown on demand.  Any lateral size (one wavefront
 * per grid point and 64 columns).  RST_EINVAL for x == y, a negative ncol, a
 * non-finite energy or another precision. */
rst_status rst_apply_h(rst_ctx *ctx, double energy, const void *x_dev, void *y_dev, int ncol,
                       int precision);

/* rst_apply_h without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operator, kernels, layouts, precisions and results as
 * rst_apply_h, with the projections h^3 B^H x kept in a fixed 16 MiB scratch array
 * that the library holds on each device until the process ends (nproj * ncol
 * complex128 values must fit: with 360 projectors up to 2912 columns, with 3420
 * up to 306; RST_EINVAL beyond, with the limit in rst_last_error).  Calls no
 * hipMalloc or hipFree and records no timing (rst_apply_timing is not updated).
 * Every call on one device shares that device's scratch array: calls that
 * overlap in time on one GPU (other threads, other contexts, other streams) race
 * and must be serialised by the caller.  Returns after the context's stream has
 * finished.  Errors as rst_apply_h; RST_EDEVICE if the scratch address of the
 * device could not be obtained. */
rst_status rst_apply_h_noalloc(rst_ctx *ctx, double energy, const void *x_dev, void *y_dev, int ncol,
                               int precision);

/* Widest column block the blocked apply supports on the current grid (a power
 * of two <= 8: a lateral plane of col_block columns must fit one workgroup at
 * two positions per thread, its padded copy the LDS).  RST_ESTATE before the
 * problem is set. */
rst_status rst_apply_block_width(rst_ctx *ctx, int *col_block);

/* y = (E - H_k + i Gamma) x in the blocked layout the solvers keep their
 * vectors in: ncol columns in ncol/col_block blocks of col_block columns; block
 * j occupies elements [j*n*col_block, (j+1)*n*col_block) and holds column
 * j*col_block + c of grid point gi at j*n*col_block + gi*col_block + c
 * (complex128, device).  The projections h^3 B^H x are formed first on the
 * FP64 matrix cores, into per-block arrays; then one workgroup streams z
 * through each block (the operator of the transmission equation's
 * G, with H_k the FD Laplacian with Bloch-phase lateral wraps, V and the KB
 * projectors).  RST_EINVAL if ncol is not a multiple of col_block, col_block is
 * not a power of two <= 8 or x == y; RST_EUNSUPPORTED if col_block exceeds
 * rst_apply_block_width. */
rst_status rst_apply_h_blocked(rst_ctx *ctx, double energy, const void *x_dev, void *y_dev, int ncol,
                               int col_block);

/* Kernel durations of the last rst_apply_h or rst_apply_h_blocked on this context, measured with HIP
 * events on the context's stream: the projector gather h^3 B^H x on the FP64
 * matrix cores (0 without projectors) and the stencil sweep.
 * Both 0 before the first apply.  RST_EINVAL for a null argument. */
rst_status rst_apply_timing(const rst_ctx *ctx, double *proj_ms, double *stencil_ms);

/* Green's function columns: x_dev[:, j] = G e_{col[j]} (complex128, n x ncol,
 * column fastest, device, caller-allocated; the retarded G of Sec. II.A) with
 * the context's solver options.  col holds ncol grid indices (host).
 * RST_EINVAL for ncol < 0, NULL arguments, an index outside 0..n-1 or a
 * non-finite energy; RST_ESTATE before the problem is set; RST_ENOCONV if a
 * column missed the tolerance (x is still written). */
rst_status rst_solve_columns(rst_ctx *ctx, double energy, int ncol, const int64_t *col,
                             void *x_dev, rst_stats *stats);

/* General right-hand sides: for every energy e < n_e and column j < ncol,
 * x_dev[gi, e, j] = (G(E_e) b_{e,j})[gi] with b_{e,j}[gi] = rhs_dev[gi, e*rhs_estride + j]
 * (complex128 device arrays; rhs_dev has ld = ncol if rhs_estride = 0, i.e. the same
 * right-hand sides for every energy, else ld = n_e*ncol with rhs_estride = ncol;
 * x_dev is (n x n_e*ncol), element (gi, e, j) at gi*(n_e*ncol) + e*ncol + j).
 * FP64 BiCGSTAB only (RST_EUNSUPPORTED otherwise); the shadow residual is
 * e_j0 with j0 = argmax |b|. */
rst_status rst_solve_rhs(rst_ctx *ctx, int n_e, const double *energies, int ncol, const void *rhs_dev,
                         int64_t rhs_estride, void *x_dev, rst_stats *stats);

/* Low-rank transmission: T = 4 ||M||_F^2 with M = Gamma_L^1/2 G Gamma_R^1/2 on the
 * left-CAP rows and right-CAP columns (the transmission equation written as a
 * Frobenius norm), by a randomised range finder instead of one solve per
 * right-CAP column: Y = M Omega from probes + heldout solves with complex
 * Gaussian right-hand sides on the right CAP; Q = orth(first probes columns of Y)
 * (Cholesky QR twice); T = 4 ||Q^H M||_F^2 from probes solves at -k
 * (G_k^H = conj(G_{-k})).  T_err[e] = 4 mean ||(I - QQ^H) y||^2 over the held-out
 * probes, an estimate of the neglected part (T_true = T + neglected >= T); while
 * it exceeds tail_tol the probe count doubles (up to max_probes).  Returns
 * RST_ENOCONV when a solve missed the tolerance or an energy ended above tail_tol.
 * FP64 BiCGSTAB (RST_BICGSTAB or RST_BICGSTAB_MC).  With direction RST_DIR_RL
 * the two CAPs exchange roles: T_RL = 4 ||Gamma_R^1/2 G Gamma_L^1/2||_F^2, equal
 * to T_LR for any Hermitian H_k and real CAPs. */
typedef struct {
  int probes;        /* initial probe count s (default 32) */
  int heldout;       /* held-out probes p for the tail estimate (default 8) */
  int max_probes;    /* largest s (default 256) */
  double tail_tol;   /* accepted 4 ||(I - QQ^H) M||_F^2 estimate (default 1e-7) */
  uint64_t seed;
} rst_lowrank_opts;
void rst_default_lowrank(rst_lowrank_opts *opts);
rst_status rst_transmission_lowrank(rst_ctx *ctx, int n_e, const double *energies, const rst_lowrank_opts *opts,
                                    double *T_out, double *T_err, rst_stats *stats);

/* Eigen route (paper Sec. II.A, the transmission trace in the eigenbasis of
 * G^-1; Sec. II.B-II.D and the Appendix, the eigenpairs of +k and -k): the
 * n_eig eigenpairs of K_k = H_k - i Gamma nearest sigma by shift-invert subspace
 * iteration (blocks of solves with G(sigma) = (sigma - K_k)^-1 on the context's
 * FP64 solver, orthonormalised by Cholesky QR twice) and Rayleigh-Ritz on the
 * subspace (the small eigenproblem by Hessenberg reduction and shifted QR on the
 * host), left eigenvectors as the conjugated right eigenvectors of K_{-k} matched
 * by eigenvalue (K_k^T = K_{-k}; at a k equal to -k modulo a reciprocal vector
 * the same run serves), normalised to L^H R = I; then for every energy
 *     T(E) = 4 sum_{m,n} GtL[m,n] GtR[n,m] / ((E - lam_n)(E - lam_m)^*),
 *     GtL = R^H Gamma_L R,  GtR = L^H Gamma_R L.
 * With n_eig equal to the grid size the sum is T exactly; with fewer it is the
 * paper's partial diagonalisation.  eig_out (nullable, 2*n_eig doubles) gets the
 * eigenvalues (re, im), nearest sigma first.  stats->max_rel_residual is the
 * largest relative eigenpair residual ||K x - lam x|| / max(1, |lam|),
 * restarts_total the subspace iterations.  RST_ENOCONV if the residuals stay
 * above tol after max_iter iterations (outputs written).  Solver options as for
 * the transmission (FP64 BiCGSTAB or IDR(s)); the caller's k is restored. */
typedef struct {
  int n_eig;         /* eigenpairs in the trace (default 32, 1..min(512, n)) */
  int subspace;      /* subspace dimension (0: min(n, 2 n_eig + 16); at most 1024) */
  int max_iter;      /* subspace iterations per Bloch vector (default 40) */
  double sigma;      /* target energy (Ha); the eigenvalues nearest it are taken (default 0) */
  double tol;        /* relative eigenpair residual accepted (default 1e-8) */
  uint64_t seed;     /* random start block */
} rst_eig_opts;
void rst_default_eig(rst_eig_opts *opts);
rst_status rst_transmission_eigen(rst_ctx *ctx, int n_e, const double *energies, const rst_eig_opts *opts,
                                  double *T_out, double *eig_out, rst_stats *stats);

/* Batched transmission (paper Appendix: the (k, spin) calculations are
 * independent; here every (structure, energy, column block) is a work item of
 * one persistent launch).  rst_batch_clear empties the batch; rst_batch_add
 * appends a structure (RST_EUNSUPPORTED if the context has projectors: the
 * batch path carries local potentials only); rst_batch_run computes T for
 * every (structure, energy) into T_out (host, sum of n_e doubles, in the order
 * the structures were added) with the context's solver options (FP64
 * BiCGSTAB, with or without the free-electron + CAP preconditioner).  With col_block = 0 the columns per workgroup are
 * chosen by timing the candidates on a sample of the batch (cached per lateral
 * shape); the launch is captured in a HIP graph and replayed while the batch is
 * unchanged.  When every structure alone has at least 64 column items per
 * compute unit (columns x energies), the structures run instead as
 * single-structure launches back to back on the context's stream (one column
 * per workgroup unless col_block says otherwise): such work already fills the
 * device, where the single-structure kernel is the faster one. */
rst_status rst_batch_clear(rst_ctx *ctx);
rst_status rst_batch_add(rst_ctx *ctx, const rst_problem *prob);
rst_status rst_batch_run(rst_ctx *ctx, double *T_out, rst_stats *stats);

/* ---- Learned correction network of the learned preconditioner ----------------
 * A three-level 3D U-Net f (16 channels, 3x3x3 convolutions without biases,
 * ReLU, 2x2x2 mean pooling over the existing children, nearest upsampling with
 * additive skips; layers W0..W8) maps the four channels (Re r, Im r, Re m, Im m)
 * of a residual r and m = M^-1 r (M the free-electron + CAP preconditioner) to
 * a two-channel correction: the learned preconditioner is z = m + f(r, m).
 * Convolutions are cross-correlations, periodic laterally and zero beyond the
 * end planes along z.  Tensors are FP32 channel-last device arrays:
 * element (column c, grid point p, channel ch) at (c*n + p)*C + ch with
 * p = (iz*nb + ib)*na + ia.  Weights (host, FP32) are the layers W0..W8 one
 * after another, each (cout, cin, 3, 3, 3) row-major, taps (dz, db, da) with
 * dz slowest; (cout, cin) = (16, 4), (16, 16) x 7, (2, 16).
 * The GPU evaluates the convolutions on FP32 matrix cores. */
int64_t rst_cnn_weight_count(void);
/* He-normal weights from `seed` (last layer scaled by 0.1); resets Adam. */
rst_status rst_cnn_seed(rst_ctx *ctx, uint64_t seed);
rst_status rst_cnn_set_weights(rst_ctx *ctx, const float *w, int64_t count);
rst_status rst_cnn_get_weights(rst_ctx *ctx, float *w, int64_t count);
/* out_dev [ncol][n][2] = f(x_dev [ncol][n][4]) on an nz x nb x na grid (n = nz*nb*na). */
rst_status rst_cnn_forward(rst_ctx *ctx, int ncol, int nz, int nb, int na, const float *x_dev, float *out_dev);
/* grad (host, rst_cnn_weight_count() floats, weight layout) = d<gout, f(x)>/dW for
 * gout_dev [ncol][n][2]. */
rst_status rst_cnn_gradient(rst_ctx *ctx, int ncol, int nz, int nb, int na, const float *x_dev,
                            const float *gout_dev, float *grad);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) on L = (1/ncol) sum_c ||f(x_c) - target_c||^2;
 * *loss = L before the step.  target_dev [ncol][n][2]. */
rst_status rst_cnn_train_step(rst_ctx *ctx, int ncol, int nz, int nb, int na, const float *x_dev,
                              const float *target_dev, float lr, double *loss);

/* Training of the network (Adam on FP32 weights).  Each step draws one energy
 * from `energies` and one lateral k from `kpts` (n_k pairs (ka, kb)), then
 * `batch` pairs (r, e) with A e = r, A = E - H_k + i Gamma; input (r, M^-1 r),
 * target e - M^-1 r, both scaled so that ||r|| = 1 (synthetic pairs) or
 * ||e|| = 1 (solver pairs).
 * source 0 (synthetic): xi complex normal (SplitMix64 counter-based,
 * Box-Muller), e = M^-1 xi, r = A e.
 * source 1 (solver): `batch` right-CAP columns b = e_c drawn at random; x* from
 * the FP64 preconditioned BiCGSTAB to 1e-10, then the iterates x_j after j =
 * 2, 4, 8, ..., 64 iterations of the same solver; pairs r_j = b - A x_j,
 * e_j = x* - x_j (the residuals and errors the solver actually leaves), one
 * Adam step per iterate.
 * steps = ceil(pairs / batch).  Starts from the context's weights (seeded from
 * `seed` if it has none); the context's k and solver options are restored on
 * return. */
typedef struct {
  int pairs;               /* training pairs */
  int batch;               /* pairs per Adam step, 1..64 */
  float lr;                /* Adam step size */
  uint64_t seed;
  int n_e;
  const double *energies;  /* host, n_e (Ha) */
  int n_k;
  const double *kpts;      /* host, 2*n_k (bohr^-1) */
  int source;              /* 0: synthetic pairs (default), 1: pairs from solver runs */
} rst_train_opts;
typedef struct {
  int steps;
  double loss_first;       /* mean loss of the first min(10, steps/4) steps */
  double loss_last;        /* mean loss of the last min(10, steps/4) steps */
  double ms;               /* device time */
} rst_train_stats;
rst_status rst_precond_train(rst_ctx *ctx, const rst_train_opts *opts, rst_train_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* RST_H */
