"""Plain FP64 CPU oracle for the Bloch-CAP transmission T(E, k).

TEST INFRASTRUCTURE ONLY.  This module is the reference the GPU library is
checked against.  Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product path never does.

What it computes (paper, Sec. II.A):
  * transmission T = Tr{ G Gamma_R G^dagger Gamma_L } with the retarded Green's
    function G = [E - H + i Gamma]^-1 and Gamma = Gamma_L + Gamma_R
    (transmission equation and the definition of G that follows it); with the
    normalisation read as a factor 4 so that one open channel gives T = 1;
  * H restricted to one lateral Bloch vector k: states of Bloch form
    u(x) exp(i k.x) (Bloch-form equation) represented on the home cell by
    twisted boundary conditions, phi(r + R) = exp(+i k.R) phi(r);
  * the k-average of T_k(E) (end of Sec. II.A).
H_k = -1/2 L_k + diag(V) + h^3 sum_p E_p |beta_k,p><beta_k,p| where L_k is the
central finite-difference Laplacian of even order 2M with Bloch-phase wraps on
the lateral faces and Dirichlet (psi = 0) outside the planes 0..Nz-1 in z.

Everything is written from the definitions: H is assembled densely and the
linear systems are solved by LU factorisation (LAPACK through scipy), one
factorisation per (E, k).  No blocking, fusion or reordering beyond that.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# Finite-difference second-derivative weights (central, order 2M)
# ----------------------------------------------------------------------------

def fd_second_derivative(order: int) -> np.ndarray:
    """Weights c_0..c_M of the central order-2M second derivative,
    f''(x) ~ h^-2 sum_{j=-M..M} c_|j| f(x + j h).

    Closed form c_j = 2 (-1)^(j+1) (M!)^2 / (j^2 (M-j)! (M+j)!) for j >= 1 and
    c_0 = -2 sum_{j>=1} c_j (the paper states no order; this is the standard
    high-order stencil used by real-space codes)."""
    if order % 2 or order < 2:
        raise ValueError("order must be even and >= 2")
    m = order // 2
    c = np.zeros(m + 1)
    fm = math.factorial(m)
    for j in range(1, m + 1):
        c[j] = 2.0 * (-1) ** (j + 1) * fm * fm / (j * j * math.factorial(m - j) * math.factorial(m + j))
    c[0] = -2.0 * c[1:].sum()
    return c


def fd_dispersion(order: int, theta):
    """s_M(theta) = -c_0 - 2 sum_j c_j cos(j theta): the symbol of -h^2 d^2/dx^2."""
    c = fd_second_derivative(order)
    theta = np.asarray(theta, dtype=float)
    s = -c[0] * np.ones_like(theta)
    for j in range(1, c.size):
        s = s - 2 * c[j] * np.cos(j * theta)
    return s


# ----------------------------------------------------------------------------
# Operator assembly
# ----------------------------------------------------------------------------

def _grid_coords(prob):
    n = prob.n
    i = np.arange(n)
    ia = i % prob.na
    ib = (i // prob.na) % prob.nb
    iz = i // (prob.na * prob.nb)
    return i, ia, ib, iz


def _laplacian_triplets(prob, k, kz=None):
    """(row, col, value) triplets of L_k.  Lateral neighbours wrap with the
    Bloch phase exp(i k_d L_d q) for q = floor((i_d + j)/N_d) (any number of
    wraps).  Along z the neighbour is dropped outside [0, Nz) unless kz is given,
    in which case z wraps with exp(i kz Lz q) (used only for bulk band structure)."""
    c = fd_second_derivative(prob.order)
    m = c.size - 1
    i, ia, ib, iz = _grid_coords(prob)
    dims = [(ia, prob.na, prob.ha, k[0], 1),
            (ib, prob.nb, prob.hb, k[1], prob.na),
            (iz, prob.nz, prob.hz, kz, prob.na * prob.nb)]
    rows, cols, vals = [], [], []
    for d, (idx, nd, hd, kd, stride) in enumerate(dims):
        ld = nd * hd
        for j in range(-m, m + 1):
            w = c[abs(j)] / (hd * hd)
            t = idx + j
            q = np.floor_divide(t, nd)
            tw = t - q * nd
            if d == 2 and kz is None:
                keep = (t >= 0) & (t < nd)
                phase = np.ones(keep.sum(), complex)
                r = i[keep]
                cc = r + (tw[keep] - idx[keep]) * stride
            else:
                phase = np.exp(1j * kd * ld * q)
                r = i
                cc = i + (tw - idx) * stride
            rows.append(r)
            cols.append(cc)
            vals.append(w * phase)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def bloch_projectors(prob, k) -> sp.csc_matrix:
    """n x nproj matrix of beta_k,p(r_i) = sum_{entries at i} beta_e exp(+i k.R_e),
    R_e = (img_a L_a, img_b L_b) the lateral image the entry comes from."""
    pj = prob.proj
    if pj.nproj == 0:
        return sp.csc_matrix((prob.n, 0), dtype=complex)
    col = np.repeat(np.arange(pj.nproj), np.diff(pj.offs))
    ph = np.exp(1j * (k[0] * prob.la * pj.img[:, 0].astype(float)
                      + k[1] * prob.lb * pj.img[:, 1].astype(float)))
    return sp.csc_matrix((pj.beta * ph, (pj.pt, col)), shape=(prob.n, pj.nproj))


def hamiltonian_sparse(prob, k, kz=None) -> sp.csr_matrix:
    """Local part -1/2 L_k + diag(V) as a sparse matrix (duplicates summed)."""
    r, c, v = _laplacian_triplets(prob, k, kz)
    lap = sp.csr_matrix((v, (r, c)), shape=(prob.n, prob.n))
    return (-0.5) * lap + sp.diags(prob.v.astype(complex))


def hamiltonian_dense(prob, k, kz=None) -> np.ndarray:
    """Dense complex128 H_k (tiny grids only)."""
    h = hamiltonian_sparse(prob, k, kz).toarray()
    if prob.proj.nproj:
        b = bloch_projectors(prob, k).toarray()
        h3 = prob.ha * prob.hb * prob.hz
        h += h3 * (b * prob.proj.ekb[None, :]) @ b.conj().T
    return h


def system_matrix(prob, k, e) -> np.ndarray:
    """A = E - H_k + i(Gamma_L + Gamma_R), dense."""
    a = -hamiltonian_dense(prob, k)
    gz = np.repeat(prob.gamma_l + prob.gamma_r, prob.na * prob.nb)
    a[np.diag_indices(prob.n)] += e + 1j * gz
    return a


def apply_system(prob, k, e, x) -> np.ndarray:
    """y = (E - H_k + i Gamma) x evaluated from the factored definition (sparse
    local part plus the low-rank projector part); any grid size.  x: (n, ncol)."""
    x = np.asarray(x, complex)
    if x.ndim == 1:
        x = x[:, None]
    e = np.broadcast_to(np.asarray(e, float), (x.shape[1],))
    hl = hamiltonian_sparse(prob, k)
    gz = np.repeat(prob.gamma_l + prob.gamma_r, prob.na * prob.nb)
    y = -(hl @ x) + (1j * gz)[:, None] * x + x * e[None, :]
    if prob.proj.nproj:
        b = bloch_projectors(prob, k)
        h3 = prob.ha * prob.hb * prob.hz
        proj = (b.conj().T @ x) * prob.proj.ekb[:, None]
        y -= h3 * (b @ proj)
    return y


# ----------------------------------------------------------------------------
# Transmission
# ----------------------------------------------------------------------------

def _gz(prob, which):
    g = prob.gamma_l if which == "L" else prob.gamma_r
    return np.repeat(g, prob.na * prob.nb)


def transmission(prob, energies, k, both=True):
    """T(E, k) for each E by LU-factorising A once per energy.

    T_LR = 4 sum_{i in R} sum_{j in L} Gamma_L,j |x_i[j]|^2 with
    x_i = A^-1 (sqrt(Gamma_R,i) e_i); T_RL the same with L and R exchanged.
    Returns dict(T_LR, T_RL, rcond, near_singular) of arrays over energies.

    Near-singular energies (a state decoupled from both CAPs makes A almost
    singular there, so T is ill-conditioned) are flagged: rcond is LAPACK's
    1-norm reciprocal condition estimate of A from its LU factors, and an energy
    is flagged when rcond < 1e-12 or, with both directions, when |T_LR - T_RL|
    exceeds 1e-9 max(1, T_LR) (the two are equal for any nonsingular A)."""
    energies = np.atleast_1d(np.asarray(energies, float))
    gl, gr = _gz(prob, "L"), _gz(prob, "R")
    rcols, lcols = prob.r_columns(), prob.l_columns()
    base = -hamiltonian_dense(prob, k)
    base[np.diag_indices(prob.n)] += 1j * (gl + gr)
    t_lr = np.zeros(energies.size)
    t_rl = np.zeros(energies.size)
    rcond = np.zeros(energies.size)
    for ie, e in enumerate(energies):
        a = base.copy()
        a[np.diag_indices(prob.n)] += e
        anorm = float(np.max(np.sum(np.abs(a), axis=0)))
        lu = sla.lu_factor(a, overwrite_a=True, check_finite=False)
        rcond[ie] = float(lapack.zgecon(lu[0], anorm, norm="1")[0])
        b = np.zeros((prob.n, rcols.size), complex)
        b[rcols, np.arange(rcols.size)] = np.sqrt(gr[rcols])
        x = sla.lu_solve(lu, b, check_finite=False)
        t_lr[ie] = 4.0 * float(np.sum(gl[:, None] * np.abs(x) ** 2))
        if both:
            b = np.zeros((prob.n, lcols.size), complex)
            b[lcols, np.arange(lcols.size)] = np.sqrt(gl[lcols])
            x = sla.lu_solve(lu, b, check_finite=False)
            t_rl[ie] = 4.0 * float(np.sum(gr[:, None] * np.abs(x) ** 2))
    flag = rcond < 1e-12
    if both:
        flag |= np.abs(t_lr - t_rl) > 1e-9 * np.maximum(1.0, t_lr)
    return dict(T_LR=t_lr, T_RL=t_rl if both else None, rcond=rcond, near_singular=flag)


def green_columns(prob, e, k, cols) -> np.ndarray:
    """Columns G e_c of G = A^-1 for the grid indices in cols: (n, len(cols))."""
    a = system_matrix(prob, k, e)
    b = np.zeros((prob.n, len(cols)), complex)
    b[np.asarray(cols), np.arange(len(cols))] = 1.0
    return sla.solve(a, b, check_finite=False)


def trace_forms(prob, e, k):
    """Full-inverse forms on tiny grids: 4 Tr[Gamma_L G Gamma_R G^+] written as
    4 sum_ij Gamma_L,i |G_ij|^2 Gamma_R,j, and the two terms of the CAP sum rule
    -4 Im Tr[Gamma_L G] and 4 Tr[Gamma_L G Gamma_L G^+]."""
    a = system_matrix(prob, k, e)
    g = np.linalg.inv(a)
    gl, gr = _gz(prob, "L"), _gz(prob, "R")
    g2 = np.abs(g) ** 2
    t = 4.0 * float(np.sum(gl[:, None] * g2 * gr[None, :]))
    t_rl = 4.0 * float(np.sum(gr[:, None] * g2 * gl[None, :]))
    im_tr = -4.0 * float(np.sum(gl * np.imag(np.diag(g))))
    t_ll = 4.0 * float(np.sum(gl[:, None] * g2 * gl[None, :]))
    return dict(T=t, T_RL=t_rl, minus4_im_tr_GLG=im_tr, T_LL=t_ll)


def residual_norms(prob, k, e, x, b):
    """Per-column true relative residual ||b - A x|| / ||b||."""
    r = b - apply_system(prob, k, e, x)
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)
