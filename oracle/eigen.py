"""Eigen route of the transmission: T(E, k) from eigenpairs of H_k - i Gamma.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the product path
never imports it.

What it computes (paper Sec. II.A, transmission in the eigenbasis of G^-1;
Sec. II.B-II.D and the Appendix for the Bloch case):
  K_k = H_k - i Gamma has right eigenvectors R (K R = R diag(lam)) and left
  eigenvectors L (L^H K = diag(lam) L^H) with L^H R = I, so that
      G(E) = (E - K)^-1 = R diag(1/(E - lam)) L^H .
  Substituting into T = 4 Tr[Gamma_L G Gamma_R G^+] (the factor 4 as in the
  transport module) gives
      T(E) = 4 sum_{m,n} GtL[m,n] GtR[n,m] / ((E - lam_n) (E - lam_m)^*),
      GtL = R^H Gamma_L R,   GtR = L^H Gamma_R L,
  the paper's eigenbasis trace with the transformed CAPs.  Restricting m, n to
  a subset of the eigenpairs (those nearest the energies of interest) is the
  paper's partial diagonalisation; with all N pairs the sum is T exactly.
  Left eigenvectors from the opposite Bloch vector: K_k^T = K_{-k} (H_k^T =
  conj(H_k) = H_{-k} for real V, beta and E_KB, and Gamma is real diagonal), so
  the left eigenvectors of K_k are the conjugated right eigenvectors of K_{-k}
  for the same eigenvalues (the paper's matching of +k and -k eigenpairs).

Everything is dense (scipy.linalg.eig): tiny grids only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .transport import hamiltonian_dense


def k_matrix(prob, k) -> np.ndarray:
    """K_k = H_k - i (Gamma_L + Gamma_R), dense."""
    kk = hamiltonian_dense(prob, k).astype(complex)
    gz = np.repeat(prob.gamma_l + prob.gamma_r, prob.na * prob.nb)
    kk[np.diag_indices(prob.n)] -= 1j * gz
    return kk


def eigenpairs(prob, k):
    """All eigenpairs of K_k: eigenvalues lam (N), right eigenvectors R and left
    eigenvectors L (columns) normalised so that L^H R = I."""
    lam, lv, rv = sla.eig(k_matrix(prob, k), left=True, right=True)
    d = np.einsum("ij,ij->j", lv.conj(), rv)  # L_n^H R_n
    lv = lv / d.conj()[None, :]
    return lam, rv, lv


def left_from_minus_k(prob, k, lam, rv):
    """Left eigenvectors of K_k from the right eigenvectors of K_{-k}: each
    eigenvalue of K_k is matched to the nearest eigenvalue of K_{-k}, the
    conjugated right eigenvector taken, and scaled so that L_n^H R_n = 1.
    Returns (L, largest eigenvalue mismatch)."""
    lam_m, rv_m = sla.eig(k_matrix(prob, (-k[0], -k[1])))
    order = [int(np.argmin(np.abs(lam_m - x))) for x in lam]
    mism = float(np.max(np.abs(lam_m[order] - lam)))
    lv = rv_m[:, order].conj()
    d = np.einsum("ij,ij->j", lv.conj(), rv)
    return lv / d.conj()[None, :], mism


def transformed_caps(prob, rv, lv):
    """GtL = R^H Gamma_L R and GtR = L^H Gamma_R L (the CAPs in the eigenbasis)."""
    gl = np.repeat(prob.gamma_l, prob.na * prob.nb)
    gr = np.repeat(prob.gamma_r, prob.na * prob.nb)
    return rv.conj().T @ (gl[:, None] * rv), lv.conj().T @ (gr[:, None] * lv)


def transmission_from_pairs(lam, gtl, gtr, energies) -> np.ndarray:
    """T(E) = 4 sum_{m,n} GtL[m,n] GtR[n,m] / ((E - lam_n)(E - lam_m)^*)."""
    energies = np.atleast_1d(np.asarray(energies, float))
    w = gtl * gtr.T  # w[m, n] = GtL[m, n] GtR[n, m]
    out = np.empty(energies.size)
    for i, e in enumerate(energies):
        d = 1.0 / (e - lam)
        out[i] = 4.0 * float(np.real(d.conj() @ w @ d))
    return out


def nearest(lam, sigma, p) -> np.ndarray:
    """Indices of the p eigenvalues nearest sigma (the partial diagonalisation's
    selection), nearest first."""
    return np.argsort(np.abs(lam - sigma), kind="stable")[:p]


def transmission_eigen(prob, energies, k, p=None, sigma=None):
    """T(E, k) by the eigen route with the p eigenpairs nearest sigma (all N by
    default), left eigenvectors from LAPACK.  Returns (T, lam_selected)."""
    lam, rv, lv = eigenpairs(prob, k)
    if p is not None:
        sel = nearest(lam, sigma if sigma is not None else float(np.mean(energies)), p)
        lam, rv, lv = lam[sel], rv[:, sel], lv[:, sel]
    gtl, gtr = transformed_caps(prob, rv, lv)
    return transmission_from_pairs(lam, gtl, gtr, energies), lam
