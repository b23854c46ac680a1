"""Pins of the oracle's eigen route (oracle/eigen.py) on tiny structures.

The eigen route writes T(E) through the eigenpairs of K_k = H_k - i Gamma
(paper Sec. II.A-II.D).  It is checked against what mathematics fixes without it:
  * with every eigenpair the trace equals the LU route's T_LR (two independent
    evaluations of the same 4 Tr[Gamma_L G Gamma_R G^+]);
  * left eigenvectors of K_k are the conjugated right eigenvectors of K_{-k}
    (K_k^T = K_{-k}), with matching eigenvalues (the paper's +-k matching);
  * Im(lam) <= 0, since the anti-Hermitian part of K is -Gamma <= 0;
  * at k = 0 K is complex symmetric: its eigenvectors are complex orthogonal
    (R^T R diagonal), the paper's U^-1 = U^T.
"""
import numpy as np

import oracle
from oracle import eigen
from tests import oracle_helpers as hp


def _problem(seed=5, k=(0.37, -0.61)):
    rng = np.random.default_rng(seed)
    p = hp.random_problem(rng, na=4, nb=3, nz=16, order=4, nproj=3, ramp=5)
    return p, k


def test_full_eigen_route_equals_lu_route():
    p, k = _problem()
    es = np.array([-0.9, 0.1, 0.55, 1.3])
    t_eig, lam = eigen.transmission_eigen(p, es, k)
    t_lu = oracle.transmission(p, es, k, both=False)["T_LR"]
    assert lam.size == p.n
    np.testing.assert_allclose(t_eig, t_lu, rtol=1e-8, atol=1e-11)


def test_full_eigen_route_equals_lu_route_order12_and_gamma_point():
    rng = np.random.default_rng(6)
    p = hp.random_problem(rng, na=7, nb=7, nz=14, order=12, nproj=2, ramp=4)
    for k in ((0.0, 0.0), (0.21, 0.4)):
        es = np.array([0.2, 0.9])
        t_eig, _ = eigen.transmission_eigen(p, es, k)
        t_lu = oracle.transmission(p, es, k, both=False)["T_LR"]
        np.testing.assert_allclose(t_eig, t_lu, rtol=1e-8, atol=1e-11)


def test_left_eigenvectors_from_minus_k():
    p, k = _problem(7)
    lam, rv, lv = eigen.eigenpairs(p, k)
    lm, mism = eigen.left_from_minus_k(p, k, lam, rv)
    assert mism <= 1e-9 * np.max(np.abs(lam))
    # both satisfy L^H R = I; where the eigenvalue is simple they are the same vectors
    err = np.linalg.norm(lm - lv, axis=0) / np.linalg.norm(lv, axis=0)
    assert np.median(err) <= 1e-8, np.median(err)
    gap = np.array([np.min(np.abs(np.delete(lam, i) - lam[i])) for i in range(lam.size)])
    assert np.all(err[gap > 1e-6 * np.max(np.abs(lam))] <= 1e-6)


def test_eigenvalues_lie_in_the_lower_half_plane():
    p, k = _problem(8)
    lam, _, _ = eigen.eigenpairs(p, k)
    assert np.all(lam.imag <= 1e-12 * np.max(np.abs(lam)))
    assert np.any(lam.imag < -1e-3)  # the CAPs absorb


def test_complex_orthogonal_eigenvectors_at_gamma():
    p, _ = _problem(9)
    lam, rv, lv = eigen.eigenpairs(p, (0.0, 0.0))
    g = rv.T @ rv
    off = g - np.diag(np.diag(g))
    assert np.max(np.abs(off)) <= 1e-8 * np.max(np.abs(np.diag(g)))
    # and the left eigenvectors are the conjugated right ones, rescaled
    s = np.einsum("ij,ij->j", lv, rv.conj()) / np.einsum("ij,ij->j", rv.conj(), rv.conj())
    np.testing.assert_allclose(lv, rv.conj() * s[None, :], rtol=0, atol=1e-8 * np.max(np.abs(lv)))


def test_partial_sums_reach_the_full_trace():
    """The partial diagonalisation's truncated sum over the p eigenpairs nearest
    the energy equals the full trace at p = N, and its error at p = N/2 is far
    smaller than the error of dropping every pair (T itself)."""
    p, k = _problem(10)
    e = 0.55
    t_full = oracle.transmission(p, [e], k, both=False)["T_LR"][0]
    t_half, _ = eigen.transmission_eigen(p, [e], k, p=p.n // 2, sigma=e)
    t_all, _ = eigen.transmission_eigen(p, [e], k, p=p.n, sigma=e)
    assert abs(t_all[0] - t_full) <= 1e-8 * max(1.0, t_full)
    assert abs(t_half[0] - t_full) < 0.5 * t_full
