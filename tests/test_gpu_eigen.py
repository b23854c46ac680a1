"""The eigen route (rst_transmission_eigen) against the oracle's eigen route and
the LU route, through the C ABI, on tiny structures.

With every eigenpair (n_eig = n) the eigenbasis trace is T exactly, so the GPU
result must equal the oracle's LU-route T_LR and the GPU solve route (the
column route); with fewer pairs it must equal the oracle's truncated sum over
the same eigenpairs (the n_eig eigenvalues nearest sigma).  Bar: 1e-6 max(1, T),
the accuracy bar of the transmission; the eigenvalues themselves to 1e-8."""
import numpy as np
import pytest

import oracle
from oracle import eigen
from paper_2208_02783_amd import rst
from tests import oracle_helpers as hp
from tests.gpu_util import make_ctx, torch_cuda

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _problem(seed, k):
    rng = np.random.default_rng(seed)
    p = hp.random_problem(rng, na=5, nb=4, nz=12, order=4, nproj=3, ramp=4)
    return p, k


@pytest.mark.parametrize("k", [(0.37, -0.61), (0.0, 0.0)])
def test_full_eigen_route_equals_lu_and_column_routes(k):
    torch = torch_cuda()
    p, k = _problem(41, k)
    es = np.array([-0.4, 0.3, 0.8])
    ctx = make_ctx(torch, p, k, precond=1, tol=1e-12)
    t, lam, st, s = ctx.rst_transmission_eigen(es, n_eig=p.n, subspace=p.n, sigma=0.3, tol=1e-8, max_iter=3)
    _say("full eigen route", t, "residual", st["max_rel_residual"], "iterations", st["restarts_total"])
    assert s == rst.RST_OK, st
    ref = oracle.transmission(p, es, k, both=False)["T_LR"]
    t_col, _, s2 = ctx.rst_transmission(es)
    assert s2 == rst.RST_OK
    for a, b, c in zip(t, ref, t_col):
        assert abs(a - b) <= 1e-6 * max(1.0, b), (a, b)
        assert abs(a - c) <= 1e-6 * max(1.0, c), (a, c)
    lam_ref = np.linalg.eigvals(eigen.k_matrix(p, k))
    assert max(np.min(np.abs(lam_ref - x)) for x in lam) <= 1e-8 * np.max(np.abs(lam_ref))


@pytest.mark.parametrize("k", [(0.37, -0.61), (0.0, 0.0)])
def test_partial_eigen_route_equals_oracle_truncated_sum(k):
    torch = torch_cuda()
    p, k = _problem(42, k)
    sigma, nev = 0.35, 40
    es = np.array([0.25, 0.35, 0.45])
    ctx = make_ctx(torch, p, k, precond=1, tol=1e-12)
    t, lam, st, s = ctx.rst_transmission_eigen(es, n_eig=nev, subspace=3 * nev, sigma=sigma, tol=1e-9, max_iter=60)
    _say("partial eigen route", t, "residual", st["max_rel_residual"], "iterations", st["restarts_total"])
    assert s == rst.RST_OK, st
    t_ref, lam_ref = eigen.transmission_eigen(p, es, k, p=nev, sigma=sigma)
    np.testing.assert_allclose(np.sort_complex(lam), np.sort_complex(lam_ref), rtol=0, atol=1e-8)
    for a, b in zip(t, t_ref):
        assert abs(a - b) <= 1e-6 * max(1.0, abs(b)), (a, b)


def test_eigen_route_option_errors():
    torch = torch_cuda()
    p, k = _problem(43, (0.1, 0.2))
    ctx = make_ctx(torch, p, k, precond=1)
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_transmission_eigen(np.array([0.3]), n_eig=p.n + 1)
    assert ei.value.status == rst.RST_EINVAL
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_transmission_eigen(np.array([0.3]), n_eig=4, tol=0.0)
    assert ei.value.status == rst.RST_EINVAL
    ctx.rst_set_solver(method=rst.RST_COCG)
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_transmission_eigen(np.array([0.3]), n_eig=4)
    assert ei.value.status == rst.RST_EUNSUPPORTED


def test_fraction_sweep_tends_to_column_route():
    """The paper's truncation to a fraction p of the eigenpairs (nearest the
    energy window): at every p the GPU sum equals the oracle's truncated sum over
    the same eigenpairs, and at p = 1 both equal the column route's T."""
    torch = torch_cuda()
    p, k = _problem(44, (0.23, 0.11))
    es = np.array([0.2, 0.5])
    ctx = make_ctx(torch, p, k, precond=1, tol=1e-12)
    t_col, _, s = ctx.rst_transmission(es)
    assert s == rst.RST_OK
    errs = []
    for frac in (0.25, 0.5, 0.75, 1.0):
        nev = int(round(frac * p.n))
        t, lam, st, s = ctx.rst_transmission_eigen(es, n_eig=nev, subspace=p.n, sigma=0.35, tol=1e-8, max_iter=2)
        assert s == rst.RST_OK, st
        t_ref, _ = eigen.transmission_eigen(p, es, k, p=nev, sigma=0.35)
        for a, b in zip(t, t_ref):
            assert abs(a - b) <= 1e-6 * max(1.0, abs(b)), (frac, a, b)
        errs.append(float(np.max(np.abs(t - t_col))))
        _say("fraction", frac, "pairs", nev, "T", t, "column route", t_col, "difference", errs[-1])
    assert errs[-1] <= 1e-6 * max(1.0, float(np.max(t_col)))
