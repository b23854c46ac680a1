"""COCG (method RST_COCG).  For a real H_k (the Gamma point and the lateral
zone boundary) A = E - H_k + i Gamma is complex symmetric and the blocked COCG
solves it; at any other k the library runs COCG on the doubled, complex
symmetric system B = [[0, A_k], [A_-k, 0]] (A_k^T = A_-k), which solves the k
and -k columns together.  Parity against the CPU oracle through the C ABI, with
and without the free-electron + CAP preconditioner, plus the option errors."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2208_02783_amd import rst
from paper_2208_02783_amd import workloads as wl
from tests import oracle_helpers as hp
from tests.gpu_util import make_ctx, n_channels, torch_cuda

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("pc", [rst.RST_PRECOND_NONE, rst.RST_PRECOND_FREE_CAP])
def test_cocg_config1_matches_oracle(pc):
    """Config 1 (8x8x40 free-electron slab at k = 0) at every fourth stored energy."""
    torch = torch_cuda()
    g = json.load(open(os.path.join(GOLD, "config1_T.json")))
    p = wl.config(1)
    es = np.array(g["energies"][::4])
    ref = np.array(g["T_LR"][::4])
    ctx = make_ctx(torch, p, method=rst.RST_COCG, precond=pc, tol=1e-10, max_iter=20000)
    t, st, s = ctx.rst_transmission(es)
    _say("cocg config1 pc", pc, "its/col", st["iterations_total"] / st["columns"], "restarts", st["restarts_total"])
    assert s == rst.RST_OK, st
    assert st["max_rel_residual"] <= 1e-10
    for e, a, b in zip(es, t, ref):
        assert abs(a - b) <= 1e-6 * max(1, n_channels(p, e, (0.0, 0.0))), (e, a, b)


@pytest.mark.parametrize("kind", ["gamma", "zone_boundary"])
def test_cocg_tiny_fcc_slab_matches_oracle(kind):
    """Tiny config-2 slab (wells and KB projectors with lateral images) at a real
    H_k: k = 0, and k_a = pi / L_a where every Bloch phase is -1 or +1."""
    torch = torch_cuda()
    p = wl.config(2, tiny=True)
    k = (0.0, 0.0) if kind == "gamma" else (math.pi / (p.na * p.ha), 0.0)
    es = p.energies[[0, 3, 6]]
    ctx = make_ctx(torch, p, k, method=rst.RST_COCG, precond=rst.RST_PRECOND_FREE_CAP, tol=1e-10, max_iter=20000)
    t, st, s = ctx.rst_transmission(es)
    _say("cocg tiny", kind, "its/col", st["iterations_total"] / st["columns"], "restarts", st["restarts_total"])
    assert s == rst.RST_OK, st
    ref = oracle.transmission(p, es, k, both=False)["T_LR"]
    np.testing.assert_allclose(t, ref, rtol=0, atol=1e-6 * max(1.0, float(ref.max())))
    # same T as the persistent preconditioned BiCGSTAB (at the zone boundary a few columns of
    # this slab need its near-breakdown / divergence restarts to converge)
    ctx.rst_set_solver(method=rst.RST_BICGSTAB, precond=rst.RST_PRECOND_FREE_CAP, tol=1e-10, max_iter=20000)
    tb, stb, sb = ctx.rst_transmission(es)
    _say("bicgstab", kind, "its/col", stb["iterations_total"] / stb["columns"], "restarts", stb["restarts_total"])
    assert sb == rst.RST_OK, stb
    np.testing.assert_allclose(tb, ref, rtol=0, atol=1e-6 * max(1.0, float(ref.max())))


def test_cocg_solve_columns_match_oracle():
    torch = torch_cuda()
    rng = np.random.default_rng(41)
    p = hp.random_problem(rng, na=5, nb=4, nz=16, order=4, nproj=3, ramp=4)
    k = (0.0, 0.0)
    cols = np.array([0, 9, p.n // 2, p.n - 1])
    for pc in (rst.RST_PRECOND_NONE, rst.RST_PRECOND_FREE_CAP):
        ctx = make_ctx(torch, p, k, method=rst.RST_COCG, precond=pc, tol=1e-12, max_iter=20000)
        x, st, s = rst.solve_columns(ctx, 0.37, cols, p.n)
        assert s == rst.RST_OK, st
        ref = oracle.green_columns(p, 0.37, k, cols)
        err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err <= 1e-9, (pc, err, st)


def test_cocg_option_and_k_errors():
    torch = torch_cuda()
    p = wl.config(2, tiny=True)
    ctx = make_ctx(torch, p, p.kpts[0])  # a generic k: H_k complex
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_set_solver(method=rst.RST_COCG, precision=rst.RST_FP32_REFINE)
    assert ei.value.status == rst.RST_EUNSUPPORTED
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_set_solver(method=rst.RST_COCG, precond=rst.RST_PRECOND_LEARNED)
    assert ei.value.status == rst.RST_EINVAL
    ctx.rst_set_solver(method=rst.RST_COCG, col_block=2)
    with pytest.raises(rst.RstError) as ei:  # launch-shape options belong to the blocked COCG
        ctx.rst_transmission(p.energies[:1])
    assert ei.value.status == rst.RST_EUNSUPPORTED
    # the batched launch and the dense right-hand sides stay BiCGSTAB-only
    ctx.rst_set_k(0.0, 0.0)
    b = torch.zeros((p.n, 1), dtype=torch.complex128, device="cuda")
    b[0, 0] = 1.0
    with pytest.raises(rst.RstError) as ei:
        rst.solve_rhs(ctx, p.energies[:1], b)
    assert ei.value.status == rst.RST_EUNSUPPORTED


@pytest.mark.parametrize("cfg,pc", [(2, 1), (3, 1)])
def test_doubled_cocg_generic_k_matches_oracle(cfg, pc):
    """COCG on the doubled k / -k system at a generic k, with the doubled
    free-electron + CAP preconditioner: T(E,k) on the tiny slabs against the
    oracle (1e-6 max(1, N_ch)), Green's columns to 1e-9, and the same T in the
    RL direction; the iteration counts are reported beside those of the
    many-column BiCGSTAB on A_k alone.  (Without a preconditioner COCG on the
    doubled system needs about ten times the applies of BiCGSTAB on A_k here,
    27,000-30,000 against 2,300-2,800 on the CPU, and is not tested.)"""
    torch = torch_cuda()
    p = wl.config(cfg, tiny=True)
    k = tuple(p.kpts[1])
    es = p.energies[[1, 5]]
    ref = oracle.transmission(p, es, k, both=False)["T_LR"]
    ctx = make_ctx(torch, p, k, method=rst.RST_COCG, precond=pc)
    t, st, s = ctx.rst_transmission(es)
    ctx_b = make_ctx(torch, p, k, method=rst.RST_BICGSTAB_MC, precond=pc)
    tb, stb, sb = ctx_b.rst_transmission(es)
    _say(f"cfg{cfg}-tiny pc={pc} k={k}: doubled COCG T={t} steps/col={st['iterations_total'] / st['columns']:.1f} "
         f"(2 applies each); BiCGSTAB steps/col={stb['iterations_total'] / stb['columns']:.1f} (2 applies each)")
    assert s == rst.RST_OK, st
    assert st["columns"] == 2 * p.r_columns().size
    for e, a, b in zip(es, t, ref):
        assert abs(a - b) <= 1e-6 * max(1, n_channels(p, e, k)), (e, a, b)
    cols = p.r_columns()[:5]
    x, st2, s2 = rst.solve_columns(ctx, float(es[0]), cols, p.n)
    assert s2 == rst.RST_OK
    g = oracle.green_columns(p, float(es[0]), k, cols)
    err = np.max(np.abs(x.cpu().numpy() - g)) / np.max(np.abs(g))
    assert err <= 1e-9, err
    ctx.rst_set_solver(method=rst.RST_COCG, precond=pc, direction=rst.RST_DIR_RL)
    t_rl, _, s3 = ctx.rst_transmission(es)
    assert s3 == rst.RST_OK
    for e, a, b in zip(es, t_rl, ref):
        assert abs(a - b) <= 1e-6 * max(1, n_channels(p, e, k)), (e, a, b)

