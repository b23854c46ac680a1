"""GPU parity of the HIP path (through the C ABI) against the CPU oracle."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2208_02783_amd import rst
from paper_2208_02783_amd import workloads as wl
from tests import oracle_helpers as hp
from tests.gpu_util import make_ctx, n_channels, rand_block, torch_cuda

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ apply

APPLY_CASES = [
    dict(na=5, nb=4, nz=11, order=4, nproj=3, k=(0.37, -0.81), ncol=5),
    dict(na=7, nb=8, nz=20, order=12, nproj=4, k=(0.2, 0.45), ncol=3),
    dict(na=9, nb=7, nz=30, order=12, nproj=0, k=(-0.6, 0.1), ncol=1),
    dict(na=3, nb=3, nz=5, order=4, nproj=2, k=(1.1, 0.3), ncol=9),
]


# The complex64 apply rounds each of its ~42 products and sums in FP32 (u = 6e-8);
# the magnitudes summed are about ten times |y| on these grids (the order-12
# Laplacian's weights), which bounds the error by ~2.5e-5 max|y|.  The input is
# rounded to complex64 first and the oracle applied to those same values.
APPLY_BAR = {"fp64": 1e-13, "fp32": 5e-5}


def _apply_vs_oracle(torch, ctx, p, k, e, x, xd, prec):
    if prec == "fp32":
        xd = xd.to(torch.complex64)
        x = xd.cpu().numpy().astype(np.complex128)
    y = rst.apply_h(ctx, e, xd).cpu().numpy().astype(np.complex128)
    ref = oracle.apply_system(p, k, e, x)
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    assert err <= APPLY_BAR[prec], (prec, err)
    return err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", APPLY_CASES)
def test_apply_matches_oracle(case, prec):
    torch = torch_cuda()
    _say("apply case", case, prec)
    rng = np.random.default_rng(13)
    p = hp.random_problem(rng, na=case["na"], nb=case["nb"], nz=case["nz"], order=case["order"],
                          nproj=case["nproj"], ramp=3)
    ctx = make_ctx(torch, p, case["k"])
    x, xd = rand_block(torch, p.n, case["ncol"], 1)
    _apply_vs_oracle(torch, ctx, p, case["k"], 0.731, x, xd, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_full_size_config2_columns(prec):
    """Config 2 at its full size (17x17x170, order 12, 360 projectors), every
    output of a few columns against the oracle's factored apply."""
    torch = torch_cuda()
    p = wl.config(2)
    k = p.kpts[5]
    ctx = make_ctx(torch, p, k)
    x, xd = rand_block(torch, p.n, 3, 2)
    _say("config-2 apply", prec, _apply_vs_oracle(torch, ctx, p, k, float(p.energies[100]), x, xd, prec))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("order,nproj", [(4, 3), (12, 4)])
def test_apply_many_columns_matches_oracle(order, nproj, prec):
    """549 columns (eight full 64-column chunks placed per XCD plus a ragged
    ninth) over 40 planes (z segments of 16, 16 and 8): every output against
    the oracle."""
    torch = torch_cuda()
    rng = np.random.default_rng(29)
    p = hp.random_problem(rng, na=7, nb=8, nz=40, order=order, nproj=nproj, ramp=5)
    k = (0.31, -0.52)
    ctx = make_ctx(torch, p, k)
    x, xd = rand_block(torch, p.n, 549, 6)
    _apply_vs_oracle(torch, ctx, p, k, 0.413, x, xd, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_wide_plane_strips_matches_oracle(prec):
    """A 29x23 plane (667 points: wider than one XCD's waves in flight, so the
    points go in strips of 6 a-columns and a ragged strip of 5) with 600
    columns (ten 64-column chunks: eight (chunk, segment) groups per XCD run and
    a remainder) over 21 planes (segments of 16 and 5): every output against
    the oracle."""
    torch = torch_cuda()
    rng = np.random.default_rng(31)
    p = hp.random_problem(rng, na=29, nb=23, nz=21, order=12, nproj=5, ramp=4)
    k = (0.27, -0.44)
    ctx = make_ctx(torch, p, k)
    x, xd = rand_block(torch, p.n, 600, 8)
    _apply_vs_oracle(torch, ctx, p, k, 0.377, x, xd, prec)


def test_apply_plane_beyond_32bit_offsets_matches_oracle():
    """A launch whose plane of rows exceeds 2^31 bytes (16 points x 8,388,645
    columns x 16 B, 12.9 GB per vector; the last 64-column chunk ragged) runs
    the 64-bit addressed kernel instead of the buffer-load one; sampled columns,
    first, middle and ragged last chunk, against the oracle."""
    torch = torch_cuda()
    rng = np.random.default_rng(37)
    p = hp.random_problem(rng, na=4, nb=4, nz=6, order=4, nproj=2, ramp=2)
    k = (0.23, -0.61)
    ncol = (1 << 31) // (p.na * p.nb * 16) + 37
    assert p.na * p.nb * ncol * 16 > (1 << 31) - 1
    need = 2 * p.n * ncol * 16 + p.proj.nproj * ncol * 16
    if torch.cuda.mem_get_info()[0] < need + (4 << 30):
        pytest.skip(f"needs {need / 1e9:.1f} GB of free device memory")
    ctx = make_ctx(torch, p, k)
    g = torch.Generator(device="cuda").manual_seed(41)
    xd = torch.randn((p.n, ncol), dtype=torch.complex128, device="cuda", generator=g)
    _say("apply past 32-bit plane offsets: ncol", ncol, "GB per vector", xd.numel() * 16 / 1e9)
    yd = rst.apply_h(ctx, 0.517, xd)
    torch.cuda.synchronize()
    cols = np.array([0, 1, 63, 64, 4_194_301, ncol - 38, ncol - 37, ncol - 20, ncol - 1])
    ci = torch.from_numpy(cols).to("cuda")
    xs = xd.index_select(1, ci).cpu().numpy()
    ys = yd.index_select(1, ci).cpu().numpy()
    del xd, yd
    torch.cuda.empty_cache()
    ref = oracle.apply_system(p, k, 0.517, xs)
    err = np.max(np.abs(ys - ref)) / np.max(np.abs(ref))
    assert err <= APPLY_BAR["fp64"], err


def test_apply_precision_argument():
    """An unknown precision is refused; both precisions accept zero columns."""
    torch = torch_cuda()
    p = wl.config(2, tiny=True)
    ctx = make_ctx(torch, p, p.kpts[0])
    x = torch.zeros((p.n, 2), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_apply_h(0.5, x.data_ptr(), y.data_ptr(), 2, 7)
    assert ei.value.status == rst.RST_EINVAL
    for prec in (rst.RST_FP64, rst.RST_FP32_REFINE):
        ctx.rst_apply_h(0.5, x.data_ptr(), y.data_ptr(), 0, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_full_size_config3_columns(prec):
    """Config 3 at its full size (54x54x252 point contact, n = 734,832, 3420
    projectors): the column-fastest apply has no per-plane workgroup limit, so
    every output of a few columns is checked against the oracle's factored
    apply.  (Its solves run on the many-column path; tests/test_gpu_mk.py checks
    them at this size.)"""
    torch = torch_cuda()
    p = wl.config(3)
    k = p.kpts[5]
    ctx = make_ctx(torch, p, k, precond=rst.RST_PRECOND_FREE_CAP)
    x, xd = rand_block(torch, p.n, 3, 4)
    e = float(p.energies[40])
    _say("config-3 apply", prec, _apply_vs_oracle(torch, ctx, p, k, e, x, xd, prec))


@pytest.mark.parametrize("case", APPLY_CASES)
def test_apply_blocked_matches_oracle(case):
    """The blocked-layout apply (the layout the solvers keep their vectors in),
    every output against the oracle, at the widest and at a one-column block."""
    torch = torch_cuda()
    _say("blocked apply case", case)
    rng = np.random.default_rng(17)
    p = hp.random_problem(rng, na=case["na"], nb=case["nb"], nz=case["nz"], order=case["order"],
                          nproj=case["nproj"], ramp=3)
    ctx = make_ctx(torch, p, case["k"])
    cwmax = ctx.rst_apply_block_width()
    assert cwmax in (1, 2, 4, 8)
    e = -0.217
    for cw in sorted({1, cwmax}):
        ncol = cw * 3
        x, xd = rand_block(torch, p.n, ncol, 5)
        y = rst.from_blocked(rst.apply_h_blocked(ctx, e, rst.to_blocked(xd, cw))).cpu().numpy()
        ref = oracle.apply_system(p, case["k"], e, x)
        err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        assert err <= 1e-13, (cw, err)


def test_apply_blocked_full_size_config2():
    """Config 2 at full size: the blocked apply over 16 columns equals the
    column-fastest apply (same operator, other kernels for the projector
    gather), and two of its columns match the oracle."""
    torch = torch_cuda()
    p = wl.config(2)
    k = p.kpts[9]
    ctx = make_ctx(torch, p, k)
    cw = ctx.rst_apply_block_width()
    assert cw == 2  # 17 x 17 plane: two columns per workgroup at two positions per thread
    x, xd = rand_block(torch, p.n, 16, 8)
    e = float(p.energies[300])
    yb = rst.from_blocked(rst.apply_h_blocked(ctx, e, rst.to_blocked(xd, cw)))
    yc = rst.apply_h(ctx, e, xd)
    d = (torch.max(torch.abs(yb - yc)) / torch.max(torch.abs(yc))).item()
    assert d <= 1e-13, d
    ref = oracle.apply_system(p, k, e, x[:, :2])
    err = np.max(np.abs(yb[:, :2].cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err <= 1e-13, err
    pm, sm = ctx.rst_apply_timing()
    assert pm > 0.0 and sm > 0.0  # the column-fastest apply ran last: gather and sweep timed


def test_apply_blocked_errors():
    torch = torch_cuda()
    p = wl.config(2)
    ctx = make_ctx(torch, p, p.kpts[0])
    x = torch.zeros((8, p.n, 1), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    for ncol, cw, want in ((6, 4, rst.RST_EINVAL), (6, 3, rst.RST_EINVAL), (8, 8, rst.RST_EUNSUPPORTED)):
        with pytest.raises(rst.RstError) as ei:
            ctx.rst_apply_h_blocked(0.5, x.data_ptr(), y.data_ptr(), ncol, cw)
        assert ei.value.status == want
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_apply_h_blocked(0.5, x.data_ptr(), x.data_ptr(), 8, 1)
    assert ei.value.status == rst.RST_EINVAL
    ctx.rst_apply_h_blocked(0.5, x.data_ptr(), y.data_ptr(), 0, 1)  # empty: nothing to do


# ----------------------------------------------------------- Green columns

def test_solve_columns_match_oracle():
    torch = torch_cuda()
    rng = np.random.default_rng(3)
    p = hp.random_problem(rng, na=5, nb=4, nz=16, order=4, nproj=3, ramp=4)
    k = (0.45, -0.2)
    ctx = make_ctx(torch, p, k, tol=1e-12)
    cols = np.array([0, 7, p.n // 2, p.n - 1])
    x, st, s = rst.solve_columns(ctx, 0.42, cols, p.n)
    assert s == rst.RST_OK, st
    ref = oracle.green_columns(p, 0.42, k, cols)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-9, (err, st)


# ----------------------------------------------------------- transmission

def test_config1_all_energies_match_oracle():
    """Config 1 as specified (8x8x40, order 4, 10-plane CAP, k = 0), 32 energies,
    all 640 right-CAP columns: |dT| <= 1e-6 max(1, N_ch)."""
    torch = torch_cuda()
    g = json.load(open(os.path.join(GOLD, "config1_T.json")))
    p = wl.config(1)
    ctx = make_ctx(torch, p)
    t, st, s = ctx.rst_transmission(np.array(g["energies"]))
    _say("config1 stats", st)
    assert s == rst.RST_OK
    for e, tg, tr in zip(g["energies"], g["T_LR"], t):
        assert abs(tr - tg) <= 1e-6 * max(1, n_channels(p, e, (0, 0))), (e, tr, tg)


def test_config1_rl_direction_equals_lr():
    torch = torch_cuda()
    g = json.load(open(os.path.join(GOLD, "config1_T.json")))
    p = wl.config(1)
    es = np.array(g["energies"][::8])
    ctx = make_ctx(torch, p, direction=rst.RST_DIR_RL)
    t, st, s = ctx.rst_transmission(es)
    assert s == rst.RST_OK
    np.testing.assert_allclose(t, np.array(g["T_RL"][::8]), atol=1e-6)
    np.testing.assert_allclose(t, np.array(g["T_LR"][::8]), atol=1e-6)


@pytest.mark.parametrize("cfg", [2, 3])
def test_tiny_structures_match_oracle(cfg):
    """Tiny variants of configs 2 and 3 from the same generator (order 12,
    Gaussian wells, KB projectors with lateral images, nonzero k)."""
    torch = torch_cuda()
    p = wl.config(cfg, tiny=True)
    k = p.kpts[1]
    es = p.energies[[0, 3, 7]]
    _say("tiny cfg", cfg, "n", p.n, "nproj", p.proj.nproj, "k", k)
    ref = oracle.transmission(p, es, k)
    ctx = make_ctx(torch, p, k)
    t, st, s = ctx.rst_transmission(es)
    _say("stats", st)
    assert s == rst.RST_OK
    assert np.max(np.abs(ref["T_LR"] - ref["T_RL"])) < 1e-9  # oracle well conditioned here
    np.testing.assert_allclose(t, ref["T_LR"], atol=1e-6, rtol=0)


def test_gpu_time_reversal_and_zone_shift():
    torch = torch_cuda()
    p = wl.config(2, tiny=True)
    k = np.array(p.kpts[1])
    es = p.energies[[2, 5]]
    out = []
    for kk in (k, -k, k + np.array([2 * math.pi / p.la, 0.0])):
        ctx = make_ctx(torch, p, kk)
        t, st, s = ctx.rst_transmission(es)
        assert s == rst.RST_OK
        out.append(t)
    np.testing.assert_allclose(out[1], out[0], atol=1e-8)
    np.testing.assert_allclose(out[2], out[0], atol=1e-8)


def test_kpoint_average_with_folding_matches_oracle():
    """T(E) = mean_k T(E,k) over the tiny config-2 slab's 2x2 Monkhorst-Pack
    grid: the +-k folding solves two k-points instead of four and still matches
    the oracle's average (and every per-k value); k + G is folded too; the
    caller's k is restored."""
    torch = torch_cuda()
    p = wl.config(2, tiny=True)
    es = p.energies[[1, 5]]
    ctx = make_ctx(torch, p, precond=rst.RST_PRECOND_FREE_CAP, tol=1e-10, max_iter=20000)
    t, tk, ns, st, s = ctx.rst_transmission_kavg(p.kpts, es, fold=True)
    assert s == rst.RST_OK, st
    assert ns == 2 and len(p.kpts) == 4
    ref_k = np.array([oracle.transmission(p, es, k, both=False)["T_LR"] for k in p.kpts])
    bar = 1e-6 * max(1.0, float(ref_k.max()))
    np.testing.assert_allclose(tk, ref_k, rtol=0, atol=bar)
    np.testing.assert_allclose(t, ref_k.mean(axis=0), rtol=0, atol=bar)
    t2, tk2, ns2, st2, s2 = ctx.rst_transmission_kavg(p.kpts, es, fold=False)
    assert s2 == rst.RST_OK and ns2 == 4
    np.testing.assert_allclose(t2, t, rtol=0, atol=bar)
    assert st2["columns"] == 2 * st["columns"]
    # the context's own k (the first k-point) is back in place: same launch, same bits
    t0, _, _ = ctx.rst_transmission(es)
    np.testing.assert_array_equal(t0, tk[0])
    # a copy shifted by a reciprocal lattice vector is not solved again
    ga = 2 * math.pi / (p.na * p.ha)
    kk = np.array([p.kpts[0], p.kpts[0] + np.array([ga, 0.0])])
    t3, tk3, ns3, _, _ = ctx.rst_transmission_kavg(kk, es, fold=True)
    assert ns3 == 1
    np.testing.assert_array_equal(tk3[0], tk3[1])
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_transmission_kavg(np.zeros((0, 2)), es)
    assert ei.value.status == rst.RST_EINVAL


def test_deterministic_bitwise():
    torch = torch_cuda()
    p = wl.config(2, tiny=True)
    es = p.energies[[1, 4]]
    ctx = make_ctx(torch, p, p.kpts[0])
    t1, _, _ = ctx.rst_transmission(es)
    t2, _, _ = ctx.rst_transmission(es)
    assert np.array_equal(t1, t2)


# ------------------------------------------------------------ edge cases

def test_edge_cases():
    torch = torch_cuda()
    p = wl.config(1)
    ctx = make_ctx(torch, p)
    t, st, s = ctx.rst_transmission(np.zeros(0))
    assert t.size == 0 and s == rst.RST_OK
    # no right CAP -> no columns -> T = 0
    ctx2 = make_ctx(torch, p.with_(gamma_r=np.zeros(p.nz)))
    t, st, s = ctx2.rst_transmission(np.array([0.3]))
    assert t[0] == 0.0
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_set_grid(3, 3, 10, 0.5, 0.5, 0.5, 12)  # radius 6 > 3 lateral points
    assert ei.value.status == rst.RST_EUNSUPPORTED
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_set_grid(8, 8, 10, 0.5, 0.5, 0.5, 5)
    assert ei.value.status == rst.RST_EINVAL
    c3 = rst.Context(0)
    c3.rst_set_grid(8, 8, 10, 0.5, 0.5, 0.5, 4)
    with pytest.raises(rst.RstError) as ei:
        c3.rst_transmission(np.array([0.3]))
    assert ei.value.status == rst.RST_ESTATE
    with pytest.raises(rst.RstError) as ei:
        c3.rst_set_abc(-np.ones(10), np.zeros(10))
    assert ei.value.status == rst.RST_EINVAL


def test_iteration_cap_reports_enoconv():
    torch = torch_cuda()
    p = wl.config(1)
    ctx = make_ctx(torch, p, max_iter=2)
    t, st, s = ctx.rst_transmission(np.array([0.7]))
    assert s == rst.RST_ENOCONV
    assert st["columns_unconverged"] > 0


# ------------------------------------------------- preconditioned solver

@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_preconditioned_matches_oracle(cfg):
    """Right-preconditioned BiCGSTAB (free-electron + CAP preconditioner) gives
    the same T as the dense oracle."""
    torch = torch_cuda()
    if cfg == 1:
        g = json.load(open(os.path.join(GOLD, "config1_T.json")))
        p = wl.config(1)
        es = np.array(g["energies"][::5])
        ref = np.array(g["T_LR"][::5])
        k = (0.0, 0.0)
    else:
        p = wl.config(cfg, tiny=True)
        k = p.kpts[1]
        es = p.energies[[0, 4, 7]]
        ref = oracle.transmission(p, es, k, both=False)["T_LR"]
    ctx = make_ctx(torch, p, k, precond=rst.RST_PRECOND_FREE_CAP)
    t, st, s = ctx.rst_transmission(es)
    _say("precond cfg", cfg, st)
    assert s == rst.RST_OK
    np.testing.assert_allclose(t, ref, atol=1e-6, rtol=0)


def test_preconditioned_solve_columns():
    torch = torch_cuda()
    p = wl.config(2, tiny=True)
    k = p.kpts[0]
    ctx = make_ctx(torch, p, k, tol=1e-12, precond=rst.RST_PRECOND_FREE_CAP)
    cols = np.array([3, p.n // 3, p.n - 5])
    x, st, s = rst.solve_columns(ctx, float(p.energies[2]), cols, p.n)
    assert s == rst.RST_OK, st
    ref = oracle.green_columns(p, float(p.energies[2]), k, cols)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-9, (err, st)


# ------------------------------------------------------ mixed precision

@pytest.mark.parametrize("cfg,pc", [(1, 0), (1, 1), (2, 1), (3, 1), (2, 0)])
def test_mixed_precision_matches_oracle(cfg, pc):
    """BiCGSTAB on FP32 vectors with FP64 reliable updates reaches the FP64
    tolerance on the FP64 true residual: T matches the dense FP64 oracle to 1e-6."""
    torch = torch_cuda()
    if cfg == 1:
        g = json.load(open(os.path.join(GOLD, "config1_T.json")))
        p = wl.config(1)
        es = np.array(g["energies"][1::6])
        ref = np.array(g["T_LR"][1::6])
        k = (0.0, 0.0)
    else:
        p = wl.config(cfg, tiny=True)
        k = p.kpts[1]
        es = p.energies[[1, 5]]
        ref = oracle.transmission(p, es, k, both=False)["T_LR"]
    ctx = make_ctx(torch, p, k, precision=rst.RST_FP32_REFINE, precond=pc)
    t, st, s = ctx.rst_transmission(es)
    _say("mixed cfg", cfg, "pc", pc, st)
    assert s == rst.RST_OK
    assert st["updates_total"] >= st["columns"]
    assert st["fallback_columns"] <= st["columns"] // 4  # most columns finish in mixed precision
    assert st["max_rel_residual"] <= 1e-10
    np.testing.assert_allclose(t, ref, atol=1e-6, rtol=0)


def test_mixed_solve_columns():
    torch = torch_cuda()
    p = wl.config(2, tiny=True)
    k = p.kpts[0]
    ctx = make_ctx(torch, p, k, tol=1e-12, precision=rst.RST_FP32_REFINE, precond=rst.RST_PRECOND_FREE_CAP)
    cols = np.array([3, p.n // 3, p.n - 5])
    x, st, s = rst.solve_columns(ctx, float(p.energies[2]), cols, p.n)
    assert s == rst.RST_OK, st
    ref = oracle.green_columns(p, float(p.energies[2]), k, cols)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-9, (err, st)


# ------------------------------------------------------------- batching

def _batch_ctx(slabs, **solver):
    p0 = slabs[0]
    ctx = rst.Context(0)
    ctx.rst_set_grid(p0.na, p0.nb, p0.nz, p0.ha, p0.hb, p0.hz, p0.order)
    ctx.rst_set_solver(**solver)
    for p in slabs:
        ctx.rst_batch_add(p.nz, p.v, p.gamma_l, p.gamma_r, p.kpts[0][0], p.kpts[0][1], p.energies)
    return ctx


@pytest.mark.parametrize("pc", [0, 1])
def test_batch_equals_individual_launches(pc):
    """Uneven slabs (config-4 generator) in one persistent launch give the same T
    as one launch per slab; with the same column block the results are bitwise
    identical, since each item is computed by one workgroup in a fixed order."""
    torch = torch_cuda()
    slabs = wl.batch_slabs(n_slabs=6, ne=3, cells=(6, 10))
    ctx = _batch_ctx(slabs, col_block=1, precond=pc)
    tb, st, s = ctx.rst_batch_run()
    _say("batch stats", st)
    assert s == rst.RST_OK and st["col_block"] == 1
    ti = []
    for p in slabs:
        c1 = make_ctx(torch, p, p.kpts[0], col_block=1, precond=pc)
        t, _, s1 = c1.rst_transmission(p.energies)
        assert s1 == rst.RST_OK
        ti.append(t)
    assert np.array_equal(tb, np.concatenate(ti))
    # autotuned column block: same T to rounding
    ctx2 = _batch_ctx(slabs, precond=pc)
    tb2, st2, s2 = ctx2.rst_batch_run()
    _say("autotuned col_block", st2["col_block"], "threads", st2["threads"])
    assert s2 == rst.RST_OK
    np.testing.assert_allclose(tb2, tb, rtol=0, atol=1e-9)


def test_batch_of_large_structures_runs_per_structure():
    """Three slabs with 32 energies each (20,480 column items per slab, enough to
    fill the device many times) take the per-structure launches: bitwise the T of
    one rst_transmission call per slab, and a second run gives the same bits."""
    torch = torch_cuda()
    slabs = wl.batch_slabs(n_slabs=3, ne=32, cells=(6, 8))
    ctx = _batch_ctx(slabs, precond=1)
    tb, st, s = ctx.rst_batch_run()
    _say("large batch stats", st)
    assert s == rst.RST_OK and st["col_block"] == 1 and st["threads"] == 64
    ti = []
    for p in slabs:
        c1 = make_ctx(torch, p, p.kpts[0], precond=1)
        t, _, s1 = c1.rst_transmission(p.energies)
        assert s1 == rst.RST_OK
        ti.append(t)
    assert np.array_equal(tb, np.concatenate(ti))
    tb2, _, s2 = ctx.rst_batch_run()
    assert s2 == rst.RST_OK and np.array_equal(tb2, tb)


@pytest.mark.parametrize("pc", [0, 1])
def test_batch_matches_oracle_and_graph_replay(pc):
    torch = torch_cuda()
    slabs = wl.batch_slabs(n_slabs=3, ne=2, cells=(6, 8), replica=1)
    ctx = _batch_ctx(slabs, precond=pc)
    t1, st, s = ctx.rst_batch_run()
    x = torch.ones(1 << 20, device="cuda")
    x.mul_(2.0)  # eager work between graph replays
    torch.cuda.synchronize()
    t2, _, _ = ctx.rst_batch_run()
    assert np.array_equal(t1, t2)
    ref = np.concatenate([oracle.transmission(p, p.energies, p.kpts[0], both=False)["T_LR"]
                          for p in slabs])
    items = [(p, e) for p in slabs for e in p.energies]
    for (p, e), tt, rr in zip(items, t1, ref):
        assert abs(tt - rr) <= 1e-6 * max(1, n_channels(p, e, p.kpts[0])), (e, tt, rr)


def test_batch_edge_cases():
    torch = torch_cuda()
    slabs = wl.batch_slabs(n_slabs=1, ne=1)
    p = slabs[0]
    c = rst.Context(0)
    c.rst_set_grid(p.na, p.nb, p.nz, p.ha, p.hb, p.hz, p.order)
    t, st, s = c.rst_batch_run(0)
    assert s == rst.RST_OK and t.size == 0
    q = wl.config(2, tiny=True)
    c2 = make_ctx(torch, q, q.kpts[0])
    with pytest.raises(rst.RstError) as ei:
        c2.rst_batch_add(q.nz, q.v, q.gamma_l, q.gamma_r, 0.0, 0.0, q.energies[:1])
    assert ei.value.status == rst.RST_EUNSUPPORTED


def test_batch_is_stale_after_set_grid():
    """A structure added before rst_set_grid carries a potential of the old grid:
    rst_batch_run refuses the batch (RST_ESTATE, nothing launched, nothing
    written) until it is cleared and rebuilt, after which it runs normally."""
    torch_cuda()
    slabs = wl.batch_slabs(n_slabs=2, ne=1, cells=(6, 7), replica=3)
    ctx = _batch_ctx(slabs, precond=0)
    t_ok, _, s_ok = ctx.rst_batch_run()
    assert s_ok == rst.RST_OK
    p0 = slabs[0]
    ctx.rst_set_grid(p0.na + 2, p0.nb, p0.nz, p0.ha, p0.hb, p0.hz, p0.order)
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_batch_run()
    assert ei.value.status == rst.RST_ESTATE
    ctx.rst_set_grid(p0.na, p0.nb, p0.nz, p0.ha, p0.hb, p0.hz, p0.order)
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_batch_run()  # same size again, but the batch was built before the call
    assert ei.value.status == rst.RST_ESTATE
    ctx.rst_batch_clear()
    for p in slabs:
        ctx.rst_batch_add(p.nz, p.v, p.gamma_l, p.gamma_r, p.kpts[0][0], p.kpts[0][1], p.energies)
    t2, _, s2 = ctx.rst_batch_run()
    assert s2 == rst.RST_OK and np.array_equal(t2, t_ok)


# ------------------------------------------------- dense right-hand sides

@pytest.mark.parametrize("pc", [0, 1])
def test_solve_rhs_matches_oracle(pc):
    """x = A^-1 b for dense right-hand sides (shared across energies and per
    energy), FP64 BiCGSTAB with and without the preconditioner, against LAPACK
    on the oracle's dense A; a zero right-hand side gives x = 0."""
    torch = torch_cuda()
    import scipy.linalg as sla
    p = wl.config(2, tiny=True)
    k = p.kpts[2]
    es = p.energies[[2, 6]]
    rng = np.random.default_rng(77)
    ncol = 5
    b = rng.standard_normal((p.n, ncol)) + 1j * rng.standard_normal((p.n, ncol))
    b[:, 3] = 0.0
    ctx = make_ctx(torch, p, k, tol=1e-12, precond=pc)
    x, st, s = rst.solve_rhs(ctx, es, torch.from_numpy(b).cuda())
    assert s == rst.RST_OK, st
    xh = x.cpu().numpy()
    for ie, e in enumerate(es):
        ref = sla.solve(oracle.system_matrix(p, k, e), b)
        got = xh[:, ie * ncol:(ie + 1) * ncol]
        assert np.all(got[:, 3] == 0)
        for j in (0, 1, 2, 4):
            err = np.linalg.norm(got[:, j] - ref[:, j]) / np.linalg.norm(ref[:, j])
            assert err <= 1e-9, (ie, j, err)
    # per-energy right-hand sides
    b2 = rng.standard_normal((p.n, 2 * 2)) + 1j * rng.standard_normal((p.n, 2 * 2))
    x2, st2, s2 = rst.solve_rhs(ctx, es, torch.from_numpy(b2).cuda(), per_energy=True)
    assert s2 == rst.RST_OK
    x2h = x2.cpu().numpy()
    for ie, e in enumerate(es):
        ref = sla.solve(oracle.system_matrix(p, k, e), b2[:, 2 * ie:2 * ie + 2])
        err = np.linalg.norm(x2h[:, 2 * ie:2 * ie + 2] - ref) / np.linalg.norm(ref)
        assert err <= 1e-9, (ie, err)


# ------------------------------------------------- low-rank transmission

@pytest.mark.parametrize("cfg,pc", [(1, 1), (2, 1), (2, 0)])
def test_lowrank_transmission_matches_oracle(cfg, pc):
    """The randomised range finder over the CAP blocks gives T to the oracle's
    1e-6 bar with far fewer solves than one per right-CAP column; its tail
    estimate bounds the neglected part."""
    torch = torch_cuda()
    if cfg == 1:
        g = json.load(open(os.path.join(GOLD, "config1_T.json")))
        p = wl.config(1)
        es = np.array(g["energies"][3::9])
        ref = np.array(g["T_LR"][3::9])
        k = (0.0, 0.0)
    else:
        p = wl.config(2, tiny=True)
        k = p.kpts[1]
        es = p.energies[[0, 3, 7]]
        ref = oracle.transmission(p, es, k, both=False)["T_LR"]
    ctx = make_ctx(torch, p, k, precond=pc, tol=1e-12)
    t, terr, st, s = ctx.rst_transmission_lowrank(es, probes=16, heldout=8, tail_tol=1e-8)
    _say("lowrank cfg", cfg, "T", t, "err", terr, "solves", st["columns"], "of", len(es) * p.r_columns().size)
    assert s == rst.RST_OK
    assert np.all(terr <= 1e-8)
    np.testing.assert_allclose(t, ref, atol=1e-6, rtol=0)
    assert np.all(t <= ref + 1e-9)  # T_Q is a lower bound up to solver error


def test_lowrank_and_rhs_edge_cases():
    """No right CAP: T = 0 with no solves; option errors; dense right-hand sides
    need FP64 BiCGSTAB; a block of zero right-hand sides returns x = 0 at once."""
    torch = torch_cuda()
    p = wl.config(1)
    ctx = make_ctx(torch, p, (0.0, 0.0), precond=1)
    ctx.rst_set_abc(p.gamma_l, np.zeros_like(p.gamma_r))
    t, terr, st, s = ctx.rst_transmission_lowrank(p.energies[:2])
    assert s == rst.RST_OK and np.all(t == 0) and st["columns"] == 0
    ctx.rst_set_abc(p.gamma_l, p.gamma_r)
    with pytest.raises(RuntimeError, match="options"):
        ctx.rst_transmission_lowrank(p.energies[:1], probes=0)
    ctx.rst_set_solver(precision=rst.RST_FP32_REFINE)
    with pytest.raises(RuntimeError, match="FP64"):
        ctx.rst_transmission_lowrank(p.energies[:1])
    b = torch.zeros((p.n, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="FP64"):
        rst.solve_rhs(ctx, p.energies[:1], b)
    ctx.rst_set_solver(precond=1)
    x, st, s = rst.solve_rhs(ctx, p.energies[:2], b)
    assert s == rst.RST_OK and torch.count_nonzero(x).item() == 0
    assert st["iterations_total"] == 0
