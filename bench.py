"""Benchmark of the Bloch-CAP transmission hot path on one MI355X.

One step = T(E, k) for one (energy, lateral k) point of the synthetic FCC bulk
slab (17x17x170 grid, h = 0.401 bohr, 12th-order FD, 40 Gaussian wells, 360
Kleinman-Bylander projectors, 34-plane quadratic CAP at each end): all 9826
right-CAP columns solved to an FP64 true relative residual of 1e-10 by the
persistent BiCGSTAB kernel (free-electron + CAP right preconditioner by
default), and T accumulated over the left CAP.  Inputs are generated and
uploaded before the timed region; the timed region is whole T(E,k) points.

Prints one JSON line (see the repository's measurement notes for the fields).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "T(E,k) points/sec at |ΔT|≤1e-6 vs FP64 oracle; stencil HBM GB/s; plain vs batched"


def src_hash():
    import hashlib
    import glob
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2208_02783_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(bytes_alg_per_launch, precond):
    """HBM traffic per launch from the committed counter profile, only if the
    kernel sources are unchanged since it was taken (else None)."""
    f = os.path.join(ROOT, "profiles", "k_bicgstab_pc_cfg2_traffic.json")
    if not precond or not os.path.exists(f):
        return None
    d = json.load(open(f))
    if d.get("src_sha256") != src_hash():
        return None
    return d["traffic_over_algorithmic"] * bytes_alg_per_launch


def step_points(prob, i):
    k = prob.kpts[(7 * i + 9) % len(prob.kpts)]
    e = float(prob.energies[(97 * i + 400) % len(prob.energies)])
    return k, e


def cpu_baseline(seconds_budget=20.0):
    """The CPU oracle (dense LU, FP64) on a bounded sample: the tiny variant of
    the same generator (8x8x48 grid, same order, wells and projector model,
    512 right-CAP columns), as many energies as fit the budget."""
    import oracle
    from paper_2208_02783_amd import workloads as wl
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    p = wl.config(2, tiny=True)
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds_budget:
        k = p.kpts[done % len(p.kpts)]
        oracle.transmission(p, [p.energies[(done // len(p.kpts)) % len(p.energies)]], k, both=False)
        done += 1
    dt = time.perf_counter() - t0
    n_tiny, n_full = p.n, 17 * 17 * 170
    per_point = dt / done
    return {"value": done / dt, "unit": "T(E,k) points/s", "cores": int(threads), "kind": "oracle",
            "sample": f"dense-LU oracle on the 8x8x48 tiny variant of the same generator "
                      f"(n={n_tiny}, 512 columns), {done} energies in {dt:.1f} s; "
                      f"at the full 17x17x170 size (n={n_full}) the dense LU scales as n^3: "
                      f"~{per_point * (n_full / n_tiny) ** 3 / 3600:.2f} h per point"}


def batched_comparison(n_slabs=96, ne=2, precond=1):
    """Config 4: 96 uneven free-electron slabs (8x8x{48..160}, order 4,
    10-plane CAPs, random k), `ne` of their 128 energies each.  Plain: one rst_transmission
    call per slab; batched: one persistent launch over every (slab, energy,
    column) item (autotuned column block, HIP-graph replay)."""
    import torch
    from paper_2208_02783_amd import rst
    from paper_2208_02783_amd import workloads as wl
    slabs = wl.batch_slabs(n_slabs=n_slabs, ne=128)
    pick = np.linspace(0, 127, ne).round().astype(int)
    p0 = slabs[0]
    # plain: per-slab launches
    ctx = rst.Context(0)
    ctx.rst_set_grid(p0.na, p0.nb, p0.nz, p0.ha, p0.hb, p0.hz, p0.order)
    ctx.rst_set_solver(precond=precond)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_plain, ok_plain, cols = [], True, 0
    for p in slabs:
        ctx.load_problem(p, p.kpts[0])
        ctx.rst_set_solver(precond=precond)
        t, st, s = ctx.rst_transmission(p.energies[pick])
        t_plain.append(t)
        ok_plain &= s == rst.RST_OK
        cols += st["columns"]
    wall_plain = time.perf_counter() - t0
    # batched: one launch (first run tunes and captures the graph; the second is timed)
    cb = rst.Context(0)
    cb.rst_set_grid(p0.na, p0.nb, p0.nz, p0.ha, p0.hb, p0.hz, p0.order)
    cb.rst_set_solver(precond=precond)
    for p in slabs:
        cb.rst_batch_add(p.nz, p.v, p.gamma_l, p.gamma_r, p.kpts[0][0], p.kpts[0][1], p.energies[pick])
    cb.rst_batch_run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_b, st_b, s_b = cb.rst_batch_run()
    wall_b = time.perf_counter() - t0
    npts = n_slabs * ne
    dmax = float(np.max(np.abs(np.concatenate(t_plain) - t_b)))
    print(f"batched comparison: plain {npts / wall_plain:.1f} pts/s, batched {npts / wall_b:.1f} pts/s",
          file=sys.stderr, flush=True)
    return {"workload": f"{n_slabs} free-electron slabs 8x8x(48..160), h=0.5, order 4, 10-plane CAPs, "
                        f"random k, {ne} energies each ({npts} T(E,k) points, {cols} column solves), "
                        f"{'free-electron + CAP preconditioned' if precond else 'plain'} BiCGSTAB",
            "plain_points_per_s": npts / wall_plain, "batched_points_per_s": npts / wall_b,
            "batched_col_block": st_b["col_block"], "batched_threads": st_b["threads"],
            "max_abs_dT_plain_vs_batched": dmax, "all_converged": bool(ok_plain and s_b == rst.RST_OK)}


def mixed_point(prob, k, e, t_ref):
    """One T(E,k) point of the same slab with FP32 BiCGSTAB and FP64 reliable
    updates (free-electron + CAP preconditioner), against the FP64 point."""
    from paper_2208_02783_amd import rst
    ctx = rst.Context(0)
    ctx.load_problem(prob, k)
    ctx.rst_set_solver(precond=1, precision=rst.RST_FP32_REFINE, max_iter=20000)
    t0 = time.perf_counter()
    t, st, s = ctx.rst_transmission(np.array([e]))
    wall = time.perf_counter() - t0
    print(f"mixed precision point: {wall:.1f} s, T={t[0]:.6f}, iters/col="
          f"{st['iterations_total'] / max(st['columns'], 1):.1f}", file=sys.stderr, flush=True)
    return {"points_per_s": (1.0 if s == rst.RST_OK else 0.0) / wall, "status": int(s), "T": float(t[0]),
            "abs_dT_vs_fp64": abs(float(t[0]) - t_ref), "iterations_per_column": st["iterations_total"] / st["columns"],
            "fp64_residual_replacements_per_column": st["updates_total"] / st["columns"],
            "max_rel_residual": st["max_rel_residual"], "kernel_ms": st["kernel_ms"],
            "algorithmic_GBps": st["bytes_algorithmic"] / (st["kernel_ms"] * 1e-3) / 1e9}


def learned_comparison(prob, ncols=32, pairs=4000, tol=1e-8):
    """Learned preconditioner on the slab's geometry: the network is trained on
    generated pairs (r = A M^-1 xi, e = M^-1 xi over the slab's energies and k
    points), then a bounded sample of right-CAP columns at one (E, k) is solved
    to `tol` by BiCGSTAB with M^-1, the unpreconditioned BiCGSTAB and FGMRES(30),
    FGMRES(30) with M^-1 and FGMRES(30) with the learned correction (every solver
    capped at 6000 iterations; its status says whether it converged)."""
    from paper_2208_02783_amd import rst
    k = prob.kpts[9]
    e = float(prob.energies[400])
    rc = prob.r_columns()
    cols = rc[np.linspace(0, rc.size - 1, ncols).round().astype(np.int64)]
    ctx = rst.Context(0)
    ctx.load_problem(prob, k)
    ctx.rst_cnn_seed(1)
    ts = ctx.rst_precond_train(prob.energies[::16], prob.kpts, pairs=pairs, batch=8, lr=1e-3, seed=2)
    print(f"learned: trained {ts['steps']} steps in {ts['ms'] / 1e3:.1f} s, loss {ts['loss_first']:.3g} -> "
          f"{ts['loss_last']:.3g}", file=sys.stderr, flush=True)
    res, xs = {}, {}
    runs = [("bicgstab_free_cap", dict(method=rst.RST_BICGSTAB, precond=rst.RST_PRECOND_FREE_CAP)),
            ("bicgstab_none", dict(method=rst.RST_BICGSTAB, precond=rst.RST_PRECOND_NONE)),
            ("fgmres_none", dict(method=rst.RST_FGMRES, precond=rst.RST_PRECOND_NONE, restart=30)),
            ("fgmres_free_cap", dict(method=rst.RST_FGMRES, precond=rst.RST_PRECOND_FREE_CAP, restart=30)),
            ("fgmres_learned", dict(method=rst.RST_FGMRES, precond=rst.RST_PRECOND_LEARNED, restart=30))]
    for name, kw in runs:
        ctx.rst_set_solver(tol=tol, max_iter=6000, **kw)
        x, st, s = rst.solve_columns(ctx, e, cols, prob.n)
        xs[name] = x.cpu().numpy()
        res[name] = {"status": int(s), "iterations_per_column": st["iterations_total"] / ncols,
                     "ms": st["kernel_ms"], "max_rel_residual": st["max_rel_residual"],
                     "fallback_columns": st["fallback_columns"], "network_tflop": st["cnn_flop"] / 1e12}
        print(f"learned comparison {name}: {st['kernel_ms']:.0f} ms, "
              f"{st['iterations_total'] / ncols:.1f} its/col", file=sys.stderr, flush=True)
    ref = xs["bicgstab_free_cap"]
    for name in res:
        d = np.linalg.norm(xs[name] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        res[name]["max_rel_dx_vs_bicgstab"] = float(np.max(d))
    return {"workload": f"config-2 slab geometry, {ncols} right-CAP columns at E={e:.4f}, k={list(map(float, k))}, "
                        f"to true relative residual {tol:g}",
            "training": {"pairs": pairs, "batch": 8, "steps": ts["steps"], "seconds": ts["ms"] / 1e3,
                         "loss_first": ts["loss_first"], "loss_last": ts["loss_last"]},
            "solvers": res}


def lowrank_comparison(prob, k, e_ref, t_ref, n_e=32):
    """Low-rank transmission on the same slab and k: a randomised range finder
    over the CAP blocks (probes + held-out solves, then adjoint solves at -k)
    instead of one solve per right-CAP column.  n_e energies (the timed step's
    energy among them) in one call; T at the step's energy is compared with the
    full-column FP64 value."""
    from paper_2208_02783_amd import rst
    es = np.unique(np.concatenate([[e_ref], prob.energies[np.linspace(0, len(prob.energies) - 1, n_e - 1)
                                                           .round().astype(int)]]))
    ctx = rst.Context(0)
    ctx.load_problem(prob, k)
    ctx.rst_set_solver(precond=1, tol=1e-10, max_iter=20000)
    t0 = time.perf_counter()
    t, terr, st, s = ctx.rst_transmission_lowrank(es, probes=16, heldout=8, tail_tol=1e-7)
    wall = time.perf_counter() - t0
    i = int(np.argmin(np.abs(es - e_ref)))
    ok = int(np.sum(terr <= 1e-7)) if s in (rst.RST_OK, rst.RST_ENOCONV) else 0
    # second full-column check at the lowest energy of the window (T near zero there)
    ctx.rst_set_solver(precond=1, tol=1e-10, max_iter=20000)
    t_low, _, s_low = ctx.rst_transmission(es[:1])
    print(f"low-rank check at E={es[0]:.4f}: full-column T={t_low[0]:.3e}, low-rank T={t[0]:.3e}",
          file=sys.stderr, flush=True)
    print(f"low-rank: {len(es)} points in {wall:.1f} s ({ok / wall:.2f} pts/s), {st['columns']} solves, "
          f"|dT| at the step point {abs(t[i] - t_ref):.2e}", file=sys.stderr, flush=True)
    return {"workload": f"same slab and k, {len(es)} energies in one call, probes 16 + 8 held out, doubling "
                        f"while the tail estimate exceeds 1e-7",
            "points_per_s": ok / wall, "status": int(s), "solves": st["columns"],
            "solves_full_column_equivalent": len(es) * prob.r_columns().size,
            "max_tail_estimate": float(np.max(terr)), "abs_dT_vs_full_column_fp64": float(abs(t[i] - t_ref)),
            "abs_dT_vs_full_column_fp64_lowest_energy": float(abs(t[0] - t_low[0])),
            "iterations_per_solve": st["iterations_total"] / max(st["columns"], 1), "kernel_ms": st["kernel_ms"]}


def stencil_apply(prob, k, e, ncol=1024, reps=5):
    """Stand-alone y = (E - H_k + i Gamma) x on ncol random columns of the slab
    (FD Laplacian with Bloch-phase lateral wraps, V, CAP, KB projectors), in the
    two layouts the library takes: column-fastest (n x ncol; the projections
    B^H x first on the FP64 matrix cores, then one wave per grid point and 64
    columns streaming z) and blocked (the solvers' layout: each block of
    col_block columns contiguous; the projections on the matrix cores into
    per-block arrays, then one workgroup streaming z through each block).  Kernel times from HIP events on the library's stream; algorithmic
    bytes = read x and write y, 32 B per point per column (V and the projector
    tables, a few MB read once per launch, are not counted).  The column-fastest
    apply is also timed on complex64 vectors (FP32 stencil, FP64 projections):
    16 B per point per column, and its largest difference from the FP64 result
    relative to max |y|."""
    import torch
    from paper_2208_02783_amd import rst
    ctx = rst.Context(0)
    ctx.load_problem(prob, k)
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randn((prob.n, ncol), dtype=torch.complex128, device="cuda", generator=g)
    y = torch.empty_like(x)
    alg = 32.0 * prob.n * ncol

    def timed(call):
        call()  # first call sizes the buffers
        pm, sm = [], []
        for _ in range(reps):
            call()
            a, b = ctx.rst_apply_timing()
            pm.append(a)
            sm.append(b)
        return float(np.mean(pm)), float(np.mean(sm))

    pm, sm = timed(lambda: ctx.rst_apply_h(e, x.data_ptr(), y.data_ptr(), ncol))
    cw = ctx.rst_apply_block_width()
    xb = rst.to_blocked(x, cw)
    yb = torch.empty_like(xb)
    pb, bm = timed(lambda: ctx.rst_apply_h_blocked(e, xb.data_ptr(), yb.data_ptr(), ncol, cw))
    dif = (torch.max(torch.abs(rst.from_blocked(yb) - y)) / torch.max(torch.abs(y))).item()
    # the two layouts run different kernels for the same operator: they must agree to rounding
    assert dif <= 1e-13, f"column-fastest and blocked applies differ by {dif:.2e}"
    gbs = alg / ((pm + sm) * 1e-3) / 1e9
    gbb = alg / ((pb + bm) * 1e-3) / 1e9
    del xb, yb
    x32 = x.to(torch.complex64)
    y32 = torch.empty_like(x32)
    pm32, sm32 = timed(lambda: ctx.rst_apply_h(e, x32.data_ptr(), y32.data_ptr(), ncol, rst.RST_FP32_REFINE))
    d32 = (torch.max(torch.abs(y32.to(torch.complex128) - y)) / torch.max(torch.abs(y))).item()
    alg32 = 16.0 * prob.n * ncol
    gb32 = alg32 / ((pm32 + sm32) * 1e-3) / 1e9
    print(f"stencil apply, {ncol} columns: column-fastest gather {pm:.3f} ms + apply {sm:.3f} ms -> "
          f"{gbs:.0f} GB/s; blocked ({cw} columns per block) {pb:.3f} + {bm:.3f} ms -> {gbb:.0f} GB/s; "
          f"max rel difference {dif:.1e}; complex64 {pm32:.3f} + {sm32:.3f} ms -> {gb32:.0f} GB/s "
          f"(vs FP64 {d32:.1e})", file=sys.stderr, flush=True)
    del x, y, x32, y32
    return {"workload": f"config-2 slab, {ncol} random columns, one apply of E - H_k + i Gamma",
            "columns": ncol, "algorithmic_bytes": alg,
            "column_fastest": {"projector_gather_ms": pm, "apply_kernel_ms": sm, "achieved_GBps": gbs,
                               "frac_of_hbm_peak": gbs / PEAK_HBM_GBS},
            "blocked": {"col_block": cw, "projector_gather_ms": pb, "kernel_ms": bm, "achieved_GBps": gbb,
                        "frac_of_hbm_peak": gbb / PEAK_HBM_GBS},
            "max_rel_difference_between_layouts": dif,
            "column_fastest_complex64": {"algorithmic_bytes": alg32, "projector_gather_ms": pm32,
                                         "apply_kernel_ms": sm32, "achieved_GBps": gb32,
                                         "frac_of_hbm_peak": gb32 / PEAK_HBM_GBS,
                                         "max_rel_difference_vs_fp64": d32}}


def cocg_comparison(prob2):
    """COCG against the persistent BiCGSTAB where H_k is real (k = 0), both with
    the free-electron + CAP preconditioner to a true relative residual of 1e-10:
    config 1 (32 energies, all 640 right-CAP columns per energy) and one
    T(E, k = 0) point of the config-2 slab (all 9826 columns)."""
    import torch
    from paper_2208_02783_amd import rst
    from paper_2208_02783_amd import workloads as wl
    out = {}
    p1 = wl.config(1)
    ctx = rst.Context(0)
    ctx.load_problem(p1, (0.0, 0.0))
    r1 = {}
    for name, m in (("bicgstab", rst.RST_BICGSTAB), ("cocg", rst.RST_COCG)):
        ctx.rst_set_solver(method=m, precond=1, tol=1e-10, max_iter=20000)
        t0 = time.perf_counter()
        t, st, s = ctx.rst_transmission(p1.energies)
        wall = time.perf_counter() - t0
        r1[name] = {"points_per_s": len(p1.energies) / wall if s == rst.RST_OK else 0.0, "kernel_ms": st["kernel_ms"],
                    "iterations_per_column": st["iterations_total"] / st["columns"], "T": t}
    dt = float(np.max(np.abs(r1["cocg"]["T"] - r1["bicgstab"]["T"])))
    for v in r1.values():
        del v["T"]
    out["config1_32_energies"] = dict(r1, max_abs_dT=dt)
    ctx2 = rst.Context(0)
    ctx2.load_problem(prob2, (0.0, 0.0))
    e = float(prob2.energies[400])
    r2 = {}
    for name, m in (("bicgstab", rst.RST_BICGSTAB), ("cocg", rst.RST_COCG)):
        ctx2.rst_set_solver(method=m, precond=1, tol=1e-10, max_iter=20000)
        t0 = time.perf_counter()
        t, st, s = ctx2.rst_transmission(np.array([e]))
        wall = time.perf_counter() - t0
        r2[name] = {"seconds": wall, "kernel_ms": st["kernel_ms"], "status": int(s), "T": float(t[0]),
                    "iterations_per_column": st["iterations_total"] / st["columns"],
                    "achieved_GBps": st["bytes_algorithmic"] / (st["kernel_ms"] * 1e-3) / 1e9}
    out["config2_gamma_point"] = dict(r2, abs_dT=abs(r2["cocg"]["T"] - r2["bicgstab"]["T"]),
                                      workload=f"config-2 slab at k = 0, E = {e:.4f}, all 9826 right-CAP columns")
    print(f"cocg vs bicgstab: config 1 {r1['cocg']['kernel_ms']:.0f} vs {r1['bicgstab']['kernel_ms']:.0f} ms; "
          f"config-2 point at Gamma {r2['cocg']['seconds']:.1f} vs {r2['bicgstab']['seconds']:.1f} s "
          f"({r2['cocg']['iterations_per_column']:.0f} vs {r2['bicgstab']['iterations_per_column']:.0f} its/col)",
          file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precond", type=int, default=1, help="1: free-electron + CAP, 0: none")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="fp64: FP64 throughout; mixed: FP32 applies inside FP64 refinement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the plain-vs-batched comparison")
    ap.add_argument("--batched-energies", type=int, default=2,
                    help="energies per slab in the batched comparison (the full configuration has 128)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision point")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--no-lowrank", action="store_true", help="skip the low-rank transmission comparison")
    ap.add_argument("--no-stencil", action="store_true", help="skip the stand-alone operator apply")
    ap.add_argument("--no-cocg", action="store_true", help="skip the COCG comparison at k = 0")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="before the run, copy this many GiB device-to-device (a reference "
                         "kernel of known traffic for hardware-counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the transmission path here runs on a single "
              "MI355X (independent (k, E, column) units; see the design notes for how it shards). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2208_02783_amd import rst
    from paper_2208_02783_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration_gib > 0:
        nel = int(args.copy_calibration_gib * (1 << 30) // 8)
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    prob = wl.config(2)
    ctx = rst.Context(0)
    ctx.load_problem(prob, prob.kpts[0])
    ctx.rst_set_solver(tol=args.tol, precond=args.precond, max_iter=20000,
                       precision=rst.RST_FP32_REFINE if args.precision == "mixed" else rst.RST_FP64)

    def one(i):
        k, e = step_points(prob, i)
        ctx.rst_set_k(k[0], k[1])
        t, st, s = ctx.rst_transmission(np.array([e]))
        print(f"step {i}: E={e:.4f} T={t[0]:.6f} status={s} iters/col="
              f"{st['iterations_total'] / max(st['columns'], 1):.1f} kernel {st['kernel_ms']:.0f} ms",
              file=sys.stderr, flush=True)
        return t[0], st, s, k, e

    for i in range(args.warmup):
        one(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [one(args.warmup + i) for i in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    ok = all(r[2] == rst.RST_OK for r in res)
    kernel_ms = sum(r[1]["kernel_ms"] for r in res)
    bytes_alg = sum(r[1]["bytes_algorithmic"] for r in res)
    iters = sum(r[1]["iterations_total"] for r in res)
    cols = sum(r[1]["columns"] for r in res)
    achieved = bytes_alg / (kernel_ms * 1e-3) / 1e9
    points_ok = sum(1 for r in res if r[2] == rst.RST_OK)
    line = {
        "metric": METRIC,
        "value": points_ok / wall,
        "unit": "T(E,k) points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "FCC bulk slab 17x17x170 (h=0.401 bohr, a=6.82, 10 cells), 12th-order FD, "
                        "40 Gaussian wells (1.5 Ha, 1.2 bohr), 360 KB projectors (l<=2, rc=2.5), "
                        "34-plane quadratic CAP peak 1 Ha, 9826 right-CAP columns per T(E,k) point",
            "solver": ("right-preconditioned BiCGSTAB, free-electron + CAP preconditioner"
                       if args.precond else "BiCGSTAB, no preconditioner"),
            "tol_true_rel_residual": args.tol,
            "precision": ("FP64 throughout" if args.precision == "fp64" else
                          "FP32 stencil/projector/preconditioner applies, FP64 refinement, "
                          "inner products and true residual"),
            "points": [{"k": [float(r[3][0]), float(r[3][1])], "E": r[4], "T": r[0],
                        "status": int(r[2])} for r in res],
            "iterations_per_column_avg": iters / max(cols, 1),
            "all_converged": ok,
            "kernel_ms_total": kernel_ms,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": (measured_traffic(bytes_alg / args.steps, args.precond)
                        if args.precision == "fp64" else None),
        },
    }
    if not args.no_stencil:
        line["stencil"] = stencil_apply(prob, res[0][3], res[0][4])
    if not args.no_batched:
        line["batched"] = batched_comparison(ne=args.batched_energies)
    if not args.no_cocg:
        line["cocg"] = cocg_comparison(prob)
    if not args.no_mixed and args.precision == "fp64":
        line["mixed"] = mixed_point(prob, res[0][3], res[0][4], res[0][0])
    if not args.no_learned:
        line["learned"] = learned_comparison(prob)
    if not args.no_lowrank and args.precision == "fp64":
        line["lowrank"] = lowrank_comparison(prob, res[0][3], res[0][4], res[0][0])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
