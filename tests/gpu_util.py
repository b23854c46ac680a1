"""Shared helpers of the GPU tests (no oracle arithmetic here)."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_ctx(torch, prob, k=None, **solver):
    from paper_2208_02783_amd import rst
    ctx = rst.Context(0)
    ctx.load_problem(prob, k)
    ctx.rst_set_solver(**solver)
    return ctx


def rand_block(torch, n, ncol, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, ncol)) + 1j * rng.standard_normal((n, ncol))
    return x, torch.from_numpy(x).to("cuda")


def n_channels(prob, e, k):
    """Open lateral channels of the free-electron dispersion (only used to scale tolerances)."""
    from tests import oracle_helpers as hp
    cnt, _ = hp.open_channels(e, prob.na, prob.nb, prob.ha, prob.hb, prob.hz, k, prob.order)
    return cnt
