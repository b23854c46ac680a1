"""GPU parity of the learned-preconditioner network against the FP64 oracle.

The GPU runs the convolutions on FP32 matrix cores; the oracle runs the same
network in FP64 on the FP32-rounded weights and inputs.  Bar: relative error
(max-norm over the tensor, or 2-norm per gradient layer) <= 1e-5 for the
forward pass and <= 2e-5 for the weight gradients (FP32 sums over up to
~10^4 points).
"""
import numpy as np
import pytest

from oracle import cnn
from paper_2208_02783_amd import rst
from tests.gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def flat(ws):
    return np.concatenate([w.reshape(-1) for w in ws]).astype(np.float32)


def unflat(v):
    out, o = [], 0
    for co, ci in cnn.LAYERS:
        k = co * ci * 27
        out.append(v[o:o + k].astype(np.float64).reshape(co, ci, 3, 3, 3))
        o += k
    return out


def rounded_weights(seed, scale_last=1.0):
    ws = cnn.init_weights(np.random.default_rng(seed), scale_last=scale_last)
    return unflat(flat(ws))  # FP32-rounded, back in FP64


def to_gpu(torch, x_nczba):
    """(ncol, C, nz, nb, na) FP64 -> channel-last FP32 CUDA tensor (ncol, nz, nb, na, C)."""
    return torch.from_numpy(np.ascontiguousarray(np.moveaxis(x_nczba, 1, -1)).astype(np.float32)).cuda()


def from_gpu(t):
    return np.moveaxis(t.cpu().numpy().astype(np.float64), -1, 1)


SHAPES = [(2, 9, 7, 5),      # several 64-point tiles and a ragged tail, odd extents at every level
          (1, 24, 17, 17),   # the lateral grid of the FCC slab, 24 planes
          (3, 1, 1, 3),      # degenerate: one plane, one row
          (1, 2, 2, 2)]


def test_weight_count_matches_the_network():
    assert rst.load().rst_cnn_weight_count() == sum(co * ci * 27 for co, ci in cnn.LAYERS)


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(shape):
    torch = torch_cuda()
    ncol, nz, nb, na = shape
    ws = rounded_weights(11)
    x = np.random.default_rng(12).standard_normal((ncol, 4, nz, nb, na)).astype(np.float32).astype(np.float64)
    ctx = rst.Context(0)
    ctx.rst_cnn_set_weights(flat(ws))
    out = from_gpu(rst.cnn_forward(ctx, to_gpu(torch, x)))
    ref = cnn.forward(ws, x)[0]
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    assert err <= 1e-5, err
    # weights round-trip through the library's packed layout
    np.testing.assert_array_equal(ctx.rst_cnn_get_weights(), flat(ws))


@pytest.mark.parametrize("shape", SHAPES[:3])
def test_weight_gradient_matches_oracle(shape):
    torch = torch_cuda()
    ncol, nz, nb, na = shape
    ws = rounded_weights(21)
    rng = np.random.default_rng(22)
    x = rng.standard_normal((ncol, 4, nz, nb, na)).astype(np.float32).astype(np.float64)
    gout = rng.standard_normal((ncol, 2, nz, nb, na)).astype(np.float32).astype(np.float64)
    ctx = rst.Context(0)
    ctx.rst_cnn_set_weights(flat(ws))
    g = unflat(rst.cnn_gradient(ctx, to_gpu(torch, x), to_gpu(torch, gout)))
    _, c = cnn.forward(ws, x)
    gref, _ = cnn.backward(ws, c, gout)
    for li, (a, b) in enumerate(zip(g, gref)):
        nrm = np.linalg.norm(b)
        if nrm == 0:
            assert np.all(a == 0)
            continue
        assert np.linalg.norm(a - b) / nrm <= 2e-5, (li, np.linalg.norm(a - b) / nrm)


def test_train_step_matches_oracle_and_lowers_the_loss():
    torch = torch_cuda()
    ncol, nz, nb, na = 2, 10, 6, 6
    ws = rounded_weights(31, scale_last=0.1)
    rng = np.random.default_rng(32)
    x = rng.standard_normal((ncol, 4, nz, nb, na)).astype(np.float32).astype(np.float64)
    tgt = (0.3 * x[:, :2] - 0.2 * x[:, 2:]).astype(np.float32).astype(np.float64)
    ctx = rst.Context(0)
    ctx.rst_cnn_set_weights(flat(ws))
    xg, tg = to_gpu(torch, x), to_gpu(torch, tgt)
    lr = 1e-3
    loss0 = rst.cnn_train_step(ctx, xg, tg, lr)
    ref_loss, gref = cnn.loss_and_grad(ws, x, tgt)
    assert abs(loss0 - ref_loss) <= 1e-5 * ref_loss
    # Adam's first step moves every weight with a non-negligible gradient by lr*sign(g)
    w1 = unflat(ctx.rst_cnn_get_weights())
    for a, w0, g in zip(w1, ws, gref):
        big = np.abs(g) > 1e-3 * np.max(np.abs(g))
        np.testing.assert_allclose((a - w0)[big], -lr * np.sign(g[big]), rtol=0, atol=2e-6)
    losses = [loss0] + [rst.cnn_train_step(ctx, xg, tg, lr) for _ in range(20)]
    assert losses[-1] < 0.8 * losses[0], losses


def test_three_adam_steps_match_oracle_elementwise():
    """Three device training steps against the oracle's Adam (Kingma and Ba,
    Algorithm 1) element by element.  Before each step the device's own weight
    gradient of the mean squared loss is taken through rst_cnn_gradient (gout =
    2 (f(x) - target) / ncol from the device forward pass); the oracle applies
    adam_step with that gradient, at t = 1, 2, 3, to its FP64 copy of the weights
    and moments.  Bar: |w_gpu - w_oracle| <= 1e-7 + 1e-6 |w| on every weight whose
    gradient is above 1e-3 of the layer's largest at all three steps (elsewhere an
    FP32 gradient of a few ulps can flip m_hat / sqrt(v_hat) by O(1), which is a
    difference in the gradient, not in the optimiser)."""
    torch = torch_cuda()
    ncol, nz, nb, na = 2, 6, 5, 5
    ws = rounded_weights(41, scale_last=0.1)
    rng = np.random.default_rng(42)
    x = rng.standard_normal((ncol, 4, nz, nb, na)).astype(np.float32).astype(np.float64)
    tgt = (0.3 * x[:, :2] - 0.2 * x[:, 2:]).astype(np.float32).astype(np.float64)
    ctx = rst.Context(0)
    ctx.rst_cnn_set_weights(flat(ws))
    xg, tg = to_gpu(torch, x), to_gpu(torch, tgt)
    w_or = [w.copy() for w in ws]
    m = [np.zeros_like(w) for w in ws]
    v = [np.zeros_like(w) for w in ws]
    big = [np.ones(w.shape, bool) for w in ws]
    lr = 2e-3
    for t in (1, 2, 3):
        out = rst.cnn_forward(ctx, xg)
        gout = ((out - tg) * (2.0 / ncol)).contiguous()
        g = unflat(rst.cnn_gradient(ctx, xg, gout))
        for b, gl in zip(big, g):
            b &= np.abs(gl) > 1e-3 * np.max(np.abs(gl))
        rst.cnn_train_step(ctx, xg, tg, lr)
        cnn.adam_step(w_or, g, m, v, t, lr=lr)
        w_gpu = unflat(ctx.rst_cnn_get_weights())
        for li, (a, b, msk) in enumerate(zip(w_gpu, w_or, big)):
            err = np.abs(a - b)[msk]
            bar = (1e-7 + 1e-6 * np.abs(b))[msk]
            assert np.all(err <= bar), (t, li, float(np.max(err - bar)))
    assert sum(int(b.sum()) for b in big) > 0.5 * sum(b.size for b in big)


def test_network_errors():
    torch = torch_cuda()
    ctx = rst.Context(0)
    x = torch.zeros((1, 2, 2, 2, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="no weights"):
        rst.cnn_forward(ctx, x)
    with pytest.raises(RuntimeError, match="count"):
        ctx.rst_cnn_set_weights(np.zeros(10, np.float32))
    bad = flat(rounded_weights(1))
    bad[5] = np.nan
    with pytest.raises(RuntimeError, match="non-finite"):
        ctx.rst_cnn_set_weights(bad)
    ctx.rst_cnn_seed(5)
    out = rst.cnn_forward(ctx, x)
    assert torch.all(out == 0)  # a bias-free network maps zero to zero
