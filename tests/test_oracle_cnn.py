"""Pins of the CPU oracle of the learned-preconditioner network (CPU only).

Each check comes from something other than the oracle's own code: a
brute-force convolution written with explicit index arithmetic, closed forms
(delta kernels, constant fields), adjoint identities between independently
written forward and backward steps, central finite differences of the whole
network, positive homogeneity of a bias-free ReLU network, and the closed form
of Adam's first step.
"""
import numpy as np
import pytest

from oracle import cnn


def brute_conv(x, w):
    """y[n,o,z,b,a] = sum_{i,dz,db,da} w[o,i,dz+1,db+1,da+1] x[n,i,z+dz,(b+db)%nb,(a+da)%na]."""
    n, ci, nz, nb, na = x.shape
    co = w.shape[0]
    y = np.zeros((n, co, nz, nb, na))
    for q in range(n):
        for o in range(co):
            for z in range(nz):
                for b in range(nb):
                    for a in range(na):
                        s = 0.0
                        for i in range(ci):
                            for dz in (-1, 0, 1):
                                zz = z + dz
                                if zz < 0 or zz >= nz:
                                    continue
                                for db in (-1, 0, 1):
                                    for da in (-1, 0, 1):
                                        s += w[o, i, dz + 1, db + 1, da + 1] * x[q, i, zz, (b + db) % nb,
                                                                                 (a + da) % na]
                        y[q, o, z, b, a] = s
    return y


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 3), (1, 2, 1)])
def test_conv_matches_brute_force(shape):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3) + shape)
    w = rng.standard_normal((2, 3, 3, 3, 3))
    np.testing.assert_allclose(cnn.conv3(x, w), brute_conv(x, w), rtol=1e-12, atol=1e-12)


def test_conv_delta_kernels():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 4, 5, 4, 6))
    w = np.zeros((4, 4, 3, 3, 3))
    w[:, :, 1, 1, 1] = np.eye(4)
    np.testing.assert_array_equal(cnn.conv3(x, w), x)          # centre tap = identity
    w = np.zeros((4, 4, 3, 3, 3))
    w[:, :, 1, 2, 0] = np.eye(4)                               # tap (0, +1, -1)
    np.testing.assert_array_equal(cnn.conv3(x, w), np.roll(x, (-1, 1), axis=(3, 4)))
    w = np.zeros((4, 4, 3, 3, 3))
    w[:, :, 2, 1, 1] = np.eye(4)                               # tap (+1, 0, 0): zero past the last plane
    y = cnn.conv3(x, w)
    np.testing.assert_array_equal(y[:, :, :-1], x[:, :, 1:])
    np.testing.assert_array_equal(y[:, :, -1], 0.0)


def test_conv_constant_field():
    """A constant field: interior planes see all 27 taps, the end planes 18."""
    w = np.random.default_rng(3).standard_normal((2, 1, 3, 3, 3))
    y = cnn.conv3(np.ones((1, 1, 4, 3, 3)), w)
    np.testing.assert_allclose(y[0, :, 1], np.broadcast_to(w.sum(axis=(1, 2, 3, 4))[:, None, None], (2, 3, 3)))
    np.testing.assert_allclose(y[0, :, 0], np.broadcast_to(w[:, :, 1:].sum(axis=(1, 2, 3, 4))[:, None, None],
                                                           (2, 3, 3)))


def test_conv_backward_is_adjoint():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 3, 4, 3, 5))
    w = rng.standard_normal((4, 3, 3, 3, 3))
    gy = rng.standard_normal((2, 4, 4, 3, 5))
    gx, gw = cnn.conv3_backward(x, w, gy)
    y = cnn.conv3(x, w)
    # <gy, conv(x, w)> is linear in x and in w
    assert np.isclose(np.sum(gy * y), np.sum(gx * x), rtol=1e-12)
    assert np.isclose(np.sum(gy * y), np.sum(gw * w), rtol=1e-12)


@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 3, 7), (1, 1, 2)])
def test_pool_and_up_adjoints_and_identities(shape):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, 2) + shape)
    cs = cnn.coarse_shape(shape)
    y = rng.standard_normal((1, 2) + cs)
    assert np.isclose(np.sum(cnn.pool2(x) * y), np.sum(x * cnn.pool2_adjoint(y, shape)), rtol=1e-12)
    assert np.isclose(np.sum(cnn.up2(y, shape) * x), np.sum(y * cnn.up2_adjoint(x)), rtol=1e-12)
    np.testing.assert_allclose(cnn.pool2(np.full((1, 1) + shape, 2.5)), 2.5)   # mean of a constant
    np.testing.assert_allclose(cnn.pool2(cnn.up2(y, shape)), y, rtol=1e-14)  # pool o up = identity
    # child counts add up to the fine grid
    assert cnn.child_counts(shape).sum() == np.prod(shape)


def test_network_gradient_by_central_differences():
    rng = np.random.default_rng(6)
    shape = (6, 5, 4)
    ws = cnn.init_weights(rng, scale_last=1.0)
    x = rng.standard_normal((2, 4) + shape)
    tgt = rng.standard_normal((2, 2) + shape)
    loss, g = cnn.loss_and_grad(ws, x, tgt)
    h = 1e-6
    for li in range(len(ws)):
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in ws[li].shape)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[li][idx] += h
            wm[li][idx] -= h
            fd = (cnn.loss_and_grad(wp, x, tgt)[0] - cnn.loss_and_grad(wm, x, tgt)[0]) / (2 * h)
            assert abs(fd - g[li][idx]) <= 1e-6 * max(1.0, abs(fd)), (li, idx, fd, g[li][idx])
    # input gradient
    out, c = cnn.forward(ws, x)
    gout = rng.standard_normal(out.shape)
    _, gx = cnn.backward(ws, c, gout)
    for _ in range(5):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (np.sum(gout * cnn.forward(ws, xp)[0]) - np.sum(gout * cnn.forward(ws, xm)[0])) / (2 * h)
        assert abs(fd - gx[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_network_positively_homogeneous():
    rng = np.random.default_rng(7)
    ws = cnn.init_weights(rng, scale_last=1.0)
    x = rng.standard_normal((1, 4, 5, 4, 4))
    f1 = cnn.forward(ws, x)[0]
    np.testing.assert_allclose(cnn.forward(ws, 3.0 * x)[0], 3.0 * f1, rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    """From zero moments, step 1 moves each weight by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(8)
    w = [rng.standard_normal((3, 4))]
    g = [rng.standard_normal((3, 4))]
    w0 = w[0].copy()
    cnn.adam_step(w, g, [np.zeros((3, 4))], [np.zeros((3, 4))], 1, lr=0.01)
    np.testing.assert_allclose(w[0], w0 - 0.01 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)


def test_adam_constant_gradient_any_step():
    """With the same gradient g at every step, both moment estimates are exactly
    unbiased after the bias correction (m_hat = g, v_hat = g^2 for every t), so
    step t moves each weight by -lr g / (|g| + eps) whatever t is: after T steps
    w = w0 - T lr g / (|g| + eps).  A wrong correction exponent (beta^(t+1),
    beta^1) or a missing correction breaks this from t = 2 on."""
    rng = np.random.default_rng(18)
    shape = (4, 5)
    g = rng.standard_normal(shape) * np.exp(rng.uniform(-6, 2, shape))
    w = [rng.standard_normal(shape)]
    w0 = w[0].copy()
    m, v = [np.zeros(shape)], [np.zeros(shape)]
    lr = 0.003
    for t in range(1, 8):
        cnn.adam_step(w, [g], m, v, t, lr=lr)
        np.testing.assert_allclose(w[0], w0 - t * lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_scale_invariance_and_zero_gradient_step():
    """Two properties of the update that hold at every t: (1) with eps = 0 the
    update is unchanged when every gradient is multiplied by c > 0 (m_hat scales
    by c, sqrt(v_hat) by c); (2) a zero gradient after one nonzero g moves the
    weight by -lr (b1/(1+b1)) / sqrt(b2/(1+b2)) sign(g) at t = 2: m_2 = b1(1-b1)g
    and v_2 = b2(1-b2)g^2 over the corrections 1-b1^2 = (1-b1)(1+b1) and
    1-b2^2 = (1-b2)(1+b2)."""
    rng = np.random.default_rng(19)
    shape = (3, 6)
    gs = [rng.standard_normal(shape) for _ in range(5)]
    runs = []
    for c in (1.0, 37.0):
        w, m, v = [np.zeros(shape)], [np.zeros(shape)], [np.zeros(shape)]
        for t, g in enumerate(gs, start=1):
            cnn.adam_step(w, [c * g], m, v, t, lr=0.01, eps=0.0)
        runs.append(w[0])
    np.testing.assert_allclose(runs[0], runs[1], rtol=1e-12, atol=1e-15)
    b1, b2, lr = 0.9, 0.999, 0.01
    g = gs[0]
    w, m, v = [np.zeros(shape)], [np.zeros(shape)], [np.zeros(shape)]
    cnn.adam_step(w, [g], m, v, 1, lr=lr, eps=0.0)
    w1 = w[0].copy()
    cnn.adam_step(w, [np.zeros(shape)], m, v, 2, lr=lr, eps=0.0)
    step2 = lr * (b1 / (1 + b1)) / np.sqrt(b2 / (1 + b2)) * np.sign(g)
    np.testing.assert_allclose(w[0] - w1, -step2, rtol=1e-12)


def test_training_reduces_loss():
    """A few Adam steps on a fixed batch lower the loss (the optimiser and the
    gradients point the same way)."""
    rng = np.random.default_rng(9)
    ws = cnn.init_weights(rng)
    x = rng.standard_normal((2, 4, 6, 4, 4))
    tgt = 0.3 * x[:, :2] - 0.2 * x[:, 2:]
    m = [np.zeros_like(w) for w in ws]
    v = [np.zeros_like(w) for w in ws]
    l0 = cnn.loss_and_grad(ws, x, tgt)[0]
    for t in range(1, 16):
        _, g = cnn.loss_and_grad(ws, x, tgt)
        cnn.adam_step(ws, g, m, v, t, lr=3e-3)
    assert cnn.loss_and_grad(ws, x, tgt)[0] < 0.8 * l0
