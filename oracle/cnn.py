"""Plain FP64 CPU oracle of the learned preconditioner network.

TEST INFRASTRUCTURE ONLY: imported by the test-suite; the product path never
imports it, and it imports nothing of the product path.

The network is a learned correction of the free-electron + CAP preconditioner
M (the learned-preconditioner growth item of the transmission path): for a
unit-norm residual r on the grid, with m = M^-1 r,

    z = m + f([Re r, Im r, Re m, Im m])

is the preconditioned vector handed to flexible GMRES.  f is a three-level
3D U-Net of 3x3x3 convolutions without biases (so f is positively
homogeneous), 16 channels at every level, ReLU activations, 2x2x2 mean
pooling and nearest-neighbour upsampling with additive skips:

    h0 = relu(conv(relu(conv(x, W0)), W1))                 full grid
    h1 = relu(conv(relu(conv(pool(h0), W2)), W3))          half grid
    h2 = relu(conv(relu(conv(pool(h1), W4)), W5))          quarter grid
    g1 = relu(conv(up(h2) + h1, W6))
    g0 = relu(conv(up(g1) + h0, W7))
    f  = conv(g0, W8)                                      2 output channels

Convolution is cross-correlation, y[o, p] = sum_{i, t} W[o, i, t] x[i, p + t],
t = (dz, db, da) in {-1, 0, 1}^3, periodic in the two lateral directions (a
plain wrap at every level) and zero outside the planes 0..nz-1 along z.
Pooling averages the children that exist (an odd extent leaves a last parent
with one child along that axis); upsampling copies a parent to its children.
Tensors are (batch, channel, z, b, a).

Everything is written from these definitions with numpy in FP64: each
convolution is a loop over its 27 taps (a shifted copy of the input times the
tap's channel matrix), the backward pass is the adjoint of each step taken in
reverse order, and Adam follows Kingma and Ba (2015), Algorithm 1.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, db, da) for dz in (-1, 0, 1) for db in (-1, 0, 1) for da in (-1, 0, 1)]
CH = 16
# (cout, cin) of W0..W8
LAYERS = [(CH, 4), (CH, CH), (CH, CH), (CH, CH), (CH, CH), (CH, CH), (CH, CH), (CH, CH), (2, CH)]


def shift(x: np.ndarray, dz: int, db: int, da: int) -> np.ndarray:
    """s[..., z, b, a] = x[..., z + dz, (b + db) mod nb, (a + da) mod na], zero
    where z + dz is outside [0, nz)."""
    s = np.roll(x, shift=(-db, -da), axis=(-2, -1))
    out = np.zeros_like(s)
    nz = x.shape[-3]
    if dz == 0:
        out[...] = s
    elif dz > 0:
        out[..., : nz - dz, :, :] = s[..., dz:, :, :]
    else:
        out[..., -dz:, :, :] = s[..., : nz + dz, :, :]
    return out


def conv3(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """y[n, o] = sum_t W[o, :, t] . shift(x, t)[n, :]; w is (cout, cin, 3, 3, 3)."""
    n, _, nz, nb, na = x.shape
    y = np.zeros((n, w.shape[0], nz, nb, na))
    for dz, db, da in TAPS:
        wt = w[:, :, dz + 1, db + 1, da + 1]
        y += np.einsum("oi,nizba->nozba", wt, shift(x, dz, db, da))
    return y


def conv3_backward(x: np.ndarray, w: np.ndarray, gy: np.ndarray):
    """Adjoint of conv3: gradients (gx, gw) of <gy, conv3(x, w)>.  The adjoint
    of shift(., t) moves values back by -t (zero-filled where the forward
    shift dropped planes)."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for dz, db, da in TAPS:
        wt = w[:, :, dz + 1, db + 1, da + 1]
        gw[:, :, dz + 1, db + 1, da + 1] = np.einsum("nozba,nizba->oi", gy, shift(x, dz, db, da))
        gx += shift(np.einsum("oi,nozba->nizba", wt, gy), -dz, -db, -da)
    return gx, gw


def coarse_shape(shape):
    return tuple((s + 1) // 2 for s in shape)


def pool2(x: np.ndarray) -> np.ndarray:
    """Mean over the existing children (2Z, 2Z+1) x (2B, 2B+1) x (2A, 2A+1)."""
    nz, nb, na = x.shape[-3:]
    cz, cb, ca = coarse_shape((nz, nb, na))
    s = np.zeros(x.shape[:-3] + (cz, cb, ca))
    cnt = np.zeros((cz, cb, ca))
    for oz in (0, 1):
        for ob in (0, 1):
            for oa in (0, 1):
                zs, bs, as_ = np.arange(oz, nz, 2), np.arange(ob, nb, 2), np.arange(oa, na, 2)
                s[..., : zs.size, : bs.size, : as_.size] += x[..., zs[:, None, None], bs[None, :, None],
                                                               as_[None, None, :]]
                cnt[: zs.size, : bs.size, : as_.size] += 1.0
    return s / cnt


def child_counts(shape):
    nz, nb, na = shape
    cz = np.array([min(2, nz - 2 * Z) for Z in range((nz + 1) // 2)], float)
    cb = np.array([min(2, nb - 2 * B) for B in range((nb + 1) // 2)], float)
    ca = np.array([min(2, na - 2 * A) for A in range((na + 1) // 2)], float)
    return cz[:, None, None] * cb[None, :, None] * ca[None, None, :]


def up2(y: np.ndarray, shape) -> np.ndarray:
    """x[..., z, b, a] = y[..., z // 2, b // 2, a // 2] on the fine grid `shape`."""
    nz, nb, na = shape
    iz, ib, ia = np.arange(nz) // 2, np.arange(nb) // 2, np.arange(na) // 2
    return y[..., iz[:, None, None], ib[None, :, None], ia[None, None, :]]


def up2_adjoint(gx: np.ndarray) -> np.ndarray:
    """Adjoint of up2: each parent receives the sum of its children."""
    nz, nb, na = gx.shape[-3:]
    cz, cb, ca = coarse_shape((nz, nb, na))
    out = np.zeros(gx.shape[:-3] + (cz, cb, ca))
    for z in range(nz):
        for b in range(nb):
            for a in range(na):
                out[..., z // 2, b // 2, a // 2] += gx[..., z, b, a]
    return out


def pool2_adjoint(gy: np.ndarray, shape) -> np.ndarray:
    """Adjoint of pool2: each child receives its parent's value / child count."""
    return up2(gy / child_counts(shape), shape)


def relu(x):
    return np.maximum(x, 0.0)


def init_weights(rng: np.random.Generator, scale_last: float = 0.1):
    """He-normal weights (std sqrt(2 / (27 cin))); the last layer scaled down so
    the untrained correction is small."""
    ws = []
    for li, (co, ci) in enumerate(LAYERS):
        w = rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci))
        if li == len(LAYERS) - 1:
            w *= scale_last
        ws.append(w)
    return ws


def forward(ws, x: np.ndarray):
    """f(x) and the cache of every intermediate (pre-activation values kept so
    the backward pass can form the ReLU masks)."""
    c = {"x": x}
    s0 = x.shape[-3:]
    s1 = coarse_shape(s0)
    c["a0"] = conv3(x, ws[0]); c["h0a"] = relu(c["a0"])
    c["a1"] = conv3(c["h0a"], ws[1]); c["h0"] = relu(c["a1"])
    c["p1"] = pool2(c["h0"])
    c["a2"] = conv3(c["p1"], ws[2]); c["h1a"] = relu(c["a2"])
    c["a3"] = conv3(c["h1a"], ws[3]); c["h1"] = relu(c["a3"])
    c["p2"] = pool2(c["h1"])
    c["a4"] = conv3(c["p2"], ws[4]); c["h2a"] = relu(c["a4"])
    c["a5"] = conv3(c["h2a"], ws[5]); c["h2"] = relu(c["a5"])
    c["u1"] = up2(c["h2"], s1) + c["h1"]
    c["a6"] = conv3(c["u1"], ws[6]); c["g1"] = relu(c["a6"])
    c["u0"] = up2(c["g1"], s0) + c["h0"]
    c["a7"] = conv3(c["u0"], ws[7]); c["g0"] = relu(c["a7"])
    out = conv3(c["g0"], ws[8])
    return out, c


def backward(ws, c, gout: np.ndarray):
    """Gradients (gW0..gW8, gx) of <gout, f(x)>: the adjoints of the forward
    steps in reverse order."""
    g = [None] * len(ws)
    s0 = c["x"].shape[-3:]
    s1 = coarse_shape(s0)
    gg0, g[8] = conv3_backward(c["g0"], ws[8], gout)
    ga7 = gg0 * (c["a7"] > 0)
    gu0, g[7] = conv3_backward(c["u0"], ws[7], ga7)
    gh0 = gu0.copy()
    gg1 = up2_adjoint(gu0)
    ga6 = gg1 * (c["a6"] > 0)
    gu1, g[6] = conv3_backward(c["u1"], ws[6], ga6)
    gh1 = gu1.copy()
    gh2 = up2_adjoint(gu1)
    ga5 = gh2 * (c["a5"] > 0)
    gh2a, g[5] = conv3_backward(c["h2a"], ws[5], ga5)
    ga4 = gh2a * (c["a4"] > 0)
    gp2, g[4] = conv3_backward(c["p2"], ws[4], ga4)
    gh1 = gh1 + pool2_adjoint(gp2, s1)
    ga3 = gh1 * (c["a3"] > 0)
    gh1a, g[3] = conv3_backward(c["h1a"], ws[3], ga3)
    ga2 = gh1a * (c["a2"] > 0)
    gp1, g[2] = conv3_backward(c["p1"], ws[2], ga2)
    gh0 = gh0 + pool2_adjoint(gp1, s0)
    ga1 = gh0 * (c["a1"] > 0)
    gh0a, g[1] = conv3_backward(c["h0a"], ws[1], ga1)
    ga0 = gh0a * (c["a0"] > 0)
    gx, g[0] = conv3_backward(c["x"], ws[0], ga0)
    return g, gx


def loss_and_grad(ws, x: np.ndarray, target: np.ndarray):
    """Mean over the batch of ||f(x_n) - target_n||^2 and its weight gradients."""
    out, c = forward(ws, x)
    nb = x.shape[0]
    d = out - target
    loss = float(np.sum(d * d)) / nb
    g, _ = backward(ws, c, 2.0 * d / nb)
    return loss, g


def adam_step(ws, grads, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015, Algorithm 1) in place; t counts from 1."""
    for w, g, mm, vv in zip(ws, grads, m, v):
        mm *= b1
        mm += (1.0 - b1) * g
        vv *= b2
        vv += (1.0 - b2) * g * g
        mhat = mm / (1.0 - b1 ** t)
        vhat = vv / (1.0 - b2 ** t)
        w -= lr * mhat / (np.sqrt(vhat) + eps)


def features(r: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Network input (4, nz, nb, na) from complex r and m = M^-1 r given on the
    grid as (nz, nb, na) arrays."""
    return np.stack([r.real, r.imag, m.real, m.imag])


def precondition(ws, r: np.ndarray, m: np.ndarray) -> np.ndarray:
    """z = m + f(r, m) (complex, grid-shaped) for one residual."""
    out, _ = forward(ws, features(r, m)[None])
    return m + out[0, 0] + 1j * out[0, 1]
