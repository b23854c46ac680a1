"""Independent helpers that pin the oracle (no import of the oracle here).

The 1D transmission below is written directly from the definitions with its own
finite-difference weights (solved from Taylor conditions, not the closed form
the oracle uses), so agreement with the oracle's 3D result is a check of the
oracle, not of itself.
"""
from __future__ import annotations

import math

import numpy as np

from paper_2208_02783_amd.workloads import Problem, Projectors


def taylor_weights(order: int) -> np.ndarray:
    """w_0..w_M with sum_{j=-M..M} w_|j| j^(2p) = 2 delta_{p,1}, p = 0..M: the
    unique symmetric stencil exact for polynomials up to degree 2M+1."""
    m = order // 2
    # unknowns w_0..w_M; equation p: w_0*[p==0] + 2 sum_{j>=1} w_j j^(2p)
    a = np.zeros((m + 1, m + 1))
    rhs = np.zeros(m + 1)
    for p in range(m + 1):
        a[p, 0] = 1.0 if p == 0 else 0.0
        for j in range(1, m + 1):
            a[p, j] = 2.0 * float(j) ** (2 * p)
    rhs[1] = 2.0
    return np.linalg.solve(a, rhs)


def symbol(order: int, theta):
    """s(theta) = -sum_j w_|j| exp(i j theta): eigenvalue of -h^2 d^2/dx^2 on exp(i j theta)."""
    w = taylor_weights(order)
    theta = np.asarray(theta, float)
    s = -w[0] * np.ones_like(theta)
    for j in range(1, w.size):
        s = s - 2.0 * w[j] * np.cos(j * theta)
    return s


def lateral_energies(na, nb, ha, hb, k, order):
    """Free-electron lateral energies eps_a(ma) + eps_b(mb) of the twisted periodic
    FD Laplacian: theta = (k + 2 pi m / L) h."""
    ma = np.arange(na)
    mb = np.arange(nb)
    ea = symbol(order, (k[0] + 2 * math.pi * ma / (na * ha)) * ha) / (2 * ha * ha)
    eb = symbol(order, (k[1] + 2 * math.pi * mb / (nb * hb)) * hb) / (2 * hb * hb)
    return (ea[:, None] + eb[None, :]).ravel()


def t1d(energy, nz, hz, order, gamma_l, gamma_r, v=None):
    """4 sum_{i in R, j in L} Gamma_L,j Gamma_R,i |G_ji|^2 for the 1D chain
    A = E - (-1/2 D2 + V) + i Gamma with Dirichlet ends."""
    w = taylor_weights(order)
    m = w.size - 1
    h = np.zeros((nz, nz))
    for j in range(-m, m + 1):
        h += -0.5 * w[abs(j)] / (hz * hz) * np.eye(nz, k=j)
    if v is not None:
        h += np.diag(v)
    a = energy * np.eye(nz) - h + 1j * np.diag(gamma_l + gamma_r)
    g = np.linalg.inv(a)
    return 4.0 * float(np.sum(gamma_l[:, None] * np.abs(g) ** 2 * gamma_r[None, :]))


def open_channels(energy, na, nb, ha, hb, hz, k, order):
    """#{lateral modes with 0 < E - eps_perp < s(pi)/(2 hz^2)}: each open mode has
    exactly one right-mover because s is increasing on [0, pi]."""
    ep = lateral_energies(na, nb, ha, hb, k, order)
    top = symbol(order, math.pi) / (2 * hz * hz)
    ek = energy - ep
    return int(np.sum((ek > 0) & (ek < top))), ep


def random_problem(rng, na=4, nb=3, nz=18, h=(0.6, 0.7, 0.5), order=4, nproj=3,
                   ramp=5, peak=0.8, vscale=0.4, images=True, sym_break=True):
    """Tiny structure with a random potential and random, non-symmetric projectors
    whose entries include lateral images (so Bloch phases matter)."""
    n = na * nb * nz
    v = vscale * rng.standard_normal(n)
    offs = [0]
    pts, imgs, betas = [], [], []
    for p in range(nproj):
        cnt = int(rng.integers(4, 9))
        pt = rng.choice(n, size=cnt, replace=False)
        if images:
            img = rng.integers(-1, 2, size=(cnt, 2))
        else:
            img = np.zeros((cnt, 2), int)
        b = rng.standard_normal(cnt)
        b /= math.sqrt(h[0] * h[1] * h[2] * float(np.sum(b * b)))
        pts.append(pt); imgs.append(img); betas.append(b)
        offs.append(offs[-1] + cnt)
    if nproj == 0:
        proj = Projectors.empty()
    else:
        proj = Projectors(np.array(offs, np.int32), np.concatenate(pts).astype(np.int32),
                          np.concatenate(imgs).astype(np.int8), np.concatenate(betas),
                          rng.uniform(-0.5, 0.5, nproj), np.arange(nproj, dtype=np.int32))
    gl = np.zeros(nz)
    gl[:ramp] = peak * ((ramp - np.arange(ramp)) / ramp) ** 2
    gr = gl[::-1].copy()
    return Problem(na, nb, nz, h[0], h[1], h[2], order, v, proj, gl, gr,
                   np.zeros((1, 2)), np.array([0.3]), "random-tiny")


def double_along_a(p: Problem) -> Problem:
    """Supercell of two copies along a.  A small-cell entry (point ia, image m)
    of the atom at tau is the point ia*h + s*L_a of the supercell, seen from
    atom copy c (at tau + c*L_a) through supercell image m' = (s - c + m)/2, with
    s = (c - m) mod 2.  Copy c of the projector is a new projector."""
    na2 = 2 * p.na
    v_small = p.v.reshape(p.nz, p.nb, p.na)
    v = np.concatenate([v_small, v_small], axis=2).reshape(-1)
    pj = p.proj
    offs = [0]
    pts, imgs, betas, ekb = [], [], [], []
    for q in range(pj.nproj):
        sl = slice(pj.offs[q], pj.offs[q + 1])
        pt = pj.pt[sl].astype(np.int64)
        ia = pt % p.na
        ib = (pt // p.na) % p.nb
        iz = pt // (p.na * p.nb)
        m = pj.img[sl, 0].astype(np.int64)
        for c in (0, 1):
            s = np.mod(c - m, 2)
            mp = (s - c + m) // 2
            new_pt = (ia + s * p.na) + na2 * (ib + p.nb * iz)
            pts.append(new_pt.astype(np.int32))
            imgs.append(np.stack([mp, pj.img[sl, 1].astype(np.int64)], 1).astype(np.int8))
            betas.append(pj.beta[sl])
            ekb.append(pj.ekb[q])
            offs.append(offs[-1] + new_pt.size)
    proj = Projectors(np.array(offs, np.int32), np.concatenate(pts), np.concatenate(imgs),
                      np.concatenate(betas), np.array(ekb))
    return Problem(na2, p.nb, p.nz, p.ha, p.hb, p.hz, p.order, v, proj, p.gamma_l, p.gamma_r,
                   p.kpts, p.energies, p.name + " x2")
