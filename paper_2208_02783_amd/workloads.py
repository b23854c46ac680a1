"""Seeded synthetic inputs for the Bloch-CAP transmission path.

This module only *produces inputs*: grids, a local potential made of Gaussian
wells, Kleinman-Bylander projector tables, absorbing-boundary (CAP) ramps,
lateral k-points and energy windows.  It contains none of the method's
arithmetic (no Laplacian, no Bloch phases, no Green's functions); both the CPU
oracle and the GPU library consume its arrays independently.

Shapes follow the paper's workloads: lateral periodic FCC cells with the
transport axis z (Sec. II.A, Bloch form), bulk electrodes of a few nm
(Sec. IV.A, V.A), a point contact with a narrowed central region (Sec. V.B),
Monkhorst-Pack lateral k-grids (Sec. IV.A), CAPs that are functions of z only
(Sec. II.A, Gaussian CAP equation).  Units are Hartree atomic units.

Every random draw uses ``numpy.random.default_rng(220802783 + 1000*cfg + replica)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 220802783


def seed_for(cfg: int, replica: int = 0) -> int:
    return SEED_BASE + 1000 * int(cfg) + int(replica)


@dataclass
class Projectors:
    """Separable nonlocal projectors in compressed-row form over projectors.

    offs[p]..offs[p+1] index the entries of projector p.  Entry e says that the
    image of the projector's atom displaced by the lateral lattice vector
    (img[e,0]*L_a, img[e,1]*L_b) has value beta[e] at home-cell grid point pt[e].
    ekb[p] is the projector energy (Ha).  The operator is
    h^3 * sum_p ekb[p] |beta_p,k><beta_p,k|.
    """
    offs: np.ndarray  # int32 (nproj+1)
    pt: np.ndarray    # int32 (nnz)
    img: np.ndarray   # int8 (nnz, 2)
    beta: np.ndarray  # float64 (nnz)
    ekb: np.ndarray   # float64 (nproj)
    atom_of: np.ndarray = None  # int32 (nproj), informational

    @property
    def nproj(self) -> int:
        return int(self.ekb.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.pt.shape[0])

    @staticmethod
    def empty() -> "Projectors":
        return Projectors(np.zeros(1, np.int32), np.zeros(0, np.int32),
                          np.zeros((0, 2), np.int8), np.zeros(0), np.zeros(0),
                          np.zeros(0, np.int32))


@dataclass
class Problem:
    """One transport structure: grid, potential, projectors, CAPs, k and E sets."""
    na: int
    nb: int
    nz: int
    ha: float
    hb: float
    hz: float
    order: int                      # even FD order 2M
    v: np.ndarray                   # (n,) local potential, index ia + na*(ib + nb*iz)
    proj: Projectors
    gamma_l: np.ndarray             # (nz,) left CAP, >= 0
    gamma_r: np.ndarray             # (nz,) right CAP, >= 0
    kpts: np.ndarray                # (nk, 2) lateral k (bohr^-1) along a, b
    energies: np.ndarray            # (ne,) Ha
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.na * self.nb * self.nz

    @property
    def la(self) -> float:
        return self.na * self.ha

    @property
    def lb(self) -> float:
        return self.nb * self.hb

    def r_columns(self) -> np.ndarray:
        """Grid indices with gamma_r > 0 (z slowest, then b, then a)."""
        planes = np.nonzero(self.gamma_r > 0)[0]
        p = self.na * self.nb
        return (planes[:, None] * p + np.arange(p)[None, :]).ravel().astype(np.int64)

    def l_columns(self) -> np.ndarray:
        planes = np.nonzero(self.gamma_l > 0)[0]
        p = self.na * self.nb
        return (planes[:, None] * p + np.arange(p)[None, :]).ravel().astype(np.int64)

    def with_(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)


# ----------------------------------------------------------------------------
# CAP profiles (Sec. II.A: CAPs depend on z only and are non-negative)
# ----------------------------------------------------------------------------

def quadratic_ramp(nz: int, width: int, peak: float) -> tuple[np.ndarray, np.ndarray]:
    """Gamma_L(iz) = peak*((width-iz)/width)^2 for iz < width; Gamma_R mirrored."""
    gl = np.zeros(nz)
    iz = np.arange(min(width, nz))
    gl[iz] = peak * ((width - iz) / width) ** 2
    gr = gl[::-1].copy()
    return gl, gr


def gaussian_cap(nz: int, hz: float, gamma0: float, sigma: float, z_l: float,
                 z_r: float, floor_rel: float = 1e-6):
    """The paper's Gaussian CAP (Gaussian CAP equation), truncated where it falls
    below floor_rel*gamma0 so that its support (the column set) is compact."""
    z = np.arange(nz) * hz
    gl = gamma0 * np.exp(-(z - z_l) ** 2 / (2 * sigma ** 2))
    gr = gamma0 * np.exp(-(z - z_r) ** 2 / (2 * sigma ** 2))
    gl[gl < floor_rel * gamma0] = 0.0
    gr[gr < floor_rel * gamma0] = 0.0
    # each CAP lives on its own side of the cell
    mid = nz // 2
    gl[mid:] = 0.0
    gr[:mid] = 0.0
    return gl, gr


# ----------------------------------------------------------------------------
# k-grids (Sec. IV.A: Monkhorst-Pack sampling of the lateral zone)
# ----------------------------------------------------------------------------

def monkhorst_pack(n_a: int, n_b: int, la: float, lb: float) -> np.ndarray:
    """k_i = (2i - N - 1)/(2N) * 2 pi / L, i = 1..N, on each lateral axis."""
    ia = np.arange(1, n_a + 1)
    ib = np.arange(1, n_b + 1)
    ka = (2 * ia - n_a - 1) / (2.0 * n_a) * 2 * math.pi / la
    kb = (2 * ib - n_b - 1) / (2.0 * n_b) * 2 * math.pi / lb
    kk = np.stack(np.meshgrid(ka, kb, indexing="ij"), -1).reshape(-1, 2)
    return kk


# ----------------------------------------------------------------------------
# Atoms, wells and projectors
# ----------------------------------------------------------------------------

FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def fcc_atoms(a: float, ncell_a: int, ncell_b: int, ncell_z: int, z_off: float) -> np.ndarray:
    pos = []
    for cz in range(ncell_z):
        for cb in range(ncell_b):
            for ca in range(ncell_a):
                for f in FCC_BASIS:
                    pos.append([(ca + f[0]) * a, (cb + f[1]) * a, (cz + f[2]) * a + z_off])
    return np.array(pos, dtype=np.float64).reshape(-1, 3)


def gaussian_wells(na, nb, nz, ha, hb, hz, atoms, depth, width, img_range=None):
    """V(r) = -depth * sum_atoms sum_lateral-images exp(-|r - tau - R|^2 / (2 width^2))."""
    la, lb = na * ha, nb * hb
    x = np.arange(na) * ha
    y = np.arange(nb) * hb
    z = np.arange(nz) * hz
    v = np.zeros((nz, nb, na))
    cut = 7.0 * width
    ra = img_range if img_range is not None else int(math.ceil(cut / la)) + 1
    rb = img_range if img_range is not None else int(math.ceil(cut / lb)) + 1
    for (ax, ay, az) in atoms:
        gz = np.exp(-(z - az) ** 2 / (2 * width ** 2))
        gx = np.zeros(na)
        gy = np.zeros(nb)
        for i in range(-ra, ra + 1):
            gx += np.exp(-(x - ax - i * la) ** 2 / (2 * width ** 2))
        for j in range(-rb, rb + 1):
            gy += np.exp(-(y - ay - j * lb) ** 2 / (2 * width ** 2))
        v -= depth * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return v.reshape(-1)


def _solid_harmonics(dx, dy, dz):
    """Real solid harmonics r^l S_lm for l <= 2 (unnormalized): 1; y, z, x;
    xy, yz, 3z^2 - r^2, xz, x^2 - y^2."""
    r2 = dx * dx + dy * dy + dz * dz
    return [np.ones_like(dx), dy, dz, dx, dx * dy, dy * dz, 3 * dz * dz - r2, dx * dz,
            dx * dx - dy * dy]


def kb_projectors(na, nb, nz, ha, hb, hz, atoms, rc, width, rng, ekb_range=(-0.5, 0.5),
                  lmax=2):
    """Kleinman-Bylander-like projectors: Gaussian radial x real solid harmonic,
    hard cutoff rc, discrete normalisation h^3 sum beta^2 = 1, energies drawn
    uniformly from ekb_range per (atom, l, m)."""
    la, lb = na * ha, nb * hb
    h3 = ha * hb * hz
    nfun = {0: 1, 1: 4, 2: 9}[lmax]
    offs = [0]
    pts, imgs, betas, ekbs, atom_of = [], [], [], [], []
    ia_rng = int(math.ceil(rc / la)) + 1
    ib_rng = int(math.ceil(rc / lb)) + 1
    for ai, (ax, ay, az) in enumerate(atoms):
        e_pt, e_img, e_dx, e_dy, e_dz = [], [], [], [], []
        # z range of grid points within rc (no z images: Dirichlet in z)
        z0 = max(0, int(math.floor((az - rc) / hz)))
        z1 = min(nz - 1, int(math.ceil((az + rc) / hz)))
        izs = np.arange(z0, z1 + 1)
        for ii in range(-ia_rng, ia_rng + 1):
            for jj in range(-ib_rng, ib_rng + 1):
                cx = ax + ii * la
                cy = ay + jj * lb
                xa0 = max(0, int(math.floor((cx - rc) / ha)))
                xa1 = min(na - 1, int(math.ceil((cx + rc) / ha)))
                yb0 = max(0, int(math.floor((cy - rc) / hb)))
                yb1 = min(nb - 1, int(math.ceil((cy + rc) / hb)))
                if xa0 > xa1 or yb0 > yb1 or izs.size == 0:
                    continue
                iz, ib, ia = np.meshgrid(izs, np.arange(yb0, yb1 + 1), np.arange(xa0, xa1 + 1),
                                         indexing="ij")
                dx = ia * ha - cx
                dy = ib * hb - cy
                dz = iz * hz - az
                m = dx * dx + dy * dy + dz * dz < rc * rc
                if not m.any():
                    continue
                e_pt.append((ia + na * (ib + nb * iz))[m])
                # the entry belongs to the atom image at tau + R with R = (ii*La, jj*Lb)
                e_img.append(np.tile(np.array([ii, jj], np.int8), (int(m.sum()), 1)))
                e_dx.append(dx[m]); e_dy.append(dy[m]); e_dz.append(dz[m])
        if not e_pt:
            continue
        pt = np.concatenate(e_pt).astype(np.int32)
        img = np.concatenate(e_img).astype(np.int8)
        dx = np.concatenate(e_dx); dy = np.concatenate(e_dy); dz = np.concatenate(e_dz)
        order = np.lexsort((img[:, 1], img[:, 0], pt))
        pt, img, dx, dy, dz = pt[order], img[order], dx[order], dy[order], dz[order]
        radial = np.exp(-(dx * dx + dy * dy + dz * dz) / (2 * width ** 2))
        harm = _solid_harmonics(dx, dy, dz)[:nfun]
        for f in range(nfun):
            b = radial * harm[f]
            nrm = math.sqrt(h3 * float(np.sum(b * b)))
            if nrm == 0.0:
                continue
            b = b / nrm
            pts.append(pt); imgs.append(img); betas.append(b)
            offs.append(offs[-1] + pt.size)
            ekbs.append(rng.uniform(*ekb_range))
            atom_of.append(ai)
    if not pts:
        return Projectors.empty()
    return Projectors(np.array(offs, np.int32), np.concatenate(pts).astype(np.int32),
                      np.concatenate(imgs).astype(np.int8), np.concatenate(betas),
                      np.array(ekbs), np.array(atom_of, np.int32))


# ----------------------------------------------------------------------------
# Presets
# ----------------------------------------------------------------------------

def free_electron_slab(na=8, nb=8, nz=40, h=0.5, order=4, ramp=10, peak=1.0,
                       energies=None, kpts=None, name="free-electron slab") -> Problem:
    gl, gr = quadratic_ramp(nz, ramp, peak)
    if energies is None:
        energies = np.linspace(0.05, 1.5, 32)
    if kpts is None:
        kpts = np.zeros((1, 2))
    return Problem(na, nb, nz, h, h, h, order, np.zeros(na * nb * nz), Projectors.empty(),
                   gl, gr, np.asarray(kpts, float), np.asarray(energies, float), name,
                   dict(abc=f"quadratic {ramp} planes, peak {peak} Ha"))


def fcc_slab(a=6.82, pts_per_a=17, ncell_a=1, ncell_b=1, ncell_z=10, order=12,
             depth=1.5, width=1.2, rc=2.5, ramp_cells=2.0, peak=1.0, nk=8, ne=512,
             cfg=2, replica=0, constriction=None, name="FCC slab") -> Problem:
    """Synthetic FCC metal slab.  constriction = (radius, first_cell, last_cell)
    keeps only atoms within `radius` of the lateral centre axis in those cells."""
    rng = np.random.default_rng(seed_for(cfg, replica))
    h = a / pts_per_a
    na = pts_per_a * ncell_a
    nb = pts_per_a * ncell_b
    nz = pts_per_a * ncell_z
    atoms = fcc_atoms(a, ncell_a, ncell_b, ncell_z, z_off=a / 4)
    if constriction is not None:
        rad, c0, c1 = constriction
        cx, cy = 0.5 * na * h, 0.5 * nb * h
        cz = np.floor((atoms[:, 2] - a / 4 + 1e-9) / a)
        inside = (cz >= c0) & (cz <= c1)
        rr = np.hypot(atoms[:, 0] - cx, atoms[:, 1] - cy)
        atoms = atoms[~inside | (rr <= rad)]
    v = gaussian_wells(na, nb, nz, h, h, h, atoms, depth, width)
    proj = kb_projectors(na, nb, nz, h, h, h, atoms, rc, rc / 4.0, rng)
    ramp = int(round(ramp_cells * pts_per_a))
    gl, gr = quadratic_ramp(nz, ramp, peak)
    vbar = float(v.mean())
    energies = np.linspace(vbar + 0.05, vbar + 1.5, ne)
    kpts = monkhorst_pack(nk, nk, na * h, nb * h)
    return Problem(na, nb, nz, h, h, h, order, v, proj, gl, gr, kpts, energies, name,
                   dict(a=a, atoms=atoms, vbar=vbar, abc=f"quadratic {ramp} planes, peak {peak} Ha",
                        seed=seed_for(cfg, replica)))


def config(cfg: int, replica: int = 0, tiny: bool = False) -> Problem:
    """The five synthetic workloads (and their tiny oracle-sized variants)."""
    if cfg == 1:
        return free_electron_slab(name="cfg1 free-electron slab 8x8x40")
    if cfg == 2:
        if tiny:
            # 8 points per a, 4 bulk cells + 1 CAP cell each end, nonzero k
            return fcc_slab(pts_per_a=8, ncell_z=6, ramp_cells=1.0, nk=2, ne=8, cfg=2,
                            replica=replica, name="cfg2-tiny FCC slab 8x8x48")
        return fcc_slab(cfg=2, replica=replica, name="cfg2 FCC bulk 17x17x170")
    if cfg == 3:
        if tiny:
            return fcc_slab(a=7.19, pts_per_a=8, ncell_a=1, ncell_b=1, ncell_z=6,
                            ramp_cells=1.0, nk=2, ne=8, cfg=3, replica=replica,
                            constriction=(2.5, 2, 3), name="cfg3-tiny point contact 8x8x48")
        return fcc_slab(a=7.19, pts_per_a=18, ncell_a=3, ncell_b=3, ncell_z=14, nk=4, ne=256,
                        cfg=3, replica=replica, constriction=(5.0, 5, 8),
                        name="cfg3 point contact 54x54x252")
    if cfg == 4:
        raise ValueError("config 4 is a batch: use batch_slabs()")
    if cfg == 5:
        return fcc_slab(cfg=5, replica=replica, nk=8, ne=64, name="cfg5 FCC geometry")
    raise ValueError(cfg)


def batch_slabs(n_slabs=96, ne=128, cells=(6, 20), replica=0, na=8, nb=8, h=0.5, ramp=10):
    """Config 4: independent free-electron slabs with z-lengths of 6..20 cells of
    8 planes (a 4-bohr lateral period) and random lateral k in the zone."""
    rng = np.random.default_rng(seed_for(4, replica))
    la = na * h
    out = []
    for s in range(n_slabs):
        nc = int(rng.integers(cells[0], cells[1] + 1))
        k = rng.uniform(-math.pi / la, math.pi / la, size=2)
        p = free_electron_slab(na=na, nb=nb, nz=8 * nc, h=h, ramp=ramp,
                               energies=np.linspace(0.05, 1.5, ne), kpts=k[None, :],
                               name=f"cfg4 slab {s} nz={8 * nc}")
        out.append(p)
    return out
