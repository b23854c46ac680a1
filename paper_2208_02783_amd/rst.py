"""Python binding of librst (ctypes): argument marshalling only.

Every step of the transmission path runs in the HIP library; this module
converts numpy arrays and torch device tensors into the pointers and sizes the
C ABI (include/rst.h) takes.  Loading fails loudly if the library is missing:
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RST_LIB") or os.path.join(_HERE, "librst.so")

RST_OK, RST_ENOCONV = 0, 1
RST_EINVAL, RST_ESTATE, RST_ENOMEM, RST_EDEVICE, RST_EUNSUPPORTED = -1, -2, -3, -4, -5
RST_BICGSTAB, RST_FGMRES, RST_COCG, RST_BICGSTAB_MC, RST_IDRS = 0, 1, 2, 3, 4
RST_FP64, RST_FP32_REFINE = 0, 1
RST_DIR_LR, RST_DIR_RL = 0, 1
RST_PRECOND_NONE, RST_PRECOND_FREE_CAP, RST_PRECOND_LEARNED = 0, 1, 2
RST_VREF_PLANE, RST_VREF_CELL = 0, 1

EXPORTED = ["rst_default_solver", "rst_create", "rst_destroy", "rst_last_error", "rst_set_grid",
            "rst_set_potential", "rst_set_projectors", "rst_set_abc", "rst_set_k", "rst_set_solver",
            "rst_transmission", "rst_transmission_kavg", "rst_apply_h", "rst_apply_timing",
            "rst_apply_block_width", "rst_apply_h_blocked", "rst_solve_columns", "rst_batch_clear",
            "rst_batch_add", "rst_batch_run", "rst_cnn_weight_count", "rst_cnn_seed",
            "rst_cnn_set_weights", "rst_cnn_get_weights", "rst_cnn_forward", "rst_cnn_gradient",
            "rst_cnn_train_step", "rst_precond_train", "rst_solve_rhs", "rst_default_lowrank",
            "rst_transmission_lowrank", "rst_apply_h_noalloc", "rst_default_eig", "rst_transmission_eigen"]


class rst_solver_opts(C.Structure):
    _fields_ = [("method", C.c_int), ("precision", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("col_block", C.c_int), ("threads", C.c_int),
                ("direction", C.c_int), ("update_delta", C.c_double), ("precond", C.c_int),
                ("restart", C.c_int), ("fallback_ratio", C.c_double), ("pc_vref", C.c_int),
                ("idr_s", C.c_int), ("pc_shift", C.c_double)]


class rst_stats(C.Structure):
    _fields_ = [("columns", C.c_int64), ("columns_unconverged", C.c_int64),
                ("iterations_total", C.c_int64), ("iterations_max", C.c_int32),
                ("restarts_total", C.c_int32), ("max_rel_residual", C.c_double),
                ("kernel_ms", C.c_double), ("bytes_algorithmic", C.c_double),
                ("updates_total", C.c_int64), ("col_block", C.c_int32),
                ("threads", C.c_int32), ("fallback_columns", C.c_int64), ("cnn_flop", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rst_eig_opts(C.Structure):
    _fields_ = [("n_eig", C.c_int), ("subspace", C.c_int), ("max_iter", C.c_int), ("sigma", C.c_double),
                ("tol", C.c_double), ("seed", C.c_uint64)]


class rst_train_opts(C.Structure):
    _fields_ = [("pairs", C.c_int), ("batch", C.c_int), ("lr", C.c_float), ("seed", C.c_uint64),
                ("n_e", C.c_int), ("energies", C.c_void_p), ("n_k", C.c_int), ("kpts", C.c_void_p),
                ("source", C.c_int)]


class rst_train_stats(C.Structure):
    _fields_ = [("steps", C.c_int), ("loss_first", C.c_double), ("loss_last", C.c_double),
                ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rst_lowrank_opts(C.Structure):
    _fields_ = [("probes", C.c_int), ("heldout", C.c_int), ("max_probes", C.c_int), ("tail_tol", C.c_double),
                ("seed", C.c_uint64)]


class rst_problem(C.Structure):
    _fields_ = [("nz", C.c_int), ("v", C.c_void_p), ("gamma_l", C.c_void_p),
                ("gamma_r", C.c_void_p), ("ka", C.c_double), ("kb", C.c_double),
                ("n_e", C.c_int), ("energies", C.c_void_p)]


class RstError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librst status {status}: {msg}")
        self.status = status


_lib = None


def _torch_runtime_first():
    """torch brings its own HIP runtime; it must initialise before the one
    librst links (the other order leaves torch without devices)."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads librst.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librst.so not found at {path}: build it with "
                           "`python -m paper_2208_02783_amd.build` (no CPU fallback exists)")
    _torch_runtime_first()
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.rst_default_solver.argtypes = [C.POINTER(rst_solver_opts)]
    lib.rst_default_solver.restype = None
    lib.rst_create.argtypes = [C.POINTER(P), C.c_int, P]
    lib.rst_destroy.argtypes = [P]
    lib.rst_destroy.restype = None
    lib.rst_last_error.argtypes = [P]
    lib.rst_last_error.restype = C.c_char_p
    lib.rst_set_grid.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int]
    lib.rst_set_potential.argtypes = [P, P]
    lib.rst_set_projectors.argtypes = [P, C.c_int, P, P, P, P, P]
    lib.rst_set_abc.argtypes = [P, P, P]
    lib.rst_set_k.argtypes = [P, C.c_double, C.c_double]
    lib.rst_set_solver.argtypes = [P, C.POINTER(rst_solver_opts)]
    lib.rst_transmission.argtypes = [P, C.c_int, P, P, C.POINTER(rst_stats)]
    lib.rst_apply_h.argtypes = [P, C.c_double, P, P, C.c_int, C.c_int]
    lib.rst_apply_h_noalloc.argtypes = [P, C.c_double, P, P, C.c_int, C.c_int]
    lib.rst_default_eig.argtypes = [C.POINTER(rst_eig_opts)]
    lib.rst_default_eig.restype = None
    lib.rst_transmission_eigen.argtypes = [P, C.c_int, P, C.POINTER(rst_eig_opts), P, P, C.POINTER(rst_stats)]
    lib.rst_transmission_kavg.argtypes = [P, C.c_int, P, C.c_int, C.c_int, P, P, P, C.POINTER(C.c_int),
                                          C.POINTER(rst_stats)]
    lib.rst_apply_timing.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.rst_apply_block_width.argtypes = [P, C.POINTER(C.c_int)]
    lib.rst_apply_h_blocked.argtypes = [P, C.c_double, P, P, C.c_int, C.c_int]
    lib.rst_solve_columns.argtypes = [P, C.c_double, C.c_int, P, P, C.POINTER(rst_stats)]
    lib.rst_batch_clear.argtypes = [P]
    lib.rst_batch_add.argtypes = [P, C.POINTER(rst_problem)]
    lib.rst_batch_run.argtypes = [P, P, C.POINTER(rst_stats)]
    lib.rst_cnn_weight_count.argtypes = []
    lib.rst_solve_rhs.argtypes = [P, C.c_int, P, C.c_int, P, C.c_int64, P, C.POINTER(rst_stats)]
    lib.rst_default_lowrank.argtypes = [C.POINTER(rst_lowrank_opts)]
    lib.rst_transmission_lowrank.argtypes = [P, C.c_int, P, C.POINTER(rst_lowrank_opts), P, P,
                                             C.POINTER(rst_stats)]
    lib.rst_precond_train.argtypes = [P, C.POINTER(rst_train_opts), C.POINTER(rst_train_stats)]
    lib.rst_cnn_seed.argtypes = [P, C.c_uint64]
    lib.rst_cnn_set_weights.argtypes = [P, P, C.c_int64]
    lib.rst_cnn_get_weights.argtypes = [P, P, C.c_int64]
    lib.rst_cnn_forward.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, P, P]
    lib.rst_cnn_gradient.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, P, P, P]
    lib.rst_cnn_train_step.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, P, P, C.c_float,
                                       C.POINTER(C.c_double)]
    for name in EXPORTED:
        if name not in ("rst_default_solver", "rst_destroy", "rst_last_error", "rst_default_lowrank",
                        "rst_default_eig"):
            getattr(lib, name).restype = C.c_int
    lib.rst_cnn_weight_count.restype = C.c_int64
    lib.rst_default_lowrank.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def default_solver() -> rst_solver_opts:
    o = rst_solver_opts()
    load().rst_default_solver(C.byref(o))
    return o


class Context:
    """One librst context (one device, one stream).  Method names follow the C ABI."""

    def __init__(self, device: int = 0, stream=None):
        # torch brings its own HIP runtime; it must initialise before librst's
        # (the other order leaves torch without devices).  Device buffers from
        # torch are then used by the library's kernels on the same GPU.
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        self.lib = load()
        self.h = C.c_void_p()
        s = self.lib.rst_create(C.byref(self.h), int(device), C.c_void_p(stream) if stream else None)
        if s != RST_OK:
            raise RstError(s, "rst_create failed")
        self._keep = []

    def close(self):
        if self.h:
            self.lib.rst_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, s, allow_noconv=False):
        if s == RST_OK or (allow_noconv and s == RST_ENOCONV):
            return s
        raise RstError(s, self.lib.rst_last_error(self.h).decode())

    def last_error(self) -> str:
        return self.lib.rst_last_error(self.h).decode()

    # -- setters
    def rst_set_grid(self, na, nb, nz, ha, hb, hz, fd_order):
        return self._chk(self.lib.rst_set_grid(self.h, na, nb, nz, ha, hb, hz, fd_order))

    def rst_set_potential(self, v):
        v = np.ascontiguousarray(v, np.float64)
        return self._chk(self.lib.rst_set_potential(self.h, _ptr(v)))

    def rst_set_projectors(self, offs, pt, img, beta, e_kb):
        nproj = int(len(e_kb))
        offs = np.ascontiguousarray(offs, np.int32)
        pt = np.ascontiguousarray(pt, np.int32)
        img = np.ascontiguousarray(img, np.int8)
        beta = np.ascontiguousarray(beta, np.float64)
        e_kb = np.ascontiguousarray(e_kb, np.float64)
        return self._chk(self.lib.rst_set_projectors(self.h, nproj, _ptr(offs), _ptr(pt), _ptr(img),
                                                     _ptr(beta), _ptr(e_kb)))

    def rst_set_abc(self, gamma_l, gamma_r):
        gl = np.ascontiguousarray(gamma_l, np.float64)
        gr = np.ascontiguousarray(gamma_r, np.float64)
        return self._chk(self.lib.rst_set_abc(self.h, _ptr(gl), _ptr(gr)))

    def rst_set_k(self, ka, kb):
        return self._chk(self.lib.rst_set_k(self.h, float(ka), float(kb)))

    def rst_set_solver(self, opts: rst_solver_opts = None, **kw):
        o = opts or default_solver()
        for k, v in kw.items():
            setattr(o, k, v)
        return self._chk(self.lib.rst_set_solver(self.h, C.byref(o)))

    # -- compute
    def rst_transmission(self, energies):
        e = np.ascontiguousarray(np.atleast_1d(energies), np.float64)
        t = np.zeros(e.size)
        st = rst_stats()
        s = self._chk(self.lib.rst_transmission(self.h, e.size, _ptr(e), _ptr(t), C.byref(st)),
                      allow_noconv=True)
        return t, st.as_dict(), s

    def rst_transmission_kavg(self, kpts, energies, fold=True):
        """(T(E) averaged over kpts, per-k T (n_k x n_e), k-points solved, stats, status)."""
        k = np.ascontiguousarray(np.asarray(kpts, np.float64).reshape(-1, 2))
        e = np.ascontiguousarray(np.atleast_1d(energies), np.float64)
        t = np.zeros(e.size)
        tk = np.zeros((k.shape[0], e.size))
        ns = C.c_int()
        st = rst_stats()
        s = self._chk(self.lib.rst_transmission_kavg(self.h, k.shape[0], _ptr(k), int(bool(fold)), e.size, _ptr(e),
                                                     _ptr(t), _ptr(tk), C.byref(ns), C.byref(st)),
                      allow_noconv=True)
        return t, tk, ns.value, st.as_dict(), s

    def rst_apply_h(self, energy, x_dev_ptr: int, y_dev_ptr: int, ncol: int, precision: int = 0):
        return self._chk(self.lib.rst_apply_h(self.h, float(energy), C.c_void_p(x_dev_ptr),
                                              C.c_void_p(y_dev_ptr), int(ncol), int(precision)))

    def rst_apply_h_noalloc(self, energy, x_dev_ptr: int, y_dev_ptr: int, ncol: int, precision: int = 0):
        return self._chk(self.lib.rst_apply_h_noalloc(self.h, float(energy), C.c_void_p(x_dev_ptr),
                                                      C.c_void_p(y_dev_ptr), int(ncol), int(precision)))

    def rst_apply_block_width(self):
        cw = C.c_int()
        self._chk(self.lib.rst_apply_block_width(self.h, C.byref(cw)))
        return cw.value

    def rst_apply_h_blocked(self, energy, x_dev_ptr: int, y_dev_ptr: int, ncol: int, col_block: int):
        return self._chk(self.lib.rst_apply_h_blocked(self.h, float(energy), C.c_void_p(x_dev_ptr),
                                                      C.c_void_p(y_dev_ptr), int(ncol), int(col_block)))

    def rst_apply_timing(self):
        """(projector gather ms, stencil sweep ms) of the last rst_apply_h."""
        a, b = C.c_double(), C.c_double()
        self._chk(self.lib.rst_apply_timing(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def rst_solve_columns(self, energy, cols, x_dev_ptr: int):
        cols = np.ascontiguousarray(cols, np.int64)
        st = rst_stats()
        s = self._chk(self.lib.rst_solve_columns(self.h, float(energy), cols.size, _ptr(cols),
                                                 C.c_void_p(x_dev_ptr), C.byref(st)), allow_noconv=True)
        return st.as_dict(), s

    def rst_solve_rhs(self, energies, ncol, rhs_dev_ptr: int, rhs_estride: int, x_dev_ptr: int):
        e = np.ascontiguousarray(np.atleast_1d(energies), np.float64)
        st = rst_stats()
        s = self._chk(self.lib.rst_solve_rhs(self.h, e.size, _ptr(e), int(ncol), C.c_void_p(rhs_dev_ptr),
                                             int(rhs_estride), C.c_void_p(x_dev_ptr), C.byref(st)),
                      allow_noconv=True)
        return st.as_dict(), s

    def rst_transmission_lowrank(self, energies, **kw):
        e = np.ascontiguousarray(np.atleast_1d(energies), np.float64)
        o = rst_lowrank_opts()
        self.lib.rst_default_lowrank(C.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        t = np.zeros(e.size)
        terr = np.zeros(e.size)
        st = rst_stats()
        s = self._chk(self.lib.rst_transmission_lowrank(self.h, e.size, _ptr(e), C.byref(o), _ptr(t), _ptr(terr),
                                                        C.byref(st)), allow_noconv=True)
        return t, terr, st.as_dict(), s

    def rst_transmission_eigen(self, energies, **kw):
        """T(E) by the eigen route; returns (T, eigenvalues (complex, nearest sigma first), stats, status)."""
        e = np.ascontiguousarray(np.atleast_1d(energies), np.float64)
        o = rst_eig_opts()
        self.lib.rst_default_eig(C.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        t = np.zeros(e.size)
        ev = np.zeros(2 * o.n_eig)
        st = rst_stats()
        s = self._chk(self.lib.rst_transmission_eigen(self.h, e.size, _ptr(e), C.byref(o), _ptr(t), _ptr(ev),
                                                      C.byref(st)), allow_noconv=True)
        return t, ev[0::2] + 1j * ev[1::2], st.as_dict(), s

    # -- batches
    def rst_batch_clear(self):
        self._batch_ne = 0
        return self._chk(self.lib.rst_batch_clear(self.h))

    def rst_batch_add(self, nz, v, gamma_l, gamma_r, ka, kb, energies):
        arrs = [np.ascontiguousarray(a, np.float64) for a in (v, gamma_l, gamma_r, energies)]
        pr = rst_problem(int(nz), _ptr(arrs[0]).value, _ptr(arrs[1]).value, _ptr(arrs[2]).value,
                         float(ka), float(kb), int(arrs[3].size), _ptr(arrs[3]).value)
        self._batch_ne = getattr(self, "_batch_ne", 0) + arrs[3].size
        return self._chk(self.lib.rst_batch_add(self.h, C.byref(pr)))

    def rst_batch_run(self, total_energies=None):
        n = int(total_energies if total_energies is not None else getattr(self, "_batch_ne", 0))
        t = np.zeros(max(n, 1))
        st = rst_stats()
        s = self._chk(self.lib.rst_batch_run(self.h, _ptr(t), C.byref(st)), allow_noconv=True)
        return t[:n], st.as_dict(), s

    # -- learned correction network
    def rst_cnn_seed(self, seed: int):
        return self._chk(self.lib.rst_cnn_seed(self.h, int(seed)))

    def rst_cnn_set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        return self._chk(self.lib.rst_cnn_set_weights(self.h, _ptr(w), w.size))

    def rst_cnn_get_weights(self):
        w = np.zeros(self.lib.rst_cnn_weight_count(), np.float32)
        self._chk(self.lib.rst_cnn_get_weights(self.h, _ptr(w), w.size))
        return w

    def rst_cnn_forward(self, x_dev_ptr: int, out_dev_ptr: int, ncol, nz, nb, na):
        return self._chk(self.lib.rst_cnn_forward(self.h, int(ncol), int(nz), int(nb), int(na),
                                                  C.c_void_p(x_dev_ptr), C.c_void_p(out_dev_ptr)))

    def rst_cnn_gradient(self, x_dev_ptr: int, gout_dev_ptr: int, ncol, nz, nb, na):
        g = np.zeros(self.lib.rst_cnn_weight_count(), np.float32)
        self._chk(self.lib.rst_cnn_gradient(self.h, int(ncol), int(nz), int(nb), int(na),
                                            C.c_void_p(x_dev_ptr), C.c_void_p(gout_dev_ptr), _ptr(g)))
        return g

    def rst_cnn_train_step(self, x_dev_ptr: int, tgt_dev_ptr: int, ncol, nz, nb, na, lr):
        loss = C.c_double(0.0)
        self._chk(self.lib.rst_cnn_train_step(self.h, int(ncol), int(nz), int(nb), int(na),
                                              C.c_void_p(x_dev_ptr), C.c_void_p(tgt_dev_ptr),
                                              float(lr), C.byref(loss)))
        return loss.value

    def rst_precond_train(self, energies, kpts, pairs, batch=8, lr=1e-3, seed=0, source=0):
        e = np.ascontiguousarray(np.atleast_1d(energies), np.float64)
        k = np.ascontiguousarray(np.asarray(kpts, np.float64).reshape(-1, 2))
        o = rst_train_opts(int(pairs), int(batch), float(lr), int(seed), e.size, _ptr(e).value,
                           k.shape[0], _ptr(k).value, int(source))
        st = rst_train_stats()
        self._chk(self.lib.rst_precond_train(self.h, C.byref(o), C.byref(st)))
        return st.as_dict()

    # -- convenience
    def load_problem(self, prob, k=None):
        """Sets grid, potential, projectors, CAPs and k from a workloads.Problem."""
        self.rst_set_grid(prob.na, prob.nb, prob.nz, prob.ha, prob.hb, prob.hz, prob.order)
        self.rst_set_potential(prob.v)
        pj = prob.proj
        if pj.nproj:
            self.rst_set_projectors(pj.offs, pj.pt, pj.img.reshape(-1), pj.beta, pj.ekb)
        self.rst_set_abc(prob.gamma_l, prob.gamma_r)
        kk = prob.kpts[0] if k is None else k
        self.rst_set_k(kk[0], kk[1])


def apply_h(ctx: Context, energy: float, x):
    """y = (E - H_k + i Gamma) x for a torch CUDA tensor x of shape (n, ncol):
    complex128 (FP64 apply) or complex64 (FP32 stencil, FP64 projections)."""
    import torch
    assert x.is_cuda and x.dtype in (torch.complex128, torch.complex64) and x.is_contiguous()
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    prec = RST_FP32_REFINE if x.dtype == torch.complex64 else RST_FP64
    ctx.rst_apply_h(energy, x.data_ptr(), y.data_ptr(), x.shape[1], prec)
    return y


def to_blocked(x, col_block: int):
    """(n, ncol) column-fastest -> the blocked layout (ncol/col_block, n, col_block)."""
    n, ncol = x.shape
    return x.reshape(n, ncol // col_block, col_block).permute(1, 0, 2).contiguous()


def from_blocked(xb):
    """Blocked (nblk, n, col_block) -> (n, nblk*col_block) column-fastest."""
    nblk, n, cw = xb.shape
    return xb.permute(1, 0, 2).reshape(n, nblk * cw)


def apply_h_blocked(ctx: Context, energy: float, xb):
    """y = (E - H_k + i Gamma) x for x in the blocked layout, a torch complex128
    CUDA tensor of shape (nblk, n, col_block)."""
    import torch
    assert xb.is_cuda and xb.dtype == torch.complex128 and xb.is_contiguous() and xb.dim() == 3
    yb = torch.empty_like(xb)
    torch.cuda.synchronize()
    ctx.rst_apply_h_blocked(energy, xb.data_ptr(), yb.data_ptr(), xb.shape[0] * xb.shape[2], xb.shape[2])
    return yb


def solve_columns(ctx: Context, energy: float, cols, n: int, device="cuda"):
    """Columns G e_c of the Green's function as a torch complex128 (n, ncol) tensor."""
    import torch
    cols = np.asarray(cols, np.int64)
    x = torch.zeros((n, cols.size), dtype=torch.complex128, device=device)
    torch.cuda.synchronize()
    st, s = ctx.rst_solve_columns(energy, cols, x.data_ptr())
    return x, st, s


def cnn_forward(ctx: Context, x):
    """f(x) for a torch float32 CUDA tensor x of shape (ncol, nz, nb, na, 4) -> (ncol, nz, nb, na, 2)."""
    import torch
    assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape[-1] == 4
    out = torch.empty(x.shape[:-1] + (2,), dtype=torch.float32, device=x.device)
    torch.cuda.synchronize()
    ctx.rst_cnn_forward(x.data_ptr(), out.data_ptr(), x.shape[0], x.shape[1], x.shape[2], x.shape[3])
    return out


def cnn_gradient(ctx: Context, x, gout):
    """Weight gradient of <gout, f(x)> (weight layout, float32 numpy)."""
    import torch
    assert x.is_contiguous() and gout.is_contiguous() and gout.dtype == torch.float32
    torch.cuda.synchronize()
    return ctx.rst_cnn_gradient(x.data_ptr(), gout.data_ptr(), x.shape[0], x.shape[1], x.shape[2], x.shape[3])


def cnn_train_step(ctx: Context, x, tgt, lr):
    import torch
    assert x.is_contiguous() and tgt.is_contiguous()
    torch.cuda.synchronize()
    return ctx.rst_cnn_train_step(x.data_ptr(), tgt.data_ptr(), x.shape[0], x.shape[1], x.shape[2],
                                  x.shape[3], lr)


def solve_rhs(ctx: Context, energies, b, per_energy=False):
    """x = G(E) b for a torch complex128 CUDA tensor b of shape (n, ncol) (the same
    right-hand sides for every energy) or (n, n_e*ncol) with per_energy; returns
    x of shape (n, n_e*ncol), column e*ncol + j for energy e."""
    import torch
    e = np.atleast_1d(np.asarray(energies, np.float64))
    assert b.is_cuda and b.dtype == torch.complex128 and b.is_contiguous()
    ncol = b.shape[1] // (e.size if per_energy else 1)
    x = torch.zeros((b.shape[0], e.size * ncol), dtype=torch.complex128, device=b.device)
    torch.cuda.synchronize()
    st, s = ctx.rst_solve_rhs(e, ncol, b.data_ptr(), ncol if per_energy else 0, x.data_ptr())
    return x, st, s
