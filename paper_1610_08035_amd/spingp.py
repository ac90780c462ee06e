"""Thin Python binding of the C ABI in include/spingp.h (argument marshalling only).

Every step of the computation runs in the gfx950 library ``libspingp.so``; this module only
turns torch tensors into device pointers and the current HIP stream into the handle's
stream.  It raises if the library is missing or no GPU is present: there is no CPU path.
The functions carry the C names; `Handle` bundles them for convenience.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspingp.so")

MATERN32, MATERN52, PERIODIC, MATERN12, MATERN72, QUASIPERIODIC, SQEXP = 1, 2, 3, 4, 5, 6, 7

ERRORS = {
    0: "ok", 1: "invalid argument", 2: "call order", 3: "unsorted times", 4: "non-finite input",
    5: "bad hyperparameter", 6: "out of device memory", 7: "HIP runtime error", 8: "unsupported",
}


class SpinGPError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {ERRORS.get(code, code)} (status {code})")
        self.code = code


class _Term(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("harmonics", ctypes.c_int32)]


_lib = None


def library_loaded() -> bool:
    return _lib is not None


def load_library():
    """Load libspingp.so (built in-tree by __graft_entry__.build()); raise loudly otherwise."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.spingp_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Term), i32, i64, i32, vp]
    lib.spingp_destroy.argtypes = [vp]
    lib.spingp_state_dim.argtypes = [vp]
    lib.spingp_n_hyper.argtypes = [vp]
    lib.spingp_assemble.argtypes = [vp, vp, vp, vp, i32, i64, vp, u32]
    lib.spingp_factor.argtypes = [vp]
    lib.spingp_logml.argtypes = [vp, vp, vp, vp]
    lib.spingp_solve.argtypes = [vp, vp, vp]
    lib.spingp_selinv.argtypes = [vp, vp, vp, vp]
    lib.spingp_logml_grad.argtypes = [vp, vp, vp, vp]
    lib.spingp_status.argtypes = [vp, ctypes.POINTER(i64)]
    lib.spingp_profile.argtypes = [vp, ctypes.c_int]
    lib.spingp_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.spingp_strerror.argtypes = [ctypes.c_int]
    lib.spingp_strerror.restype = ctypes.c_char_p
    lib.spingp_workspace_bytes.argtypes = [vp]
    lib.spingp_workspace_bytes.restype = i64
    lib.spingp_tile_count.argtypes = []
    lib.spingp_tile_shape.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.spingp_get_tile.argtypes = [vp, ctypes.POINTER(i32)]
    lib.spingp_set_tile.argtypes = [vp, i32]
    lib.spingp_tune.argtypes = [vp, i32]
    lib.spingp_blocks.argtypes = [vp, vp, vp, vp, vp]
    lib.spingp_predict.argtypes = [vp, vp, vp, i64, vp, vp]
    lib.spingp_logml_grad_noalloc.argtypes = [ctypes.POINTER(_Term), i32, vp, vp, i64, vp, vp, vp, vp]
    for name in ("spingp_create", "spingp_destroy", "spingp_state_dim", "spingp_n_hyper", "spingp_assemble",
                 "spingp_factor", "spingp_logml", "spingp_solve", "spingp_selinv", "spingp_logml_grad",
                 "spingp_status", "spingp_profile", "spingp_profile_read", "spingp_tile_count",
                 "spingp_tile_shape", "spingp_get_tile", "spingp_set_tile", "spingp_tune", "spingp_blocks", "spingp_predict",
                 "spingp_logml_grad_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc, where):
    if rc != 0:
        raise SpinGPError(rc, where)


def _dev(x, name, n=None):
    if x is None:
        return None
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor on the GPU")
    if n is not None and x.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {x.numel()}")
    return ctypes.c_void_p(x.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# --------------------------------------------------------------------------- C-named calls
def spingp_create(terms, max_points, max_series=1, stream=None):
    lib = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the SpInGP library runs on the GPU only")
    arr = (_Term * len(terms))(*[_Term(k, h) for k, h in terms])
    h = ctypes.c_void_p()
    _check(lib.spingp_create(ctypes.byref(h), arr, len(terms), int(max_points), int(max_series),
                             _stream_ptr(stream)), "spingp_create")
    return h


def spingp_destroy(h):
    _check(load_library().spingp_destroy(h), "spingp_destroy")


FLAG_GRAPH = 1
FLAG_AUTOTUNE = 2


def spingp_assemble(h, t, y, hyper, offsets=None, n_series=1, flags=0):
    n = t.numel()
    lib = load_library()
    off = None
    if offsets is not None:
        if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
            raise ValueError("offsets must be a contiguous int64 tensor on the GPU")
        if offsets.numel() != int(n_series) + 1:
            raise ValueError(f"offsets must have n_series + 1 = {int(n_series) + 1} entries")
        off = ctypes.c_void_p(offsets.data_ptr())
    nh = lib.spingp_n_hyper(h) * int(n_series)
    _check(lib.spingp_assemble(h, _dev(t, "t"), _dev(y, "y", n), off, int(n_series), int(n),
                               _dev(hyper, "hyper", nh), int(flags)), "spingp_assemble")


def spingp_factor(h):
    _check(load_library().spingp_factor(h), "spingp_factor")


def spingp_logml(h, logml, datafit=None, logdet=None):
    _check(load_library().spingp_logml(h, _dev(logml, "logml"), _dev(datafit, "datafit"), _dev(logdet, "logdet")),
           "spingp_logml")


def spingp_solve(h, f_mean=None, z_mean=None):
    _check(load_library().spingp_solve(h, _dev(f_mean, "f_mean"), _dev(z_mean, "z_mean")), "spingp_solve")


def spingp_selinv(h, f_var=None, S_diag=None, S_sub=None):
    _check(load_library().spingp_selinv(h, _dev(f_var, "f_var"), _dev(S_diag, "S_diag"), _dev(S_sub, "S_sub")),
           "spingp_selinv")


def spingp_logml_grad(h, logml, grad, mask=None):
    """mask: None (every gradient component) or a sequence of n_hyper truth values (host); the
    components masked off are written as 0."""
    m = None
    if mask is not None:
        m = (ctypes.c_uint8 * len(mask))(*[1 if v else 0 for v in mask])
    _check(load_library().spingp_logml_grad(h, _dev(logml, "logml"), _dev(grad, "grad"), m), "spingp_logml_grad")


def spingp_logml_grad_noalloc(terms, t, y, hyper, logml, grad, stream=None):
    """logML and gradient of one Matern series without a handle or any device allocation (the
    library's fixed workspace array); for callers that cannot allocate."""
    n = t.numel()
    arr = (_Term * len(terms))(*[_Term(k, h) for k, h in terms])
    _check(load_library().spingp_logml_grad_noalloc(arr, len(terms), _dev(t, "t"), _dev(y, "y", n), int(n),
                                                    _dev(hyper, "hyper", 3), _dev(logml, "logml", 1),
                                                    _dev(grad, "grad", 3), _stream_ptr(stream)),
           "spingp_logml_grad_noalloc")


def spingp_predict(h, t_star, f_mean=None, f_var=None, offsets_star=None):
    m = t_star.numel()
    off = None
    if offsets_star is not None:
        if offsets_star.dtype != torch.int64 or not offsets_star.is_cuda or not offsets_star.is_contiguous():
            raise ValueError("offsets_star must be a contiguous int64 tensor on the GPU")
        off = ctypes.c_void_p(offsets_star.data_ptr())
    _check(load_library().spingp_predict(h, _dev(t_star, "t_star"), off, int(m), _dev(f_mean, "f_mean", m),
                                         _dev(f_var, "f_var", m)), "spingp_predict")


def spingp_blocks(h, A=None, Q=None, D=None, Bsub=None):
    _check(load_library().spingp_blocks(h, _dev(A, "A"), _dev(Q, "Q"), _dev(D, "D"), _dev(Bsub, "Bsub")),
           "spingp_blocks")


def spingp_status(h):
    bad = ctypes.c_int64(-1)
    rc = load_library().spingp_status(h, ctypes.byref(bad))
    return rc, bad.value


N_KERNELS = 6
KERNEL_NAMES = ("validate", "fwd_fold_tree", "top_tree", "bwd_elim_adjoint", "series_reduce", "graph")


def spingp_workspace_bytes(h):
    return int(load_library().spingp_workspace_bytes(h))


def spingp_tile_count():
    return int(load_library().spingp_tile_count())


def spingp_tile_shape(i):
    r, l = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().spingp_tile_shape(int(i), ctypes.byref(r), ctypes.byref(l)), "spingp_tile_shape")
    return r.value, l.value


def spingp_get_tile(h):
    i = ctypes.c_int32()
    _check(load_library().spingp_get_tile(h, ctypes.byref(i)), "spingp_get_tile")
    return i.value


def spingp_set_tile(h, i):
    _check(load_library().spingp_set_tile(h, int(i)), "spingp_set_tile")


def spingp_tune(h, reps=3):
    _check(load_library().spingp_tune(h, int(reps)), "spingp_tune")


def spingp_profile(h, enable):
    _check(load_library().spingp_profile(h, int(bool(enable))), "spingp_profile")


def spingp_profile_read(h):
    ms = (ctypes.c_double * N_KERNELS)()
    cnt = (ctypes.c_int64 * N_KERNELS)()
    _check(load_library().spingp_profile_read(h, ms, cnt), "spingp_profile_read")
    return {KERNEL_NAMES[i]: (ms[i], cnt[i]) for i in range(N_KERNELS)}


# --------------------------------------------------------------------------- convenience
class Handle:
    """One model, one stream, workspace sized for `max_points`."""

    def __init__(self, terms, max_points, max_series=1, stream=None):
        self.terms = [tuple(x) for x in terms]
        self.stream = stream            # None: torch's current stream at creation
        self._h = spingp_create(self.terms, max_points, max_series, stream)
        lib = load_library()
        self.b = lib.spingp_state_dim(self._h)
        self.n_hyper = lib.spingp_n_hyper(self._h)
        self.n = 0
        self.n_series = 1
        self._keep = ()

    def close(self):
        if self._h is not None:
            spingp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assemble(self, t, y, hyper, offsets=None, graph=False, autotune=False):
        n_series = 1 if offsets is None else offsets.numel() - 1
        flags = (FLAG_GRAPH if graph else 0) | (FLAG_AUTOTUNE if autotune else 0)
        spingp_assemble(self._h, t, y, hyper, offsets, n_series, flags)
        self.n = t.numel()
        self.n_series = n_series
        self._keep = (t, y, hyper, offsets)   # keep the bound buffers alive

    def factor(self):
        spingp_factor(self._h)

    def logml(self, parts=False):
        dev = self._keep[0].device
        out = torch.empty(self.n_series, dtype=torch.float64, device=dev)
        if not parts:
            spingp_logml(self._h, out)
            return out
        fit = torch.empty_like(out)
        ld = torch.empty_like(out)
        spingp_logml(self._h, out, fit, ld)
        return out, fit, ld

    def solve(self, states=False):
        dev = self._keep[0].device
        f = torch.empty(self.n, dtype=torch.float64, device=dev)
        z = torch.empty(self.b, self.n, dtype=torch.float64, device=dev) if states else None
        spingp_solve(self._h, f, z)
        return (f, z) if states else f

    def selinv(self, blocks=False):
        dev = self._keep[0].device
        v = torch.empty(self.n, dtype=torch.float64, device=dev)
        if not blocks:
            spingp_selinv(self._h, v)
            return v
        sd = torch.empty(self.b * (self.b + 1) // 2, self.n, dtype=torch.float64, device=dev)
        ss = torch.zeros(self.b * self.b, self.n, dtype=torch.float64, device=dev)
        spingp_selinv(self._h, v, sd, ss)
        return v, sd, ss

    def logml_grad(self, mask=None):
        dev = self._keep[0].device
        ll = torch.empty(self.n_series, dtype=torch.float64, device=dev)
        g = torch.empty(self.n_series, self.n_hyper, dtype=torch.float64, device=dev)
        spingp_logml_grad(self._h, ll, g, mask)
        return ll, g

    def status(self):
        return spingp_status(self._h)

    @property
    def tile(self):
        return spingp_get_tile(self._h)

    @tile.setter
    def tile(self, i):
        spingp_set_tile(self._h, i)

    def tune(self, reps=3):
        spingp_tune(self._h, reps)
        return self.tile

    def workspace_bytes(self):
        return spingp_workspace_bytes(self._h)

    def predict(self, t_star, offsets_star=None):
        """Latent predictive mean and variance at the times t_star (sorted within each series;
        offsets_star [n_series + 1] splits them by series on a batched handle)."""
        if offsets_star is not None and offsets_star.numel() != self.n_series + 1:
            raise ValueError(f"offsets_star must have n_series + 1 = {self.n_series + 1} entries")
        fm = torch.empty_like(t_star)
        fv = torch.empty_like(t_star)
        spingp_predict(self._h, t_star, fm, fv, offsets_star)
        return fm, fv

    def blocks(self):
        """Materialised (A, Q, D, Bsub) SoA blocks (see spingp_blocks)."""
        dev = self._keep[0].device
        b, n = self.b, self.n
        A = torch.zeros(b * b, n, dtype=torch.float64, device=dev)
        Q = torch.zeros(b * (b + 1) // 2, n, dtype=torch.float64, device=dev)
        D = torch.zeros_like(Q)
        Bs = torch.zeros_like(A)
        spingp_blocks(self._h, A, Q, D, Bs)
        return A, Q, D, Bs
