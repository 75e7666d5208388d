"""Thin ctypes binding of the HIP library ``libhobi.so`` (C ABI in ``include/hobi.h``).

Argument marshalling only: every step of the method runs in the library's kernels.  The
module-level functions carry the C names; ``Context`` and ``Problem`` wrap the handles.
Host arrays are numpy; device vectors may be torch tensors on the GPU (their
``data_ptr()`` is passed with ``on_device=1``), torch being used for device memory and
streams only.  There is no fallback: if the library is missing or a call fails, an
exception is raised.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhobi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hobi.h")

HOBI_FP64 = 0
HOBI_MIXED = 1
HOBI_HIGHER_ORDER = 0
HOBI_LOWER_ORDER = 1

STATUS = {0: "HOBI_OK", 1: "HOBI_E_ARG", 2: "HOBI_E_MESH", 3: "HOBI_E_CHARGE_OUTSIDE",
          4: "HOBI_E_NOCONV", 5: "HOBI_E_OOM", 6: "HOBI_E_HIP", 7: "HOBI_E_NUMERIC",
          8: "HOBI_E_BUSY"}


class HobiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class hobi_params(ctypes.Structure):
    _fields_ = [("eps1", ctypes.c_double), ("eps2", ctypes.c_double), ("kappa", ctypes.c_double),
                ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("method", ctypes.c_int32), ("diag_scaling", ctypes.c_int32),
                ("tree_theta", ctypes.c_double), ("tree_degree", ctypes.c_int32), ("tree_leaf", ctypes.c_int32),
                ("tree_batch", ctypes.c_int32), ("tree_refine", ctypes.c_int32)]


class hobi_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("est_residual", ctypes.c_double), ("true_residual", ctypes.c_double),
                ("ms_setup", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("ms_energy", ctypes.c_double), ("pairs_per_matvec", ctypes.c_int64),
                ("ms_pair_kernel", ctypes.c_double), ("pair_launches", ctypes.c_int64),
                ("ms_gather", ctypes.c_double), ("ms_combine", ctypes.c_double),
                ("ms_krylov", ctypes.c_double), ("ms_field_kernel", ctypes.c_double),
                ("field_launches", ctypes.c_int64), ("tree_far_pairs", ctypes.c_int64),
                ("tree_near_pairs", ctypes.c_int64), ("field_tree_far_pairs", ctypes.c_int64),
                ("field_tree_near_pairs", ctypes.c_int64), ("refine_steps", ctypes.c_int32),
                ("dense_matvecs", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)
_SIGS = {
    "hobi_params_default": (None, [ctypes.POINTER(hobi_params)]),
    "hobi_ctx_create": (ctypes.c_int, [ctypes.c_int, _P, ctypes.POINTER(_P)]),
    "hobi_ctx_destroy": (None, [_P]),
    "hobi_last_error": (ctypes.c_char_p, [_P]),
    "hobi_ctx_set_profiling": (ctypes.c_int, [_P, ctypes.c_int32]),
    "hobi_ctx_stream": (_P, [_P]),
    "hobi_problem_create": (ctypes.c_int, [_P, ctypes.c_int32, _D, _D, ctypes.c_int32, _I,
                                           ctypes.c_int32, _D, _D, ctypes.POINTER(hobi_params),
                                           ctypes.POINTER(_P)]),
    "hobi_problem_destroy": (None, [_P]),
    "hobi_problem_set_precision": (ctypes.c_int, [_P, ctypes.c_int32]),
    "hobi_problem_set_solver": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]),
    "hobi_problem_set_dielectric": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "hobi_solve": (ctypes.c_int, [_P, _D, _D, _D, ctypes.POINTER(hobi_stats)]),
    "hobi_matvec": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "hobi_matvec_noalloc": (ctypes.c_int, [_P, _P, _P]),
    "hobi_device_math": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _D, _D]),
    "hobi_energy": (ctypes.c_int, [_P, _P, ctypes.c_int32, _D]),
    "hobi_field": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _D, _D, _D, _D, _D, _I]),
    "hobi_get_nodes": (ctypes.c_int, [_P, _D, _D, _D]),
    "hobi_get_rhs": (ctypes.c_int, [_P, _D]),
    "hobi_reset_stats": (ctypes.c_int, [_P]),
    "hobi_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(hobi_stats)]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1301_5914_amd.build`")
        # torch ships its own HIP runtime under the same soname; loading torch first makes
        # the library bind to that one, so that a process holds a single HIP runtime and
        # torch's device pointers and streams are valid in the library.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols(path: str = HEADER):
    """Function names declared in the C header."""
    text = open(path).read()
    return sorted(set(re.findall(r"\b(hobi_[a-z_0-9]+)\s*\(", text)))


def _dptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---------------------------------------------------------------- C-named functions

def hobi_params_default() -> hobi_params:
    p = hobi_params()
    lib().hobi_params_default(ctypes.byref(p))
    return p


def hobi_ctx_create(device: int = 0, stream: int | None = None):
    h = _P()
    st = lib().hobi_ctx_create(int(device), _P(stream) if stream else None, ctypes.byref(h))
    if st != 0:
        raise HobiError(st, "hobi_ctx_create failed")
    return h


HOBI_MATH_EXP_NEG, HOBI_MATH_RSQRT = 0, 1


def hobi_device_math(ctx, fn: int, x) -> np.ndarray:
    """The FP64 pair kernel's exp(-x) (fn 0) or 1/sqrt(x) (fn 1) on the device, host arrays."""
    x = _f64(x).ravel()
    y = np.empty_like(x)
    _check(ctx.handle, lib().hobi_device_math(ctx.handle, fn, x.shape[0], _dptr(x), _dptr(y)))
    return y


def hobi_last_error(ctx) -> str:
    msg = lib().hobi_last_error(ctx)
    return msg.decode() if msg else ""


def _check(ctx, st):
    if st != 0:
        raise HobiError(st, hobi_last_error(ctx))


class Context:
    """A device + stream (``stream`` may be a torch.cuda.Stream or a raw hipStream_t)."""

    def __init__(self, device: int = 0, stream=None, profiling: bool = False):
        raw = getattr(stream, "cuda_stream", stream)
        if stream is not None and not raw:
            raise ValueError("the legacy default stream (handle 0) cannot be shared; pass a "
                             "non-default stream, or None for a stream owned by the context")
        self.handle = hobi_ctx_create(device, raw)
        self.device = device
        if profiling:
            self.set_profiling(True)

    def set_profiling(self, on: bool):
        _check(self.handle, lib().hobi_ctx_set_profiling(self.handle, 1 if on else 0))

    @property
    def stream(self) -> int:
        return lib().hobi_ctx_stream(self.handle) or 0

    def close(self):
        if getattr(self, "handle", None):
            lib().hobi_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """One surface + charge set with its setup resident on the device."""

    def __init__(self, ctx: Context, xyz, nrm, tri, qpos, q, eps1=1.0, eps2=80.0, kappa=0.1257,
                 rtol=1e-6, max_iter=200, restart=200, precision=HOBI_FP64, method=HOBI_HIGHER_ORDER,
                 diag_scaling=2, tree_theta=0.0, tree_degree=5, tree_leaf=256, tree_batch=128, tree_refine=0):
        self.ctx = ctx
        xyz = _f64(xyz).reshape(-1, 3)
        nrm = _f64(nrm).reshape(-1, 3)
        tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32).reshape(-1, 3))
        qpos = _f64(qpos).reshape(-1, 3)
        q = _f64(q).ravel()
        self.nv, self.nf, self.nc = xyz.shape[0], tri.shape[0], q.shape[0]
        self.method = method
        # unknowns per site: vertices (higher-order) or triangles (lower-order)
        self.nu = self.nf if method == HOBI_LOWER_ORDER else self.nv
        p = hobi_params_default()
        p.eps1, p.eps2, p.kappa, p.rtol = eps1, eps2, kappa, rtol
        p.max_iter, p.restart, p.precision, p.method = max_iter, restart, precision, method
        p.diag_scaling = diag_scaling
        p.tree_theta, p.tree_degree, p.tree_leaf, p.tree_batch = tree_theta, tree_degree, tree_leaf, tree_batch
        p.tree_refine = tree_refine
        h = _P()
        st = lib().hobi_problem_create(ctx.handle, self.nv, _dptr(xyz), _dptr(nrm), self.nf,
                                       tri.ctypes.data_as(_I), self.nc, _dptr(qpos), _dptr(q),
                                       ctypes.byref(p), ctypes.byref(h))
        _check(ctx.handle, st)
        self.handle = h

    @classmethod
    def from_inputs(cls, ctx, prob, **kw):
        return cls(ctx, prob.xyz, prob.nrm, prob.tri, prob.qpos, prob.q, prob.eps1, prob.eps2,
                   prob.kappa, **kw)

    def _chk(self, st):
        _check(self.ctx.handle, st)

    def set_precision(self, precision: int):
        self._chk(lib().hobi_problem_set_precision(self.handle, precision))

    def set_dielectric(self, eps1, eps2, kappa):
        """New eps1, eps2, kappa; re-runs the device setup on the resident surface."""
        self._chk(lib().hobi_problem_set_dielectric(self.handle, eps1, eps2, kappa))

    def set_solver(self, rtol=1e-6, max_iter=200, restart=200):
        self._chk(lib().hobi_problem_set_solver(self.handle, rtol, max_iter, restart))

    def matvec(self, u, out=None):
        """y = A u.  numpy in -> numpy out (host copies); a device tensor in -> the
        result is written into ``out`` (a device tensor of the same size)."""
        if hasattr(u, "data_ptr"):
            if out is None:
                raise ValueError("device input needs a device output tensor")
            self._chk(lib().hobi_matvec(self.handle, _P(u.data_ptr()), _P(out.data_ptr()), 1))
            return out
        u = _f64(u).ravel()
        if u.shape[0] != 2 * self.nu:
            raise ValueError("u must have 2 entries per site")
        y = np.empty_like(u)
        self._chk(lib().hobi_matvec(self.handle, _P(u.ctypes.data), _P(y.ctypes.data), 0))
        return y

    def matvec_noalloc(self, u, out):
        """y = A u from device tensors into ``out`` through the allocation-free entry point
        (partial sums in the library's static work space; dense sum only)."""
        if not (hasattr(u, "data_ptr") and hasattr(out, "data_ptr")):
            raise ValueError("hobi_matvec_noalloc takes device tensors")
        if u.numel() != 2 * self.nu or out.numel() != 2 * self.nu:
            raise ValueError("u and out must have 2 entries per site")
        self._chk(lib().hobi_matvec_noalloc(self.handle, _P(u.data_ptr()), _P(out.data_ptr())))
        return out

    def energy(self, u) -> float:
        e = ctypes.c_double()
        if hasattr(u, "data_ptr"):
            self._chk(lib().hobi_energy(self.handle, _P(u.data_ptr()), 1, ctypes.byref(e)))
        else:
            u = _f64(u).ravel()
            self._chk(lib().hobi_energy(self.handle, _P(u.ctypes.data), 0, ctypes.byref(e)))
        return e.value

    def field(self, u, points):
        """Potential and field at points off the surface for the internal-unit solution u
        (numpy or a device tensor): dict of phi [np], field [np,3], reac [np],
        reac_field [np,3] (kcal/(mol e) [/A]) and inside [np] (int32)."""
        pts = _f64(points).reshape(-1, 3)
        n = pts.shape[0]
        out = dict(phi=np.empty(n), field=np.empty((n, 3)), reac=np.empty(n), reac_field=np.empty((n, 3)),
                   inside=np.empty(n, dtype=np.int32))
        if hasattr(u, "data_ptr"):
            uptr, dev = _P(u.data_ptr()), 1
        else:
            u = _f64(u).ravel()
            if u.shape[0] != 2 * self.nu:
                raise ValueError("u must have 2 entries per site")
            uptr, dev = _P(u.ctypes.data), 0
        self._chk(lib().hobi_field(self.handle, uptr, dev, n, _dptr(pts), _dptr(out["phi"]), _dptr(out["field"]),
                                   _dptr(out["reac"]), _dptr(out["reac_field"]),
                                   out["inside"].ctypes.data_as(_I)))
        return out

    def solve(self, allow_noconv: bool = False):
        phi = np.empty(self.nu)
        dphi = np.empty(self.nu)
        e = ctypes.c_double()
        st = hobi_stats()
        code = lib().hobi_solve(self.handle, _dptr(phi), _dptr(dphi), ctypes.byref(e), ctypes.byref(st))
        if code != 0 and not (allow_noconv and code == 4):
            self._chk(code)
        return dict(phi=phi, dphi=dphi, energy=e.value, stats=st.as_dict(), status=STATUS[code])

    def nodes(self):
        per = 1 if self.method == HOBI_LOWER_ORDER else 4
        y = np.empty((self.nf, per, 3))
        ny = np.empty((self.nf, per, 3))
        w = np.empty((self.nf, per))
        self._chk(lib().hobi_get_nodes(self.handle, _dptr(y), _dptr(ny), _dptr(w)))
        return y, ny, w

    def rhs(self):
        b = np.empty(2 * self.nu)
        self._chk(lib().hobi_get_rhs(self.handle, _dptr(b)))
        return b

    def reset_stats(self):
        self._chk(lib().hobi_reset_stats(self.handle))

    def stats(self):
        st = hobi_stats()
        self._chk(lib().hobi_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().hobi_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- request server

class hobi_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("active", ctypes.c_int32), ("pending", ctypes.c_int32),
                ("mean_batch", ctypes.c_double), ("bytes_in_use", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("busy_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_SIGS.update({
    "hobi_server_create": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    "hobi_server_submit": (ctypes.c_int, [_P, ctypes.c_int32, _D, _D, ctypes.c_int32, _I, ctypes.c_int32, _D, _D,
                                          ctypes.POINTER(hobi_params), ctypes.POINTER(ctypes.c_uint64)]),
    "hobi_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, _D, _D, _D, ctypes.POINTER(hobi_stats)]),
    "hobi_server_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(hobi_server_stats)]),
    "hobi_server_last_error": (ctypes.c_char_p, [_P]),
    "hobi_server_destroy": (None, [_P]),
})


class Server:
    """Continuous-batching request server on one device (hobi_server_* in the C ABI)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 8 << 30, max_slots: int = 64,
                 use_graph: bool = True):
        h = _P()
        _check(ctx.handle, lib().hobi_server_create(ctx.handle, int(hbm_budget_bytes), int(max_slots),
                                                    1 if use_graph else 0, ctypes.byref(h)))
        self.ctx = ctx
        self.handle = h
        self._nv = {}

    def _err(self, st):
        msg = lib().hobi_server_last_error(self.handle)
        raise HobiError(st, msg.decode() if msg else "")

    def submit(self, prob, rtol=1e-6, max_iter=300, precision=HOBI_MIXED, eps1=None, eps2=None,
               kappa=None, method=HOBI_HIGHER_ORDER, diag_scaling=2, tree_theta=0.0, tree_degree=5, tree_leaf=256,
               tree_batch=128, tree_refine=0) -> int:
        xyz = _f64(prob.xyz).reshape(-1, 3)
        nrm = _f64(prob.nrm).reshape(-1, 3)
        tri = np.ascontiguousarray(np.asarray(prob.tri, dtype=np.int32).reshape(-1, 3))
        qpos = _f64(prob.qpos).reshape(-1, 3)
        q = _f64(prob.q).ravel()
        p = hobi_params_default()
        p.eps1 = prob.eps1 if eps1 is None else eps1
        p.eps2 = prob.eps2 if eps2 is None else eps2
        p.kappa = prob.kappa if kappa is None else kappa
        p.rtol, p.max_iter, p.restart, p.precision, p.method = rtol, max_iter, max_iter, precision, method
        p.diag_scaling = diag_scaling
        p.tree_theta, p.tree_degree, p.tree_leaf, p.tree_batch = tree_theta, tree_degree, tree_leaf, tree_batch
        p.tree_refine = tree_refine
        t = ctypes.c_uint64()
        st = lib().hobi_server_submit(self.handle, xyz.shape[0], _dptr(xyz), _dptr(nrm), tri.shape[0],
                                      tri.ctypes.data_as(_I), q.shape[0], _dptr(qpos), _dptr(q),
                                      ctypes.byref(p), ctypes.byref(t))
        if st != 0:
            self._err(st)
        self._nv[t.value] = tri.shape[0] if method == HOBI_LOWER_ORDER else xyz.shape[0]
        return t.value

    def poll(self, ticket: int, raise_errors: bool = True):
        """None while the request is waiting or running, else its result dict."""
        nv = self._nv.get(ticket)
        phi = np.empty(nv) if nv else None
        dphi = np.empty(nv) if nv else None
        e = ctypes.c_double()
        st = hobi_stats()
        code = lib().hobi_server_poll(self.handle, ticket, _dptr(phi), _dptr(dphi), ctypes.byref(e),
                                      ctypes.byref(st))
        if code == 8:
            return None
        self._nv.pop(ticket, None)
        if code not in (0, 4) and raise_errors:
            self._err(code)
        return dict(phi=phi, dphi=dphi, energy=e.value, stats=st.as_dict(), status=STATUS[code])

    def stats(self):
        s = hobi_server_stats()
        lib().hobi_server_get_stats(self.handle, ctypes.byref(s))
        return s.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().hobi_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
