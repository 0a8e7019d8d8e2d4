"""ctypes access to the C reference (oracle/lb_oracle.c): the library's C ABI
on host (numpy) arrays.

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.
"""

import ctypes
import os

import numpy as np

from .build import LIB

_vp, _i32, _int = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
_lib = None


def _params_type():
    """The lb_params struct of include/lb.h (field order and types)."""
    class P(ctypes.Structure):
        _fields_ = [("nx", _i32), ("ny", _i32), ("nz", _i32), ("model", _i32), ("storage", _i32), ("vvl", _i32),
                    ("collision", _i32), ("binary_step", _i32), ("tau_f", ctypes.c_double), ("A", ctypes.c_double),
                    ("B", ctypes.c_double), ("kappa", ctypes.c_double), ("mobility", ctypes.c_double),
                    ("gamma", ctypes.c_double), ("rho0", ctypes.c_double), ("phi0", ctypes.c_double),
                    ("tau_minus", ctypes.c_double), ("tau_bulk", ctypes.c_double),
                    ("tau_ghost_even", ctypes.c_double), ("tau_ghost_odd", ctypes.c_double)]
    return P


Params = _params_type()


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError("C reference not built (python -m oracle.build)")
        lib = ctypes.CDLL(LIB)
        sig = {"lb_workspace_bytes": [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)],
               "lb_create": [ctypes.POINTER(Params), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)],
               "lb_init_equilibrium": [_vp, _vp, _vp, _vp], "lb_collide": [_vp], "lb_propagate": [_vp],
               "lb_step": [_vp, _i32], "lb_moments": [_vp, _vp, _vp, _vp], "lb_conserved_sums": [_vp, _vp],
               "lb_get_state": [_vp, _vp, _vp], "lb_set_state": [_vp, _vp, _vp], "lb_destroy": [_vp]}
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.restype, fn.argtypes = _int, args
        lib.lb_strerror.restype, lib.lb_strerror.argtypes = ctypes.c_char_p, [_int]
        lib.lb_oracle_set_threads.restype, lib.lb_oracle_set_threads.argtypes = _int, [_int]
        _lib = lib
    return _lib


def set_threads(n):
    """Threads of the C reference's site loops (n <= 0: all host cores);
    returns the count used.  Results do not depend on it."""
    return int(load().lb_oracle_set_threads(int(n)))


def _workspace(count):
    """Zeroed host array for the reference's fields.  numpy asks for
    transparent huge pages on large arrays; the reference's 19-direction
    arrays are N doubles apart, so on 2 MiB pages all of a site's values
    fall into the same cache sets (measured 2.2x slower at 64^3).  Small
    pages scatter them."""
    hp = np._core.multiarray
    was = hp._set_madvise_hugepage(False)
    try:
        return np.zeros(count, dtype=np.float64)
    finally:
        hp._set_madvise_hugepage(was)


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data


class CLattice:
    """One context of the C reference on a host workspace.  Shapes as in
    the numpy reference: (nz, ny, nx) scalars, (19, nz, ny, nx) states."""

    def __init__(self, nx, ny, nz, model=0, tau_f=1.0, A=-0.0625, B=0.0625, kappa=0.04, mobility=0.45,
                 gamma=1.0, storage=0, collision=0):
        lib = load()
        self.p = Params(nx, ny, nz, model, storage, 1, collision, 0, tau_f, A, B, kappa, mobility, gamma,
                        1.0, 0.0, tau_f, tau_f, tau_f, tau_f)
        self.shape = (nz, ny, nx)
        self.binary = model == 1
        n = ctypes.c_size_t(0)
        self.status = lib.lb_workspace_bytes(ctypes.byref(self.p), ctypes.byref(n))
        if self.status != 0:
            raise ValueError(lib.lb_strerror(self.status).decode())
        self.ws = _workspace(n.value // 8)
        self.ctx = _vp()
        rc = lib.lb_create(ctypes.byref(self.p), _ptr(self.ws), n.value, None, ctypes.byref(self.ctx))
        assert rc == 0, rc

    def _call(self, name, *args):
        rc = getattr(load(), name)(self.ctx, *args)
        assert rc == 0, (name, rc)

    def init_equilibrium(self, rho, u, phi=None):
        c = lambda a: np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
        self._in = (c(rho), c(u), c(phi))
        self._call("lb_init_equilibrium", *(_ptr(a) for a in self._in))

    def collide(self):
        self._call("lb_collide")

    def propagate(self):
        self._call("lb_propagate")

    def step(self, n):
        self._call("lb_step", int(n))

    def state(self):
        f = np.empty((19,) + self.shape)
        g = np.empty_like(f) if self.binary else None
        self._call("lb_get_state", _ptr(f), _ptr(g))
        return f, g

    def set_state(self, f, g=None):
        self._st = (np.ascontiguousarray(f, dtype=np.float64),
                    np.ascontiguousarray(g, dtype=np.float64) if g is not None else None)
        self._call("lb_set_state", *(_ptr(a) for a in self._st))

    def moments(self):
        rho, u = np.empty(self.shape), np.empty((3,) + self.shape)
        phi = np.empty(self.shape) if self.binary else None
        self._call("lb_moments", _ptr(rho), _ptr(u), _ptr(phi))
        return rho, u, phi

    def sums(self):
        out = np.empty(5)
        self._call("lb_conserved_sums", _ptr(out))
        return out

    def close(self):
        if self.ctx:
            load().lb_destroy(self.ctx)
            self.ctx = None
