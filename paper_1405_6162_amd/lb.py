"""Python binding of liblb.so: the C ABI of include/lb.h, same names,
argument marshalling only.

Device memory and streams come from PyTorch: the workspace is a uint8 CUDA
(HIP) tensor, every array passed in or out is a contiguous device tensor,
and calls are queued on ``torch.cuda.current_stream()``.  Every step of the
update runs in the HIP kernels of liblb.so; there is no CPU fallback, and
``load()`` raises if the library has not been built.
"""

import ctypes
import os

import torch

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ENOTSUP, LB_ERANGE = 0, -1, -2, -3, -4, -5
LB_NOALLOC_MAX_BLOCKS = 262144
LB_SINGLE, LB_BINARY = 0, 1
LB_F64, LB_F32, LB_F16 = 0, 1, 2
LB_BGK, LB_TRT, LB_MRT = 0, 1, 2
LB_STEP_AUTO, LB_STEP_MARCH, LB_STEP_TWO_PASS = 0, 1, 2
LB_K_COLLIDE, LB_K_PHI, LB_K_STREAM, LB_K_ADJOINT, LB_K_OTHER = 0, 1, 2, 3, 4
Q = 19

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "liblb.so")

STORAGE_DTYPE = {LB_F64: torch.float64, LB_F32: torch.float32, LB_F16: torch.float16}


class LBError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        msg = _lib.lb_strerror(status).decode() if _lib is not None else str(status)
        super().__init__("%s failed: %s (%d)" % (fn, msg, status))


class lb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("model", ctypes.c_int32), ("storage", ctypes.c_int32), ("vvl", ctypes.c_int32),
        ("collision", ctypes.c_int32), ("binary_step", ctypes.c_int32),
        ("tau_f", ctypes.c_double),
        ("A", ctypes.c_double), ("B", ctypes.c_double), ("kappa", ctypes.c_double),
        ("mobility", ctypes.c_double), ("gamma", ctypes.c_double),
        ("rho0", ctypes.c_double), ("phi0", ctypes.c_double),
        ("tau_minus", ctypes.c_double),
        ("tau_bulk", ctypes.c_double), ("tau_ghost_even", ctypes.c_double), ("tau_ghost_odd", ctypes.c_double),
    ]


def make_params(nx, ny, nz, model=LB_SINGLE, storage=LB_F64, tau_f=1.0, A=-0.0625, B=0.0625,
                kappa=0.04, mobility=0.45, gamma=1.0, rho0=1.0, phi0=0.0, vvl=1, collision=LB_BGK,
                tau_minus=None, tau_bulk=None, tau_ghost_even=None, tau_ghost_odd=None, binary_step=0):
    """lb_params with defaults; the relaxation times not given default to the
    ones that make each collision reduce to the simpler one (TRT to BGK, MRT
    to TRT)."""
    tm = tau_f if tau_minus is None else tau_minus
    tb = tau_f if tau_bulk is None else tau_bulk
    tge = tau_f if tau_ghost_even is None else tau_ghost_even
    tgo = tm if tau_ghost_odd is None else tau_ghost_odd
    return lb_params(nx, ny, nz, model, storage, vvl, collision, binary_step, tau_f, A, B, kappa, mobility, gamma,
                     rho0, phi0, tm, tb, tge, tgo)


_lib = None
_vp, _i32, _int = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
_SIGNATURES = {
    "lb_workspace_bytes": (_int, [ctypes.POINTER(lb_params), ctypes.POINTER(ctypes.c_size_t)]),
    "lb_create": (_int, [ctypes.POINTER(lb_params), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "lb_set_stream": (_int, [_vp, _vp]),
    "lb_init_equilibrium": (_int, [_vp, _vp, _vp, _vp]),
    "lb_collide": (_int, [_vp]),
    "lb_propagate": (_int, [_vp]),
    "lb_step": (_int, [_vp, _i32]),
    "lb_moments": (_int, [_vp, _vp, _vp, _vp]),
    "lb_conserved_sums": (_int, [_vp, _vp]),
    "lb_field_stats": (_int, [_vp, _vp]),
    "lb_set_params": (_int, [_vp, _vp]),
    "lb_adjoint_step_binary": (_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp]),
    "lb_adjoint_init_binary": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lb_get_state": (_int, [_vp, _vp, _vp]),
    "lb_set_state": (_int, [_vp, _vp, _vp]),
    "lb_set_tau": (_int, [_vp, ctypes.c_double]),
    "lb_step_record": (_int, [_vp, _i32, _vp, _vp]),
    "lb_adjoint_step": (_int, [_vp, _vp, _int, _vp, _vp, _vp]),
    "lb_adjoint_segment": (_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "lb_adjoint_segment_binary": (_int, [_vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "lb_mask_index": (_int, [_vp, _vp, _vp, _vp]),
    "lb_get_sites": (_int, [_vp, _vp, ctypes.c_int64, _vp, _vp]),
    "lb_set_sites": (_int, [_vp, _vp, ctypes.c_int64, _vp, _vp]),
    "lb_profile": (_int, [_vp, _int]),
    "lb_profile_mask": (_int, [_vp, ctypes.c_uint]),
    "lb_kernel_times": (_int, [_vp, _int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "lb_destroy": (_int, [_vp]),
    "lb_stream_copy": (_int, [_vp, _vp, ctypes.c_size_t, _vp]),
    "lb_conserved_sums_noalloc": (_int, [ctypes.POINTER(lb_params), _vp, _vp, _vp, _vp]),
    "lb_strerror": (ctypes.c_char_p, [_int]),
}


def load(path=LIB_PATH):
    """Load liblb.so (once).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("liblb.so not built (%s); run python -m paper_1405_6162_amd.build" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype, fn.argtypes = res, args
    _lib = lib
    return lib


def _check(fn, rc):
    if rc != LB_OK:
        raise LBError(fn, rc)


def _ptr(t, dtype=None):
    """Device address of a contiguous CUDA tensor (None -> NULL); with dtype
    given, the tensor must have it (the C side reads raw memory)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("liblb.so takes device tensors")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected a %s tensor, got %s" % (dtype, t.dtype))
    return t.data_ptr()


def _f64(t):
    return _ptr(t, torch.float64)


def _stream():
    return torch.cuda.current_stream().cuda_stream


# ---- the C ABI, one Python function per symbol -----------------------------

def lb_workspace_bytes(params):
    load()
    n = ctypes.c_size_t(0)
    _check("lb_workspace_bytes", _lib.lb_workspace_bytes(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def lb_create(params, workspace, stream=None):
    load()
    ctx = _vp()
    nbytes = workspace.numel() * workspace.element_size()
    _check("lb_create", _lib.lb_create(ctypes.byref(params), _ptr(workspace), nbytes,
                                       _stream() if stream is None else stream, ctypes.byref(ctx)))
    return ctx


def lb_set_stream(ctx, stream):
    _check("lb_set_stream", _lib.lb_set_stream(ctx, stream))


def lb_init_equilibrium(ctx, rho, u, phi=None):
    _check("lb_init_equilibrium", _lib.lb_init_equilibrium(ctx, _f64(rho), _f64(u), _f64(phi)))


def lb_collide(ctx):
    _check("lb_collide", _lib.lb_collide(ctx))


def lb_propagate(ctx):
    _check("lb_propagate", _lib.lb_propagate(ctx))


def lb_step(ctx, nsteps):
    _check("lb_step", _lib.lb_step(ctx, int(nsteps)))


def lb_moments(ctx, rho, u, phi=None):
    _check("lb_moments", _lib.lb_moments(ctx, _f64(rho), _f64(u), _f64(phi)))


def lb_conserved_sums(ctx, out):
    _check("lb_conserved_sums", _lib.lb_conserved_sums(ctx, _f64(out)))


def lb_field_stats(ctx, out):
    _check("lb_field_stats", _lib.lb_field_stats(ctx, _f64(out)))


def lb_get_state(ctx, f, g=None):
    _check("lb_get_state", _lib.lb_get_state(ctx, _ptr(f), _ptr(g)))


def lb_set_state(ctx, f, g=None):
    _check("lb_set_state", _lib.lb_set_state(ctx, _ptr(f), _ptr(g)))


def lb_set_tau(ctx, tau_f):
    _check("lb_set_tau", _lib.lb_set_tau(ctx, float(tau_f)))


def lb_step_record(ctx, nsteps, post, phi=None):
    _check("lb_step_record", _lib.lb_step_record(ctx, int(nsteps), _ptr(post), _ptr(phi)))


def lb_adjoint_step(ctx, f, lam_next, lam_n, domega, f_pending=False):
    _check("lb_adjoint_step", _lib.lb_adjoint_step(ctx, _f64(f), 1 if f_pending else 0, _f64(lam_next),
                                                   _f64(lam_n), _f64(domega)))


def lb_set_params(ctx, params):
    _check("lb_set_params", _lib.lb_set_params(ctx, ctypes.byref(params)))


def lb_adjoint_step_binary(ctx, f, g, lf_next, lg_next, lf_n, lg_n, grads, pending=False, phi=None):
    _check("lb_adjoint_step_binary", _lib.lb_adjoint_step_binary(
        ctx, _f64(f), _f64(g), _f64(phi), 1 if pending else 0, _f64(lf_next), _f64(lg_next), _f64(lf_n),
        _f64(lg_n), _f64(grads)))


def lb_adjoint_init_binary(ctx, rho, u, phi, lf0, lg0, dphi, drho, du, dkappa):
    _check("lb_adjoint_init_binary", _lib.lb_adjoint_init_binary(
        ctx, _f64(rho), _f64(u), _f64(phi), _f64(lf0), _f64(lg0), _f64(dphi), _f64(drho), _f64(du),
        _f64(dkappa)))


def lb_adjoint_segment(ctx, f0, post, length, lam, work, domega):
    _check("lb_adjoint_segment", _lib.lb_adjoint_segment(ctx, _f64(f0), _f64(post), int(length), _f64(lam),
                                                         _f64(work), _f64(domega)))


def lb_adjoint_segment_binary(ctx, f0, g0, post, phi, length, lf, lg, work, grads):
    _check("lb_adjoint_segment_binary", _lib.lb_adjoint_segment_binary(
        ctx, _f64(f0), _f64(g0), _f64(post), _f64(phi), int(length), _f64(lf), _f64(lg), _f64(work), _f64(grads)))


def lb_mask_index(ctx, mask, index, count):
    _check("lb_mask_index", _lib.lb_mask_index(ctx, _ptr(mask, torch.uint8), _ptr(index, torch.int32),
                                               _ptr(count, torch.int64)))


def lb_get_sites(ctx, index, m, f_packed, g_packed=None):
    _check("lb_get_sites", _lib.lb_get_sites(ctx, _ptr(index, torch.int32), int(m), _ptr(f_packed), _ptr(g_packed)))


def lb_set_sites(ctx, index, m, f_packed, g_packed=None):
    _check("lb_set_sites", _lib.lb_set_sites(ctx, _ptr(index, torch.int32), int(m), _ptr(f_packed), _ptr(g_packed)))


def lb_profile(ctx, enable):
    _check("lb_profile", _lib.lb_profile(ctx, 1 if enable else 0))


def lb_profile_mask(ctx, kinds):
    """Time only the launches of the given kernel classes (an iterable of
    LB_K_* values); an empty one stops."""
    mask = 0
    for k in kinds:
        mask |= 1 << int(k)
    _check("lb_profile_mask", _lib.lb_profile_mask(ctx, mask))


def lb_kernel_times(ctx, kind):
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check("lb_kernel_times", _lib.lb_kernel_times(ctx, kind, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def lb_destroy(ctx):
    if _lib is not None and ctx is not None:
        _check("lb_destroy", _lib.lb_destroy(ctx))


def lb_conserved_sums_noalloc(params, f, g, out, stream=None):
    """Allocation-free sums of a canonical state (f, g device tensors of the
    storage dtype of `params`; g None for the single fluid) into out[5]."""
    load()
    dt = STORAGE_DTYPE[params.storage]
    _check("lb_conserved_sums_noalloc", _lib.lb_conserved_sums_noalloc(
        ctypes.byref(params), _ptr(f, dt), _ptr(g, dt), _f64(out), _stream() if stream is None else stream))


def lb_strerror(status):
    load()
    return _lib.lb_strerror(status).decode()


def lb_stream_copy(dst, src, nbytes=None, stream=None):
    """Streaming copy of the first `nbytes` bytes (default: all of src) of
    device tensor src into dst, on `stream` (default: the current one)."""
    load()
    nbytes = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    if nbytes > src.numel() * src.element_size() or nbytes > dst.numel() * dst.element_size():
        raise ValueError("copy larger than its tensors")
    _check("lb_stream_copy", _lib.lb_stream_copy(_ptr(dst), _ptr(src), nbytes,
                                                 _stream() if stream is None else stream))


# ---- a small owner object ---------------------------------------------------

class Lattice:
    """One context plus the torch-owned workspace it borrows.

    Shapes: scalar fields (nz, ny, nx); vector fields (3, nz, ny, nx);
    distributions (19, nz, ny, nx), all contiguous on the device.
    """

    def __init__(self, nx, ny, nz, model=LB_SINGLE, storage=LB_F64, device="cuda", **phys):
        self.params = make_params(nx, ny, nz, model=model, storage=storage, **phys)
        self.shape = (nz, ny, nx)
        self.model, self.storage = model, storage
        self.device = torch.device(device)
        nbytes = lb_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = lb_create(self.params, self.workspace)

    @property
    def nsite(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    def _dev(self, a, count, dtype=torch.float64, name="array"):
        t = torch.as_tensor(a, dtype=dtype, device=self.device).contiguous()
        if t.numel() != count:
            raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), count))
        return t

    def init_equilibrium(self, rho, u, phi=None):
        n = self.nsite
        rho, u = self._dev(rho, n, name="rho"), self._dev(u, 3 * n, name="u")
        if (phi is None) != (self.model != LB_BINARY):
            raise ValueError("phi is required for the binary model and only for it")
        phi = self._dev(phi, n, name="phi") if phi is not None else None
        lb_set_stream(self.ctx, _stream())
        lb_init_equilibrium(self.ctx, rho, u, phi)
        self._keep = (rho, u, phi)          # inputs stay alive until the queued kernel ran

    def step(self, n=1):
        lb_set_stream(self.ctx, _stream())
        lb_step(self.ctx, n)

    def collide(self):
        lb_set_stream(self.ctx, _stream())
        lb_collide(self.ctx)

    def propagate(self):
        lb_set_stream(self.ctx, _stream())
        lb_propagate(self.ctx)

    def moments(self):
        lb_set_stream(self.ctx, _stream())
        rho = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        phi = torch.empty(self.shape, dtype=torch.float64, device=self.device) \
            if self.model == LB_BINARY else None
        lb_moments(self.ctx, rho, u, phi)
        return rho, u, phi

    def conserved_sums(self):
        lb_set_stream(self.ctx, _stream())
        out = torch.empty(5, dtype=torch.float64, device=self.device)
        lb_conserved_sums(self.ctx, out)
        return out

    def field_stats(self):
        """(10,) device tensor: sum rho, sum j (3), sum phi, sum rho u.u,
        min phi, max phi, sum phi^2, max u.u."""
        lb_set_stream(self.ctx, _stream())
        out = torch.empty(10, dtype=torch.float64, device=self.device)
        lb_field_stats(self.ctx, out)
        return out

    def get_state(self):
        lb_set_stream(self.ctx, _stream())
        dt = STORAGE_DTYPE[self.storage]
        f = torch.empty((Q,) + self.shape, dtype=dt, device=self.device)
        g = torch.empty_like(f) if self.model == LB_BINARY else None
        lb_get_state(self.ctx, f, g)
        return f, g

    def set_state(self, f, g=None):
        lb_set_stream(self.ctx, _stream())
        dt = STORAGE_DTYPE[self.storage]
        if (g is None) != (self.model != LB_BINARY):
            raise ValueError("g is required for the binary model and only for it")
        f = self._dev(f, Q * self.nsite, dt, "f")
        g = self._dev(g, Q * self.nsite, dt, "g") if g is not None else None
        lb_set_state(self.ctx, f, g)
        self._keep = (f, g)

    def mask_index(self, mask):
        """Included sites of a boolean (nz, ny, nx) mask, in site order, as a
        device int32 tensor (the count is read back to size it)."""
        lb_set_stream(self.ctx, _stream())
        m = torch.as_tensor(mask, device=self.device).to(torch.uint8).contiguous()
        if m.numel() != self.nsite:
            raise ValueError("mask has %d elements, expected %d" % (m.numel(), self.nsite))
        index = torch.empty(self.nsite, dtype=torch.int32, device=self.device)
        count = torch.empty(1, dtype=torch.int64, device=self.device)
        lb_mask_index(self.ctx, m, index, count)
        return index[: int(count.item())]

    def get_sites(self, index):
        """State at the listed sites, packed (19, m) (and g for the binary model)."""
        lb_set_stream(self.ctx, _stream())
        index = index.to(torch.int32).contiguous()
        m = index.numel()
        dt = STORAGE_DTYPE[self.storage]
        f = torch.empty((Q, m), dtype=dt, device=self.device)
        g = torch.empty_like(f) if self.model == LB_BINARY else None
        lb_get_sites(self.ctx, index, m, f, g)
        return f, g

    def set_sites(self, index, f, g=None):
        lb_set_stream(self.ctx, _stream())
        index = index.to(torch.int32).contiguous()
        m = index.numel()
        dt = STORAGE_DTYPE[self.storage]
        if (g is None) != (self.model != LB_BINARY):
            raise ValueError("g is required for the binary model and only for it")
        f = self._dev(f, Q * m, dt, "f")
        g = self._dev(g, Q * m, dt, "g") if g is not None else None
        lb_set_sites(self.ctx, index, m, f, g)
        self._keep = (index, f, g)

    def copy_from_masked(self, mask, f_host, g_host=None):
        """Update the host arrays (19, nz, ny, nx) at the masked sites only,
        moving only those sites' values across (packed on the device)."""
        index = self.mask_index(mask)
        f, g = self.get_sites(index)
        idx = index.cpu().numpy()
        f_host.reshape(Q, -1)[:, idx] = f.cpu().numpy()
        if g_host is not None:
            g_host.reshape(Q, -1)[:, idx] = g.cpu().numpy()

    def copy_to_masked(self, mask, f_host, g_host=None):
        """Write the host arrays' values at the masked sites into the state."""
        index = self.mask_index(mask)
        idx = index.cpu().numpy()
        f = f_host.reshape(Q, -1)[:, idx]
        g = g_host.reshape(Q, -1)[:, idx] if g_host is not None else None
        self.set_sites(index, f, g)

    def set_tau(self, tau_f):
        lb_set_tau(self.ctx, tau_f)
        self.params.tau_f = float(tau_f)

    def set_params(self, **phys):
        """Change physical parameters (tau_f, A, B, kappa, mobility, gamma,
        tau_minus) for subsequent calls; the state is kept."""
        allowed = {"tau_f", "A", "B", "kappa", "mobility", "gamma", "tau_minus", "tau_bulk", "tau_ghost_even",
                   "tau_ghost_odd"}
        bad = set(phys) - allowed
        if bad:
            raise ValueError("cannot change %s after creation" % ", ".join(sorted(bad)))
        p = lb_params()
        ctypes.memmove(ctypes.byref(p), ctypes.byref(self.params), ctypes.sizeof(lb_params))
        for k, v in phys.items():
            setattr(p, k, float(v))
        lb_set_params(self.ctx, p)
        self.params = p

    def close(self):
        if self.ctx is not None:
            lb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
