"""Python binding of the UGKS C ABI (include/ugks.h).

Argument marshalling only: every step of the time step runs in the gfx950 kernels of
``lib/libugks.so``.  PyTorch supplies device memory (the workspace) and the stream.  The
functions keep the C names; ``Solver`` bundles them for convenience.  There is no CPU
fallback: a missing library raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libugks.so")

UGKS_OK = 0
UGKS_E_INVAL = -1
UGKS_E_NOMEM = -2
UGKS_E_DEVICE = -3
UGKS_E_STATE = -4
UGKS_E_BUSY = -5
UGKS_BC_PERIODIC = 0
UGKS_BC_CHANNEL = 1
UGKS_FP64 = 0
UGKS_FP32_STORE = 1

KERNELS = ("ghost", "moments", "interfaces", "update")


class ugks_mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double)]


class ugks_vgrid(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int), ("nv", ctypes.c_int),
                ("umax", ctypes.c_double), ("vmax", ctypes.c_double),
                ("internal_dof", ctypes.c_int)]


class ugks_bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("inlet_fixed_u", ctypes.c_int),
                ("p_ratio", ctypes.c_double), ("T_in", ctypes.c_double),
                ("T_wall", ctypes.c_double), ("U_in", ctypes.c_double),
                ("U_noise", ctypes.c_double)]


class ugks_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("velocity_chunks", ctypes.c_int),
                ("cfl", ctypes.c_double), ("rho0", ctypes.c_double), ("T0", ctypes.c_double),
                ("noise", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("dt_override", ctypes.c_double), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("prandtl", ctypes.c_double), ("adaptive_dt", ctypes.c_int)]


class ugks_info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nu", ctypes.c_int),
                ("nv", ctypes.c_int), ("plane_stride", ctypes.c_int), ("precision", ctypes.c_int),
                ("internal_dof", ctypes.c_int), ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
                ("tau_ref", ctypes.c_double), ("steps", ctypes.c_int64),
                ("device_bytes", ctypes.c_size_t), ("prandtl", ctypes.c_double),
                ("moment_chunks", ctypes.c_int), ("update_chunks", ctypes.c_int),
                ("update_chunks_per_workgroup", ctypes.c_int), ("update_v_chunks", ctypes.c_int)]


_dp = ctypes.POINTER(ctypes.c_double)
_lib = None

# C ABI functions: name -> (restype, argtypes)
SIGNATURES = {
    "ugks_required_bytes": (ctypes.c_int, [ctypes.POINTER(ugks_mesh), ctypes.POINTER(ugks_vgrid),
                                           ctypes.POINTER(ugks_opts),
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "ugks_create": (ctypes.c_int, [ctypes.POINTER(ugks_mesh), ctypes.POINTER(ugks_vgrid),
                                   ctypes.c_double, ctypes.POINTER(ugks_bc),
                                   ctypes.POINTER(ugks_opts), ctypes.POINTER(ctypes.c_void_p)]),
    "ugks_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ugks_step_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ugks_moments": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "ugks_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ugks_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "ugks_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ugks_info)]),
    "ugks_get_time": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "ugks_get_state": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "ugks_set_state": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "ugks_get_face_flux": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "ugks_set_kernel_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ugks_get_kernel_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "ugks_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "ugks_step_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.c_int, ctypes.c_int]),
    "ugks_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ugks_batch_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
}


class UgksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ugks error {code}: {msg}")
        self.code = code


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libugks.so not built ({LIB_PATH}); run python paper_1810_08137_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, h=None):
    if rc != UGKS_OK:
        msg = lib().ugks_last_error(h)
        raise UgksError(rc, msg.decode() if msg else "")
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


# ----------------------------------------------------------------------------- C names
def ugks_required_bytes(mesh, vgrid, opts):
    n = ctypes.c_size_t(0)
    _check(lib().ugks_required_bytes(ctypes.byref(mesh), ctypes.byref(vgrid),
                                     ctypes.byref(opts), ctypes.byref(n)))
    return int(n.value)


def ugks_create(mesh, vgrid, kn, bc, opts):
    h = ctypes.c_void_p(None)
    _check(lib().ugks_create(ctypes.byref(mesh), ctypes.byref(vgrid), float(kn),
                             ctypes.byref(bc), ctypes.byref(opts), ctypes.byref(h)))
    return h


def ugks_step(h, n):
    return _check(lib().ugks_step(h, int(n)), h)


def ugks_step_static(h, n):
    return _check(lib().ugks_step_static(h, int(n)), h)


def ugks_moments(h, out=None):
    info = ugks_get_info(h)
    if out is None:
        out = np.empty((info.ny, info.nx, 4))
    rc = lib().ugks_moments(h, _ptr(out))
    _check(rc, h)
    return out


def ugks_destroy(h):
    return _check(lib().ugks_destroy(h))


def ugks_last_error(h=None):
    msg = lib().ugks_last_error(h)
    return msg.decode() if msg else ""


def ugks_get_info(h):
    info = ugks_info()
    _check(lib().ugks_get_info(h, ctypes.byref(info)), h)
    return info


def ugks_get_time(h):
    t = ctypes.c_double(0)
    dt = ctypes.c_double(0)
    _check(lib().ugks_get_time(h, ctypes.byref(t), ctypes.byref(dt)), h)
    return float(t.value), float(dt.value)


def values_per_cell(info):
    """f values per cell: nu*nv, twice that (G then H) with internal degrees of freedom."""
    return info.nu * info.nv * (2 if info.internal_dof > 0 else 1)


def ugks_get_state(h, want_f=True, want_W=True):
    info = ugks_get_info(h)
    f = np.empty((info.ny, info.nx, values_per_cell(info))) if want_f else None
    W = np.empty((info.ny, info.nx, 4)) if want_W else None
    _check(lib().ugks_get_state(h, _ptr(f), _ptr(W)), h)
    return f, W


def ugks_set_state(h, f=None, W=None):
    info = ugks_get_info(h)
    fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    Wa = None if W is None else np.ascontiguousarray(W, dtype=np.float64)
    if fa is not None and fa.size != info.nx * info.ny * values_per_cell(info):
        raise ValueError("f has the wrong size")
    if Wa is not None and Wa.size != info.nx * info.ny * 4:
        raise ValueError("W has the wrong size")
    _check(lib().ugks_set_state(h, _ptr(fa), _ptr(Wa)), h)


def ugks_get_face_flux(h):
    info = ugks_get_info(h)
    Fx = np.empty((info.ny, info.nx + 1, 4))
    Fy = np.empty((info.ny + 1, info.nx, 4))
    _check(lib().ugks_get_face_flux(h, _ptr(Fx), _ptr(Fy)), h)
    return Fx, Fy


def ugks_set_kernel_timing(h, on):
    return _check(lib().ugks_set_kernel_timing(h, int(bool(on))), h)


def ugks_get_kernel_timing(h, kernel):
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(lib().ugks_get_kernel_timing(h, int(kernel), ctypes.byref(ms), ctypes.byref(n)), h)
    return float(ms.value), int(n.value)


def ugks_batch_create(stream_ptr, max_instances):
    b = ctypes.c_void_p(None)
    _check(lib().ugks_batch_create(ctypes.c_void_p(stream_ptr), int(max_instances),
                                   ctypes.byref(b)))
    return b


def ugks_step_batch(b, handles, n):
    arr = (ctypes.c_void_p * len(handles))(*[h.value for h in handles])
    rc = lib().ugks_step_batch(b, arr, len(handles), int(n))
    if rc != UGKS_OK:
        msg = lib().ugks_batch_last_error(b)
        raise UgksError(rc, msg.decode() if msg else "")
    return rc


def ugks_batch_destroy(b):
    return _check(lib().ugks_batch_destroy(b))


def ugks_batch_last_error(b):
    msg = lib().ugks_batch_last_error(b)
    return msg.decode() if msg else ""


# ----------------------------------------------------------------------------- structs
def make_structs(nx, ny, lx, ly, nu, nv, umax, vmax, bc="channel", p_ratio=2.0, T_in=1.0,
                 T_wall=1.0, inlet_fixed_u=0, U_in=0.0, U_noise=0.0, precision="fp64", cfl=0.8,
                 rho0=1.0, T0=1.0, noise=0.01, seed=1, dt_override=0.0, velocity_chunks=0,
                 dof=0, prandtl=1.0, adaptive_dt=0, **_):
    mesh = ugks_mesh(int(nx), int(ny), float(lx), float(ly))
    vgrid = ugks_vgrid(int(nu), int(nv), float(umax), float(vmax), int(dof))
    kind = {"periodic": UGKS_BC_PERIODIC, "channel": UGKS_BC_CHANNEL}[bc] if isinstance(bc, str) else int(bc)
    b = ugks_bc(kind, int(inlet_fixed_u), float(p_ratio), float(T_in), float(T_wall),
                float(U_in), float(U_noise))
    prec = {"fp64": UGKS_FP64, "fp32_store": UGKS_FP32_STORE}[precision] if isinstance(precision, str) else int(precision)
    o = ugks_opts(prec, int(velocity_chunks), float(cfl), float(rho0), float(T0), float(noise),
                  int(seed), float(dt_override), None, None, 0, float(prandtl), int(adaptive_dt))
    return mesh, vgrid, b, o


class Solver:
    """One UGKS solve on the current GPU.

    The workspace is a torch uint8 tensor on the current device and the work runs on torch's
    current stream (or ``stream``).  Keyword arguments are those of ``make_structs`` plus
    ``kn``.
    """

    def __init__(self, kn, stream=None, **case):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the UGKS library runs only on the GPU")
        self.case = dict(case, kn=kn)
        self.mesh, self.vgrid, self.bc, self.opts = make_structs(**case)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self._alloc_stream = self._stream
        nbytes = ugks_required_bytes(self.mesh, self.vgrid, self.opts)
        with torch.cuda.stream(self._stream):
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.opts.stream = ctypes.c_void_p(self._stream.cuda_stream)
        self.opts.workspace = ctypes.c_void_p(self._ws.data_ptr())
        self.opts.workspace_bytes = nbytes
        self.h = ugks_create(self.mesh, self.vgrid, kn, self.bc, self.opts)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            ugks_destroy(self.h)
            self.h = None
            if self._stream is not self._alloc_stream:
                # the workspace was last used on another stream (a batch adopted the handle)
                self._ws.record_stream(self._stream)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        return ugks_get_info(self.h)

    @property
    def dt(self):
        return self.info.dt

    @property
    def stream(self):
        return self._stream

    def step(self, n=1):
        ugks_step(self.h, n)

    def step_static(self, n=1):
        ugks_step_static(self.h, n)

    def moments(self):
        return ugks_moments(self.h)

    def state(self):
        return ugks_get_state(self.h)

    def set_state(self, f=None, W=None):
        ugks_set_state(self.h, f, W)

    def face_flux(self):
        return ugks_get_face_flux(self.h)

    def time(self):
        """(simulated time, dt of the next step)"""
        return ugks_get_time(self.h)

    def kernel_timing(self, on=None):
        if on is not None:
            ugks_set_kernel_timing(self.h, on)
            return None
        return {name: ugks_get_kernel_timing(self.h, k) for k, name in enumerate(KERNELS)}


def updates_per_step(info):
    return info.nx * info.ny * info.nu * info.nv


class Batch:
    """A batch of solvers stepped together (one launch per phase for all of them)."""

    def __init__(self, max_instances, stream=None):
        import torch

        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self.b = ugks_batch_create(self._stream.cuda_stream, max_instances)

    def step(self, solvers, n):
        ugks_step_batch(self.b, [s.h for s in solvers], n)
        for s in solvers:   # members now live on the batch's stream
            s._stream = self._stream

    def close(self):
        if getattr(self, "b", None) is not None and self.b.value:
            ugks_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = [n for n in SIGNATURES] + ["Solver", "Batch", "make_structs", "UgksError", "lib",
                                     "updates_per_step"]
