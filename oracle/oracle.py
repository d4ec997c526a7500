"""ctypes view of the plain FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark import this module.
It loads ``libugks_oracle.so`` built from ``ugks_oracle.c`` and never touches the HIP library.
Arrays come back as numpy float64 in the oracle's layout: f[ny, nx, NF] with the velocity
index k*nv + m (NF = nu*nv; with internal degrees of freedom NF = 2*nu*nv, G then H),
W[ny, nx, 4] = (rho, rho U, rho V, rho E).
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libugks_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)


class RefCase(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("nu", ctypes.c_int), ("nv", ctypes.c_int),
        ("umax", ctypes.c_double), ("vmax", ctypes.c_double),
        ("kn", ctypes.c_double),
        ("bc", ctypes.c_int), ("inlet_fixed_u", ctypes.c_int),
        ("p_ratio", ctypes.c_double), ("T_in", ctypes.c_double), ("T_wall", ctypes.c_double),
        ("U_in", ctypes.c_double), ("U_noise", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("rho0", ctypes.c_double), ("T0", ctypes.c_double), ("noise", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("dt_override", ctypes.c_double),
        ("dof", ctypes.c_int),
        ("prandtl", ctypes.c_double),
        ("adaptive_dt", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run oracle/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        L.ugks_ref_create.restype = ctypes.c_void_p
        L.ugks_ref_create.argtypes = [ctypes.POINTER(RefCase)]
        L.ugks_ref_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ugks_ref_get_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.ugks_ref_set_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.ugks_ref_get_face_flux.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.ugks_ref_get_ghost.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.ugks_ref_get_micro_flux.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.ugks_ref_dt.restype = ctypes.c_double
        L.ugks_ref_dt.argtypes = [ctypes.c_void_p]
        L.ugks_ref_time.restype = ctypes.c_double
        L.ugks_ref_time.argtypes = [ctypes.c_void_p]
        L.ugks_ref_adaptive_dt.restype = ctypes.c_double
        L.ugks_ref_adaptive_dt.argtypes = [_dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.ugks_ref_tau_ref.restype = ctypes.c_double
        L.ugks_ref_tau_ref.argtypes = [ctypes.c_void_p]
        L.ugks_ref_destroy.argtypes = [ctypes.c_void_p]
        L.ugks_ref_set_threads.argtypes = [ctypes.c_int]
        L.ugks_ref_get_threads.restype = ctypes.c_int
        L.ugks_ref_splitmix64.restype = ctypes.c_uint64
        L.ugks_ref_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.ugks_ref_unit_noise.restype = ctypes.c_double
        L.ugks_ref_unit_noise.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.ugks_ref_nodes.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.ugks_ref_maxwellian.restype = ctypes.c_double
        L.ugks_ref_maxwellian.argtypes = [_dp, ctypes.c_double, ctypes.c_double]
        L.ugks_ref_prim.argtypes = [_dp, _dp, ctypes.c_int]
        L.ugks_ref_vanleer.restype = ctypes.c_double
        L.ugks_ref_vanleer.argtypes = [ctypes.c_double, ctypes.c_double]
        L.ugks_ref_moments_1d.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        L.ugks_ref_micro_slope.argtypes = [_dp, _dp, _dp, ctypes.c_int]
        L.ugks_ref_time_weights.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
        L.ugks_ref_time_slope.argtypes = [_dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        L.ugks_ref_equilibrium_flux.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                                ctypes.c_int]
        L.ugks_ref_face.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                    ctypes.c_double]
        L.ugks_ref_shakhov.restype = ctypes.c_double
        L.ugks_ref_shakhov.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _vec(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


# ----------------------------------------------------------------------------- blocks
def splitmix64(seed, k):
    return int(lib().ugks_ref_splitmix64(seed, k))


def unit_noise(seed, k):
    return float(lib().ugks_ref_unit_noise(seed, k))


def nodes(n, a):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().ugks_ref_nodes(n, a, _ptr(x), _ptr(w))
    return x, w


def maxwellian(prim, u, v):
    p = _vec(prim, 4)
    return float(lib().ugks_ref_maxwellian(_ptr(p), u, v))


def prim(W, dof=0):
    w = _vec(W, 4)
    p = np.zeros(4)
    rc = lib().ugks_ref_prim(_ptr(w), _ptr(p), int(dof))
    return rc, p


def vanleer(p, q):
    return float(lib().ugks_ref_vanleer(p, q))


def moments_1d(U, lam):
    full, pos, neg = np.zeros(7), np.zeros(7), np.zeros(7)
    lib().ugks_ref_moments_1d(U, lam, _ptr(full), _ptr(pos), _ptr(neg))
    return full, pos, neg


def micro_slope(prim, s, dof=0):
    p, sv, a = _vec(prim, 4), _vec(s, 4), np.zeros(4)
    lib().ugks_ref_micro_slope(_ptr(p), _ptr(sv), _ptr(a), int(dof))
    return a


def time_weights(dt, tau):
    Mt = np.zeros(5)
    lib().ugks_ref_time_weights(dt, tau, _ptr(Mt))
    return Mt


def time_slope(prim, aL, aR, b, dof=0):
    A = np.zeros(4)
    args = [_vec(x, 4) for x in (prim, aL, aR, b)]
    lib().ugks_ref_time_slope(*[_ptr(x) for x in args], _ptr(A), int(dof))
    return A


def equilibrium_flux(prim, aL, aR, b, A, Mt, dof=0):
    F = np.zeros(4)
    args = [_vec(x, 4) for x in (prim, aL, aR, b, A)] + [_vec(Mt, 5)]
    lib().ugks_ref_equilibrium_flux(*[_ptr(x) for x in args], _ptr(F), int(dof))
    return F


def face(un, ut, w, fhat, sn, st, WL, WR, dn, length, dt, mu_ref, collisionless=False, dof=0,
         prandtl=1.0):
    """fhat, sn, st: nvel values (G), followed by nvel values of H when dof > 0."""
    n = len(un)
    nf = n * (2 if dof > 0 else 1)
    u3 = [_vec(x, n) for x in (un, ut, w)]
    f3 = [_vec(x, nf) for x in (fhat, sn, st)]
    wl, wr = _vec(WL, 4), _vec(WR, 4)
    FW = np.zeros(4)
    Ff = np.zeros(nf)
    rc = lib().ugks_ref_face(n, *[_ptr(a) for a in u3 + f3], _ptr(wl), _ptr(wr), dn, length,
                             dt, mu_ref, int(collisionless), _ptr(FW), _ptr(Ff), int(dof),
                             float(prandtl))
    return rc, FW, Ff


def shakhov(prim, q, prandtl, u, v):
    """S of the Shakhov equilibrium g (1 + S) at (u, v)."""
    p, qq = _vec(prim, 4), _vec(q, 2)
    return float(lib().ugks_ref_shakhov(_ptr(p), _ptr(qq), float(prandtl), float(u), float(v)))


def adaptive_dt(W, cfl, umax, vmax, dx, dy):
    """The adaptive step of a state W[..., 4] (see ugks_ref_adaptive_dt)."""
    w = np.ascontiguousarray(np.asarray(W, dtype=np.float64).reshape(-1, 4))
    return float(lib().ugks_ref_adaptive_dt(_ptr(w), w.shape[0], cfl, umax, vmax, dx, dy))


def set_threads(n):
    lib().ugks_ref_set_threads(int(n))


def get_threads():
    return int(lib().ugks_ref_get_threads())


def mu_ref_of_kn(kn):
    """Hard-sphere reference viscosity for a Knudsen number (same reading as the C oracle)."""
    return 5.0 * math.sqrt(math.pi) * kn / 16.0


# ----------------------------------------------------------------------------- state
CASE_DEFAULTS = dict(lx=1.0, ly=1.0, umax=5.0, vmax=5.0, kn=0.1, bc=1, inlet_fixed_u=0,
                     p_ratio=2.0, T_in=1.0, T_wall=1.0, U_in=0.0, U_noise=0.0, cfl=0.8,
                     rho0=1.0, T0=1.0, noise=0.01, seed=1, dt_override=0.0, dof=0,
                     prandtl=1.0, adaptive_dt=0)


class Oracle:
    """One oracle solve.  Keyword arguments are the fields of ``ugks_ref_case``."""

    def __init__(self, **kw):
        c = dict(CASE_DEFAULTS)
        c.update(kw)
        self.case = c
        self._c = RefCase(**c)
        self.nx, self.ny, self.nu, self.nv = c["nx"], c["ny"], c["nu"], c["nv"]
        self.NV = self.nu * self.nv
        self.dof = c["dof"]
        self.NF = self.NV * (2 if self.dof > 0 else 1)   # G, then H
        h = lib().ugks_ref_create(ctypes.byref(self._c))
        if not h:
            raise ValueError("ugks_ref_create rejected the case")
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().ugks_ref_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, n=1):
        return int(lib().ugks_ref_step(self._h, int(n)))

    @property
    def dt(self):
        return float(lib().ugks_ref_dt(self._h))

    @property
    def time(self):
        return float(lib().ugks_ref_time(self._h))

    @property
    def tau_ref(self):
        return float(lib().ugks_ref_tau_ref(self._h))

    def state(self):
        f = np.empty((self.ny, self.nx, self.NF))
        W = np.empty((self.ny, self.nx, 4))
        lib().ugks_ref_get_state(self._h, _ptr(f), _ptr(W))
        return f, W

    def set_state(self, f=None, W=None):
        fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        Wa = None if W is None else np.ascontiguousarray(W, dtype=np.float64)
        if fa is not None:
            assert fa.size == self.ny * self.nx * self.NF
        if Wa is not None:
            assert Wa.size == self.ny * self.nx * 4
        lib().ugks_ref_set_state(self._h, _ptr(fa) if fa is not None else None,
                                 _ptr(Wa) if Wa is not None else None)

    def face_flux(self):
        Fx = np.empty((self.ny, self.nx + 1, 4))
        Fy = np.empty((self.ny + 1, self.nx, 4))
        lib().ugks_ref_get_face_flux(self._h, _ptr(Fx), _ptr(Fy))
        return Fx, Fy

    def micro_flux(self):
        Ffx = np.empty((self.ny, self.nx + 1, self.NF))
        Ffy = np.empty((self.ny + 1, self.nx, self.NF))
        lib().ugks_ref_get_micro_flux(self._h, _ptr(Ffx), _ptr(Ffy))
        return Ffx, Ffy

    def ghost(self):
        Wg = np.empty((2, self.ny, 4))
        fg = np.empty((2, self.ny, self.NF))
        lib().ugks_ref_get_ghost(self._h, _ptr(Wg), _ptr(fg))
        return Wg, fg

    def velocity_grid(self):
        uk, wk = nodes(self.nu, self.case["umax"])
        vm, wm = nodes(self.nv, self.case["vmax"])
        return uk, vm, wk, wm

    def moments(self):
        """(rho, U, V, T) per cell from W, in the oracle's own arithmetic."""
        _, W = self.state()
        out = np.empty((self.ny, self.nx, 4))
        for j in range(self.ny):
            for i in range(self.nx):
                rc, p = prim(W[j, i], self.dof)
                out[j, i] = (p[0], p[1], p[2], 1.0 / p[3]) if rc == 0 else (np.nan,) * 4
        return out
