"""Pins for the oracle's gas with internal degrees of freedom (CPU only).

With dof internal coordinates xi the distribution is carried as G = int f dxi and
H = int |xi|^2 f dxi, and the energy variable is (u^2 + v^2 + |xi|^2)/2.  The checks integrate
over xi numerically (Gauss-Hermite in dof dimensions) and over (u, v) with the independent
panel quadrature, so none of them re-uses the oracle's closed forms for the moments of xi.
State-level checks: the gas constant (gamma), conservation, the equilibrium fixed point,
relaxation, equipartition, free transport of H and channel symmetry.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import quadrature as Q


# ------------------------------------------------------------------ xi quadrature
def _xi_nodes(lam, dof, order=8):
    """Nodes s = |xi|^2 and weights of the normalised Gaussian (lam/pi)^(dof/2) e^(-lam|xi|^2)
    on the tensor Gauss-Hermite grid in dof dimensions."""
    x, w = np.polynomial.hermite.hermgauss(order)
    x = x / math.sqrt(lam)
    w = w / math.sqrt(math.pi)
    s = np.zeros(1)
    ws = np.ones(1)
    for _ in range(dof):
        s = (s[:, None] + x[None, :] ** 2).ravel()
        ws = (ws[:, None] * w[None, :]).ravel()
    return s, ws


def _xi_mean(lam, dof, poly):
    """E over xi of poly(s), poly a numpy-aware function of s = |xi|^2."""
    s, w = _xi_nodes(lam, dof)
    return float(np.sum(w * poly(s)))


def _psi(uu, vv, s):
    return [np.ones_like(uu), uu, vv, 0.5 * (uu ** 2 + vv ** 2 + s)]


def _dot(c, uu, vv, s):
    return c[0] + c[1] * uu + c[2] * vv + c[3] * 0.5 * (uu ** 2 + vv ** 2 + s)


def _moment(prim, poly, half_sign, dof):
    """int over the half plane sign(u) = half_sign (0: whole plane) and over xi of
    poly(u, v, s) g(u, v) with the normalised xi Gaussian; poly is at most quadratic in s,
    so it is taken at s = 0, 1, 2 and combined with E[s] and E[s^2] from the xi quadrature."""
    rho, U, V, lam = prim
    hu = {1: "pos", -1: "neg", 0: None}[half_sign]
    u, wu = Q.line(U, lam, half=hu)
    v, wv = Q.line(V, lam)
    uu, vv = np.meshgrid(u, v, indexing="ij")
    g = Q.maxwellian_2d(prim, uu, vv)
    ww = np.outer(wu, wv) * g
    P = [np.sum(ww * poly(uu, vv, float(s))) for s in (0, 1, 2)]
    p2 = 0.5 * (P[2] - 2 * P[1] + P[0])
    p1 = P[1] - P[0] - p2
    m1 = _xi_mean(lam, dof, lambda s: s)
    m2 = _xi_mean(lam, dof, lambda s: s * s)
    return P[0] + p1 * m1 + p2 * m2


# ------------------------------------------------------------------ gas constant
@pytest.mark.parametrize("dof,gamma", [(0, 2.0), (1, 5.0 / 3.0), (3, 7.0 / 5.0)])
def test_energy_follows_the_ratio_of_specific_heats(dof, gamma):
    """rho E = rho |U|^2 / 2 + p / (gamma - 1) with p = rho T / 2 and gamma = (n + 2)/n for
    n = 2 + dof degrees of freedom (5/3: a monatomic gas seen in 2D; 7/5: diatomic)."""
    rho, U, V, T = 1.3, 0.2, -0.4, 0.8
    p = rho * T / 2
    W = [rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V) + p / (gamma - 1)]
    rc, pr = O.prim(W, dof)
    assert rc == 0
    np.testing.assert_allclose(pr, [rho, U, V, 1 / T], rtol=1e-14)


# ------------------------------------------------------------------ micro slope
def _gh_moments_of(prim, c, dof, order=12):
    """rho * int psi g (c . psi) du dv dxi on Gauss-Hermite grids (exact for these
    polynomial x Gaussian integrands)."""
    rho, U, V, lam = prim
    x, w = np.polynomial.hermite.hermgauss(order)
    sc = 1.0 / math.sqrt(lam)
    wu = w / math.sqrt(math.pi)
    uu, vv = np.meshgrid(U + sc * x, V + sc * x, indexing="ij")
    ww = np.outer(wu, wu)
    s, ws = _xi_nodes(lam, dof, order)
    out = np.zeros(4)
    for sk, wk in zip(s, ws):
        psi = _psi(uu, vv, sk)
        cp = _dot(c, uu, vv, sk)
        out += wk * np.array([rho * np.sum(ww * p * cp) for p in psi])
    return out


@pytest.mark.parametrize("dof", [1, 2, 3])
def test_micro_slope_inverts_the_moment_map_with_internal_dof(dof):
    rng = np.random.default_rng(20 + dof)
    for _ in range(10):
        prim = (rng.uniform(0.3, 2.0), rng.uniform(-1, 1), rng.uniform(-1, 1),
                rng.uniform(0.4, 3.0))
        c = rng.normal(size=4)
        s = _gh_moments_of(prim, c, dof)
        np.testing.assert_allclose(O.micro_slope(prim, s, dof), c, rtol=1e-10, atol=1e-11)
        # the monatomic solve gets the energy row wrong for this gas
        assert np.max(np.abs(O.micro_slope(prim, s, 0) - c)) > 1e-3


# ------------------------------------------------------------------ time slope, flux
@pytest.mark.parametrize("dof", [1, 3])
def test_time_slope_with_internal_dof_satisfies_compatibility(dof):
    rng = np.random.default_rng(30 + dof)
    for _ in range(3):
        prim = (rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5),
                rng.uniform(0.6, 1.6))
        aL, aR, b = rng.normal(size=(3, 4)) * 0.3
        A = O.time_slope(prim, aL, aR, b, dof)
        for q in range(4):
            def f(a_side):
                return lambda u, v, s: _psi(u, v, s)[q] * (
                    _dot(A, u, v, s) + u * _dot(a_side, u, v, s) + v * _dot(b, u, v, s))
            tot = _moment(prim, f(aL), 1, dof) + _moment(prim, f(aR), -1, dof)
            assert abs(tot) < 1e-11, (q, tot)


@pytest.mark.parametrize("dof", [1, 3])
def test_equilibrium_flux_with_internal_dof_against_quadrature(dof):
    rng = np.random.default_rng(40 + dof)
    for _ in range(3):
        prim = (rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5),
                rng.uniform(0.6, 1.6))
        aL, aR, b, A = rng.normal(size=(4, 4)) * 0.3
        Mt = O.time_weights(0.01, 0.05)
        F = O.equilibrium_flux(prim, aL, aR, b, A, Mt, dof)
        for q in range(4):
            def f(a_side):
                return lambda u, v, s: _psi(u, v, s)[q] * u * (
                    Mt[0] + Mt[1] * (u * _dot(a_side, u, v, s) + v * _dot(b, u, v, s))
                    + Mt[2] * _dot(A, u, v, s))
            exact = _moment(prim, f(aL), 1, dof) + _moment(prim, f(aR), -1, dof)
            assert abs(F[q] - exact) < 1e-12 * max(1.0, abs(exact)), (q, F[q], exact)


# ------------------------------------------------------------------ one face
def _face_grid(n, a):
    x, w = O.nodes(n, a)
    un, ut = np.meshgrid(x, x, indexing="ij")
    return un.ravel(), ut.ravel(), np.outer(w, w).ravel()


def test_uniform_equilibrium_face_with_internal_dof_gives_euler_flux():
    """G and H in equilibrium, zero slopes: dt * len * the Euler flux of a gas with
    gamma = 5/3 (one internal degree of freedom)."""
    un, ut, w = _face_grid(40, 6.0)
    rho, U, V, T = 1.1, 0.25, -0.15, 0.95
    g = Q.maxwellian_2d((rho, U, V, 1 / T), un, ut)
    h = 0.5 * T * g                              # <xi^2> = T/2 for one coordinate
    p = rho * T / 2
    E = 0.5 * rho * (U * U + V * V) + 1.5 * p
    Wc = np.array([rho, rho * U, rho * V, E])
    dt, length = 1e-3, 0.25
    z = np.zeros(2 * un.size)
    rc, FW, Ff = O.face(un, ut, w, np.concatenate([g, h]), z, z, Wc, Wc, 0.1, length, dt,
                        O.mu_ref_of_kn(0.05), dof=1)
    assert rc == 0
    euler = np.array([rho * U, rho * U * U + p, rho * U * V, U * (E + p)])
    np.testing.assert_allclose(FW, dt * length * euler, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("dof", [1, 3])
def test_face_macro_flux_equals_moments_of_distribution_flux_with_internal_dof(dof):
    """The analytic flux (S5 + S7) against the discrete moments of the per-velocity G and H
    fluxes (S8), energy = sum w (u^2+v^2)/2 F_G + sum w F_H / 2: a wrong factor or shift in
    the equilibrium of H shows in the energy row."""
    un, ut, w = _face_grid(257, 9.0)
    primL = (1.05, 0.2, 0.05, 1 / 1.05)
    primR = (0.95, 0.1, -0.05, 1 / 0.97)
    gL = Q.maxwellian_2d(primL, un, ut)
    gR = Q.maxwellian_2d(primR, un, ut)
    fL = np.concatenate([gL * (1 + 0.02 * np.sin(un)), 0.5 * dof * 1.1 * gL * (1 + 0.03 * np.cos(un))])
    fR = np.concatenate([gR * (1 + 0.02 * np.cos(ut)), 0.5 * dof * 0.9 * gR])
    H = np.tile(np.where(un > 0, 1.0, np.where(un < 0, 0.0, 0.5)), 2)
    sL = np.concatenate([0.3 * gL * un, 0.2 * dof * gL * un])
    sR = np.concatenate([-0.2 * gR * ut, 0.1 * dof * gR * ut])
    fh = H * fL + (1 - H) * fR
    sn = H * sL + (1 - H) * sR
    st = 0.1 * fh * (np.tile(ut, 2) - 0.05)
    n = un.size

    def cons(f):
        psi = [np.ones_like(un), un, ut, 0.5 * (un ** 2 + ut ** 2)]
        W = np.array([np.sum(w * p * f[:n]) for p in psi])
        W[3] += 0.5 * np.sum(w * f[n:])
        return W

    for kn in (0.01, 0.1, 1.0):
        rc, FW, Ff = O.face(un, ut, w, fh, sn, st, cons(fL), cons(fR), 0.05, 0.1, 2e-3,
                            O.mu_ref_of_kn(kn), dof=dof)
        assert rc == 0
        psi = [np.ones_like(un), un, ut, 0.5 * (un ** 2 + ut ** 2)]
        micro = np.array([np.sum(w * p * Ff[:n]) for p in psi])
        micro[3] += 0.5 * np.sum(w * Ff[n:])
        np.testing.assert_allclose(FW, micro, rtol=0, atol=2e-10 * np.max(np.abs(FW)))


# ------------------------------------------------------------------ states
PERIODIC = dict(nx=12, ny=8, lx=1.5, ly=1.0, nu=16, nv=16, umax=5.0, vmax=5.0, kn=0.05, bc=0,
                noise=0.05, seed=9, dof=1)


def _grid(o):
    uk, vm, wk, wm = o.velocity_grid()
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    return uu.ravel(), vv.ravel(), np.outer(wk, wm).ravel()


def _cons_of_f(o, f):
    """sum w psi G + (0, 0, 0, sum w H / 2) per cell (test-side arithmetic)"""
    uu, vv, w = _grid(o)
    NV = uu.size
    psi = np.stack([np.ones(NV), uu, vv, 0.5 * (uu ** 2 + vv ** 2)])
    W = np.einsum("...v,qv->...q", f[..., :NV] * w, psi)
    W[..., 3] += 0.5 * np.sum(f[..., NV:] * w, axis=-1)
    return W


def test_initial_state_with_internal_dof():
    o = O.Oracle(**PERIODIC)
    f, W = o.state()
    assert f.shape == (8, 12, 2 * 256)
    # H = T/2 G per cell at T0 = 1, and W holds the energy of both
    np.testing.assert_allclose(f[..., 256:], 0.5 * f[..., :256], rtol=1e-15)
    rho = W[..., 0]
    np.testing.assert_allclose(W[..., 3], 0.75 * rho, rtol=1e-15)     # (2 + 1)/4 rho T


def test_periodic_box_with_internal_dof_conserves():
    o = O.Oracle(**PERIODIC)
    _, W0 = o.state()
    tot0 = W0.sum(axis=(0, 1))
    assert o.step(20) == 0
    f, W = o.state()
    tot = W.sum(axis=(0, 1))
    scale = np.array([tot0[0], tot0[0], tot0[0], tot0[3]])
    assert np.all(np.abs(tot - tot0) <= 1e-13 * scale), (tot - tot0) / scale
    assert np.ptp(W[..., 0]) > 1e-4
    # the distribution keeps carrying W, up to the gap between the analytic equilibrium flux
    # and the discrete moments of its per-velocity form on this coarse 16^2 grid (about 1e-7
    # after 20 steps, the same as for the monatomic gas)
    np.testing.assert_allclose(_cons_of_f(o, f), W, rtol=0, atol=2e-7)


def test_uniform_equilibrium_with_internal_dof_is_a_fixed_point():
    o = O.Oracle(**PERIODIC)
    uu, vv, _ = _grid(o)
    rho, U, V, T = 1.1, 0.3, -0.2, 0.9
    g = Q.maxwellian_2d((rho, U, V, 1 / T), uu, vv)
    f0 = np.broadcast_to(np.concatenate([g, 0.5 * T * g]), (o.ny, o.nx, 2 * uu.size)).copy()
    W0 = np.broadcast_to([rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V) + 0.75 * rho * T],
                         (o.ny, o.nx, 4)).copy()
    o.set_state(f0, W0)
    assert o.step(10) == 0
    f, W = o.state()
    assert np.array_equal(W, W0)
    assert np.max(np.abs(f - f0)) <= 1e-14 * np.max(f0)


def test_channel_with_internal_dof_at_rest_stays_at_rest():
    o = O.Oracle(nx=10, ny=6, lx=2.0, ly=1.0, nu=40, nv=40, umax=6.0, vmax=6.0, kn=0.1, bc=1,
                 p_ratio=1.0, noise=0.0, dof=1)
    f0, W0 = o.state()
    assert o.step(5) == 0
    f, W = o.state()
    assert np.max(np.abs(W - W0)) < 1e-13
    assert np.max(np.abs(f - f0)) < 1e-13 * np.max(f0)


def test_internal_energy_relaxes_to_equipartition():
    """Uniform gas whose translational and internal temperatures differ (2.0 vs 0.5), W the
    moments of f: no flux, so each step must conserve W (the collision term conserves
    energy only if the equilibrium of H carries dof/(2 lambda) of it) and
    H - dof/(2 lambda) g must shrink by the trapezoid factor (1 - h)/(1 + h)."""
    o = O.Oracle(nx=4, ny=4, lx=1.0, ly=1.0, nu=40, nv=40, umax=9.0, vmax=9.0, kn=0.02, bc=0,
                 noise=0.0, dof=1)
    uu, vv, w = _grid(o)
    Tt, Ti = 2.0, 0.5
    G = Q.maxwellian_2d((1.0, 0.0, 0.0, 1 / Tt), uu, vv)
    H = 0.5 * Ti * G
    f0 = np.broadcast_to(np.concatenate([G, H]), (4, 4, 2 * uu.size)).copy()
    W0 = _cons_of_f(o, f0)
    o.set_state(f0, W0)
    assert o.step(1) == 0
    f1, W1 = o.state()
    assert np.array_equal(W1, W0)
    np.testing.assert_allclose(_cons_of_f(o, f1), W0, rtol=0, atol=1e-12)
    rc, p = O.prim(W0[0, 0], 1)
    T = 1 / p[3]
    assert abs(T - (2 * Tt + Ti) / 3) < 1e-10          # equipartition over 3 degrees
    tau = 2 * O.mu_ref_of_kn(0.02) * math.sqrt(p[3]) / p[0]
    h = o.dt / (2 * tau)
    g = Q.maxwellian_2d((p[0], 0.0, 0.0, p[3]), uu, vv)
    np.testing.assert_allclose(f1[0, 0, uu.size:] - 0.5 * T * g,
                               (H - 0.5 * T * g) * (1 - h) / (1 + h), rtol=0, atol=1e-14)
    assert o.step(400) == 0
    f, _ = o.state()
    np.testing.assert_allclose(f[0, 0, uu.size:], 0.5 * T * f[0, 0, :uu.size], rtol=1e-9)


def test_collisionless_internal_energy_is_transported_like_the_mass():
    """tau = inf with H = c G everywhere: H is advected by the same limited upwind scheme, and
    the limiter is homogeneous of degree one, so H stays c G."""
    o = O.Oracle(nx=10, ny=8, lx=1.0, ly=1.0, nu=12, nv=12, umax=3.0, vmax=3.0,
                 kn=float("inf"), bc=0, noise=0.3, seed=5, dof=2)
    f0, W0 = o.state()
    uu, vv, _ = _grid(o)
    NV = uu.size
    f0[..., :NV] *= 1 + 0.3 * np.cos(uu)[None, None, :] * np.linspace(0, 1, 10)[None, :, None]
    f0[..., NV:] = 0.7 * f0[..., :NV]
    o.set_state(f0, W0)
    assert o.step(6) == 0
    f, _ = o.state()
    assert np.max(np.abs(f[..., :NV] - f0[..., :NV])) > 1e-3
    np.testing.assert_allclose(f[..., NV:], 0.7 * f[..., :NV], rtol=1e-13,
                               atol=1e-15 * np.max(f0))


def test_channel_with_internal_dof_is_mirror_symmetric():
    o = O.Oracle(nx=8, ny=6, lx=2.0, ly=1.0, nu=16, nv=16, umax=5.0, vmax=5.0, kn=0.1, bc=1,
                 p_ratio=2.0, noise=0.0, dof=1)
    assert o.step(10) == 0
    m = o.moments()
    mirror = m[::-1]
    np.testing.assert_allclose(m[..., [0, 1, 3]], mirror[..., [0, 1, 3]], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(m[..., 2], -mirror[..., 2], rtol=0, atol=1e-13)
    assert np.max(m[..., 1]) > 1e-3                     # the pressure drop drives a flow


def test_walls_with_internal_dof_reflect_internal_energy_at_the_wall_temperature():
    """The gas leaving a wall at T_w carries H = T_w/2 G (per internal degree)."""
    o = O.Oracle(nx=6, ny=4, lx=1.5, ly=1.0, nu=16, nv=16, umax=5.0, vmax=5.0, kn=0.1, bc=1,
                 p_ratio=1.5, noise=0.02, T_wall=1.3, dof=2)
    assert o.step(1) == 0
    Ffx, Ffy = o.micro_flux()
    uk, vm, _, _ = o.velocity_grid()
    NV = 256
    vv = np.tile(vm, 16)
    up = vv > 0
    bottom = Ffy[0]                                  # y = 0: gas leaves the wall upwards
    np.testing.assert_allclose(bottom[:, NV:][:, up], 2 * 1.3 / 2 * bottom[:, :NV][:, up],
                               rtol=1e-14)
