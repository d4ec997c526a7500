"""Pins for the oracle's Shakhov collision model (CPU only).

The correction g S must carry no mass, momentum or energy and a heat flux of exactly (1 - Pr) q;
both are checked by Gauss-Hermite quadrature, not by the oracle's formula.  Then: Pr = 1 is
BGK bit for bit, the face flux matches the moments of its per-velocity form, a periodic box
conserves, a uniform equilibrium stays fixed, and a uniform gas with a heat flux relaxes it
by the factor the trapezoidal Eq. (3) gives with the heat flux of f^n in both equilibria.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import quadrature as Q


def _gh_grid(prim, order=16):
    rho, U, V, lam = prim
    x, w = np.polynomial.hermite.hermgauss(order)
    s = 1.0 / math.sqrt(lam)
    uu, vv = np.meshgrid(U + s * x, V + s * x, indexing="ij")
    ww = np.outer(w, w) / math.pi
    return uu.ravel(), vv.ravel(), ww.ravel() * rho      # weights of rho times the Gaussian


@pytest.mark.parametrize("pr", [2.0 / 3.0, 0.2, 1.0])
def test_shakhov_correction_carries_only_its_heat_flux(pr):
    rng = np.random.default_rng(int(pr * 100))
    for _ in range(5):
        prim = (rng.uniform(0.5, 2.0), rng.uniform(-0.7, 0.7), rng.uniform(-0.7, 0.7),
                rng.uniform(0.5, 2.5))
        q = rng.normal(size=2) * 0.3
        uu, vv, gw = _gh_grid(prim)
        S = np.array([O.shakhov(prim, q, pr, u, v) for u, v in zip(uu, vv)])
        cx, cy = uu - prim[1], vv - prim[2]
        c2 = cx * cx + cy * cy
        for psi in (np.ones_like(uu), uu, vv, 0.5 * (uu * uu + vv * vv)):
            assert abs(np.sum(gw * psi * S)) < 1e-13 * prim[0]
        heat = [0.5 * np.sum(gw * cx * c2 * S), 0.5 * np.sum(gw * cy * c2 * S)]
        np.testing.assert_allclose(heat, (1 - pr) * q, rtol=1e-12, atol=1e-15)


CASE = dict(nx=12, ny=8, lx=1.5, ly=1.0, nu=16, nv=16, umax=5.0, vmax=5.0, kn=0.05, bc=1,
            noise=0.05, seed=9, p_ratio=2.0)


def test_prandtl_one_is_bgk_bit_for_bit():
    a = O.Oracle(**CASE)
    b = O.Oracle(**dict(CASE, prandtl=1.0))
    c = O.Oracle(**dict(CASE, prandtl=1.0 - 2.0 ** -40))
    for o in (a, b, c):
        assert o.step(5) == 0
    fa, Wa = a.state()
    fb, Wb = b.state()
    fc, Wc = c.state()
    assert np.array_equal(fa, fb) and np.array_equal(Wa, Wb)
    assert not np.array_equal(fa, fc)                 # a Prandtl number below 1 is in effect
    assert np.max(np.abs(fa - fc)) < 1e-10 * np.max(fa)


def test_shakhov_rejects_internal_dof_and_bad_prandtl():
    for kw in (dict(prandtl=0.5, dof=1), dict(prandtl=0.0), dict(prandtl=1.5)):
        with pytest.raises(ValueError):
            O.Oracle(**dict(CASE, **kw))


def _face_grid(n, a):
    x, w = O.nodes(n, a)
    un, ut = np.meshgrid(x, x, indexing="ij")
    return un.ravel(), ut.ravel(), np.outer(w, w).ravel()


def test_shakhov_face_macro_flux_equals_moments_of_distribution_flux():
    """S5 + S7 with the Shakhov energy flux (1 - Pr) q0_n against the discrete moments of the
    per-velocity flux carrying Mt1 g0 S0."""
    un, ut, w = _face_grid(257, 9.0)
    primL = (1.05, 0.2, 0.05, 1 / 1.05)
    primR = (0.95, 0.1, -0.05, 1 / 0.97)
    fL = Q.maxwellian_2d(primL, un, ut) * (1 + 0.05 * np.sin(un) + 0.03 * un * (un * un + ut * ut - 2))
    fR = Q.maxwellian_2d(primR, un, ut) * (1 + 0.02 * np.cos(ut) - 0.02 * ut * (un * un - 1))
    H = np.where(un > 0, 1.0, np.where(un < 0, 0.0, 0.5))
    sL = 0.3 * Q.maxwellian_2d(primL, un, ut) * un
    sR = -0.2 * Q.maxwellian_2d(primR, un, ut) * ut
    fh = H * fL + (1 - H) * fR
    sn = H * sL + (1 - H) * sR
    st = 0.1 * fh * (ut - 0.05)
    psi = [np.ones_like(un), un, ut, 0.5 * (un ** 2 + ut ** 2)]
    WL = np.array([np.sum(w * p * fL) for p in psi])
    WR = np.array([np.sum(w * p * fR) for p in psi])
    for kn in (0.01, 0.1, 1.0):
        rc, FW, Ff = O.face(un, ut, w, fh, sn, st, WL, WR, 0.05, 0.1, 2e-3, O.mu_ref_of_kn(kn),
                            prandtl=2.0 / 3.0)
        assert rc == 0
        micro = np.array([np.sum(w * p * Ff) for p in psi])
        np.testing.assert_allclose(FW, micro, rtol=0, atol=2e-10 * np.max(np.abs(FW)))
        rc, FB, _ = O.face(un, ut, w, fh, sn, st, WL, WR, 0.05, 0.1, 2e-3, O.mu_ref_of_kn(kn))
        assert abs(FW[3] - FB[3]) > 1e-8 * abs(FB[3])      # the heat flux term is present
        np.testing.assert_array_equal(FW[:3], FB[:3])      # and touches only the energy


def test_shakhov_periodic_box_conserves():
    o = O.Oracle(**dict(CASE, bc=0, prandtl=2.0 / 3.0))
    _, W0 = o.state()
    tot0 = W0.sum(axis=(0, 1))
    assert o.step(20) == 0
    _, W = o.state()
    tot = W.sum(axis=(0, 1))
    scale = np.array([tot0[0], tot0[0], tot0[0], tot0[3]])
    assert np.all(np.abs(tot - tot0) <= 1e-13 * scale)


def test_shakhov_uniform_equilibrium_is_a_fixed_point():
    """On a grid that resolves the Maxwellian (40^2 on [-6,6]^2) its discrete heat flux is
    round-off, and so is the drift; on the coarse 16^2 grid the discrete heat flux of a moving
    Maxwellian is ~1e-9 and the Shakhov term acts on it (BGK does not see it)."""
    o = O.Oracle(**dict(CASE, bc=0, nu=40, nv=40, umax=6.0, vmax=6.0, prandtl=2.0 / 3.0))
    uk, vm, wk, wm = o.velocity_grid()
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    rho, U, V, T = 1.1, 0.3, -0.2, 0.9
    g = Q.maxwellian_2d((rho, U, V, 1 / T), uu.ravel(), vv.ravel())
    f0 = np.broadcast_to(g, (o.ny, o.nx, g.size)).copy()
    W0 = np.broadcast_to([rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V) + 0.5 * rho * T],
                         (o.ny, o.nx, 4)).copy()
    o.set_state(f0, W0)
    assert o.step(10) == 0
    f, W = o.state()
    assert np.array_equal(W, W0)
    assert np.max(np.abs(f - f0)) <= 1e-12 * np.max(f0)


@pytest.mark.parametrize("pr", [2.0 / 3.0, 0.4])
def test_uniform_heat_flux_relaxes_by_the_trapezoid_factor(pr):
    """Uniform gas with a heat flux, no net face flux: W stays, the collision conserves the
    moments of f, and with the heat flux of f^n in both equilibria of Eq. (3) the heat flux
    becomes q (1 + h (1 - 2 Pr)/2)/(1 + h/2), h = dt/tau."""
    o = O.Oracle(nx=4, ny=4, lx=1.0, ly=1.0, nu=48, nv=48, umax=8.0, vmax=8.0, kn=0.02, bc=0,
                 noise=0.0, prandtl=pr)
    uk, vm, wk, wm = o.velocity_grid()
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    u, v, w = uu.ravel(), vv.ravel(), np.outer(wk, wm).ravel()
    g = Q.maxwellian_2d((1.0, 0.0, 0.0, 1.0), u, v)
    f0 = g * (1 + 0.05 * (0.6 * u + 0.8 * v) * (u * u + v * v - 2.0))   # heat flux, same W
    psi = np.stack([np.ones_like(u), u, v, 0.5 * (u * u + v * v)])
    W = psi @ (w * f0)
    q0 = 0.5 * np.array([np.sum(w * u * (u * u + v * v) * f0), np.sum(w * v * (u * u + v * v) * f0)])
    assert np.linalg.norm(q0) > 1e-2
    o.set_state(np.broadcast_to(f0, (4, 4, u.size)).copy(), np.broadcast_to(W, (4, 4, 4)).copy())
    assert o.step(1) == 0
    f, W1 = o.state()
    assert np.array_equal(W1[0, 0], W)
    f1 = f[0, 0]
    np.testing.assert_allclose(psi @ (w * f1), W, rtol=0, atol=1e-12)
    rc, p = O.prim(W)
    tau = 2 * O.mu_ref_of_kn(0.02) * math.sqrt(p[3]) / p[0]
    h = o.dt / tau
    q1 = 0.5 * np.array([np.sum(w * (u - p[1]) * ((u - p[1]) ** 2 + (v - p[2]) ** 2) * f1),
                         np.sum(w * (v - p[2]) * ((u - p[1]) ** 2 + (v - p[2]) ** 2) * f1)])
    np.testing.assert_allclose(q1, q0 * (1 + 0.5 * h * (1 - 2 * pr)) / (1 + 0.5 * h),
                               rtol=1e-9, atol=1e-14)
