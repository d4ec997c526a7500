"""State-level pins for the oracle (CPU only): conservation, fixed points, the collisionless
limit against an independently written advection scheme, the relaxation factor of Eq. (3),
channel symmetry and wall behaviour."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import quadrature as Q


def _psi_moments(f, uk, vm, wk, wm):
    """sum w psi f over the velocity grid, f[..., K*M] -> [..., 4] (test-side arithmetic)."""
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    w = np.outer(wk, wm).ravel()
    psi = np.stack([np.ones(uu.size), uu.ravel(), vv.ravel(), 0.5 * (uu ** 2 + vv ** 2).ravel()])
    return np.einsum("...v,qv->...q", f * w, psi)


def _maxwell_field(prim_field, uk, vm):
    """discrete Maxwellian per cell from (rho, U, V, lambda) fields, test-side arithmetic"""
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    uu, vv = uu.ravel(), vv.ravel()
    rho, U, V, lam = [prim_field[..., q][..., None] for q in range(4)]
    return Q.maxwellian_2d((rho, U, V, lam), uu, vv)


def _cons(prim_field):
    rho, U, V, lam = [prim_field[..., q] for q in range(4)]
    return np.stack([rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V) + 0.5 * rho / lam], -1)


PERIODIC = dict(nx=12, ny=8, lx=1.5, ly=1.0, nu=16, nv=16, umax=5.0, vmax=5.0, kn=0.05, bc=0,
                noise=0.05, seed=9)


# ------------------------------------------------------------------ Eq. (4) telescopes
def test_periodic_box_conserves_mass_momentum_energy():
    o = O.Oracle(**PERIODIC)
    _, W0 = o.state()
    tot0 = W0.sum(axis=(0, 1))
    assert o.step(20) == 0
    _, W = o.state()
    tot = W.sum(axis=(0, 1))
    scale = np.array([tot0[0], tot0[0], tot0[0], tot0[3]])   # momentum normalised by mass
    assert np.all(np.abs(tot - tot0) <= 1e-13 * scale), (tot - tot0) / scale
    assert np.ptp(W[..., 0]) > 1e-4     # the state did evolve


# ------------------------------------------------------------------ equilibrium fixed point
def test_uniform_moving_maxwellian_is_a_fixed_point_periodic():
    o = O.Oracle(**PERIODIC)
    uk, vm, _, _ = o.velocity_grid()
    prim = np.zeros((o.ny, o.nx, 4))
    prim[...] = (1.1, 0.3, -0.2, 1 / 0.9)
    f0 = _maxwell_field(prim, uk, vm)
    W0 = _cons(prim)
    o.set_state(f0, W0)
    assert o.step(10) == 0
    f, W = o.state()
    assert np.array_equal(W, W0)      # every face sees the same state: fluxes cancel exactly
    assert np.max(np.abs(f - f0)) <= 1e-14 * np.max(f0)


def test_channel_at_rest_stays_at_rest():
    """Equal inlet/outlet pressure, walls at the gas temperature, no noise: up to the
    difference between discrete and analytic Maxwellian moments (< 1e-14 on this grid)
    nothing moves."""
    o = O.Oracle(nx=10, ny=6, lx=2.0, ly=1.0, nu=40, nv=40, umax=6.0, vmax=6.0, kn=0.1, bc=1,
                 p_ratio=1.0, noise=0.0)
    f0, W0 = o.state()
    assert o.step(5) == 0
    f, W = o.state()
    assert np.max(np.abs(W - W0)) < 1e-13
    assert np.max(np.abs(f - f0)) < 1e-13 * np.max(f0)


# ------------------------------------------------------------------ Eq. (3) collision term
def test_uniform_nonequilibrium_relaxes_by_the_trapezoid_factor():
    """A spatially uniform f away from equilibrium sees no net flux; Eq. (3) then reduces to
    the trapezoid rule for df/dt = (g - f)/tau, so f - g shrinks by (1 - h)/(1 + h),
    h = dt/(2 tau), with W (hence g and tau) unchanged."""
    o = O.Oracle(**PERIODIC)
    uk, vm, wk, wm = o.velocity_grid()
    prim = np.zeros((o.ny, o.nx, 4))
    prim[...] = (1.0, 0.1, 0.0, 1.0)
    g = _maxwell_field(prim, uk, vm)
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    bump = 0.05 * np.exp(-((uu.ravel() - 1.0) ** 2 + vv.ravel() ** 2))
    f0 = g * (1 + 0.2 * np.cos(uu.ravel())) + bump
    W0 = _cons(prim)
    o.set_state(f0, W0)
    assert o.step(1) == 0
    f, W = o.state()
    assert np.array_equal(W, W0)
    tau = 2 * O.mu_ref_of_kn(PERIODIC["kn"]) * math.sqrt(prim[0, 0, 3]) / prim[0, 0, 0]
    h = o.dt / (2 * tau)
    np.testing.assert_allclose(f - g, (f0 - g) * (1 - h) / (1 + h), rtol=0,
                               atol=1e-14 * np.max(np.abs(f0)))


# ------------------------------------------------------------------ free transport
FREE = dict(nx=8, ny=8, lx=1.0, ly=1.0, nu=3, nv=3, umax=1.0, vmax=1.0, kn=float("inf"), bc=0,
            dt_override=0.125, noise=0.0)


def test_collisionless_axis_velocities_shift_exactly_one_cell():
    o = O.Oracle(**FREE)
    rng = np.random.default_rng(4)
    f0 = rng.uniform(0.5, 1.5, size=(8, 8, 9))
    uk, vm, wk, wm = o.velocity_grid()
    W0 = _psi_moments(f0, uk, vm, wk, wm)
    o.set_state(f0, W0)
    assert o.step(1) == 0
    f, W = o.state()
    for k, u in enumerate(uk):
        for m, v in enumerate(vm):
            q = k * 3 + m
            if u != 0 and v != 0:
                continue                  # diagonal velocities are not a pure shift
            expect = np.roll(f0[..., q], shift=(int(v), int(u)), axis=(0, 1))
            np.testing.assert_allclose(f[..., q], expect, rtol=0, atol=1e-14)
    # in the collisionless limit the macro flux is the moment of the micro flux
    np.testing.assert_allclose(W, _psi_moments(f, uk, vm, wk, wm), rtol=0, atol=1e-14)


def _vl(a, b):
    prod = a * b
    den = np.where(prod > 0, a + b, 1.0)
    return np.where(prod > 0, 2 * prod / den, 0.0)


def _muscl_hancock_step(f, uk, vm, dx, dy, dt):
    """Independent periodic 2D MUSCL-Hancock step with van Leer slopes and upwind faces,
    written with array shifts (no oracle code)."""
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    u, v = uu.ravel(), vv.ravel()
    sx = _vl(np.roll(f, -1, 1) - f, f - np.roll(f, 1, 1)) / dx
    sy = _vl(np.roll(f, -1, 0) - f, f - np.roll(f, 1, 0)) / dy
    pred = lambda g, s_n, s_t, sign, d, un, ut: g + sign * 0.5 * d * s_n - 0.5 * dt * (un * s_n + ut * s_t)
    # x-face to the left of cell i: cell i-1 on its right edge, cell i on its left edge
    left = pred(np.roll(f, 1, 1), np.roll(sx, 1, 1), np.roll(sy, 1, 1), +1, dx, u, v)
    right = pred(f, sx, sy, -1, dx, u, v)
    face_x = np.where(u > 0, left, np.where(u < 0, right, 0.5 * (left + right)))
    Fx = u * face_x * dt * dy
    low = pred(np.roll(f, 1, 0), np.roll(sy, 1, 0), np.roll(sx, 1, 0), +1, dy, v, u)
    high = pred(f, sy, sx, -1, dy, v, u)
    face_y = np.where(v > 0, low, np.where(v < 0, high, 0.5 * (low + high)))
    Fy = v * face_y * dt * dx
    return f + (Fx - np.roll(Fx, -1, 1) + Fy - np.roll(Fy, -1, 0)) / (dx * dy)


def test_collisionless_matches_independent_muscl_hancock():
    case = dict(FREE, nx=10, ny=7, lx=1.0, ly=0.7, nu=5, nv=4, umax=1.3, vmax=0.9, dt_override=0.0,
                cfl=0.7)
    o = O.Oracle(**case)
    uk, vm, wk, wm = o.velocity_grid()
    rng = np.random.default_rng(6)
    x = (np.arange(10) + 0.5) / 10
    y = (np.arange(7) + 0.5) / 7 * 0.7
    base = 1 + 0.3 * np.sin(2 * np.pi * x)[None, :, None] * np.cos(2 * np.pi * y / 0.7)[:, None, None]
    f0 = base * rng.uniform(0.5, 1.5, size=(1, 1, 20)) + 0.05 * rng.uniform(size=(7, 10, 20))
    o.set_state(f0, _psi_moments(f0, uk, vm, wk, wm))
    ref = f0.copy()
    for _ in range(6):
        assert o.step(1) == 0
        ref = _muscl_hancock_step(ref, uk, vm, 0.1, 0.1, o.dt)
        f, _ = o.state()
        np.testing.assert_allclose(f, ref, rtol=0, atol=1e-14)


# ------------------------------------------------------------------ channel
C1 = dict(nx=40, ny=10, lx=4.0, ly=1.0, nu=24, nv=24, umax=5.0, vmax=5.0, kn=0.1, bc=1,
          p_ratio=2.0, noise=0.01, seed=1)


def test_channel_ghost_states_follow_the_pressure_readings():
    o = O.Oracle(**C1)
    assert o.step(4) == 0
    _, W = o.state()               # the next step builds its ghosts from this state
    assert o.step(1) == 0
    Wg, fg = o.ghost()
    p0 = 0.5
    p_in, p_out = 2 * 2.0 * p0 / 3.0, 2 * p0 / 3.0
    for j in range(o.ny):
        rc, pin = O.prim(Wg[0, j])
        rc2, pout = O.prim(Wg[1, j])
        _, first = O.prim(W[j, 0])
        _, last = O.prim(W[j, -1])
        assert rc == 0 and rc2 == 0
        assert math.isclose(pin[0] / pin[3] / 2, p_in, rel_tol=1e-13)      # p = rho T / 2
        assert math.isclose(1 / pin[3], 1.0, rel_tol=1e-13)                  # T_in
        np.testing.assert_allclose(pin[1:3], first[1:3], rtol=1e-13, atol=1e-16)
        assert math.isclose(pout[0] / pout[3] / 2, p_out, rel_tol=1e-13)
        np.testing.assert_allclose(pout[1:], last[1:], rtol=1e-13, atol=1e-16)
    # ghosts are Maxwellians of their states on the grid
    uk, vm, _, _ = o.velocity_grid()
    rc, pin = O.prim(Wg[0, 3])
    np.testing.assert_allclose(fg[0, 3], _maxwell_field(pin[None, :], uk, vm)[0], rtol=1e-13)


def test_channel_inlet_with_seeded_velocity():
    o = O.Oracle(**dict(C1, inlet_fixed_u=1, U_in=0.1, U_noise=0.05, noise=0.0, seed=3))
    assert o.step(1) == 0
    Wg, _ = o.ghost()
    for j in range(o.ny):
        _, pin = O.prim(Wg[0, j])
        xi = O.unit_noise(3, o.nx * o.ny + j)
        assert math.isclose(pin[1], 0.1 * (1 + 0.05 * xi), rel_tol=1e-13)
        assert abs(pin[2]) < 1e-16


# Boundary temperatures away from 1 (Sec. 3.A fixes the inlet temperature; the walls are a
# reading): with T_in = T_wall = 1 a slip of lambda for T in either place would pass unseen.
HOT = dict(C1, T_in=1.2, T_wall=1.3)


def test_inlet_ghost_holds_the_inlet_temperature_and_pressure():
    """The inlet ghost state has T = T_in and rho = 2 p_in / T_in (p = rho T / 2), taken here
    from W by the energy relation rho E = rho |U|^2/2 + rho T/2, and its f is the Maxwellian
    rho/(pi T_in) exp(-|c - U|^2 / T_in) on the grid."""
    o = O.Oracle(**HOT)
    assert o.step(3) == 0
    Wg, fg = o.ghost()
    p_in = 2 * 2.0 * 0.5 / 3.0
    uk, vm, _, _ = o.velocity_grid()
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    for j in range(o.ny):
        rho, mx, my, E = Wg[0, j]
        U, V = mx / rho, my / rho
        T = (E - 0.5 * rho * (U * U + V * V)) / (0.5 * rho)
        assert math.isclose(T, 1.2, rel_tol=1e-13)
        assert math.isclose(rho, 2.0 * p_in / 1.2, rel_tol=1e-13)
        g = rho / (math.pi * 1.2) * np.exp(-((uu - U) ** 2 + (vv - V) ** 2) / 1.2)
        np.testing.assert_allclose(fg[0, j], g.ravel(), rtol=1e-13, atol=0)
        # the ratio of two grid values depends on T_in alone, whatever rho is
        r = fg[0, j][0] / fg[0, j][o.nv * (o.nu // 2) + o.nv // 2]
        d = ((uk[0] - U) ** 2 + (vm[0] - V) ** 2) - ((uk[o.nu // 2] - U) ** 2 + (vm[o.nv // 2] - V) ** 2)
        assert math.isclose(r, math.exp(-d / 1.2), rel_tol=1e-12)


def test_outlet_ghost_keeps_the_last_column_temperature_at_a_hot_inlet():
    """The outlet ghost copies (U, V, T) of the last column and fixes p_out, also when the
    inlet and walls are not at the reference temperature."""
    o = O.Oracle(**HOT)
    assert o.step(6) == 0
    _, W = o.state()
    assert o.step(1) == 0
    Wg, _ = o.ghost()
    p_out = 2 * 0.5 / 3.0
    for j in range(o.ny):
        rho, mx, my, E = W[j, -1]
        T_last = (E - 0.5 * (mx * mx + my * my) / rho) / (0.5 * rho)
        rg, gx, gy, Eg = Wg[1, j]
        Tg = (Eg - 0.5 * (gx * gx + gy * gy) / rg) / (0.5 * rg)
        assert math.isclose(Tg, T_last, rel_tol=1e-13)
        assert math.isclose(0.5 * rg * Tg, p_out, rel_tol=1e-13)


@pytest.mark.parametrize("top", [False, True])
def test_hot_wall_emits_its_own_maxwellian(top):
    """Particles leaving a wall at T_wall = 1.3 carry rho_w exp(-|c|^2 / T_wall): the ratio of
    the distribution flux per unit normal velocity at two leaving velocities is
    exp(-(|c1|^2 - |c2|^2) / T_wall) whatever rho_w is, and the net mass flux through the wall
    is zero."""
    o = O.Oracle(**HOT)
    assert o.step(4) == 0
    _, Ffy = o.micro_flux()
    uk, vm, wk, wm = o.velocity_grid()
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    u, v, w = uu.ravel(), vv.ravel(), np.outer(wk, wm).ravel()
    face = Ffy[-1] if top else Ffy[0]
    leave = (v < 0) if top else (v > 0)
    idx = np.flatnonzero(leave)
    a, b = idx[0], idx[len(idx) // 2]
    expect = math.exp(-((u[a] ** 2 + v[a] ** 2) - (u[b] ** 2 + v[b] ** 2)) / 1.3)
    for i in range(o.nx):
        r = (face[i, a] / v[a]) / (face[i, b] / v[b])
        assert math.isclose(r, expect, rel_tol=1e-12), (i, r, expect)
    # one emitted density per face: flux / (v exp(-|c|^2/T_w)) is the same for every leaving c
    dens = face[:, idx] / (v[idx] * np.exp(-(u[idx] ** 2 + v[idx] ** 2) / 1.3))
    np.testing.assert_allclose(dens, dens[:, :1] * np.ones_like(dens), rtol=1e-12)
    assert np.all(dens > 0)
    net = (face * w).sum(axis=1)
    assert np.max(np.abs(net)) < 1e-14 * np.max(np.abs(face * w).sum(axis=1))


def test_wall_rows_reconstruct_without_y_slope():
    """Reading: next to a wall the y-slope of f is zero, so in the collisionless limit the
    flux through the face above the bottom wall row, for v > 0, is pure upwind transport of
    that row with its x-slope only."""
    case = dict(C1, nx=8, ny=5, lx=1.0, ly=0.625, nu=6, nv=6, kn=float("inf"), noise=0.0)
    o = O.Oracle(**case)
    rng = np.random.default_rng(12)
    f0 = rng.uniform(0.5, 1.5, size=(5, 8, 36))
    uk, vm, wk, wm = o.velocity_grid()
    o.set_state(f0, _psi_moments(f0, uk, vm, wk, wm))
    assert o.step(1) == 0
    Wg, fg = o.ghost()
    _, Ffy = o.micro_flux()
    dx, dt = 0.125, o.dt
    row = f0[0]
    left = np.vstack([fg[0, 0][None], row[:-1]])
    right = np.vstack([row[1:], fg[1, 0][None]])
    sx = _vl(right - row, row - left) / dx
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    u, v = uu.ravel(), vv.ravel()
    up = v > 0
    expect = dx * v * (dt * row - 0.5 * dt * dt * (u * sx))
    np.testing.assert_allclose(Ffy[1][:, up], expect[:, up], rtol=1e-13, atol=1e-16)


def test_channel_without_noise_is_mirror_symmetric():
    o = O.Oracle(**dict(C1, noise=0.0))
    assert o.step(40) == 0
    m = o.moments()
    flip = m[::-1]
    for q, parity in [(0, 1), (1, 1), (2, -1), (3, 1)]:
        np.testing.assert_allclose(m[..., q], parity * flip[..., q], rtol=0, atol=1e-13)
    assert np.max(np.abs(m[..., 2])) > 1e-4       # a real transverse flow exists


def test_walls_have_zero_net_mass_flux():
    o = O.Oracle(**C1)
    assert o.step(3) == 0
    Fx, Fy = o.face_flux()
    scale = np.max(np.abs(Fx[..., 0]))
    assert np.max(np.abs(Fy[0, :, 0])) < 1e-15 * max(scale, 1.0)
    assert np.max(np.abs(Fy[-1, :, 0])) < 1e-15 * max(scale, 1.0)


def test_invalid_state_is_reported():
    o = O.Oracle(**PERIODIC)
    f, W = o.state()
    W[2, 3, 3] = 0.0            # no internal energy
    o.set_state(f, W)
    assert o.step(1) == -4


def test_channel_pressure_difference_drives_flow_towards_outlet():
    o = O.Oracle(**C1)
    assert o.step(100) == 0
    m = o.moments()
    assert np.mean(m[:, :, 1]) > 0.0
    assert np.all(m[..., 0] > 0) and np.all(m[..., 3] > 0)


# ------------------------------------------------------------------ Eq. (3) and Eq. (4) as printed
def test_update_satisfies_eq3_and_eq4_in_their_printed_form():
    """After a step in which W changes, the new state satisfies the paper's update equations
    as written: Eq. (4) with the face fluxes, and Eq. (3) with the collision term evaluated
    at both time levels (implicit in f^{n+1}), each to rounding."""
    o = O.Oracle(**C1)
    assert o.step(5) == 0
    fn, Wn = o.state()
    assert o.step(1) == 0
    f1, W1 = o.state()
    Fx, Fy = o.face_flux()
    Ffx, Ffy = o.micro_flux()
    dx, dy, dt = 0.1, 0.1, o.dt
    np.testing.assert_allclose(
        W1, Wn + (Fx[:, :-1] - Fx[:, 1:] + Fy[:-1] - Fy[1:]) / (dx * dy), rtol=0, atol=1e-14)
    assert np.max(np.abs(W1 - Wn)) > 1e-6
    uk, vm, _, _ = o.velocity_grid()

    def prim_tau(W):
        rho = W[..., 0]
        U, V = W[..., 1] / rho, W[..., 2] / rho
        lam = rho / (2 * (W[..., 3] - 0.5 * rho * (U * U + V * V)))
        tau = 2 * O.mu_ref_of_kn(C1["kn"]) * np.sqrt(lam) / rho
        return np.stack([rho, U, V, lam], -1), tau[..., None]

    pn, tn = prim_tau(Wn)
    p1, t1 = prim_tau(W1)
    gn, g1 = _maxwell_field(pn, uk, vm), _maxwell_field(p1, uk, vm)
    dF = (Ffx[:, :-1] - Ffx[:, 1:] + Ffy[:-1] - Ffy[1:]) / (dx * dy)
    resid = f1 - (fn + dF + 0.5 * dt * ((g1 - f1) / t1 + (gn - fn) / tn))
    assert np.max(np.abs(resid)) < 1e-15 * 50 * np.max(fn)


# ------------------------------------------------------------------ geometric symmetries
def _smooth_state(nx, ny, uk, vm, seed):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)              # [ny, nx]
    prim = np.stack([1 + 0.1 * np.sin(2 * np.pi * X + rng.uniform()) * np.cos(2 * np.pi * Y),
                     0.2 * np.cos(2 * np.pi * Y + rng.uniform()),
                     0.15 * np.sin(2 * np.pi * X),
                     1 / (1 + 0.05 * np.cos(2 * np.pi * (X + Y)))], -1)
    f = _maxwell_field(prim, uk, vm) * (1 + 0.05 * rng.uniform(size=(1, 1, uk.size * vm.size)))
    return f, _cons(prim)


def test_transposing_x_and_y_commutes_with_the_step():
    """Swap x<->y and u<->v: on a square periodic box with a square velocity grid the step
    must commute with the swap.  Catches a wrong local frame on the y-faces."""
    case = dict(PERIODIC, nx=9, ny=9, lx=1.0, ly=1.0, nu=12, nv=12)
    a, b = O.Oracle(**case), O.Oracle(**case)
    uk, vm, _, _ = a.velocity_grid()
    f, W = _smooth_state(9, 9, uk, vm, 1)
    ft = f.reshape(9, 9, 12, 12).transpose(1, 0, 3, 2).reshape(9, 9, 144)
    Wt = W.transpose(1, 0, 2)[..., [0, 2, 1, 3]]
    a.set_state(f, W)
    b.set_state(ft, Wt)
    assert a.step(3) == 0 and b.step(3) == 0
    fa, Wa = a.state()
    fb, Wb = b.state()
    np.testing.assert_allclose(fb, fa.reshape(9, 9, 12, 12).transpose(1, 0, 3, 2).reshape(9, 9, 144),
                               rtol=0, atol=1e-14)
    np.testing.assert_allclose(Wb, Wa.transpose(1, 0, 2)[..., [0, 2, 1, 3]], rtol=0, atol=1e-14)


def test_reflecting_x_commutes_with_the_step():
    """x -> -x together with u -> -u (and U -> -U) on a periodic box."""
    case = dict(PERIODIC, nx=10, ny=6, nu=12, nv=10)
    a, b = O.Oracle(**case), O.Oracle(**case)
    uk, vm, _, _ = a.velocity_grid()
    f, W = _smooth_state(10, 6, uk, vm, 2)
    fr = f.reshape(6, 10, 12, 10)[:, ::-1, ::-1, :].reshape(6, 10, 120)
    Wr = W[:, ::-1].copy()
    Wr[..., 1] *= -1
    a.set_state(f, W)
    b.set_state(fr, Wr)
    assert a.step(3) == 0 and b.step(3) == 0
    fa, Wa = a.state()
    fb, Wb = b.state()
    np.testing.assert_allclose(fb, fa.reshape(6, 10, 12, 10)[:, ::-1, ::-1, :].reshape(6, 10, 120),
                               rtol=0, atol=1e-14)
    Wa_r = Wa[:, ::-1].copy()
    Wa_r[..., 1] *= -1
    np.testing.assert_allclose(Wb, Wa_r, rtol=0, atol=1e-14)
