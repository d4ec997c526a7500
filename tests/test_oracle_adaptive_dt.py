"""Pins for the oracle's adaptive time step (CPU only).

Reading (the paper fixes no time step): with ``adaptive_dt`` each step n takes
dt^n = cfl / max over cells of [(umax + |U|)/dx + (vmax + |V|)/dy] on the state W^n at its
start, a global max-reduction; at rest it is the fixed CFL step.  The pins: the closed form at
rest and for a uniform flow (a fixed point, so the step stays put), the time level (a step
with the adaptive dt equals a step of a fixed-dt solver given that same dt, bitwise), the
simulated time as the sum of the steps, and the bound by the fixed step."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import quadrature as Q

PERIODIC = dict(nx=12, ny=8, lx=1.5, ly=1.0, nu=16, nv=16, umax=5.0, vmax=4.0, kn=0.05, bc=0,
                noise=0.05, seed=9, cfl=0.7)


def _uniform_state(o, prim):
    uk, vm, _, _ = o.velocity_grid()
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    rho, U, V, lam = prim
    f = Q.maxwellian_2d((rho, U, V, lam), uu.ravel(), vv.ravel())
    fcell = np.broadcast_to(f, (o.ny, o.nx, f.size)).copy()
    W = np.array([rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V) + 0.5 * rho / lam])
    return fcell, np.broadcast_to(W, (o.ny, o.nx, 4)).copy()


def _fixed_dt(c):
    dx, dy = c["lx"] / c["nx"], c["ly"] / c["ny"]
    return c["cfl"] / (c["umax"] / dx + c["vmax"] / dy)


def test_at_rest_the_adaptive_step_is_the_fixed_cfl_step():
    o = O.Oracle(**dict(PERIODIC, adaptive_dt=1, noise=0.0))
    assert o.dt == pytest.approx(_fixed_dt(PERIODIC), rel=1e-15)
    assert o.step(3) == 0
    assert o.dt == pytest.approx(_fixed_dt(PERIODIC), rel=1e-15)
    assert o.time == pytest.approx(3 * _fixed_dt(PERIODIC), rel=1e-15)


def test_uniform_flow_closed_form_and_steady():
    c = dict(PERIODIC, adaptive_dt=1)
    o = O.Oracle(**c)
    U, V = 0.35, -0.25
    f, W = _uniform_state(o, (1.2, U, V, 1 / 0.8))
    o.set_state(f, W)
    dx, dy = c["lx"] / c["nx"], c["ly"] / c["ny"]
    expect = c["cfl"] / ((c["umax"] + abs(U)) / dx + (c["vmax"] + abs(V)) / dy)
    assert o.dt == pytest.approx(expect, rel=1e-14)
    assert o.dt < _fixed_dt(c)
    assert o.step(5) == 0
    # a uniform state is a fixed point, so the step stays; time is the sum of five equal steps
    assert o.dt == pytest.approx(expect, rel=1e-13)
    assert o.time == pytest.approx(5 * expect, rel=1e-13)


def test_each_step_uses_the_dt_of_the_state_it_starts_from():
    """Step by step, the adaptive solver equals a fixed-step solver handed dt^n computed
    from W^n: bitwise for f and W."""
    case = dict(PERIODIC, noise=0.08)
    a = O.Oracle(**dict(case, adaptive_dt=1))
    f, W = a.state()
    # give the gas a non-uniform flow so that dt changes from step to step
    uk, vm, _, _ = a.velocity_grid()
    prim = np.zeros((a.ny, a.nx, 4))
    x = (np.arange(a.nx) + 0.5) / a.nx
    prim[..., 0] = W[..., 0]
    prim[..., 1] = 0.4 * np.sin(2 * np.pi * x)[None, :]
    prim[..., 2] = 0.1
    prim[..., 3] = 1.0
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    rho, U, V, lam = [prim[..., q][..., None] for q in range(4)]
    f = Q.maxwellian_2d((rho, U, V, lam), uu.ravel(), vv.ravel())
    W = np.stack([prim[..., 0], prim[..., 0] * prim[..., 1], prim[..., 0] * prim[..., 2],
                  0.5 * prim[..., 0] * (prim[..., 1] ** 2 + prim[..., 2] ** 2)
                  + 0.5 * prim[..., 0] / prim[..., 3]], -1)
    a.set_state(f, W)
    dts, t = [], 0.0
    for n in range(4):
        f_n, W_n = a.state()
        dx, dy = case["lx"] / case["nx"], case["ly"] / case["ny"]
        dt_n = O.adaptive_dt(W_n, case["cfl"], case["umax"], case["vmax"], dx, dy)
        assert a.dt == dt_n
        b = O.Oracle(**dict(case, dt_override=dt_n))
        b.set_state(f_n, W_n)
        assert a.step(1) == 0 and b.step(1) == 0
        fa, Wa = a.state()
        fb, Wb = b.state()
        assert np.array_equal(fa, fb) and np.array_equal(Wa, Wb), n
        dts.append(dt_n)
        t += dt_n
        assert a.time == t
    assert len(set(dts)) > 1                  # the step did change
    assert max(dts) <= _fixed_dt(case)


def test_adaptive_with_an_override_is_rejected():
    with pytest.raises(ValueError):
        O.Oracle(**dict(PERIODIC, adaptive_dt=1, dt_override=1e-3))
