"""GPU parity for the adaptive time step (each step's dt from a device max-reduction over the
state it starts from): the HIP path through the C ABI against the FP64 oracle, whose adaptive
step is pinned on the CPU (tests/test_oracle_adaptive_dt.py).  The step sequence and the
simulated time agree to rounding; the states to the FP64 bar (1e-12) and the FP32-store bar
(1e-5)."""
import numpy as np
import pytest

from paper_1810_08137_amd import ugks
from paper_1810_08137_amd import workloads as WL
from tests import parity as PR

pytestmark = pytest.mark.gpu

C1_ADAPT = dict(WL.C1, adaptive_dt=1)
# a periodic box whose gas is set moving: the step shrinks as the flow speeds up
PERIODIC_ADAPT = dict(WL.CHANNEL_DEFAULTS, nx=20, ny=9, lx=2.0, ly=1.0, nu=16, nv=18, umax=5.0,
                      vmax=5.0, kn=0.05, bc=0, seed=51, noise=0.05, adaptive_dt=1)


def test_c1_channel_adaptive_step_100_steps():
    PR.oracle_threads()
    g, o = PR.make_pair(C1_ADAPT)
    try:
        dts = []
        for n in range(10):
            t_g, dt_g = g.time()
            assert abs(dt_g - o.dt) <= 1e-14 * o.dt, (n, dt_g, o.dt)
            assert abs(t_g - o.time) <= 1e-14 * max(o.time, o.dt), (n, t_g, o.time)
            dts.append(o.dt)
            g.step(10)
            assert o.step(10) == 0
        t_g, dt_g = g.time()
        assert abs(t_g - o.time) <= 1e-13 * o.time
        f_gpu, W_gpu = g.state()
        f_ref, W_ref = o.state()
        e = PR.errors(g.moments(), PR.moments_of_W(W_ref), f_gpu, f_ref)
        print(f"[parity] C1 adaptive dt 100 steps: {e}, dt {dts[0]:.6g} -> {o.dt:.6g}", flush=True)
        PR.assert_within(e, PR.FP64_TOL, "C1 adaptive dt")
        assert o.dt < dts[0]          # the channel flow sped up and the step shrank
    finally:
        g.close()
        o.close()


def _moving(g, o):
    """Give both sides the same non-uniform moving Maxwellian state."""
    f, W = o.state()
    uk, vm, _, _ = o.velocity_grid()
    x = (np.arange(o.nx) + 0.5) / o.nx
    rho = W[..., 0]
    U = np.broadcast_to(0.5 * np.sin(2 * np.pi * x)[None, :], rho.shape)
    V = np.full(rho.shape, -0.15)
    lam = np.ones(rho.shape)
    uu, vv = np.meshgrid(uk, vm, indexing="ij")
    f = (rho * lam / np.pi)[..., None] * np.exp(
        -lam[..., None] * ((uu.ravel() - U[..., None]) ** 2 + (vv.ravel() - V[..., None]) ** 2))
    W = np.stack([rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V) + 0.5 * rho / lam], -1)
    o.set_state(f, W)
    g.set_state(f, W)


@pytest.mark.parametrize("precision,tol", [("fp64", PR.FP64_TOL), ("fp32_store", PR.FP32_STORE_TOL)])
def test_periodic_moving_gas_adaptive_step(precision, tol):
    PR.oracle_threads()
    g, o = PR.make_pair(PERIODIC_ADAPT, precision)
    try:
        _moving(g, o)
        t_g, dt_g = g.time()
        assert abs(dt_g - o.dt) <= 1e-14 * o.dt
        g.step(40)
        assert o.step(40) == 0
        t_g, dt_g = g.time()
        rel = 1e-13 if precision == "fp64" else 1e-6
        assert abs(t_g - o.time) <= rel * o.time
        assert abs(dt_g - o.dt) <= rel * o.dt
        f_gpu, W_gpu = g.state()
        f_ref, W_ref = o.state()
        e = PR.errors(g.moments(), PR.moments_of_W(W_ref), f_gpu, f_ref)
        print(f"[parity] periodic moving gas, adaptive dt, 40 steps, {precision}: {e}", flush=True)
        PR.assert_within(e, tol, f"periodic adaptive {precision}")
    finally:
        g.close()
        o.close()


def test_adaptive_solvers_in_a_batch_equal_alone_and_static_path():
    import torch

    cases = [C1_ADAPT, dict(PERIODIC_ADAPT, seed=52), dict(WL.C1, seed=53)]   # the last fixed
    alone = []
    for c in cases:
        kn, kw = WL.solver_kwargs(c)
        s = ugks.Solver(kn, **kw)
        s.step(6)
        alone.append((s.state(), s.time()))
        s.close()
    stream = torch.cuda.Stream()
    batch = ugks.Batch(8, stream=stream)
    solvers = []
    for c in cases:
        kn, kw = WL.solver_kwargs(c)
        solvers.append(ugks.Solver(kn, stream=stream, **kw))
    batch.step(solvers, 6)
    for (st, tm), s in zip(alone, solvers):
        f, W = s.state()
        assert np.array_equal(f, st[0]) and np.array_equal(W, st[1])
        assert s.time() == tm
    batch.close()
    for s in solvers:
        s.close()
    # the allocation-free entry point keeps the same step sequence
    kn, kw = WL.solver_kwargs(C1_ADAPT)
    s = ugks.Solver(kn, **kw)
    s.step_static(6)
    f, W = s.state()
    assert np.array_equal(f, alone[0][0][0]) and np.array_equal(W, alone[0][0][1])
    assert s.time() == alone[0][1]
    s.close()


def test_adaptive_with_an_override_is_refused():
    kn, kw = WL.solver_kwargs(dict(C1_ADAPT, dt_override=1e-3))
    with pytest.raises(ugks.UgksError) as e:
        ugks.Solver(kn, **kw)
    assert e.value.code == ugks.UGKS_E_INVAL
