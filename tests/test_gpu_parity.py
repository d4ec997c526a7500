"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded inputs.

FP64 bar: rho and T relative, U and V absolute, f per-cell max |df| / max f, all <= 1e-12.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_08137_amd import ugks
from paper_1810_08137_amd import workloads as WL
from tests import parity as PR

pytestmark = pytest.mark.gpu


def _case(**kw):
    c = dict(WL.CHANNEL_DEFAULTS)
    c.update(kw)
    return c


def test_c1_first_step_face_fluxes():
    """One step of the parity case: every interface flux and the new state."""
    PR.oracle_threads()
    g, o = PR.make_pair(WL.C1)
    try:
        g.step(1)
        assert o.step(1) == 0
        Fx, Fy = g.face_flux()
        Rx, Ry = o.face_flux()
        scale = np.max(np.abs(Rx), axis=(0, 1))
        ex = np.max(np.abs(Fx - Rx), axis=(0, 1)) / scale
        ey = np.max(np.abs(Fy - Ry), axis=(0, 1)) / np.maximum(np.max(np.abs(Ry), axis=(0, 1)), scale)
        print("[parity] C1 step 1 face flux errors", ex, ey, flush=True)
        assert np.all(ex < 1e-12) and np.all(ey < 1e-12)
        f_gpu, W_gpu = g.state()
        f_ref, W_ref = o.state()
        PR.assert_within(PR.errors(PR.moments_of_W(W_gpu), PR.moments_of_W(W_ref), f_gpu, f_ref),
                         PR.FP64_TOL, "C1 step 1")
    finally:
        g.close()
        o.close()


def test_c1_parity_full_run():
    PR.run_and_compare(WL.C1, WL.C1_STEPS, label="C1 40x10 24^2 channel")


@pytest.mark.parametrize("nx,ny,nu,nv", [(13, 7, 11, 9), (5, 9, 8, 13), (17, 3, 6, 6)])
def test_ragged_periodic_boxes(nx, ny, nu, nv):
    """Velocity counts that are not multiples of 64 and odd cell counts, periodic."""
    case = _case(nx=nx, ny=ny, lx=1.3, ly=0.9, nu=nu, nv=nv, umax=4.5, vmax=5.5, kn=0.07, bc=0,
                 noise=0.05, seed=11 + nx)
    PR.run_and_compare(case, 25, label=f"periodic {nx}x{ny} {nu}x{nv}")


@pytest.mark.parametrize("nx,ny,nu,nv", [(9, 5, 7, 7), (6, 4, 9, 5)])
def test_ragged_channels_with_zero_velocities(nx, ny, nu, nv):
    """Odd velocity counts put u = 0 and v = 0 on the grid (upwind weight 1/2)."""
    case = _case(nx=nx, ny=ny, lx=2.0, ly=1.0, nu=nu, nv=nv, umax=5.0, vmax=5.0, kn=0.2,
                 noise=0.02, seed=4)
    PR.run_and_compare(case, 30, label=f"channel {nx}x{ny} {nu}x{nv}")


@pytest.mark.parametrize("nx", [60, 61, 62, 63, 121, 124])
def test_channel_widths_at_segment_edges(nx):
    """Channel widths at the row-segment edges of the two cell kernels (60 cells per update
    segment, 62 per moment segment): the outlet ghost column then falls on a segment's last
    lane, on the halo of the segment before the last, or next to a one-cell last segment."""
    case = _case(nx=nx, ny=3, lx=nx / 10.0, ly=0.3, nu=8, nv=6, umax=4.0, vmax=4.0, kn=0.1,
                 noise=0.02, seed=21 + nx)
    PR.run_and_compare(case, 20, label=f"channel {nx}x3 8x6")


@pytest.mark.parametrize("bc,precision,extra", [(1, "fp64", {}), (0, "fp64", {}),
                                                 (1, "fp32_store", {}),
                                                 (1, "fp64", {"prandtl": 2.0 / 3.0}),
                                                 (1, "fp64", {"dof": 1})])
def test_odd_row_count_with_unequal_v_chunks(bc, precision, extra):
    """Seven rows (the last row pair overlaps the one before it and writes only its upper row)
    with each v half of 33 nodes split into four chunks of unequal length (17 nodes on the
    v >= 0 side, 16 on the other), each chunk starting its Gauss recurrences at its own first
    node; also with the Shakhov model and with internal degrees of freedom (whose chunks of H
    follow those of G)."""
    case = _case(nx=23, ny=7, lx=2.3, ly=0.7, nu=33, nv=33, umax=5.0, vmax=5.0, kn=0.1, bc=bc,
                 noise=0.03, seed=31, **extra)
    kn, kw = WL.solver_kwargs(case, precision)
    s = ugks.Solver(kn, **kw)
    try:
        assert s.info.update_v_chunks == 4
    finally:
        s.close()
    tol = PR.FP64_TOL if precision == "fp64" else PR.FP32_STORE_TOL
    PR.run_and_compare(case, 20, precision=precision, tol=tol,
                       label=f"23x7 33^2 bc={bc} {precision} {extra}, 4 v chunks")


@pytest.mark.parametrize("bc", [0, 1])
def test_collisionless_limit(bc):
    case = _case(nx=12, ny=6, lx=2.0, ly=1.0, nu=10, nv=9, umax=3.0, vmax=3.0, kn=float("inf"),
                 bc=bc, noise=0.05, seed=8)
    PR.run_and_compare(case, 20, label=f"collisionless bc={bc}")


@pytest.mark.parametrize("nx,ny,bc", [(1, 6, 1), (8, 1, 1), (1, 1, 0), (1, 5, 0), (2, 2, 1)])
def test_degenerate_meshes(nx, ny, bc):
    """Single row (both walls on one row), single column (inlet and outlet ghosts on one
    cell), a 1x1 periodic box (every neighbour is the cell itself)."""
    case = _case(nx=nx, ny=ny, lx=0.5 * nx, ly=0.5 * ny, nu=8, nv=8, umax=4.0, vmax=4.0, kn=0.3,
                 bc=bc, noise=0.03, seed=21)
    PR.run_and_compare(case, 15, label=f"degenerate {nx}x{ny} bc={bc}")


def test_wide_velocity_space_inlet_noise():
    """The wide-grid configuration's boundary treatment (seeded inlet U) on a small mesh."""
    case = dict(WL.C3, nx=20, ny=6, nu=41, nv=41)
    PR.run_and_compare(case, 20, label="C3-shaped small")


def test_c2_full_size_steps():
    """The 400x100 x 40^2 configuration the benchmark times, compared in full."""
    PR.run_and_compare(WL.C2, 3, label="C2 400x100 40^2")


def test_c3_full_size_steps():
    """200x50 x 101^2 (10201 velocities per cell, padded to 10240)."""
    PR.run_and_compare(WL.C3, 2, label="C3 200x50 101^2")


def test_fp32_store_error_c1():
    e = PR.run_and_compare(WL.C1, WL.C1_STEPS, precision="fp32_store", tol=PR.FP32_STORE_TOL,
                           label="C1 FP32-store")
    assert max(e.values()) > 1e-12      # it really is stored in FP32


def test_fp32_store_c4_against_oracle_50_steps():
    """The FP32-store form of the 400x100 x 40^2 case against the FP64 oracle."""
    e = PR.run_and_compare(WL.C4, 50, precision="fp32_store", tol=PR.FP32_STORE_TOL,
                           label="C4 FP32-store 50 steps")
    assert max(e.values()) > 1e-12


def test_fp32_store_with_velocity_chunks():
    """FP32-store on the paper's M1 mesh at 49^2 (16 velocity chunks per quadrant)."""
    e = PR.run_and_compare(WL.paper_mesh(40, 20, 49), 20, precision="fp32_store",
                           tol=PR.FP32_STORE_TOL, label="paper M1 49^2 FP32-store")
    assert max(e.values()) > 1e-12


def test_fp32_store_wide_velocity_grid():
    """FP32-store on 200x50 x 101^2 (3 velocity chunks, Gaussians over 51 v nodes)."""
    e = PR.run_and_compare(WL.C3, 2, precision="fp32_store", tol=PR.FP32_STORE_TOL,
                           label="C3 FP32-store")
    assert max(e.values()) > 1e-12


def test_runs_are_bitwise_deterministic():
    kn, kw = WL.solver_kwargs(WL.C1)
    a, b = ugks.Solver(kn, **kw), ugks.Solver(kn, **kw)
    try:
        a.step(20)
        b.step(20)
        fa, Wa = a.state()
        fb, Wb = b.state()
        assert np.array_equal(fa, fb) and np.array_equal(Wa, Wb)
    finally:
        a.close()
        b.close()


RESUME_CASES = {
    "C1 fp64": (WL.C1, "fp64", 10),
    "C1 fp32 (odd step count)": (WL.C1, "fp32_store", 11),
    "channel 121x5, three segments": (
        _case(nx=121, ny=5, lx=12.1, ly=0.5, nu=10, nv=8, umax=4.0, vmax=4.0, kn=0.1, seed=71),
        "fp64", 7),
}


@pytest.mark.parametrize("name", list(RESUME_CASES))
def test_checkpoint_resume_is_bitwise(name):
    """A state copied into a second solver steps on bitwise as the first: the channel ghost
    columns a set state gets from the update kernel's fill mode equal those a running solver's
    update kernel writes."""
    case, precision, steps = RESUME_CASES[name]
    kn, kw = WL.solver_kwargs(case, precision)
    a, b = ugks.Solver(kn, **kw), ugks.Solver(kn, **dict(kw, seed=99))
    try:
        a.step(steps)
        f, W = a.state()
        b.set_state(f, W)
        a.step(15)
        b.step(15)
        fa, Wa = a.state()
        fb, Wb = b.state()
        assert np.array_equal(fa, fb) and np.array_equal(Wa, Wb)
    finally:
        a.close()
        b.close()


def test_invalid_state_is_reported_by_moments():
    kn, kw = WL.solver_kwargs(WL.C1)
    a = ugks.Solver(kn, **kw)
    try:
        f, W = a.state()
        W[3, 7, 3] = -1.0
        a.set_state(f, W)
        a.step(1)
        with pytest.raises(ugks.UgksError) as ex:
            a.moments()
        assert ex.value.code == ugks.UGKS_E_STATE
    finally:
        a.close()


@pytest.mark.parametrize("bc", [1, 0])
def test_kernel_timing_counts_launches(bc):
    """Every launch of a step is timed; a channel has no ghost launch (its update kernel
    writes the next step's ghost columns), a periodic box has one per step."""
    kn, kw = WL.solver_kwargs(dict(WL.C1, bc=bc))
    a = ugks.Solver(kn, **kw)
    try:
        a.kernel_timing(True)
        a.step(5)
        t = a.kernel_timing()
        launched = [k for k in ugks.KERNELS if not (k == "ghost" and bc == 1)]
        assert all(t[k][1] == 5 and t[k][0] > 0 for k in launched)
        if bc == 1:
            assert t["ghost"][1] == 0
    finally:
        a.close()


def test_moving_maxwellian_fixed_point_on_gpu():
    case = _case(nx=10, ny=10, lx=1.0, ly=1.0, nu=40, nv=40, umax=6.0, vmax=6.0, kn=0.05, bc=0,
                 noise=0.0)
    kn, kw = WL.solver_kwargs(case)
    a = ugks.Solver(kn, **kw)
    try:
        f, W = a.state()
        uk, _ = O.nodes(40, 6.0)
        uu, vv = np.meshgrid(uk, uk, indexing="ij")
        rho, U, V, T = 1.05, 0.2, -0.1, 0.95
        g = rho / (math.pi * T) * np.exp(-((uu - U) ** 2 + (vv - V) ** 2) / T)
        f[...] = g.ravel()
        W[...] = (rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V) + rho * T / 2)
        a.set_state(f, W)
        a.step(10)
        f1, W1 = a.state()
        assert np.array_equal(W1, W)
        assert np.max(np.abs(f1 - f)) < 1e-14 * np.max(f)
    finally:
        a.close()


@pytest.mark.parametrize("nvel", [29, 49])
def test_paper_mesh_m1(nvel):
    """The paper's channel on its mesh M1 (40x20, L/W = 2, Kn 0.1, p_in/p_out 1.5) at its
    29^2 and 49^2 velocity grids (odd counts: u = 0 and v = 0 are nodes)."""
    PR.run_and_compare(WL.paper_mesh(40, 20, nvel), 20, label=f"paper M1 {nvel}^2")


def test_velocity_grid_at_the_limit():
    """nu = nv = 1024, the documented maximum: 512 v nodes per half for the Gauss
    recurrences, 16 velocity chunks and an 8 KB v-node table in the update kernel's LDS."""
    case = _case(nx=3, ny=2, lx=1.5, ly=1.0, nu=1024, nv=1024, umax=12.0, vmax=12.0, kn=0.1,
                 bc=1, noise=0.02, seed=17)
    PR.run_and_compare(case, 2, label="1024x1024 velocities")


def _tiny_grid(nu, nv):
    return _case(nx=5, ny=4, lx=1.0, ly=0.8, nu=nu, nv=nv, umax=2.0, vmax=2.0, kn=0.2, bc=0,
                 noise=0.05, seed=31)


@pytest.mark.parametrize("nu,nv", [(2, 3), (3, 2)])
def test_two_node_velocity_axes(nu, nv):
    """The smallest velocity axes: one node per half (with three nodes the zero node is
    shared by the two halves of the moment sums)."""
    PR.run_and_compare(_tiny_grid(nu, nv), 10, label=f"periodic {nu}x{nv} velocities")


def test_two_by_two_velocity_grid_within_its_conditioning():
    """With u, v in {-2, 2} every velocity has |c|^2 = 8, far from the Maxwellian the cells
    hold, and the step amplifies a one-rounding change of f about 3e5-fold: no rounding
    order reaches 1e-12 here.  The bar is ten times the oracle's own spread under such a
    change (measured in the test, about 5e-11 after 3 steps)."""
    case = _tiny_grid(2, 2)
    s = PR.oracle_sensitivity(case, 3)
    assert s > PR.FP64_TOL  # the case really is that sensitive
    PR.run_and_compare(case, 3, tol=10 * s, label="periodic 2x2 velocities")


def test_largest_velocity_grid():
    """291 x 291 velocities on a 3 x 2 channel: long Gauss recurrences along v (146 nodes per
    half) and a single row segment per row."""
    case = _case(nx=3, ny=2, lx=1.5, ly=1.0, nu=291, nv=291, umax=12.0, vmax=12.0, kn=0.1,
                 bc=1, noise=0.02, seed=17)
    PR.run_and_compare(case, 3, label="291x291 velocities")


@pytest.mark.parametrize("V,flagged", [(20.0, False), (30.0, True)])
def test_transverse_speed_ratio_limit(V, flagged):
    """The v-direction Gaussians start at the innermost node of each half of v.  A Maxwellian
    centred so far out that its start value underflows (speed ratio |V| lambda^(1/2) = 30 here)
    is reported as an invalid state instead of being updated wrongly; ratio 20 is inside the
    range and runs normally."""
    case = _case(nx=4, ny=4, lx=1.0, ly=1.0, nu=16, nv=16, umax=40.0, vmax=40.0, kn=0.1, bc=0,
                 noise=0.0)
    kn, kw = WL.solver_kwargs(case)
    a = ugks.Solver(kn, **kw)
    try:
        f, W = a.state()
        W[..., 1] = 0.0
        W[..., 2] = V * W[..., 0]
        W[..., 3] = 0.5 * W[..., 0] * V * V + 0.5 * W[..., 0]  # T = 1
        a.set_state(f, W)
        a.step(1)
        if flagged:
            with pytest.raises(ugks.UgksError) as ex:
                a.moments()
            assert ex.value.code == ugks.UGKS_E_STATE
        else:
            m = a.moments()
            assert np.all(np.isfinite(m))
    finally:
        a.close()


def test_zero_steps_change_nothing():
    """ugks_step(h, 0) and a zero-step batch enqueue no work: the state stays bitwise."""
    kn, kw = WL.solver_kwargs(WL.C1)
    a = ugks.Solver(kn, **kw)
    b = ugks.Batch(1)
    try:
        a.step(3)
        f0, W0 = a.state()
        a.step(0)
        b.step([a], 0)
        f1, W1 = a.state()
        assert np.array_equal(f0, f1) and np.array_equal(W0, W1)
        assert a.info.steps == 3
    finally:
        b.close()
        a.close()


def test_paper_length_run_stays_valid_and_settles():
    """10,000 steps (the length of the paper's runs) of the parity channel: the state stays
    valid and the flow settles (the step-to-step change of W decays)."""
    kn, kw = WL.solver_kwargs(WL.C1)
    s = ugks.Solver(kn, **kw)
    try:
        changes = []
        for _ in range(5):
            s.step(1999)
            _, Wa = s.state()
            s.step(1)
            _, Wb = s.state()
            changes.append(float(np.max(np.abs(Wb - Wa))))
        m = s.moments()                        # raises on an invalid state
        assert s.info.steps == 10000
    finally:
        s.close()
    print("[long run] max |W^{n+1} - W^n| every 2000 steps", changes, flush=True)
    assert np.all(np.isfinite(m)) and m[..., 0].min() > 0 and m[..., 3].min() > 0
    assert changes[-1] < 0.1 * changes[0]
    assert np.max(m[..., 1]) > 1e-3            # a pressure-driven flow remains


def test_periodic_box_conserves_over_10000_steps():
    case = _case(nx=24, ny=16, lx=1.5, ly=1.0, nu=16, nv=16, umax=5.0, vmax=5.0, kn=0.05, bc=0,
                 noise=0.05, seed=9)
    kn, kw = WL.solver_kwargs(case)
    s = ugks.Solver(kn, **kw)
    try:
        _, W0 = s.state()
        s.step(10000)
        _, W = s.state()
    finally:
        s.close()
    tot0, tot = W0.sum(axis=(0, 1)), W.sum(axis=(0, 1))
    scale = np.array([tot0[0], tot0[0], tot0[0], tot0[3]])
    print("[long run] periodic conservation", (tot - tot0) / scale, flush=True)
    assert np.all(np.abs(tot - tot0) <= 1e-12 * scale)


def test_c1_parity_holds_over_2000_steps():
    """Rounding differences do not accumulate: after 2,000 steps (the flow near its steady
    state) the GPU still matches the oracle within the FP64 bar."""
    PR.run_and_compare(WL.C1, 2000, label="C1 2000 steps")


def test_hot_inlet_and_hot_walls():
    """Inlet ghost at T_in = 1.2 and diffuse walls at T_wall = 1.3 for the gas without internal
    degrees of freedom: the ghost density 2 p_in / T_in, the ghost and wall Maxwellians at their
    own temperatures."""
    PR.run_and_compare(dict(WL.C1, T_in=1.2, T_wall=1.3), 50, label="C1 T_in 1.2 T_wall 1.3")


@pytest.mark.parametrize("nvel", [29, 69])
def test_paper_mesh_m4(nvel):
    """The paper's largest mesh M4 (160x80) at its smallest and largest velocity grids
    (Table 1), compared in full after a few steps."""
    PR.run_and_compare(WL.paper_mesh(160, 80, nvel), 3, label=f"paper M4 {nvel}^2")


def test_paper_mesh_m3_69():
    """M3 (120x60) at 69^2, the largest grid the paper ran on its smaller GPU."""
    PR.run_and_compare(WL.paper_mesh(120, 60, 69), 5, label="paper M3 69^2")


def test_fp32_store_c4_after_1000_steps_against_fp64():
    """The precision workload's accuracy statement: after its 1,000 steps the FP32-store form
    is within 1e-5 of the FP64 form (rho, T relative; U, V absolute), both from the same seeded
    state; the FP64 form matches the oracle within 1e-12 in the tests above."""
    steps = WL.C4_STEPS
    m = {}
    for prec in ("fp64", "fp32_store"):
        kn, kw = WL.solver_kwargs(WL.C4, prec)
        s = ugks.Solver(kn, **kw)
        try:
            s.step(steps)
            m[prec] = s.moments()
        finally:
            s.close()
    e = PR.errors(m["fp32_store"], m["fp64"])
    print(f"[parity] C4 FP32-store vs FP64 after {steps} steps: {e}", flush=True)
    PR.assert_within(e, PR.FP32_STORE_TOL, "C4 FP32-store 1000 steps")
    assert max(e.values()) > 1e-12
