"""GPU tests of the serving form: batched multi-instance launches give each solve exactly the
result it gets alone, members may join (from another stream) and leave between batches, one
failing member does not disturb the others, and the request loop runs end to end."""
import ctypes

import numpy as np
import pytest

from paper_1810_08137_amd import serving as SV
from paper_1810_08137_amd import ugks
from paper_1810_08137_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _case(**kw):
    c = dict(WL.CHANNEL_DEFAULTS)
    c.update(kw)
    return c


CASES = [
    _case(nx=20, ny=6, lx=4.0, ly=1.0, nu=24, nv=24, umax=6.0, vmax=6.0, kn=0.07, seed=31),
    _case(nx=13, ny=9, lx=2.0, ly=1.0, nu=17, nv=11, umax=5.0, vmax=5.0, kn=0.3, seed=32,
          p_ratio=1.7),
    _case(nx=9, ny=7, lx=1.0, ly=1.0, nu=12, nv=12, umax=4.0, vmax=4.0, kn=0.02, bc=0,
          seed=33),
    _case(nx=30, ny=8, lx=4.0, ly=1.0, nu=48, nv=48, umax=6.0, vmax=6.0, kn=0.5, seed=34),
]


def _solver(case, precision="fp64", stream=None, velocity_chunks=0):
    kn, kw = WL.solver_kwargs(case, precision)
    return ugks.Solver(kn, stream=stream, velocity_chunks=velocity_chunks, **kw)


@pytest.mark.parametrize("precision", ["fp64", "fp32_store"])
def test_batched_steps_are_bitwise_the_steps_alone(precision):
    import torch

    alone = [_solver(c, precision) for c in CASES]
    for s in alone:
        s.step(24)
    run = torch.cuda.Stream()
    side = torch.cuda.Stream()
    batch = ugks.Batch(8, stream=run)
    mixed = [_solver(c, precision, stream=run) for c in CASES[:2]]
    try:
        batch.step(mixed, 6)
        mixed.append(_solver(CASES[2], precision, stream=side))   # joins from another stream
        batch.step(mixed, 5)
        mixed.append(_solver(CASES[3], precision, stream=side))
        batch.step(mixed, 13)                 # members 0, 1 reach 24 steps
        batch.step(mixed[2:], 24 - 18)        # member 2: 5 + 13 + 6
        mixed[3].step(24 - 19)                # member 3 finishes alone, on the batch stream
        for a, m in zip(alone, mixed):
            fa, Wa = a.state()
            fm, Wm = m.state()
            assert np.array_equal(fa, fm) and np.array_equal(Wa, Wm)
            assert a.info.steps == m.info.steps == 24
    finally:
        for s in alone + mixed:
            s.close()
        batch.close()


def test_batch_rejects_invalid_member_lists():
    import torch

    run = torch.cuda.Stream()
    a = _solver(CASES[0], "fp64", stream=run)
    b = _solver(CASES[1], "fp32_store", stream=run)
    batch = ugks.Batch(2, stream=run)
    try:
        for members in ([a, a], [a, b], [a, a, a]):
            with pytest.raises(ugks.UgksError) as ex:
                batch.step(members, 1)
            assert ex.value.code == ugks.UGKS_E_INVAL
        arr = (ctypes.c_void_p * 0)()
        assert ugks.lib().ugks_step_batch(batch.b, arr, 0, 1) == ugks.UGKS_E_INVAL
        batch.step([a], 2)
        assert a.info.steps == 2
    finally:
        a.close()
        b.close()
        batch.close()


def test_one_invalid_member_does_not_disturb_the_others():
    import torch

    run = torch.cuda.Stream()
    good = [_solver(c, "fp64", stream=run) for c in (CASES[0], CASES[1])]
    bad = _solver(CASES[3], "fp64", stream=run)
    ref = _solver(CASES[0], "fp64")
    batch = ugks.Batch(4, stream=run)
    try:
        f, W = bad.state()
        W[2, 5, 3] = -1.0
        bad.set_state(f, W)
        batch.step(good + [bad], 10)
        ref.step(10)
        with pytest.raises(ugks.UgksError) as ex:
            bad.moments()
        assert ex.value.code == ugks.UGKS_E_STATE
        m = good[0].moments()
        assert np.array_equal(m, ref.moments())
        good[1].moments()
    finally:
        for s in good + [bad, ref]:
            s.close()
        batch.close()


def test_request_loop_end_to_end():
    reqs = SV.serving_requests(12, rate=400.0, seed=7, steps=20, precision="fp32_store",
                               meshes=[(50, 12), (100, 25)], vgrids=[24, 32])
    ex = SV.GpuExecutor(max_slots=16)
    try:
        srv = SV.Server(ex, budget_bytes=8 << 30, max_slots=16, quantum=7)
        stats = srv.run(reqs)
    finally:
        ex.close()
    print("[serving] small run", stats, "batches", srv.batches, "resident", srv.max_resident,
          flush=True)
    assert stats["done"] == 12
    assert srv.max_resident >= 2
    for r in reqs[:3]:
        # stepped alone with the executor's cap on velocity chunks: the same sum order
        s = _solver(r.case, "fp32_store", velocity_chunks=ex.velocity_chunks)
        try:
            s.step(r.steps)
            assert np.array_equal(s.moments(), r.result)
        finally:
            s.close()


def test_cancelled_request_leaves_and_the_others_end_as_alone():
    """A request cancelled while its batch runs is released after that batch; the requests
    still resident keep stepping and end bitwise as they would alone."""
    reqs = SV.serving_requests(6, rate=float("inf"), seed=13, steps=12, precision="fp32_store",
                               meshes=[(50, 12), (100, 25)], vgrids=[24])
    ex = SV.GpuExecutor(max_slots=8)
    try:
        srv = SV.Server(ex, budget_bytes=8 << 30, max_slots=8, quantum=4)
        step = ex.step

        def step_and_cancel(solvers, n):
            step(solvers, n)
            if srv.batches == 0:
                srv.cancel(reqs[2].rid)

        ex.step = step_and_cancel
        stats = srv.run(reqs)
    finally:
        ex.close()
    print("[serving] cancel run", stats, flush=True)
    assert reqs[2].status == "cancelled" and reqs[2].result is None
    assert stats["done"] == 5 and stats["cancelled"] == 1
    for r in [r for r in reqs if r is not reqs[2]][:2]:
        s = _solver(r.case, "fp32_store", velocity_chunks=ex.velocity_chunks)
        try:
            s.step(r.steps)
            assert np.array_equal(s.moments(), r.result)
        finally:
            s.close()


def test_request_loop_with_mixed_gases_and_collision_models():
    """BGK, Shakhov and internal-degree-of-freedom requests in one request loop: the executor
    steps one batch per collision model and every request ends as it would alone."""
    reqs = SV.serving_requests(9, rate=400.0, seed=11, steps=15, precision="fp32_store",
                               meshes=[(50, 12), (100, 25)], vgrids=[24])
    for k, r in enumerate(reqs):
        if k % 3 == 1:
            r.case["prandtl"] = 2.0 / 3.0
        elif k % 3 == 2:
            r.case["dof"] = 1
    ex = SV.GpuExecutor(max_slots=16)
    try:
        srv = SV.Server(ex, budget_bytes=8 << 30, max_slots=16, quantum=5)
        stats = srv.run(reqs)
        groups = sorted(ex.batches)
    finally:
        ex.close()
    print("[serving] mixed run", stats, "groups", groups, flush=True)
    assert stats["done"] == 9 and len(groups) == 2
    for r in reqs[:3]:
        s = _solver(r.case, "fp32_store", velocity_chunks=ex.velocity_chunks)
        try:
            s.step(r.steps)
            assert np.array_equal(s.moments(), r.result)
        finally:
            s.close()


def test_batch_mixing_chunked_and_unchunked_solvers():
    """A solver capped at one velocity chunk (no chunk-sum workgroups) between chunked ones:
    the chunk-sum launch must still find each chunked member, and every member steps
    bitwise as it does alone with the same cap."""
    import torch

    caps = [0, 1, 0, 2]
    alone = [_solver(c, "fp64", velocity_chunks=k) for c, k in zip(CASES, caps)]
    for s in alone:
        s.step(9)
    run = torch.cuda.Stream()
    batch = ugks.Batch(4, stream=run)
    members = [_solver(c, "fp64", stream=run, velocity_chunks=k) for c, k in zip(CASES, caps)]
    try:
        batch.step(members, 9)
        for a, m in zip(alone, members):
            fa, Wa = a.state()
            fm, Wm = m.state()
            assert np.array_equal(fa, fm) and np.array_equal(Wa, Wm)
    finally:
        for s in alone + members:
            s.close()
        batch.close()
