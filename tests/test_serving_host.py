"""Scheduler of the serving form on the CPU: admission by footprint, FIFO order, exact step
counts, latency bookkeeping and failure isolation, with a fake executor whose solves are the
FP64 oracle (a test double, not a second product path) and a virtual clock."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_08137_amd import serving as SV
from paper_1810_08137_amd import workloads as WL


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class FakeExecutor:
    """Oracle solves; each batched step costs `cost` virtual seconds per million updates."""

    def __init__(self, clock, cost=0.01):
        self.clock = clock
        self.cost = cost
        self.resident = 0
        self.peak = 0
        self.order = []
        self.steps_done = {}

    def footprint(self, req):
        return WL.updates(req.case) * 8 * 2

    def create(self, req):
        if req.case.get("fail_create"):
            raise RuntimeError("cannot start")
        o = O.Oracle(**WL.oracle_kwargs(req.case))
        o.req = req
        self.resident += self.footprint(req)
        self.peak = max(self.peak, self.resident)
        self.order.append(req.rid)
        self.steps_done[req.rid] = 0
        return o

    def step(self, solvers, n):
        for o in solvers:
            assert o.step(n) == 0 or o.req.case.get("poison")
            self.steps_done[o.req.rid] += n
        self.clock.t += self.cost * n * sum(WL.updates(o.req.case) for o in solvers) / 1e6

    def wait(self):
        pass

    def finish(self, o):
        if o.req.case.get("poison"):
            raise RuntimeError("invalid state")
        return o.moments()

    def release(self, o):
        self.resident -= self.footprint(o.req)
        o.close()


def small_requests(n, rate, seed=3, steps=6):
    return SV.serving_requests(n, rate, seed=seed, steps=steps, precision="fp64",
                               meshes=[(6, 3), (8, 4), (10, 5)], vgrids=[6, 8])


def test_all_requests_finish_with_exact_steps_and_latency():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = small_requests(10, rate=50.0)
    srv = SV.Server(ex, budget_bytes=10**9, max_slots=4, quantum=4, clock=clock,
                    sleep=clock.sleep)
    stats = srv.run(reqs)
    assert stats["done"] == 10 and stats["failed"] == 0
    for r in reqs:
        assert ex.steps_done[r.rid] == r.steps
        assert r.admitted >= r.arrival - 1e-12 and r.finished >= r.admitted
        assert r.latency > 0
    assert stats["p99_latency_s"] >= stats["p50_latency_s"] > 0
    assert srv.max_resident <= 4


def test_results_are_those_of_a_solve_alone():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = small_requests(5, rate=float("inf"), steps=7)
    SV.Server(ex, budget_bytes=10**9, max_slots=2, quantum=3, clock=clock,
              sleep=clock.sleep).run(reqs)
    for r in reqs:
        o = O.Oracle(**WL.oracle_kwargs(r.case))
        assert o.step(r.steps) == 0
        np.testing.assert_array_equal(r.result, o.moments())


def test_admission_respects_the_memory_budget_and_fifo_order():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = small_requests(12, rate=100.0)
    budget = 3 * max(ex.footprint(r) for r in reqs)
    SV.Server(ex, budget_bytes=budget, max_slots=64, quantum=2, clock=clock,
              sleep=clock.sleep).run(reqs)
    assert ex.peak <= budget
    assert ex.order == sorted(ex.order, key=lambda rid: (reqs[rid].arrival, rid))
    assert all(r.status == "done" for r in reqs)


def test_request_larger_than_the_budget_is_rejected_others_run():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = small_requests(4, rate=float("inf"))
    big = SV.Request(99, dict(reqs[0].case, nx=40, ny=20), 3, 0.0, "fp64")
    budget = 2 * max(ex.footprint(r) for r in reqs)
    assert ex.footprint(big) > budget
    stats = SV.Server(ex, budget_bytes=budget, max_slots=8, quantum=2, clock=clock,
                      sleep=clock.sleep).run(reqs + [big])
    assert big.status == "rejected"
    assert stats["done"] == 4 and stats["rejected"] == 1


def test_a_failing_request_does_not_take_others_down():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = small_requests(6, rate=float("inf"))
    reqs[2].case = dict(reqs[2].case, poison=True)
    reqs[4].case = dict(reqs[4].case, fail_create=True)
    stats = SV.Server(ex, budget_bytes=10**9, max_slots=8, quantum=3, clock=clock,
                      sleep=clock.sleep).run(reqs)
    assert reqs[2].status == "failed" and reqs[4].status == "failed"
    assert stats["done"] == 4 and stats["failed"] == 2
    assert ex.resident == 0


def test_requests_arriving_during_a_batch_join_the_next_one():
    clock = Clock()
    ex = FakeExecutor(clock, cost=0.5)
    reqs = small_requests(6, rate=20.0, steps=8)
    srv = SV.Server(ex, budget_bytes=10**9, max_slots=8, quantum=2, clock=clock,
                    sleep=clock.sleep)
    srv.run(reqs)
    assert srv.max_resident >= 2          # solves overlapped
    assert all(ex.steps_done[r.rid] == 8 for r in reqs)


def test_request_generator_shape_and_seed():
    a = SV.serving_requests(50, rate=10.0, seed=4)
    b = SV.serving_requests(50, rate=10.0, seed=4)
    assert [r.case for r in a] == [r.case for r in b]
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    for r in a:
        assert (r.case["nx"], r.case["ny"]) in SV.MESHES
        assert r.case["nu"] in SV.VGRIDS and r.case["nu"] == r.case["nv"]
        assert 0.01 <= r.case["kn"] <= 1.0 and 1.5 <= r.case["p_ratio"] <= 3.0
        assert r.steps == 500 and r.precision == "fp32_store"


def test_a_burst_is_created_in_rounds_while_the_first_requests_run():
    """With admit_per_round = 3, a burst of 10 arrivals is created three at a time between
    batches: the first batch runs with three members, later ones with more, every request
    still gets exactly its steps, and admission stays in arrival order."""
    clock = Clock()
    ex = FakeExecutor(clock)
    sizes = []
    step = ex.step

    def counting_step(solvers, n):
        sizes.append(len(solvers))
        step(solvers, n)

    ex.step = counting_step
    reqs = small_requests(10, rate=float("inf"))
    srv = SV.Server(ex, budget_bytes=10**9, max_slots=10, quantum=2, admit_per_round=3,
                    clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs)
    assert stats["done"] == 10
    assert sizes[0] == 3 and max(sizes) > 3
    assert ex.order == sorted(ex.order)
    assert all(ex.steps_done[r.rid] == r.steps for r in reqs)


def test_cancelling_a_running_request_releases_it_after_the_batch_in_flight():
    """A request cancelled while its batch runs leaves when that batch ends: its solver is
    released and its memory returned, it keeps the steps it got, and the others finish."""
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = small_requests(4, rate=float("inf"), steps=9)
    srv = SV.Server(ex, budget_bytes=10**9, max_slots=8, quantum=3, clock=clock,
                    sleep=clock.sleep)
    step = ex.step

    def step_and_cancel(solvers, n):
        step(solvers, n)
        if srv.batches == 0:          # the client cancels request 1 during the first batch
            srv.cancel(reqs[1].rid)

    ex.step = step_and_cancel
    stats = srv.run(reqs)
    assert reqs[1].status == "cancelled" and reqs[1].result is None
    assert ex.steps_done[reqs[1].rid] == 3
    assert all(r.status == "done" and ex.steps_done[r.rid] == 9 for r in reqs if r is not reqs[1])
    assert stats["done"] == 3 and stats["cancelled"] == 1
    assert ex.resident == 0


def test_cancelling_a_queued_request_never_starts_it():
    """With one slot, a request cancelled while it waits in the queue is never created."""
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = small_requests(3, rate=float("inf"), steps=4)
    reqs[2].cancel_at = 0.0
    stats = SV.Server(ex, budget_bytes=10**9, max_slots=1, quantum=2, clock=clock,
                      sleep=clock.sleep).run(reqs)
    assert reqs[2].status == "cancelled" and reqs[2].rid not in ex.order
    assert stats["done"] == 2 and stats["cancelled"] == 1
    assert ex.resident == 0


def test_cancelling_a_resident_request_between_batches():
    """A request cancelled at a time that falls between two batches leaves before the next
    batch: it is not stepped again."""
    clock = Clock()
    ex = FakeExecutor(clock, cost=1.0)
    reqs = small_requests(2, rate=float("inf"), steps=10)
    per_batch = 1.0 * 2 * sum(WL.updates(r.case) for r in reqs) / 1e6   # two steps a batch
    reqs[0].cancel_at = 1.5 * per_batch                               # after the first batch
    stats = SV.Server(ex, budget_bytes=10**9, max_slots=4, quantum=2, clock=clock,
                      sleep=clock.sleep).run(reqs)
    assert reqs[0].status == "cancelled"
    assert ex.steps_done[reqs[0].rid] in (2, 4)   # the batch in flight at cancel_at completes
    assert reqs[1].status == "done" and ex.steps_done[reqs[1].rid] == 10
    assert stats["cancelled"] == 1 and ex.resident == 0
