"""The velocity chunks a solver's launches use, as ugks_info reports them, against the rules
the kernels document (restated here): the moment kernel's chunks fixed at create so that its
workgroups fill the GPU about three times per CU; the update kernel's v-range chunks, fixed at
create, more than one only when its workgroups with every u range split would leave more than
half the GPU idle; and its u-range chunk count U that minimises rounds x (2 + u nodes per
chunk / v chunks) for a solver alone, with FP64 workgroups of two chunks (eight wavefronts)
unless that would leave more than half the CUs without one."""
import math

import pytest

from paper_1810_08137_amd import ugks
from paper_1810_08137_amd import workloads as WL

pytestmark = pytest.mark.gpu

CUS = 256
SEG = 60  # cells per update segment; the moment-chunk rule counts the same segments


def moment_chunks(nx, ny, K, NC, cap=0):
    base = math.ceil(nx / SEG) * ny * NC
    G = max(1, min(3 * CUS // base, K // 2, 16))
    return cap if 0 < cap < G else G


def update_v_chunks(nx, ny, K, M, NC, fp32, shak, cap=0):
    base = math.ceil(nx / SEG) * ((ny + 1) // 2) * NC
    umax = max(1, min(K // 2, 16))
    slots = CUS * ((2 if shak else 4) if fp32 else 2)
    if 2 * base * umax >= slots:
        return 1
    vs = min(slots // (base * umax), (M // 2) // 4)
    if cap > 0:
        vs = min(vs, cap)
    return max(vs, 1)


def _single(base, slots, cap, per_wg, half, vs):
    best, best_cost = 1, None
    for U in range(1, min(cap, 16) + 1):
        rounds = -(-base * U // slots)
        cost = rounds * (2 * vs + -(-half // (per_wg * U)))
        if best_cost is None or cost <= best_cost:
            best, best_cost = U, cost
    return best


def update_chunks(nx, ny, K, M, NC, fp32, shak):
    vs = update_v_chunks(nx, ny, K, M, NC, fp32, shak)
    base = math.ceil(nx / SEG) * ((ny + 1) // 2) * NC * vs
    waves = (2 if shak else 4) if fp32 else 2   # waves per SIMD of the update kernel
    per = 1 if fp32 else 2
    cap = lambda ch: max(1, K // 2 // ch)
    U = _single(base, CUS * waves // per, cap(per), per, K // 2, vs)
    if per == 2 and base * U < CUS // 2:
        per = 1
        U = _single(base, CUS * waves, cap(1), 1, K // 2, vs)
    return U, per, vs


CASES = {"C1": (WL.C1, "fp64"), "C2": (WL.C2, "fp64"), "C2 fp32": (WL.C2, "fp32_store"),
         "C3": (WL.C3, "fp64"), "C2 dof": (WL.C2_DOF, "fp64"),
         "C2 Shakhov fp32": (WL.C2_SHAKHOV, "fp32_store")}
for _nx, _ny in WL.PAPER_MESHES:
    for _nv in WL.PAPER_VGRIDS:
        CASES[f"{_nx}x{_ny} {_nv}^2"] = (WL.paper_mesh(_nx, _ny, _nv), "fp64")


@pytest.mark.parametrize("name", list(CASES))
def test_solver_reports_the_documented_velocity_chunks(name):
    case, precision = CASES[name]
    kn, kw = WL.solver_kwargs(case, precision)
    s = ugks.Solver(kn, **kw)
    try:
        info = s.info
        NC = 2 if case.get("dof", 0) else 1
        shak = 0.0 < case.get("prandtl", 1.0) < 1.0
        K = case["nu"]
        assert info.moment_chunks == moment_chunks(case["nx"], case["ny"], K, NC), name
        U, per, vs = update_chunks(case["nx"], case["ny"], K, case["nv"], NC,
                                   precision == "fp32_store", shak)
        assert (info.update_chunks, info.update_chunks_per_workgroup, info.update_v_chunks) == \
            (U, per, vs), name
    finally:
        s.close()


def test_velocity_chunk_cap_is_kept():
    kn, kw = WL.solver_kwargs(WL.paper_mesh(40, 20, 49), "fp64")
    s = ugks.Solver(kn, velocity_chunks=3, **{k: v for k, v in kw.items() if k != "velocity_chunks"})
    try:
        assert s.info.moment_chunks == 3
        assert s.info.update_v_chunks == 3  # the automatic choice there is 3, within the cap
    finally:
        s.close()
