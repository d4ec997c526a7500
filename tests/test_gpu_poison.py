"""Every value a step reads was written by the step before it: with UGKS_DEBUG_POISON=1 the
library starts the buffers the first step writes as NaN in every cell (and, in a channel, in
the ghost columns, which the update kernel writes for the next step), so a value a step failed
to write would surface as a NaN in the state, and the poisoned solver would differ from a
plain one.  Cases cover the update kernel's row pairs (odd row counts, one row), velocity
chunks, both storage precisions, internal degrees of freedom, the Shakhov model and periodic
boxes."""
import numpy as np
import pytest

from paper_1810_08137_amd import ugks
from paper_1810_08137_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _case(**kw):
    c = dict(WL.CHANNEL_DEFAULTS)
    c.update(kw)
    return c


CASES = {
    "channel 40x10 fp64": (WL.C1, "fp64"),
    "channel 40x10 fp32": (WL.C1, "fp32_store"),
    "channel 23x7 (odd rows), 17x13 velocities": (
        _case(nx=23, ny=7, lx=2.3, ly=1.0, nu=17, nv=13, umax=5.0, vmax=5.0, kn=0.2, seed=61),
        "fp64"),
    "channel one row": (_case(nx=31, ny=1, lx=3.0, ly=0.1, nu=12, nv=12, umax=5.0, vmax=5.0,
                              kn=0.3, seed=62), "fp32_store"),
    "paper mesh 40x20 at 29^2 (velocity chunks)": (WL.paper_mesh(40, 20, 29), "fp64"),
    "internal dof": (WL.C1_DOF, "fp64"),
    "shakhov": (WL.C1_SHAKHOV, "fp32_store"),
    "channel 61x5 (outlet column on a segment's halo)": (
        _case(nx=61, ny=5, lx=6.1, ly=0.5, nu=10, nv=8, umax=4.0, vmax=4.0, kn=0.1, seed=64),
        "fp64"),
    "periodic 19x9": (_case(nx=19, ny=9, lx=1.9, ly=1.0, nu=14, nv=14, umax=5.0, vmax=5.0,
                            kn=0.05, bc=0, seed=63), "fp64"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_steps_write_every_value_they_later_read(name, monkeypatch):
    case, precision = CASES[name]
    kn, kw = WL.solver_kwargs(case, precision)
    monkeypatch.setenv("UGKS_DEBUG_POISON", "1")
    a = ugks.Solver(kn, **kw)
    monkeypatch.delenv("UGKS_DEBUG_POISON")
    b = ugks.Solver(kn, **kw)
    try:
        for n in (1, 2):
            a.step(1)
            b.step(1)
            fa, Wa = a.state()
            fb, Wb = b.state()
            assert np.isfinite(fa).all() and np.isfinite(Wa).all(), (name, n)
            assert np.array_equal(fa, fb) and np.array_equal(Wa, Wb), (name, n)
    finally:
        a.close()
        b.close()
