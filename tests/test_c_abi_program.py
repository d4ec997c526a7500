"""The C ABI used from plain C (tests/c_abi/channel.c: gcc, no HIP headers, no Python): the
program links against the library and, on a GPU, gives bitwise the moments the Python binding
gives for the same case."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

from paper_1810_08137_amd import ugks
from paper_1810_08137_amd import workloads as WL

PROG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "channel")


def _prog():
    if not os.path.exists(PROG):
        raise RuntimeError(f"{PROG} not built: run python __graft_entry__.py")
    return PROG


def test_c_program_links_against_the_library():
    r = subprocess.run([_prog()], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr


@pytest.mark.gpu
def test_c_program_matches_the_python_binding_bitwise():
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "m.bin")
        r = subprocess.run([_prog(), "100", out], capture_output=True, text=True, timeout=120)
        print("[c abi]", r.stdout.strip(), r.stderr.strip(), flush=True)
        assert r.returncode == 0, r.stderr
        m_c = np.fromfile(out, dtype=np.float64).reshape(10, 40, 4)
    kn, kw = WL.solver_kwargs(WL.C1)
    s = ugks.Solver(kn, **kw)
    try:
        s.step(100)
        m_py = s.moments()
    finally:
        s.close()
    assert np.array_equal(m_c, m_py)
