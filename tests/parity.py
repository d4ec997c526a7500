"""Shared helpers for GPU-vs-oracle parity tests: run both sides on the same seeded case and
compare with the metrics of the stated tolerance (relative for rho and T, absolute for U and
V in units of sqrt(2kT0/m), per-cell max |df| / max f for the distribution)."""
import os

import numpy as np

from oracle import oracle as O
from paper_1810_08137_amd import ugks
from paper_1810_08137_amd import workloads as WL

FP64_TOL = 1e-12       # GPU FP64 against the FP64 oracle
FP32_STORE_TOL = 1e-5  # GPU FP32-store against the FP64 oracle


def oracle_threads():
    n = min(16, os.cpu_count() or 1)
    O.set_threads(n)
    return n


def moments_of_W(W, dof=0):
    """(rho, U, V, T): rho E = rho |U|^2/2 + (2 + dof) rho T/4."""
    rho = W[..., 0]
    U = W[..., 1] / rho
    V = W[..., 2] / rho
    T = 4.0 * (W[..., 3] - 0.5 * rho * (U * U + V * V)) / ((2 + dof) * rho)
    return np.stack([rho, U, V, T], -1)


def errors(m_gpu, m_ref, f_gpu=None, f_ref=None, nv=None):
    """With internal degrees of freedom (f holding G then H, nv values each) the two
    distributions are measured separately, H as "h"."""
    if f_gpu is not None and nv is not None and f_ref.shape[-1] == 2 * nv:
        e = errors(m_gpu, m_ref, f_gpu[..., :nv], f_ref[..., :nv])
        e["h"] = errors(m_gpu, m_ref, f_gpu[..., nv:], f_ref[..., nv:])["f"]
        return e
    e = {
        "rho": float(np.max(np.abs(m_gpu[..., 0] - m_ref[..., 0]) / np.abs(m_ref[..., 0]))),
        "U": float(np.max(np.abs(m_gpu[..., 1] - m_ref[..., 1]))),
        "V": float(np.max(np.abs(m_gpu[..., 2] - m_ref[..., 2]))),
        "T": float(np.max(np.abs(m_gpu[..., 3] - m_ref[..., 3]) / np.abs(m_ref[..., 3]))),
    }
    if f_gpu is not None:
        scale = np.max(np.abs(f_ref), axis=-1)
        e["f"] = float(np.max(np.max(np.abs(f_gpu - f_ref), axis=-1) / scale))
    return e


def assert_within(e, tol, what=""):
    bad = {k: v for k, v in e.items() if not (v <= tol)}
    assert not bad, f"{what}: errors above {tol}: {bad} (all: {e})"


def make_pair(case, precision="fp64"):
    kn, kw = WL.solver_kwargs(case, precision)
    g = ugks.Solver(kn, **kw)
    o = O.Oracle(**WL.oracle_kwargs(case))
    return g, o


def oracle_sensitivity(case, steps):
    """How far the oracle's own f moves (per-cell max |df| / max f) after `steps` steps when
    its initial f changes by one rounding: the accuracy any other rounding order can reach."""
    oracle_threads()
    a = O.Oracle(**WL.oracle_kwargs(case))
    b = O.Oracle(**WL.oracle_kwargs(case))
    f, W = b.state()
    sign = np.where(np.sin(np.arange(f.size)) >= 0.0, 1.0, -1.0).reshape(f.shape)
    b.set_state(f * (1.0 + 2.0 ** -53 * sign), W)
    assert a.step(steps) == 0 and b.step(steps) == 0
    fa, _ = a.state()
    fb, _ = b.state()
    return float(np.max(np.max(np.abs(fa - fb), axis=-1) / np.max(np.abs(fa), axis=-1)))


def run_and_compare(case, steps, precision="fp64", tol=FP64_TOL, check_f=True, label=""):
    oracle_threads()
    g, o = make_pair(case, precision)
    try:
        assert abs(g.dt - o.dt) <= 1e-15 * o.dt
        g.step(steps)
        m_gpu = g.moments()
        f_gpu, W_gpu = g.state() if check_f else (None, None)
        assert o.step(steps) == 0
        f_ref, W_ref = o.state()
        e = errors(m_gpu, moments_of_W(W_ref, case.get("dof", 0)), f_gpu,
                   f_ref if check_f else None, nv=case["nu"] * case["nv"])
        print(f"[parity] {label} steps={steps} {precision}: {e}", flush=True)
        assert_within(e, tol, label)
        return e
    finally:
        g.close()
        o.close()
