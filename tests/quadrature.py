"""Independent quadrature used to pin the oracle (no oracle code is used here).

Gauss-Legendre panels integrate polynomial-times-Gaussian integrands over a line or a half
line to near machine precision, so moments and fluxes of a Maxwellian can be checked by brute
force rather than by re-deriving the oracle's recurrences.
"""
import numpy as np


def legendre_panels(a, b, panels=20, order=20):
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(a, b, panels + 1)
    xs, ws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        xs.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w)
    return np.concatenate(xs), np.concatenate(ws)


def line(center, lam, half=None, width=14.0, **kw):
    """Nodes and weights covering a Gaussian exp(-lam (x - center)^2) on the whole line
    (half=None), on x > 0 (half='pos') or on x < 0 (half='neg')."""
    s = width / np.sqrt(lam)
    lo, hi = center - s, center + s
    if half == "pos":
        lo = max(lo, 0.0)
        hi = max(hi, 1e-300)
    elif half == "neg":
        hi = min(hi, 0.0)
        lo = min(lo, -1e-300)
    if hi <= lo:
        return np.zeros(1), np.zeros(1)
    return legendre_panels(lo, hi, **kw)


def maxwellian_2d(prim, u, v):
    rho, U, V, lam = prim
    return rho * lam / np.pi * np.exp(-lam * ((u - U) ** 2 + (v - V) ** 2))
