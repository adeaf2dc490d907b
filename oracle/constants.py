"""Derivation of the quadrature step h_M and of the short-range cutoff r_c.

The paper cites the sinc quadrature without fixing its step (Sec. 2, eq. 2.2) and
bounds the short-range support only by the van der Waals distance (Prop. 3.2).
Readings used here:
  * L_s = 2 sqrt(3) b (the box diagonal), and h_M is the step that minimises the
    largest relative error |r g(r) - 1| on r in geomspace(1 A, L_s, 4000),
    rounded to 4 significant digits;
  * r_c is the smallest radius beyond which the short-range Gaussians are below
    1e-16/r, i.e. the last crossing of r * g_short(r) = 1e-16.
Running this module prints the values frozen in ``workloads.configs``.
"""
from __future__ import annotations

import math

import numpy as np

from . import sinc as _sinc


def scale_length(b: float) -> float:
    return 2.0 * math.sqrt(3.0) * b


def optimal_step(M: int, b: float, lo: float = 0.05, hi: float = 0.6) -> float:
    """h_M minimising the radial-sweep error, rounded to 4 significant digits."""
    L_s = scale_length(b)
    hs = np.linspace(lo, hi, 1101)
    errs = [_sinc.max_rel_error(M, h, L_s, 1.0, L_s) for h in hs]
    j = int(np.argmin(errs))
    a, c = hs[max(j - 1, 0)], hs[min(j + 1, len(hs) - 1)]
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(60):
        x1 = c - g * (c - a)
        x2 = a + g * (c - a)
        if _sinc.max_rel_error(M, x1, L_s, 1.0, L_s) < _sinc.max_rel_error(M, x2, L_s, 1.0, L_s):
            c = x2
        else:
            a = x1
    return float(f"{0.5 * (a + c):.4g}")


def short_cutoff(M: int, h_M: float, L_s: float, K_long: int, tol: float = 1e-16) -> float:
    """Last radius where r * sum_{k >= K_long} w_k exp(-t_k^2 r^2) crosses tol."""
    t, w = _sinc.sinc_table(M, h_M, L_s)
    ts, ws = t[K_long:], w[K_long:]
    if ts.size == 0:
        return 0.0

    def f(r):
        return r * float(np.sum(ws * np.exp(-(ts * ts) * r * r))) - tol

    rs = np.geomspace(1e-3, 4.0 * L_s, 20000)
    vals = np.array([f(r) for r in rs])
    pos = np.nonzero(vals > 0.0)[0]
    if pos.size == 0:
        return 0.0
    j = pos[-1]
    a, c = rs[j], rs[min(j + 1, rs.size - 1)]
    for _ in range(200):
        mid = 0.5 * (a + c)
        if f(mid) > 0.0:
            a = mid
        else:
            c = mid
    return c


if __name__ == "__main__":  # pragma: no cover - documentation helper
    for (M, b, K) in [(24, 24.0, 12), (32, 52.0, 22), (32, 60.0, 22)]:
        h = optimal_step(M, b)
        L = scale_length(b)
        print(f"M={M} b={b} h_M={h} L_s={L!r} err={_sinc.max_rel_error(M, h, L, 1.0, L):.3e} "
              f"r_c(K_long={K})={short_cutoff(M, h, L, K)!r}")
