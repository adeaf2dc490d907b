"""Sinc-quadrature Gaussian sum for the Newton kernel 1/r (Sec. 2, eq. 2.2).

1/r = (2/sqrt(pi)) * int_0^inf exp(-r^2 t^2) dt.  With t = sinh(u)/L_s the
integrand becomes even in u, and the trapezoid (sinc) rule with step h_M over
u = k*h_M, k = -M..M gives

    1/r ~ sum_{k=-M}^{M} a_k exp(-t_k^2 r^2),
    t_k = sinh(k h_M) / L_s,   a_k = h_M cosh(k h_M) / (sqrt(pi) L_s).

Terms +k and -k share t_k^2, so they fold into M+1 distinct Gaussians with
weights w_0 = a_0, w_k = 2 a_k (k >= 1).  The paper gives only the form of the
sum (eq. 2.2); the sinh substitution and the folding are this project's
reading.  Terms are ordered widest first (k = 0 is the widest Gaussian), and
the first K_long of them form the long-range part (range separation, eq. 2.4).
"""
from __future__ import annotations

import numpy as np


def sinc_table(M: int, h_M: float, L_s: float) -> tuple[np.ndarray, np.ndarray]:
    """Folded nodes t_k and weights w_k, k = 0..M (eq. 2.2, folded +-k)."""
    k = np.arange(M + 1, dtype=np.float64)
    t = np.sinh(k * h_M) / L_s
    a = h_M * np.cosh(k * h_M) / (np.sqrt(np.pi) * L_s)
    w = a.copy()
    w[1:] = 2.0 * a[1:]
    return t, w


def gaussian_sum(r: np.ndarray, t: np.ndarray, w: np.ndarray) -> np.ndarray:
    """g(r) = sum_k w_k exp(-t_k^2 r^2) over the given terms (eq. 2.2)."""
    r = np.asarray(r, dtype=np.float64)
    return np.sum(w[None, :] * np.exp(-np.outer(r * r, t * t)), axis=1).reshape(r.shape)


def split(t: np.ndarray, w: np.ndarray, K_long: int):
    """Range separation (eq. 2.4): the K_long widest terms are long-range, the rest short-range."""
    return (t[:K_long], w[:K_long]), (t[K_long:], w[K_long:])


def max_rel_error(M: int, h_M: float, L_s: float, r_min: float, r_max: float,
                  samples: int = 4000) -> float:
    """max over r in geomspace(r_min, r_max) of |r g(r) - 1| (radial sweep against 1/r)."""
    t, w = sinc_table(M, h_M, L_s)
    r = np.geomspace(r_min, r_max, samples)
    return float(np.max(np.abs(r * gaussian_sum(r, t, w) - 1.0)))
