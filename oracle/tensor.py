"""Grid, 1-D Gaussian factors and the uncompressed long-range tensor (Sec. 2, eqs. 2.1-2.6).

Grid (Sec. 2, before eq. 2.1; origin at node n/2 as in Sec. 3.2): box [-b, b]^3,
mesh h = 2b/n, nodes X_j = -b + (j+1) h for j = 0..n-1 (the paper's i = 1..n).

Long-range collective potential of the protein (eq. 2.6, Algorithm TEP steps 2-3):

    T0[i1,i2,i3] = sum_m sum_{k in long} z_m w_k prod_d exp(-t_k^2 (X_{i_d} - x_{m,d})^2),

a canonical tensor of rank N*K_long.  The build collocates the Gaussians at the
true (off-grid) atom positions instead of shifting a reference tensor onto
grid-snapped atoms (eq. 2.5); this is a reading recorded in the design notes.
"""
from __future__ import annotations

import numpy as np


def grid(n: int, b: float):
    """(h, X0, inv_h, nodes) for the n-point grid on [-b, b]; nodes X_j = -b + (j+1) h."""
    h = (2.0 * b) / n
    X0 = -b + h
    inv_h = 1.0 / h
    nodes = -b + (np.arange(n, dtype=np.float64) + 1.0) * h
    return h, X0, inv_h, nodes


def factor_columns(coord: np.ndarray, t_long: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """1-D Gaussian factors of one mode: G[j, m, k] = exp(-t_k^2 (X_j - x_m)^2).

    coord: (N,) atom coordinates along the mode.  Returns (n, N, K) float64.
    """
    diff = nodes[:, None] - coord[None, :]
    return np.exp(-(t_long * t_long)[None, None, :] * (diff * diff)[:, :, None])


def galerkin_columns(coord: np.ndarray, t_long: np.ndarray, nodes: np.ndarray, h: float) -> np.ndarray:
    """1-D Galerkin factors of eq. 2.1 (projection onto piecewise-constant basis functions),
    normalised as cell averages so that they approximate the same potential values as the
    collocated factors: G[j, m, k] = (1/h) int_{X_j - h/2}^{X_j + h/2} exp(-t_k^2 (x - x_m)^2) dx
      = sqrt(pi) / (2 t_k h) * (erf(t_k (X_j + h/2 - x_m)) - erf(t_k (X_j - h/2 - x_m))),
    and 1 for t_k = 0.  Where both arguments share a sign the difference is taken of erfc
    values, which keeps the digits of the tails.  Returns (n, N, K) float64."""
    from scipy.special import erf, erfc
    diff = (nodes[:, None] - coord[None, :])[:, :, None]                 # X_j - x_m
    t = np.asarray(t_long, dtype=np.float64)[None, None, :]
    u1 = t * (diff - 0.5 * h)
    u2 = t * (diff + 0.5 * h)
    d = np.where(u1 >= 0.0, erfc(u1) - erfc(u2), np.where(u2 <= 0.0, erfc(-u2) - erfc(-u1), erf(u2) - erf(u1)))
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.sqrt(np.pi) / (2.0 * t * h) * d
    return np.where(t > 0.0, g, 1.0)


def long_range_at_nodes(charges, positions, t_long, w_long, n, b, idx):
    """Uncompressed long-range tensor T0 at grid multi-indices idx (Q, 3) (eq. 2.6).

    Evaluated term by term from the separable factors, looping over atoms.
    """
    _, _, _, nodes = grid(n, b)
    idx = np.asarray(idx)
    out = np.zeros(idx.shape[0])
    X = nodes[idx]  # (Q, 3)
    t2 = t_long * t_long
    for m in range(positions.shape[0]):
        d = X - positions[m][None, :]                            # (Q, 3)
        g = np.exp(-t2[None, :, None] * (d * d)[:, None, :])     # (Q, K, 3)
        out += charges[m] * np.sum(w_long[None, :] * g[:, :, 0] * g[:, :, 1] * g[:, :, 2], axis=1)
    return out


def long_range_continuous(charges, positions, t_long, w_long, y):
    """Long-range potential sum_m z_m sum_{k long} w_k exp(-t_k^2 |y - x_m|^2) at points y (Q, 3)."""
    y = np.atleast_2d(y)
    out = np.zeros(y.shape[0])
    t2 = t_long * t_long
    for m in range(positions.shape[0]):
        d = y - positions[m][None, :]
        r2 = np.sum(d * d, axis=1)
        out += charges[m] * np.sum(w_long[None, :] * np.exp(-np.outer(r2, t2)), axis=1)
    return out


def materialize_canonical(F1, F2, F3) -> np.ndarray:
    """Full n^3 array of the canonical tensor sum_p F1[:,p] x F2[:,p] x F3[:,p] (small n only)."""
    return np.einsum("ip,jp,kp->ijk", F1, F2, F3, optimize=True)
