"""Grid, 1-D Gaussian factors and the uncompressed long-range tensor (Sec. 2, eqs. 2.1-2.6).

Grid (Sec. 2, before eq. 2.1; origin at node n/2 as in Sec. 3.2): box [-b, b]^3,
mesh h = 2b/n, nodes X_j = -b + (j+1) h for j = 0..n-1 (the paper's i = 1..n).

Long-range collective potential of the protein (eq. 2.6, Algorithm TEP steps 2-3):

    T0[i1,i2,i3] = sum_m sum_{k in long} z_m w_k prod_d exp(-t_k^2 (X_{i_d} - x_{m,d})^2),

a canonical tensor of rank N*K_long.  The default build collocates the Gaussians at
the true (off-grid) atom positions; the paper's own construction -- a reference tensor
on a twice larger grid shifted onto each charge moved to its nearest node and windowed
onto the grid (eq. 2.5) -- is `shifted_columns`, the snapped variant.
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


def snap_to_nodes(coord: np.ndarray, n: int, b: float) -> np.ndarray:
    """Index of the grid node nearest to each coordinate, the grid point a charge is moved to
    before the reference tensor is shifted onto it (eq. 2.5): j = floor((x - X0)/h + 1/2),
    clipped to [0, n-1] (a coordinate half-way between two nodes goes to the upper one)."""
    _, X0, inv_h, _ = grid(n, b)
    j = np.floor((np.asarray(coord, dtype=np.float64) - X0) * inv_h + 0.5)
    return np.clip(j, 0, n - 1).astype(np.int64)


def snapped_positions(positions: np.ndarray, n: int, b: float) -> np.ndarray:
    """The atoms moved to their nearest grid nodes (every coordinate a node X_j)."""
    _, _, _, nodes = grid(n, b)
    return nodes[snap_to_nodes(positions, n, b)]


def reference_vectors(t_long: np.ndarray, n: int, h: float, galerkin: bool = False) -> np.ndarray:
    """1-D factors of the reference tensor on the twice larger grid (the single-charge kernel of
    eq. 2.5, long-range terms): for term k, the Gaussian exp(-t_k^2 (o h)^2) at offsets o = -n..n-1
    from the node that holds the charge (row o + n), or its cell average (eq. 2.1, normalised as in
    `galerkin_columns`).  Returns (2n, K)."""
    offsets = (np.arange(2 * n, dtype=np.float64) - n) * h
    t_long = np.asarray(t_long, dtype=np.float64)
    if galerkin:
        return galerkin_columns(np.zeros(1), t_long, offsets, h)[:, 0, :]
    return np.exp(-(t_long * t_long)[None, :] * (offsets * offsets)[:, None])


def shifted_columns(coord: np.ndarray, t_long: np.ndarray, n: int, b: float, galerkin: bool = False) -> np.ndarray:
    """Shift-and-window transform of the reference vectors (eq. 2.5): the charge m moves to its
    nearest node j_m, the reference's centre is shifted there and the result is restricted to the
    n grid nodes, G[i, m, k] = ref[i - j_m + n, k].  Returns (n, N, K)."""
    h = (2.0 * b) / n
    ref = reference_vectors(t_long, n, h, galerkin)
    j = snap_to_nodes(coord, n, b)
    rows = np.arange(n)[:, None] - j[None, :] + n          # (n, N), always in [1, 2n - 1]
    return ref[rows]


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
