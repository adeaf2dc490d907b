"""The electrostatic energy of one molecule from its own RS tensor (Prop. 3.2, eqs. 3.8-3.9).

Test infrastructure, like every module of this package: a plain FP64 statement of what the
device computes, used only to check it.

The energy E_N = 1/2 sum_j z_j sum_{m != j} z_m / |x_j - x_m| splits with the range-separated
kernel.  Prop. 3.2 evaluates the long-range part from the tensor at the atoms themselves and
removes each atom's own long-range term, which is its charge times the long-range reference
kernel at distance zero, P_{R_l}(0) = sum_{k < K_long} w_k:

    E_long  = 1/2 sum_j z_j (P_l(x_j) - z_j sum_{k < K_long} w_k)

(P_l(x_j) here is the trilinear value of the canonical tensor at x_j, as everywhere else).
The proposition assumes the short-range Gaussians vanish beyond the smallest pair distance;
the short-range pairs are kept separately so that the sum is the whole energy otherwise:

    E_short = 1/2 sum_j z_j sum_{m != j, |x_j - x_m|^2 < r_c^2} z_m sum_{k >= K_long} w_k exp(-t_k^2 |x_j - x_m|^2).
"""
from __future__ import annotations

import numpy as np

from . import score as _score


def self_energy(F, n, b, atoms, z, w_long, t_short, w_short, r_cut):
    """(E_long, E_short) of the molecule whose long-range tensor has factors F."""
    atoms = np.asarray(atoms, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    v, inside, *_ = _score.long_range(F, n, b, atoms)
    if not np.all(inside):
        raise ValueError("every atom must lie on the grid")
    w0 = float(np.sum(w_long))
    E_long = 0.5 * float(np.sum(z * (v - z * w0)))
    D2 = _score.pair_d2(atoms, atoms)
    np.fill_diagonal(D2, np.inf)
    j, m = np.nonzero(D2 < r_cut * r_cut)
    if j.size:
        g = np.exp(-np.outer(D2[j, m], np.asarray(t_short) ** 2)) @ np.asarray(w_short)
        E_short = 0.5 * float(np.sum(z[j] * z[m] * g))
    else:
        E_short = 0.0
    return E_long, E_short


def coulomb(atoms, z) -> float:
    """The direct sum 1/2 sum_{j != m} z_j z_m / |x_j - x_m|."""
    atoms = np.asarray(atoms, dtype=np.float64)
    D = np.sqrt(_score.pair_d2(atoms, atoms))
    np.fill_diagonal(D, np.inf)
    return 0.5 * float(np.sum(np.outer(z, z) / D))
