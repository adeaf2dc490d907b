"""Direct Coulomb binding energy and forces (the plain definitions the RS method approximates).

E(M, L) = sum_l sum_m zeta_l z_m / |y_l - x_m|            (eq. 3.5)
F_l = zeta_l sum_m z_m (y_l - x_m) / |y_l - x_m|^3 = -grad_{y_l} E   (Sec. 3.3, force on a ligand atom)
Rigid-body gradient: dE/dt = -sum_l F_l, dE/domega = -sum_l (y_l - t) x F_l.
Units: Angstrom and elementary charge with Coulomb constant 1 (energies in e^2/A).
"""
from __future__ import annotations

import numpy as np

from . import score as _score


def energies(atoms, z, lig_charges, lig_positions, quats, trans, want_grad: bool = False):
    """Direct E (P,) and optionally the rigid-body gradient (P, 6) for every pose."""
    atoms = np.asarray(atoms, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    zeta = np.asarray(lig_charges, dtype=np.float64)
    _, u = _score.ligand_frame(lig_positions)
    R = _score.rotation_matrix(quats)
    v = _score.rotate(R, u)
    y = v + np.atleast_2d(trans)[:, None, :]
    P, L = y.shape[0], y.shape[1]
    E = np.zeros(P)
    G = np.zeros((P, 6)) if want_grad else None
    for p in range(P):
        diff = y[p][:, None, :] - atoms[None, :, :]          # (L, N, 3)
        r = np.sqrt(np.sum(diff * diff, axis=2))
        E[p] = np.sum(zeta[:, None] * z[None, :] / r)
        if want_grad:
            force = zeta[:, None] * np.sum((z[None, :] / r ** 3)[:, :, None] * diff, axis=1)  # (L, 3)
            G[p, :3] = -force.sum(axis=0)
            G[p, 3:] = -np.cross(v[p], force).sum(axis=0)
    return (E, G) if want_grad else E
