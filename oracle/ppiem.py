"""The posing search of Algorithm PPIEM (Sec. 3.5, steps A0-A7): energies of the ligand at
first contact along every orbit direction and in every orientation, and the minima.

Test infrastructure, like every module of this package: a plain FP64 statement of what the
device computes, used only to check it.

Steps, in the paper's order (A1, the tensor, is the build; A0's angle grids are inputs):
  A2  the geometric centres: x_P of the protein and the ligand centre used by the pose
      transform (both unweighted means of the atom positions).
  A3  radial approach.  The ligand, rotated by q about its centre, has its centre on the ray
      x_P + rho u (u a unit orbit direction).  Moving in from far away, it first touches the
      van der Waals distance at the largest rho where some pair (ligand atom l, protein atom
      m) is exactly sigma apart.  With a_l = x_P + R(q) u_l and w = a_l - x_m the pair distance
      is |rho u + w|, and |rho u + w|^2 = sigma^2 has the roots
          rho = -(u . w) +- sqrt((u . w)^2 - (|w|^2 - sigma^2));
      between its roots the pair is closer than sigma, outside farther.  So the first contact
      is rho* = the largest root over all pairs, and every rho > rho* is admissible; a ray
      whose pairs have no real root never comes within sigma (rho* = -inf).  The pose is put
      at rho* + gap (gap > 0 keeps it strictly admissible; the energy is scored there).
  A4/A5  the energy of every (orbit position, orientation) pose at its contact radius,
      scored like any pose (flags included).
  A6  minima: for each orbit position the lowest energy over the orientations whose pose is
      accepted (the minimum of A4's array, lowest index on ties); orbit positions whose value
      is not larger than any neighbour's (on the orbit grid's neighbour graph) are the minima.
  A7  the poses of those minima (orientation, translation), sorted by energy.
"""
from __future__ import annotations

import numpy as np

from . import score as _score


def geometric_centre(positions) -> np.ndarray:
    """Unweighted mean, summed in index order and divided by the count (as the ligand centre)."""
    return _score.ligand_frame(positions)[0]


def contact_radius(lig_positions, quats, dirs, centre, atoms, sigma):
    """rho*[u, q] of step A3 for every orbit direction u and orientation q (brute force over
    all protein-ligand pairs)."""
    _, ul = _score.ligand_frame(lig_positions)
    R = _score.rotation_matrix(np.asarray(quats, dtype=np.float64))
    v = _score.rotate(R, ul)                               # (Q, L, 3): R(q) u_l
    atoms = np.asarray(atoms, dtype=np.float64)
    dirs = np.asarray(dirs, dtype=np.float64)
    c = np.asarray(centre, dtype=np.float64)
    rho = np.full((dirs.shape[0], v.shape[0]), -np.inf)
    s2 = float(sigma) * float(sigma)
    for q in range(v.shape[0]):
        a = c[None, :] + v[q]                              # (L, 3)
        w = a[:, None, :] - atoms[None, :, :]              # (L, N, 3)
        ww = np.sum(w * w, axis=2) - s2                    # |w|^2 - sigma^2
        for i, u in enumerate(dirs):
            bu = w @ u                                     # u . w
            disc = bu * bu - ww
            ok = disc >= 0.0
            if np.any(ok):
                rho[i, q] = np.max(-bu[ok] + np.sqrt(disc[ok]))
    return rho


def contact_poses(quats, dirs, centre, rho, gap):
    """Quaternions and translations (U*Q poses, orbit-major) at rho* + gap; rays that never
    meet the protein get a NaN translation (an invalid pose)."""
    dirs = np.asarray(dirs, dtype=np.float64)
    quats = np.asarray(quats, dtype=np.float64)
    U, Q = rho.shape
    r = np.where(np.isfinite(rho), rho + gap, np.nan)
    t = np.asarray(centre)[None, None, :] + r[:, :, None] * dirs[:, None, :]
    return np.broadcast_to(quats[None], (U, Q, 4)).reshape(-1, 4).copy(), t.reshape(-1, 3)


def orbit_minima(E, flags, U, Q, nbr_off, nbr_idx):
    """Step A6.  Returns (best_rotation[U] (-1 if no accepted pose), best_energy[U] (+inf then),
    is_minimum[U])."""
    E = np.asarray(E).reshape(U, Q)
    acc = (np.asarray(flags).reshape(U, Q) & _score.FLAG_ACCEPT) != 0
    best = np.full(U, -1, dtype=np.int64)
    bestE = np.full(U, np.inf)
    for i in range(U):
        for q in range(Q):
            if acc[i, q] and E[i, q] < bestE[i]:
                bestE[i] = E[i, q]
                best[i] = q
    is_min = np.zeros(U, dtype=bool)
    for i in range(U):
        if best[i] < 0:
            continue
        is_min[i] = all(bestE[i] <= bestE[j] for j in nbr_idx[nbr_off[i]:nbr_off[i + 1]])
    return best, bestE, is_min


def ppiem(F, n, b, atoms, z, t_short, w_short, r_cut, lig_charges, lig_positions, dirs, quats, sigma, gap,
          nbr_off, nbr_idx, grid_spec=None):
    """Steps A2-A7 with the oracle's scorer.  Returns a dict with rho, the scored poses, their
    results, the per-orbit minima and the sorted list of (energy, orbit, rotation)."""
    xP = geometric_centre(atoms)
    rho = contact_radius(lig_positions, quats, dirs, xP, atoms, sigma)
    qs, ts = contact_poses(quats, dirs, xP, rho, gap)
    res = _score.score(F, n, b, atoms, z, t_short, w_short, r_cut, lig_charges, lig_positions, qs, ts, sigma,
                       grid_spec=grid_spec)
    U, Q = rho.shape
    best, bestE, is_min = orbit_minima(res["E"], res["flags"], U, Q, nbr_off, nbr_idx)
    minima = sorted((bestE[i], i, int(best[i])) for i in range(U) if is_min[i])
    return dict(centre=xP, rho=rho, quats=qs, trans=ts, result=res, best=best, best_energy=bestE,
                is_minimum=is_min, minima=minima)
