"""The long-range tensor restricted to a sub-box and recompressed (Sec. 3.3, schemes (B)/(C)).

Test infrastructure, like every module of this package: a plain FP64 statement of what the
device computes, used only to check it.

The paper observes (Table 3.1) that the long-range potential restricted to a small box Pi
next to the molecule has a much smaller canonical rank R_Pi than on the whole box, and
proposes to compute it once per box and then score every ligand position inside the box
at cost R_Pi * L (scheme (B)), or to obtain it from the global rank-R tensor by rank
reduction (scheme (C), the hybrid).  This module follows scheme (C):

1. Restriction.  For each mode keep the grid rows that trilinear evaluation inside
   [lo_d, hi_d] can touch: i_lo = floor((lo_d - X0) / h) .. i_hi = floor((hi_d - X0) / h) + 1,
   clipped to the grid.  The restricted tensor has the same mesh h, origin
   X0_d = node i_lo (-b + (i_lo + 1) h) and n_d = i_hi - i_lo + 1 rows in mode d; its
   factors are the kept rows of the global ones.  Nothing is approximated here: inside the
   sub-box it evaluates exactly as the global tensor.
2. Rank reduction of the canonical tensor sum_p f1p x f2p x f3p by the same
   canonical -> Tucker -> canonical transform as the build (RHOSVD): unit-norm side
   matrices A_d[:, p] = f_dp / ||f_dp||, weights xi_p = prod_d ||f_dp||, left singular
   vectors with s >= eps * s_1, the Tucker core sum_p xi_p (U1^T a1p) x (U2^T a2p) x (U3^T a3p),
   then slice SVDs kept at eps times the largest over all slices.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import rhosvd as _rhosvd
from . import tensor as _tensor


@dataclass
class Restricted:
    F: list            # three (n_d, R) factor matrices (rows of the global factors)
    X0s: np.ndarray    # (3,) origin of each mode: the first kept node
    inv_h: float
    ns: np.ndarray     # (3,) rows per mode
    rows: list         # per mode (i_lo, i_hi) in the global grid

    @property
    def grid_spec(self):
        return (self.X0s, self.inv_h, self.ns)


def restrict(F, n: int, b: float, lo, hi) -> Restricted:
    """Rows of the global factors that the sub-box [lo, hi] needs (step 1)."""
    h, X0, inv_h, nodes = _tensor.grid(n, b)
    X0s, ns, rows, Fr = np.zeros(3), np.zeros(3, dtype=np.int64), [], []
    for d in range(3):
        i_lo = int(np.floor((lo[d] - X0) * inv_h))
        i_hi = int(np.floor((hi[d] - X0) * inv_h)) + 1
        i_lo = min(max(i_lo, 0), n - 2)
        i_hi = min(max(i_hi, i_lo + 1), n - 1)
        X0s[d] = nodes[i_lo]
        ns[d] = i_hi - i_lo + 1
        rows.append((i_lo, i_hi))
        Fr.append(np.array(F[d][i_lo:i_hi + 1], dtype=np.float64))
    return Restricted(F=Fr, X0s=X0s, inv_h=inv_h, ns=ns, rows=rows)


def recompress(F, eps):
    """Canonical -> Tucker -> canonical rank reduction of explicit factors (step 2).

    Returns (TuckerResult, CanonicalResult); the Tucker result carries the RHOSVD error
    bound ||xi|| * sum_d (sum of the dropped squared singular values of mode d)^(1/2)."""
    nrm = [np.sqrt(np.sum(np.asarray(F[d]) ** 2, axis=0)) for d in range(3)]
    live = (nrm[0] > 0.0) & (nrm[1] > 0.0) & (nrm[2] > 0.0)   # a zero column is a zero term
    A = [np.asarray(F[d])[:, live] / nrm[d][live][None, :] for d in range(3)]
    xi = nrm[0][live] * nrm[1][live] * nrm[2][live]
    U, sing, ranks, B = [], [], [], []
    for d in range(3):
        Ud, sd = _rhosvd._left_svd(A[d])
        rd = int(np.count_nonzero(sd >= eps * sd[0])) if sd.size else 0
        Ud = Ud[:, :rd]
        U.append(Ud)
        sing.append(sd)
        ranks.append(rd)
        B.append(Ud.T @ A[d])
    r1, r2, r3 = ranks
    kr = (B[0][:, None, :] * B[1][None, :, :]).reshape(r1 * r2, -1)
    core = (kr @ (B[2] * xi[None, :]).T).reshape(r1, r2, r3)
    xi_norm = float(np.linalg.norm(xi))
    bound = xi_norm * sum(float(np.sqrt(np.sum(sing[d][ranks[d]:] ** 2))) for d in range(3))
    tk = _rhosvd.TuckerResult(U=U, sing=sing, ranks=tuple(ranks), core=core, xi_norm=xi_norm, bound=bound)
    return tk, _rhosvd.tucker_to_canonical(tk, eps)


def combine(F_list, eps):
    """The long-range tensor of a complex of molecules (eq. 5.1 sums their potentials): the
    canonical factors of tensors on one grid are concatenated (a sum of canonical tensors is
    the canonical tensor of all their terms) and the rank of the sum is reduced as in
    `recompress` (the add-and-compress of Sec. 5)."""
    F = [np.concatenate([np.asarray(Fi[d], dtype=np.float64) for Fi in F_list], axis=1) for d in range(3)]
    return F, recompress(F, eps)
