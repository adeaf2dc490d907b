"""Rank reduction of the long-range sum: canonical -> Tucker (RHOSVD) -> canonical.

Algorithm TEP step 4 reduces the rank-N*K_long canonical sum of eq. 2.6 by the
canonical-to-Tucker-to-canonical transform, using the reduced HOSVD (RHOSVD)
of Khoromskij and Khoromskaia (2009, cited in the introduction).  The paper
gives no formulas for it; this module follows the standard RHOSVD:

1. Per mode d, the side matrix A_d (n x N*K) has the Gaussian factor columns
   normalised to unit 2-norm; the weights collect the norms:
   xi_{m,k} = z_m w_k prod_d ||g_{k,m,d}||.
2. SVD A_d = U_d S_d V_d^T; keep r_d = #{s_i >= eps * s_1} left vectors.
   (Computed as the SVD of the triangular factor of A_d^T, which has the same
   singular values and left singular vectors as A_d.)
3. Tucker core beta = sum_{m,k} xi_{m,k} (U_1^T a1) x (U_2^T a2) x (U_3^T a3).
   The RHOSVD error bound is
   ||T0 - T_tucker||_F <= ||xi||_2 * sum_d (sum_{i > r_d} s_{d,i}^2)^{1/2}.
4. Tucker -> canonical: for each mode-3 index c, SVD of the slice
   beta[:, :, c] = sum_q s_cq u_cq v_cq^T, keeping s_cq >= eps * max_{c,q} s_cq;
   each kept term becomes one canonical term
   F1[:, p] = s_cq U_1 u_cq,  F2[:, p] = U_2 v_cq,  F3[:, p] = U_3[:, c].

The same eps is used in steps 2 and 4.  Factors are unique only up to
rotation and sign, so results are compared through evaluated tensor values.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import tensor as _tensor


@dataclass
class TuckerResult:
    U: list          # per mode: (n, r_d) orthonormal columns
    sing: list       # per mode: all singular values of the normalised side matrix
    ranks: tuple     # (r_1, r_2, r_3)
    core: np.ndarray  # (r_1, r_2, r_3)
    xi_norm: float   # ||xi||_2
    bound: float     # RHOSVD Frobenius error bound


@dataclass
class CanonicalResult:
    F: list          # three (n, R) factor matrices; the weight s_cq is folded into F[0]
    R: int
    dropped_fro: float  # sqrt(sum of squared dropped slice singular values)


def _left_svd(A: np.ndarray):
    """Singular values and left singular vectors of a wide matrix A (n x C), C >= n or not."""
    n, C = A.shape
    if C > n:
        Rf = np.linalg.qr(A.T, mode="r")          # A^T = Q R  ->  A = R^T Q^T
        U, s, _ = np.linalg.svd(Rf.T, full_matrices=False)
    else:
        U, s, _ = np.linalg.svd(A, full_matrices=False)
    return U, s


def rhosvd(charges, positions, t_long, w_long, n, b, eps, col_chunk: int = 8192, galerkin: bool = False,
           snapped: bool = False) -> TuckerResult:
    """Canonical-to-Tucker transform of the long-range sum (steps 1-3 above); galerkin=True
    takes the cell-average factors of eq. 2.1 instead of collocated ones; snapped=True builds
    the columns by the shift-and-window transform of eq. 2.5 (charges at their nearest nodes)."""
    charges = np.asarray(charges, dtype=np.float64)
    positions = np.asarray(positions, dtype=np.float64)
    N = positions.shape[0]
    K = t_long.shape[0]
    _, _, _, nodes = _tensor.grid(n, b)
    U, sing, ranks, B, norms = [], [], [], [], []
    for d in range(3):
        if snapped:
            G = _tensor.shifted_columns(positions[:, d], t_long, n, b, galerkin).reshape(n, N * K)
        elif galerkin:
            G = _tensor.galerkin_columns(positions[:, d], t_long, nodes, (2.0 * b) / n).reshape(n, N * K)
        else:
            G = _tensor.factor_columns(positions[:, d], t_long, nodes).reshape(n, N * K)
        nrm = np.sqrt(np.sum(G * G, axis=0))
        G /= np.where(nrm > 0.0, nrm, 1.0)[None, :]
        Ud, sd = _left_svd(G)
        rd = int(np.count_nonzero(sd >= eps * sd[0]))
        Ud = Ud[:, :rd]
        B.append(Ud.T @ G)        # (r_d, N*K)
        U.append(Ud)
        sing.append(sd)
        ranks.append(rd)
        norms.append(nrm)
        del G
    xi = (charges[:, None] * w_long[None, :]).reshape(N * K) * norms[0] * norms[1] * norms[2]
    r1, r2, r3 = ranks
    core = np.zeros((r1 * r2, r3))
    for c0 in range(0, N * K, col_chunk):
        c1 = min(N * K, c0 + col_chunk)
        kr = (B[0][:, None, c0:c1] * B[1][None, :, c0:c1]).reshape(r1 * r2, c1 - c0)
        core += kr @ (B[2][:, c0:c1] * xi[None, c0:c1]).T
    core = core.reshape(r1, r2, r3)
    xi_norm = float(np.linalg.norm(xi))
    bound = xi_norm * sum(float(np.sqrt(np.sum(sing[d][ranks[d]:] ** 2))) for d in range(3))
    return TuckerResult(U=U, sing=sing, ranks=tuple(ranks), core=core, xi_norm=xi_norm, bound=bound)


def tucker_to_canonical(tk: TuckerResult, eps) -> CanonicalResult:
    """Step 4: slice-wise SVD of the Tucker core into canonical terms."""
    r1, r2, r3 = tk.core.shape
    svds = [np.linalg.svd(tk.core[:, :, c], full_matrices=False) for c in range(r3)]
    smax = max(float(s[0]) for _, s, _ in svds) if r3 > 0 else 0.0
    cols1, cols2, cols3 = [], [], []
    dropped = 0.0
    for c, (u, s, vt) in enumerate(svds):
        keep = s >= eps * smax
        dropped += float(np.sum(s[~keep] ** 2))
        for q in np.nonzero(keep)[0]:
            cols1.append(s[q] * (tk.U[0] @ u[:, q]))
            cols2.append(tk.U[1] @ vt[q, :])
            cols3.append(tk.U[2][:, c].copy())
    n = tk.U[0].shape[0]
    if cols1:
        F = [np.stack(cols1, axis=1), np.stack(cols2, axis=1), np.stack(cols3, axis=1)]
    else:
        F = [np.zeros((n, 0)) for _ in range(3)]
    return CanonicalResult(F=F, R=F[0].shape[1], dropped_fro=float(np.sqrt(dropped)))


def build(charges, positions, t_long, w_long, n, b, eps, galerkin: bool = False, snapped: bool = False):
    """Algorithm TEP steps 3-5: the rank-reduced canonical long-range tensor."""
    tk = rhosvd(charges, positions, t_long, w_long, n, b, eps, galerkin=galerkin, snapped=snapped)
    return tk, tucker_to_canonical(tk, eps)


def uncompressed_factors(charges, positions, t_long, w_long, n, b):
    """The rank N*K_long canonical factors of eq. 2.6 with weights folded into mode 1 (no compression)."""
    _, _, _, nodes = _tensor.grid(n, b)
    N = positions.shape[0]
    K = t_long.shape[0]
    F = [_tensor.factor_columns(positions[:, d], t_long, nodes).reshape(n, N * K) for d in range(3)]
    F[0] = F[0] * (np.asarray(charges)[:, None] * w_long[None, :]).reshape(N * K)[None, :]
    return F
