"""Pose scoring: transform, long-range and short-range potential, energy, flags, gradients.

Follows, in order:
  * the rigid motion F = R o T about the ligand's geometric centre (Sec. 3.4, eq. 3.14);
  * the binding energy E(M, L) = sum_l zeta_l P_M(y_l) (eq. 3.7), with the long-range
    part evaluated from the rank-R canonical factors (Lemma 3.3, eq. 3.10; Algorithm
    PLIE steps 2-3) and the short-range part summed over protein atoms closer than
    the cutoff r_c (the RS-canonical format, Def. 2.1, eq. 2.7);
  * the van der Waals constraint dist(M, F(L)) >= sigma (eq. 3.14);
  * gradients: the one-sided difference of the factor rows inside the grid cell
    (eq. 3.12) and the rigid-body reduction of per-atom forces to a translation and
    a rotation part (Sec. 5.2, eqs. 5.2-5.3, written as the torque about the centre).

Off-grid ligand atoms are evaluated by the trilinear interpolant of the canonical
tensor, i.e. per-mode linear interpolation of two adjacent factor rows.

Exactness contract.  Everything that decides an integer (grid row, in-domain,
d^2 < r_c^2, d^2 >= sigma^2) is computed here in one fixed IEEE-754 operation
order with no fused multiply-add; numpy's elementwise ufuncs round every
operation separately, so these values are reproducible by any FP64 code that
performs the same operations in the same order:
  centre  c = ((0 + x_0) + x_1) + ... ; c = c / L       (index order)
  u_l     = x_l - c
  R(q)    rows [1-2(y*y+z*z), 2(x*y-w*z), 2(x*z+w*y)], [2(x*y+w*z), 1-2(x*x+z*z), 2(y*z-w*x)],
              [2(x*z-w*y), 2(y*z+w*x), 1-2(x*x+y*y)]
  y_i     = ((R_i0 u_0 + R_i1 u_1) + R_i2 u_2) + t_i
  s_d     = (y_d - X_0) * inv_h,  X_0 = -b + h,  h = (2b)/n,  inv_h = 1/h
  d^2     = ((y_0-x_0)^2 + (y_1-x_1)^2) + (y_2-x_2)^2
  |q|^2   = ((w*w + x*x) + y*y) + z*z
Flags: bit0 accept (in domain and min d^2 >= sigma^2), bit1 in domain
(0 <= s_d <= n-1 for every atom and axis), bit2 invalid pose (non-finite input
or | |q|^2 - 1 | > 1e-12).
"""
from __future__ import annotations

import numpy as np

from . import tensor as _tensor

FLAG_ACCEPT = 1
FLAG_IN_DOMAIN = 2
FLAG_INVALID = 4
QUAT_TOL = 1e-12


def ligand_frame(lig_positions: np.ndarray):
    """Geometric centre (summed in index order, then divided by L) and centred coordinates."""
    lig = np.asarray(lig_positions, dtype=np.float64)
    c = np.zeros(3)
    for ell in range(lig.shape[0]):
        c = c + lig[ell]
    c = c / lig.shape[0]
    return c, lig - c[None, :]


def rotation_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrices (P, 3, 3) of quaternions q = (w, x, y, z), used as given."""
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1.0 - 2.0 * (y * y + z * z)
    R[:, 0, 1] = 2.0 * (x * y - w * z)
    R[:, 0, 2] = 2.0 * (x * z + w * y)
    R[:, 1, 0] = 2.0 * (x * y + w * z)
    R[:, 1, 1] = 1.0 - 2.0 * (x * x + z * z)
    R[:, 1, 2] = 2.0 * (y * z - w * x)
    R[:, 2, 0] = 2.0 * (x * z - w * y)
    R[:, 2, 1] = 2.0 * (y * z + w * x)
    R[:, 2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return R


def rotate(R: np.ndarray, u: np.ndarray) -> np.ndarray:
    """v[p, l, i] = (R_i0 u_0 + R_i1 u_1) + R_i2 u_2."""
    v = np.empty((R.shape[0], u.shape[0], 3))
    for i in range(3):
        v[:, :, i] = (R[:, i, 0][:, None] * u[None, :, 0] + R[:, i, 1][:, None] * u[None, :, 1]) \
            + R[:, i, 2][:, None] * u[None, :, 2]
    return v


def transform(q: np.ndarray, t: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Atom positions y (P, L, 3) of the posed ligand: y = R(q) u + t."""
    return rotate(rotation_matrix(q), u) + np.atleast_2d(t)[:, None, :]


def quat_valid(q: np.ndarray, t: np.ndarray) -> np.ndarray:
    q = np.atleast_2d(q)
    t = np.atleast_2d(t)
    qq = ((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3]
    fin = np.all(np.isfinite(q), axis=1) & np.all(np.isfinite(t), axis=1)
    return fin & (np.abs(qq - 1.0) <= QUAT_TOL)


def long_range(F, n: int, b: float, y: np.ndarray, want_grad: bool = False, grid_spec=None):
    """Trilinear evaluation of the canonical tensor sum_p F1[:,p] x F2[:,p] x F3[:,p] (Lemma 3.3).

    y: (Q, 3) points.  Returns (value, in_domain, abs_scale, grad, grad_abs) per point;
    value/grad are NaN where the point is outside the grid.
    Row i_d = min(floor(s_d), n_d-2) and weight f_d = s_d - i_d; the mode-d factor row
    is (1-f_d) F_d[i_d] + f_d F_d[i_d+1]; its derivative (F_d[i_d+1]-F_d[i_d]) inv_h
    is the one-sided difference of eq. 3.12 inside the cell.
    grid_spec = (X0s, inv_h, ns): per-mode origins and row counts (a tensor restricted to a
    sub-box); default: the n-point grid on [-b, b] in every mode.
    """
    if grid_spec is None:
        _, X0, inv_h, _ = _tensor.grid(n, b)
        X0s = np.full(3, X0)
        ns = np.full(3, n, dtype=np.int64)
    else:
        X0s, inv_h, ns = grid_spec
        X0s = np.asarray(X0s, dtype=np.float64)
        ns = np.asarray(ns, dtype=np.int64)
    y = np.atleast_2d(y)
    s = (y - X0s[None, :]) * inv_h
    inside = np.all((s >= 0.0) & (s <= (ns - 1)[None, :]), axis=1)
    Q = y.shape[0]
    val = np.full(Q, np.nan)
    scale = np.zeros(Q)
    grad = np.full((Q, 3), np.nan) if want_grad else None
    gabs = np.zeros(Q) if want_grad else None
    ok = np.nonzero(inside)[0]
    if ok.size == 0:
        return val, inside, scale, grad, gabs
    so = s[ok]
    i = np.minimum(np.floor(so), (ns - 2)[None, :]).astype(np.int64)
    f = so - i
    lerp, alerp, dl, adl = [], [], [], []
    for d in range(3):
        a = F[d][i[:, d]]
        c = F[d][i[:, d] + 1]
        fd = f[:, d][:, None]
        lerp.append((1.0 - fd) * a + fd * c)
        alerp.append((1.0 - fd) * np.abs(a) + fd * np.abs(c))
        if want_grad:
            dl.append((c - a) * inv_h)
            adl.append((np.abs(c) + np.abs(a)) * inv_h)
    val[ok] = np.sum(lerp[0] * lerp[1] * lerp[2], axis=1)
    scale[ok] = np.sum(alerp[0] * alerp[1] * alerp[2], axis=1)
    if want_grad:
        g = np.stack([np.sum(dl[0] * lerp[1] * lerp[2], axis=1),
                      np.sum(lerp[0] * dl[1] * lerp[2], axis=1),
                      np.sum(lerp[0] * lerp[1] * dl[2], axis=1)], axis=1)
        grad[ok] = g
        gabs[ok] = (np.sum(adl[0] * alerp[1] * alerp[2], axis=1)
                    + np.sum(alerp[0] * adl[1] * alerp[2], axis=1)
                    + np.sum(alerp[0] * alerp[1] * adl[2], axis=1))
    return val, inside, scale, grad, gabs


def pair_d2(y: np.ndarray, atoms: np.ndarray) -> np.ndarray:
    """d^2[q, m] = ((y0-x0)^2 + (y1-x1)^2) + (y2-x2)^2 for points y (Q,3) and atoms (N,3)."""
    d0 = y[:, None, 0] - atoms[None, :, 0]
    d1 = y[:, None, 1] - atoms[None, :, 1]
    d2 = y[:, None, 2] - atoms[None, :, 2]
    return (d0 * d0 + d1 * d1) + d2 * d2


def short_range(atoms, z, t_short, w_short, r_cut, y, want_grad: bool = False):
    """Short-range potential sum_{m: d^2 < r_c^2} z_m sum_{k short} w_k exp(-t_k^2 d^2) (Def. 2.1).

    Brute force over all protein atoms.  Returns (value, count, min_d2, abs_scale,
    grad, grad_abs) per point.
    """
    y = np.atleast_2d(y)
    D2 = pair_d2(y, atoms)                           # (Q, N)
    rc2 = r_cut * r_cut
    mask = D2 < rc2
    count = np.sum(mask, axis=1)
    min_d2 = np.min(D2, axis=1) if atoms.shape[0] else np.full(y.shape[0], np.inf)
    t2 = t_short * t_short
    val = np.zeros(y.shape[0])
    scale = np.zeros(y.shape[0])
    grad = np.zeros((y.shape[0], 3)) if want_grad else None
    gabs = np.zeros(y.shape[0]) if want_grad else None
    qi, mi = np.nonzero(mask)
    if qi.size:
        d2 = D2[qi, mi]
        e = np.exp(-np.outer(d2, t2))                # (pairs, S)
        gsum = e @ w_short
        zm = z[mi]
        np.add.at(val, qi, zm * gsum)
        np.add.at(scale, qi, np.abs(zm) * gsum)
        if want_grad:
            dg = e @ (w_short * (-2.0 * t2))          # d/d(d^2) * 2 -> coefficient of (y - x)
            diff = y[qi] - atoms[mi]
            np.add.at(grad, qi, (zm * dg)[:, None] * diff)
            np.add.at(gabs, qi, np.abs(zm) * np.abs(dg) * np.sqrt(d2))
    return val, count, min_d2, scale, grad, gabs


def score(F, n, b, atoms, z, t_short, w_short, r_cut, lig_charges, lig_positions,
          quats, trans, vdw_min, want_grad: bool = False, pose_chunk: int = 16, grid_spec=None):
    """Score P poses (Algorithm PLIE with the short-range term and the vdW flag).

    Returns a dict with E, E_long (P,), flags (P,) uint8, counts (P,) int32,
    scale (P,) = FP64 summation-error scale of E, and with want_grad also
    grads (P, 6) = (dE/dt, dE/domega) and grad_scale (P,).
    """
    atoms = np.asarray(atoms, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    zeta = np.asarray(lig_charges, dtype=np.float64)
    quats = np.atleast_2d(np.asarray(quats, dtype=np.float64))
    trans = np.atleast_2d(np.asarray(trans, dtype=np.float64))
    P = quats.shape[0]
    L = zeta.shape[0]
    _, u = ligand_frame(lig_positions)
    sig2 = vdw_min * vdw_min
    E = np.full(P, np.nan)
    El = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.uint8)
    counts = np.zeros(P, dtype=np.int32)
    scale = np.zeros(P)
    grads = np.full((P, 6), np.nan) if want_grad else None
    gscale = np.zeros(P) if want_grad else None
    valid = quat_valid(quats, trans)
    flags[~valid] = FLAG_INVALID
    for p0 in range(0, P, pose_chunk):
        p1 = min(P, p0 + pose_chunk)
        idx = np.arange(p0, p1)[valid[p0:p1]]
        if idx.size == 0:
            continue
        R = rotation_matrix(quats[idx])
        v = rotate(R, u)                                  # (Pc, L, 3) = R u
        y = v + trans[idx][:, None, :]
        pts = y.reshape(-1, 3)
        lv, inside, lsc, lg, lga = long_range(F, n, b, pts, want_grad, grid_spec)
        sv, cnt, md2, ssc, sg, sga = short_range(atoms, z, t_short, w_short, r_cut, pts, want_grad)
        Pc = idx.size
        inside = inside.reshape(Pc, L).all(axis=1)
        cnt = cnt.reshape(Pc, L).sum(axis=1)
        md2 = md2.reshape(Pc, L).min(axis=1)
        el = (zeta[None, :] * lv.reshape(Pc, L)).sum(axis=1)
        et = (zeta[None, :] * (lv + sv).reshape(Pc, L)).sum(axis=1)
        sc = (np.abs(zeta)[None, :] * (lsc + ssc).reshape(Pc, L)).sum(axis=1)
        E[idx] = np.where(inside, et, np.nan)
        El[idx] = np.where(inside, el, np.nan)
        counts[idx] = cnt
        scale[idx] = sc
        f = np.where(inside, FLAG_IN_DOMAIN, 0)
        f = f | np.where(inside & (md2 >= sig2), FLAG_ACCEPT, 0)
        flags[idx] = f.astype(np.uint8)
        if want_grad:
            gp = (lg + sg).reshape(Pc, L, 3) * zeta[None, :, None]      # zeta_l grad P(y_l)
            gt = gp.sum(axis=1)
            gw = np.cross(v, gp).sum(axis=1)
            g = np.concatenate([gt, gw], axis=1)
            g[~inside] = np.nan
            grads[idx] = g
            vn = np.linalg.norm(v, axis=2)
            gscale[idx] = (np.abs(zeta)[None, :] * (1.0 + vn) * (lga + sga).reshape(Pc, L)).sum(axis=1)
    out = dict(E=E, E_long=El, flags=flags, counts=counts, scale=scale)
    if want_grad:
        out["grads"] = grads
        out["grad_scale"] = gscale
    return out


def long_range_uncompressed(charges, positions, t_long, w_long, n: int, b: float, y: np.ndarray,
                            want_grad: bool = False, corners_out: dict | None = None):
    """Trilinear interpolant of the uncompressed long-range tensor T0 (eq. 2.6) at points y (Q, 3).

    The 8 corner values of each point's grid cell are evaluated term by term from the
    definition of T0; the value is sum_corners w0 w1 w2 T0(corner) with weights (1-f_d, f_d),
    and its derivative along axis d replaces (1-f_d, f_d) by (-inv_h, +inv_h).  Points
    outside the grid give NaN.  Used at sizes where the factor matrices of T0 are too large.
    """
    _, X0, inv_h, _ = _tensor.grid(n, b)
    y = np.atleast_2d(y)
    s = (y - X0) * inv_h
    inside = np.all((s >= 0.0) & (s <= n - 1), axis=1)
    val = np.full(y.shape[0], np.nan)
    grad = np.full((y.shape[0], 3), np.nan) if want_grad else None
    ok = np.nonzero(inside)[0]
    if ok.size == 0:
        return val, inside, grad
    so = s[ok]
    i = np.minimum(np.floor(so), n - 2).astype(np.int64)
    f = so - i
    corners = np.array([[a, bb, c] for a in (0, 1) for bb in (0, 1) for c in (0, 1)])
    V = np.stack([_tensor.long_range_at_nodes(charges, positions, t_long, w_long, n, b, i + cr) for cr in corners],
                 axis=1)                                              # (Q, 8)
    wts = [np.stack([1.0 - f[:, d], f[:, d]], axis=1) for d in range(3)]
    dws = np.array([-inv_h, inv_h])
    W = np.stack([wts[0][:, a] * wts[1][:, bb] * wts[2][:, c] for a, bb, c in corners], axis=1)
    val[ok] = np.sum(W * V, axis=1)
    if corners_out is not None:   # node indices, node values and weights of every evaluated point
        corners_out.update(points=ok, index=i[:, None, :] + corners[None, :, :], value=V, weight=W)
    if want_grad:
        G0 = np.stack([dws[a] * wts[1][:, bb] * wts[2][:, c] for a, bb, c in corners], axis=1)
        G1 = np.stack([wts[0][:, a] * dws[bb] * wts[2][:, c] for a, bb, c in corners], axis=1)
        G2 = np.stack([wts[0][:, a] * wts[1][:, bb] * dws[c] for a, bb, c in corners], axis=1)
        grad[ok] = np.stack([np.sum(G0 * V, axis=1), np.sum(G1 * V, axis=1), np.sum(G2 * V, axis=1)], axis=1)
    return val, inside, grad


def score_uncompressed(charges, positions, t_long, w_long, n, b, t_short, w_short, r_cut, lig_charges,
                       lig_positions, quats, trans, vdw_min, want_grad: bool = False, corners_out: dict | None = None):
    """Energies, flags, counts (and gradients) of poses from the uncompressed tensor T0.

    Same quantities as `score`, with the long-range part taken from the interpolant of T0
    itself (no rank reduction); the short-range part, flags and counts are identical.
    """
    atoms = np.asarray(positions, dtype=np.float64)
    z = np.asarray(charges, dtype=np.float64)
    zeta = np.asarray(lig_charges, dtype=np.float64)
    quats = np.atleast_2d(quats)
    trans = np.atleast_2d(trans)
    _, u = ligand_frame(lig_positions)
    R = rotation_matrix(quats)
    v = rotate(R, u)
    y = v + trans[:, None, :]
    P, L = y.shape[0], y.shape[1]
    pts = y.reshape(-1, 3)
    lv, inside, lg = long_range_uncompressed(z, atoms, t_long, w_long, n, b, pts, want_grad, corners_out)
    sv, cnt, md2, _, sg, _ = short_range(atoms, z, t_short, w_short, r_cut, pts, want_grad)
    inside = inside.reshape(P, L).all(axis=1)
    E = np.where(inside, (zeta[None, :] * (lv + sv).reshape(P, L)).sum(axis=1), np.nan)
    flags = np.where(inside, FLAG_IN_DOMAIN, 0) | np.where(inside & (md2.reshape(P, L).min(axis=1) >= vdw_min * vdw_min),
                                                           FLAG_ACCEPT, 0)
    valid = quat_valid(quats, trans)
    flags = np.where(valid, flags, FLAG_INVALID).astype(np.uint8)
    out = dict(E=np.where(valid, E, np.nan), flags=flags, counts=np.where(valid, cnt.reshape(P, L).sum(axis=1), 0))
    if want_grad:
        gp = (lg + sg).reshape(P, L, 3) * zeta[None, :, None]
        g = np.concatenate([gp.sum(axis=1), np.cross(v, gp).sum(axis=1)], axis=1)
        g[~(inside & valid)] = np.nan
        out["grads"] = g
    return out
