"""Constrained rigid-pose minimisation driven by the adjoint (problem of eq. 3.14).

Each step moves every pose down its gradient (translation dE/dt, rotation dE/domega),
with the step lengths clipped to a trust radius, and then restores the van der Waals
constraint by the radial approach of Algorithm PPIEM (step A3), run in reverse: a pose
that lost its accept flag is pushed out along the line from the protein centre through
the ligand centre, by the smallest offset (bisection) that accepts it again; a pose no
offset can repair keeps its previous position.  Energies, flags and gradients all come
from rsd_score_poses; the tensor algebra here is only the pose update.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import rsdock
from .autograd import _hamilton


def quat_from_rotvec(w: torch.Tensor) -> torch.Tensor:
    """Unit quaternions (w, x, y, z) of rotation vectors (P, 3)."""
    ang = torch.linalg.norm(w, dim=-1, keepdim=True)
    half = 0.5 * ang
    small = ang < 1e-12
    scale = torch.where(small, 0.5 - ang * ang / 48.0, torch.sin(half) / torch.where(small, torch.ones_like(ang), ang))
    return torch.cat([torch.cos(half), scale * w], dim=-1)


def _normalise(q: torch.Tensor) -> torch.Tensor:
    return q / torch.linalg.norm(q, dim=-1, keepdim=True)


@dataclass
class PGResult:
    quats: torch.Tensor
    trans: torch.Tensor
    energy: torch.Tensor
    flags: torch.Tensor
    history: list = field(default_factory=list)


def _accepts(ctx, tensor, lz, lx, q, t, vdw_min):
    out = rsdock.score_poses(ctx, tensor, lz, lx, q.contiguous(), t.contiguous(), vdw_min)
    return (out["flags"] & rsdock.FLAG_ACCEPT) != 0


def _restore(ctx, tensor, lz, lx, q, t, t_prev, q_prev, centre, vdw_min, push_max, iters):
    ok = _accepts(ctx, tensor, lz, lx, q, t, vdw_min)
    bad = ~ok
    if not bool(bad.any()):
        return q, t
    idx = torch.nonzero(bad).squeeze(1)
    qb, tb = q[idx], t[idx]
    d = tb - centre
    d = d / torch.linalg.norm(d, dim=-1, keepdim=True).clamp_min(1e-12)
    lo = torch.zeros(idx.numel(), dtype=t.dtype, device=t.device)
    hi = torch.full_like(lo, push_max)
    ok_hi = _accepts(ctx, tensor, lz, lx, qb, tb + hi[:, None] * d, vdw_min)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        acc = _accepts(ctx, tensor, lz, lx, qb, tb + mid[:, None] * d, vdw_min)
        hi = torch.where(acc, mid, hi)
        lo = torch.where(acc, lo, mid)
    t_fix = torch.where(ok_hi[:, None], tb + hi[:, None] * d, t_prev[idx])
    q_fix = torch.where(ok_hi[:, None], qb, q_prev[idx])
    t = t.clone()
    q = q.clone()
    t[idx] = t_fix
    q[idx] = q_fix
    return q, t


def projected_gradient(ctx, tensor, lig_charges, lig_positions, quats, trans, vdw_min, steps=50, eta_t=0.5,
                       eta_r=0.5, max_t=0.25, max_r=0.05, centre=None, push_max=8.0, bisect=12) -> PGResult:
    """`steps` projected-gradient steps on (t, omega) for every pose (device tensors, FP64)."""
    q = _normalise(quats.clone())
    t = trans.clone()
    c = torch.zeros(3, dtype=t.dtype, device=t.device) if centre is None else centre
    q, t = _restore(ctx, tensor, lig_charges, lig_positions, q, t, t, q, c, vdw_min, push_max, bisect)
    hist = []
    for _ in range(steps):
        out = rsdock.score_poses(ctx, tensor, lig_charges, lig_positions, q, t, vdw_min, grads=True)
        g = torch.nan_to_num(out["grads"], nan=0.0)
        acc = (out["flags"] & rsdock.FLAG_ACCEPT) != 0
        hist.append(dict(mean_E=float(out["E"][acc].mean()) if bool(acc.any()) else float("nan"),
                         accepted=int(acc.sum())))
        st = -eta_t * g[:, :3]
        sr = -eta_r * g[:, 3:]
        st = st * torch.clamp(max_t / torch.linalg.norm(st, dim=-1, keepdim=True).clamp_min(1e-300), max=1.0)
        sr = sr * torch.clamp(max_r / torch.linalg.norm(sr, dim=-1, keepdim=True).clamp_min(1e-300), max=1.0)
        t_new = t + st
        q_new = _normalise(_hamilton(quat_from_rotvec(sr), q))
        q, t = _restore(ctx, tensor, lig_charges, lig_positions, q_new, t_new, t, q, c, vdw_min, push_max, bisect)
    out = rsdock.score_poses(ctx, tensor, lig_charges, lig_positions, q, t, vdw_min, grads=True)
    acc = (out["flags"] & rsdock.FLAG_ACCEPT) != 0
    hist.append(dict(mean_E=float(out["E"][acc].mean()) if bool(acc.any()) else float("nan"),
                     accepted=int(acc.sum())))
    return PGResult(q, t, out["E"], out["flags"], hist)
