"""torch.autograd.Function around rsd_score_poses and its hand-written adjoint.

Forward returns the binding energy E (Algorithm PLIE with the short-range term) per pose;
backward uses the gradients the scoring kernel writes in the same pass: dE/dt and the
derivative dE/domega with respect to a rotation vector applied on the left of the pose
quaternion (the rigid-body force reduction of Sec. 5.2).  For the quaternion input the
gradient returned is the one tangent to the unit sphere: along q' = quat(omega) q the
derivative of q is (1/2)(0, omega) q, so grad_q = 2 (0, dE/domega) q, which is the unique
tangent vector whose inner product with every such direction gives dE/domega.
"""
from __future__ import annotations

import torch

from . import rsdock


def _hamilton(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Quaternion products a b for (P, 4) tensors (w, x, y, z)."""
    aw, ax, ay, az = a.unbind(-1)
    bw, bx, by, bz = b.unbind(-1)
    return torch.stack([aw * bw - ax * bx - ay * by - az * bz,
                        aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw], dim=-1)


class RigidPoseEnergy(torch.autograd.Function):
    """E(q, t) per pose; non-differentiable flags and pair counts are returned alongside."""

    @staticmethod
    def forward(fctx, quats, trans, rs_ctx, tensor, lig_charges, lig_positions, vdw_min):
        out = rsdock.score_poses(rs_ctx, tensor, lig_charges, lig_positions, quats.contiguous(), trans.contiguous(),
                                 vdw_min, grads=True)
        fctx.save_for_backward(quats, out["grads"])
        fctx.mark_non_differentiable(out["flags"], out["counts"])
        return out["E"], out["flags"], out["counts"]

    @staticmethod
    def backward(fctx, gE, _gflags, _gcounts):
        quats, g = fctx.saved_tensors
        gE = gE.unsqueeze(-1)
        g_t = gE * g[:, :3]
        g_w = g[:, 3:]
        pure = torch.cat([torch.zeros_like(g_w[:, :1]), g_w], dim=-1)
        g_q = gE * 2.0 * _hamilton(pure, quats)
        return g_q, g_t, None, None, None, None, None


def pose_energy(rs_ctx, tensor, lig_charges, lig_positions, quats, trans, vdw_min):
    """(E, flags, counts) with autograd through E to quats and trans (device tensors)."""
    return RigidPoseEnergy.apply(quats, trans, rs_ctx, tensor, lig_charges, lig_positions, float(vdw_min))
