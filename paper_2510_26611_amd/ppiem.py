"""Posing search of Algorithm PPIEM (steps A2-A7) on the device.

The angle grids (step A0) and the tensor (step A1, rsd_build_rs_tensor) are the caller's.
Each step below is one C-ABI call whose kernels do the work; this module only moves the
arrays to the device and reads the few minima back:
  A2  rsd_tensor_centre          the protein's geometric centre x_P
  A3  rsd_contact_poses          first contact along x_P + rho u for every (u, q)
  A4/A5  rsd_score_poses         energies and flags of all U*Q contact poses
  A6  rsd_orbit_minima           best orientation per orbit position, local minima on the orbit grid
  A7  the minima's poses, sorted by energy (host, a handful of entries)
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from .rsdock import Context, Tensor, _check, score_poses


def _dev(x, dtype):
    import torch
    if isinstance(x, torch.Tensor):
        if x.dtype != dtype or not x.is_cuda or not x.is_contiguous():
            raise TypeError(f"expected a contiguous CUDA tensor of {dtype}")
        return x
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def tensor_centre(t: Tensor) -> np.ndarray:
    c = (C.c_double * 3)()
    _check(_lib.lib().rsd_tensor_centre(t.handle, c))
    return np.array(c[:])


def contact_poses(ctx: Context, tensor: Tensor, lig_positions, dirs, quats, sigma: float, gap: float = 1e-6,
                  centre=None) -> dict:
    """rsd_contact_poses: rho [U, Q] and the contact poses (U*Q quaternions and translations)."""
    import torch
    lp = _dev(lig_positions, torch.float64)
    dp = _dev(dirs, torch.float64)
    qp = _dev(quats, torch.float64)
    U, Q, L = int(dp.shape[0]), int(qp.shape[0]), int(lp.shape[0])
    c = tensor_centre(tensor) if centre is None else np.asarray(centre, dtype=np.float64)
    dev = dp.device
    rho = torch.empty((U, Q), dtype=torch.float64, device=dev)
    pq = torch.empty((U * Q, 4), dtype=torch.float64, device=dev)
    pt = torch.empty((U * Q, 3), dtype=torch.float64, device=dev)
    c3 = (C.c_double * 3)(*[float(x) for x in c])
    _check(_lib.lib().rsd_contact_poses(ctx.handle, tensor.handle, lp.data_ptr(), L, dp.data_ptr(), U, qp.data_ptr(),
                                        Q, c3, float(sigma), float(gap), rho.data_ptr(), pq.data_ptr(),
                                        pt.data_ptr()))
    return dict(centre=c, rho=rho, quats=pq, trans=pt)


def orbit_minima(ctx: Context, energies, flags, U: int, Q: int, nbr_off, nbr_idx) -> dict:
    """rsd_orbit_minima: best_rotation [U] (-1: none accepted), best_energy [U], is_minimum [U]."""
    import torch
    E = _dev(energies, torch.float64)
    F = _dev(flags, torch.uint8)
    off = _dev(nbr_off, torch.int32)
    idx = _dev(nbr_idx, torch.int32) if len(nbr_idx) else torch.zeros(1, dtype=torch.int32, device=E.device)
    dev = E.device
    bq = torch.empty(U, dtype=torch.int32, device=dev)
    be = torch.empty(U, dtype=torch.float64, device=dev)
    im = torch.empty(U, dtype=torch.uint8, device=dev)
    _check(_lib.lib().rsd_orbit_minima(ctx.handle, E.data_ptr(), F.data_ptr(), U, Q, off.data_ptr(), idx.data_ptr(),
                                       bq.data_ptr(), be.data_ptr(), im.data_ptr()))
    return dict(best_rotation=bq, best_energy=be, is_minimum=im)


def ppiem(ctx: Context, tensor: Tensor, lig_charges, lig_positions, dirs, quats, sigma: float, nbr_off, nbr_idx,
          gap: float = 1e-6) -> dict:
    """Steps A2-A7 for orbit directions `dirs` (U x 3, unit) and orientations `quats` (Q x 4).
    Returns the device arrays of every step and `minima`: (energy, orbit index, orientation
    index, quaternion, translation) of each local minimum, lowest energy first."""
    import torch
    cp = contact_poses(ctx, tensor, lig_positions, dirs, quats, sigma, gap)
    U, Q = cp["rho"].shape
    zc = _dev(lig_charges, torch.float64)
    lp = _dev(lig_positions, torch.float64)
    res = score_poses(ctx, tensor, zc, lp, cp["quats"], cp["trans"], sigma)
    mins = orbit_minima(ctx, res["E"], res["flags"], U, Q, nbr_off, nbr_idx)
    im = mins["is_minimum"].cpu().numpy().astype(bool)
    bq = mins["best_rotation"].cpu().numpy()
    be = mins["best_energy"].cpu().numpy()
    sel = np.nonzero(im)[0]
    rows = sel * Q + bq[sel]
    qs = cp["quats"][torch.from_numpy(rows).to(cp["quats"].device)].cpu().numpy() if sel.size else np.zeros((0, 4))
    ts = cp["trans"][torch.from_numpy(rows).to(cp["trans"].device)].cpu().numpy() if sel.size else np.zeros((0, 3))
    minima = sorted(((float(be[u]), int(u), int(bq[u]), qs[i], ts[i]) for i, u in enumerate(sel)),
                    key=lambda m: (m[0], m[1]))
    return dict(contact=cp, result=res, orbit=mins, minima=minima)
