"""Deterministic angle grids of the posing search (Algorithm PPIEM, step A0) and their
neighbour graphs, shared as inputs by the oracle tests, the GPU tests and the bench.

Like ``generators``, this module holds none of the method's arithmetic: it only lays out
sample points of the parametric space (orbit directions of the ligand centre around the
protein centre, orientations of the ligand about its own centre) and says which orbit
samples are adjacent.  The paper scans 12 orbit angles x 12 self-rotation angles in a plane
(Sec. 4, steps 2*pi/12); ``orbit_ring`` / ``spins`` are that planar grid, ``orbit_sphere`` /
``orientations`` its 3-D counterpart.

Neighbour graphs are CSR arrays (offsets[U + 1], index[offsets[U]]) over the orbit samples.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


def orbit_ring(m: int) -> np.ndarray:
    """m unit directions in the xy-plane at angles 2*pi*i/m (delta_M = 2*pi/m_P)."""
    a = 2.0 * math.pi * np.arange(m) / m
    return np.stack([np.cos(a), np.sin(a), np.zeros(m)], axis=1)


def ring_neighbours(m: int):
    """Each ring sample is adjacent to the previous and the next one (cyclically)."""
    if m == 1:
        return np.array([0, 0], dtype=np.int32), np.zeros(0, dtype=np.int32)
    if m == 2:
        return np.array([0, 1, 2], dtype=np.int32), np.array([1, 0], dtype=np.int32)
    idx = np.stack([(np.arange(m) - 1) % m, (np.arange(m) + 1) % m], axis=1).reshape(-1)
    return np.arange(0, 2 * m + 1, 2, dtype=np.int32), idx.astype(np.int32)


def orbit_sphere(m: int) -> np.ndarray:
    """m nearly uniform unit directions (Fibonacci lattice): z_i = 1 - (2i + 1)/m, azimuth
    i times the golden angle."""
    i = np.arange(m, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / m
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = GOLDEN_ANGLE * i
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def sphere_neighbours(dirs: np.ndarray, k: int = 6):
    """The k directions with the largest dot product with each direction (itself excluded;
    ties by index), made symmetric: i ~ j if either is among the other's k nearest."""
    d = np.asarray(dirs, dtype=np.float64)
    m = d.shape[0]
    k = min(k, m - 1)
    adj = [set() for _ in range(m)]
    for i0 in range(0, m, 1024):
        blk = d[i0:i0 + 1024] @ d.T
        for r in range(blk.shape[0]):
            i = i0 + r
            blk[r, i] = -np.inf
            near = np.lexsort((np.arange(m), -blk[r]))[:k]
            for j in near:
                adj[i].add(int(j))
                adj[int(j)].add(i)
    off = np.zeros(m + 1, dtype=np.int32)
    for i in range(m):
        off[i + 1] = off[i] + len(adj[i])
    idx = np.concatenate([np.array(sorted(a), dtype=np.int32) for a in adj]) if m else np.zeros(0, np.int32)
    return off, idx.astype(np.int32)


def spins(m: int, axis=(0.0, 0.0, 1.0)) -> np.ndarray:
    """m unit quaternions (w, x, y, z) turning by 2*pi*k/m about `axis` (delta_L = 2*pi/m_L)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    th = 2.0 * math.pi * np.arange(m) / m
    return np.concatenate([np.cos(th / 2)[:, None], np.sin(th / 2)[:, None] * a[None, :]], axis=1)


def _qmul(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    w1, x1, y1, z1 = p[..., 0], p[..., 1], p[..., 2], p[..., 3]
    w2, x2, y2, z2 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def orientations(m_axes: int, m_spin: int) -> np.ndarray:
    """m_axes * m_spin unit quaternions: a spin by 2*pi*k/m_spin about z, then the rotation
    taking z to the i-th Fibonacci direction (about the axis z x a_i).  Renormalised so that
    | |q|^2 - 1 | stays at rounding level."""
    a = orbit_sphere(m_axes)
    out = np.empty((m_axes, m_spin, 4))
    s = spins(m_spin)
    for i in range(m_axes):
        c = float(np.clip(a[i, 2], -1.0, 1.0))
        ax = np.array([-a[i, 1], a[i, 0], 0.0])
        nrm = float(np.linalg.norm(ax))
        if nrm < 1e-300:
            al = np.array([1.0, 0.0, 0.0, 0.0]) if c > 0 else np.array([0.0, 1.0, 0.0, 0.0])
        else:
            th = math.acos(c)
            al = np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * ax / nrm])
        out[i] = _qmul(al[None, :], s)
    out = out.reshape(-1, 4)
    return out / np.linalg.norm(out, axis=1, keepdims=True)
