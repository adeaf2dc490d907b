"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic (no sinc table, no tensor, no transform, no distances
beyond the 1.2 A minimum-separation rule that defines the synthetic
clusters).  Every stream is a ``numpy.random.Generator(PCG64(seed))`` with
``seed = 1000 * config + stream``:

    1 protein positions   2 protein charges   3 ligand positions
    4 ligand charges      5 quaternions       6 translations
    7 sizes / pose counts 8 arrivals

The workloads stand in for the paper's own data (synthetic flat clusters in
Sec. 4.1 and a 379-atom protein in Sec. 4.2, neither of which is available):
clusters are random points in a ball with a minimum pair separation, and the
ligand is posed by a uniform rotation about its geometric centre plus a
translation of that centre (the rigid motion of Sec. 3.4, eq. 3.14).
"""
from __future__ import annotations

import math

import numpy as np

MIN_SEPARATION = 1.2  # Angstrom, minimum distance between atoms of one cluster
_BATCH = 4096         # candidate batch size of the rejection sampler (fixed: part of the stream definition)


def rng(config: int, stream: int, item: int | None = None) -> np.random.Generator:
    """Generator for (config, stream); seed = 1000*config + stream.  Workloads made of many
    independent items (protein/ligand pairs, requests) add the item index as a second seed word."""
    base = 1000 * int(config) + int(stream)
    if item is None:
        return np.random.Generator(np.random.PCG64(base))
    return np.random.Generator(np.random.PCG64([base, int(item)]))


def ball_points(g: np.random.Generator, count: int, radius: float,
                min_sep: float = MIN_SEPARATION) -> np.ndarray:
    """``count`` points uniform in a ball of ``radius`` with pairwise distance >= min_sep.

    Sequential rejection: candidates are uniform in the cube [-radius, radius]^3,
    kept if inside the ball and at least ``min_sep`` from every point kept so far
    (checked through a hash of cells of edge ``min_sep``).  Returns (count, 3) float64.
    """
    if count <= 0:
        return np.zeros((0, 3))
    out = np.empty((count, 3))
    cells: dict[tuple[int, int, int], list[int]] = {}
    kept = 0
    r2 = radius * radius
    s2 = min_sep * min_sep
    tries = 0
    while kept < count:
        cand = g.uniform(-radius, radius, size=(_BATCH, 3))
        for p in cand:
            tries += 1
            if tries > 200 * count + 10 * _BATCH:
                raise RuntimeError("ball_points: packing too dense for the minimum separation")
            if p[0] * p[0] + p[1] * p[1] + p[2] * p[2] > r2:
                continue
            key = (int(math.floor(p[0] / min_sep)), int(math.floor(p[1] / min_sep)),
                   int(math.floor(p[2] / min_sep)))
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        for j in cells.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                            q = out[j]
                            if ((p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2 + (p[2] - q[2]) ** 2) < s2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                continue
            out[kept] = p
            cells.setdefault(key, []).append(kept)
            kept += 1
            if kept == count:
                break
    return out


def charges(g: np.random.Generator, count: int, std: float, net_zero: bool) -> np.ndarray:
    """N(0, std) charges; ``net_zero`` subtracts the mean."""
    z = g.normal(0.0, std, size=count)
    if net_zero and count > 0:
        z = z - z.mean()
    return z


def unit_quaternions(g: np.random.Generator, count: int) -> np.ndarray:
    """Uniform random rotations as unit quaternions (w, x, y, z), Shoemake's subgroup method."""
    u = g.random((count, 3))
    a = np.sqrt(1.0 - u[:, 0])
    c = np.sqrt(u[:, 0])
    t1 = 2.0 * np.pi * u[:, 1]
    t2 = 2.0 * np.pi * u[:, 2]
    return np.stack([c * np.cos(t2), a * np.sin(t1), a * np.cos(t1), c * np.sin(t2)], axis=1)


def directions(g: np.random.Generator, count: int) -> np.ndarray:
    """Uniform directions on the unit sphere: normalised N(0, I3) draws."""
    v = g.normal(size=(count, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def sphere_translations(g: np.random.Generator, count: int, radius: float) -> np.ndarray:
    """Ligand-centre positions on a sphere of ``radius`` about the origin."""
    return radius * directions(g, count)


def shell_translations(g: np.random.Generator, count: int, r_in: float, r_out: float) -> np.ndarray:
    """Ligand-centre positions uniform by volume in the shell r_in <= |t| <= r_out."""
    d = directions(g, count)
    u = g.random(count)
    r = np.cbrt(r_in ** 3 + u * (r_out ** 3 - r_in ** 3))
    return d * r[:, None]


def protein_radius(n_atoms: int, density: float) -> float:
    """Radius of a ball holding ``n_atoms`` at ``density`` atoms per cubic Angstrom."""
    return (3.0 * n_atoms / (4.0 * math.pi * density)) ** (1.0 / 3.0)
