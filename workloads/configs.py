"""Workload definitions: sizes, distributions and frozen numeric constants.

The constants h_M, L_s and r_cut are numbers here, not computations: they were
produced by ``python -m oracle.constants`` and a CPU test re-derives them from
the oracle and checks these frozen values.

Config 1: 200-atom protein in a 12 A ball, 12-atom ligand in a 4 A ball, n=512
on [-24,24]^3, M=24 (49 Gaussians, 25 distinct), 12 long-range terms,
128 poses with the ligand centre on an 18 A sphere, vdW distance 2.5 A.
Config 2: 5,000-atom protein at 0.05 atoms/A^3, 50-atom ligand in a 6 A ball,
n=2048 on [-52,52]^3, M=32, 22 long-range terms, RHOSVD eps 1e-8,
1,000,000 poses with the ligand centre uniform in the shell 5-15 A beyond the
protein surface, vdW distance 2.5 A.
Config 4: 10,000-atom protein, 60-atom ligand, n=4096 on [-60,60]^3, 65,536
poses in the same kind of shell, energies plus rigid-body gradients.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import generators as gen


@dataclass(frozen=True)
class Config:
    index: int
    name: str
    N: int                   # protein atoms
    protein_radius: float    # A
    protein_charge_std: float
    L: int                   # ligand atoms
    ligand_radius: float     # A
    ligand_charge_std: float
    n: int                   # grid points per axis (even)
    b: float                 # box [-b, b]^3, A
    M: int                   # sinc terms k = 0..M after folding +-k
    h_M: float               # quadrature step (frozen)
    L_s: float               # quadrature scale 2*sqrt(3)*b (frozen)
    K_long: int              # number of long-range (widest) terms
    r_cut: float             # short-range cutoff, A (frozen)
    eps: float               # RHOSVD / T2C relative truncation
    P: int                   # poses
    pose_kind: str           # "sphere" or "shell"
    pose_r_in: float
    pose_r_out: float
    sigma: float             # van der Waals minimum distance, A


CONFIG1 = Config(
    index=1, name="cfg1-N200-L12-n512", N=200, protein_radius=12.0, protein_charge_std=0.3,
    L=12, ligand_radius=4.0, ligand_charge_std=0.3, n=512, b=24.0, M=24, h_M=0.2622,
    L_s=83.13843876330611, K_long=12, r_cut=43.836027469049675, eps=1e-8, P=128,
    pose_kind="sphere", pose_r_in=18.0, pose_r_out=18.0, sigma=2.5)

_RP2 = gen.protein_radius(5000, 0.05)
CONFIG2 = Config(
    index=2, name="cfg2-N5000-L50-n2048", N=5000, protein_radius=_RP2, protein_charge_std=0.4,
    L=50, ligand_radius=6.0, ligand_charge_std=0.4, n=2048, b=52.0, M=32, h_M=0.2239,
    L_s=180.13328398716322, K_long=22, r_cut=15.962725425480096, eps=1e-8, P=1_000_000,
    pose_kind="shell", pose_r_in=_RP2 + 5.0, pose_r_out=_RP2 + 15.0, sigma=2.5)

_RP4 = gen.protein_radius(10000, 0.05)
CONFIG4 = Config(
    index=4, name="cfg4-N10000-L60-n4096-grad", N=10000, protein_radius=_RP4, protein_charge_std=0.4,
    L=60, ligand_radius=6.0 * (60 / 50) ** (1.0 / 3.0), ligand_charge_std=0.4, n=4096, b=60.0,
    M=32, h_M=0.228, L_s=207.84609690826525, K_long=22, r_cut=16.833903442913364, eps=1e-8,
    P=65_536, pose_kind="shell", pose_r_in=_RP4 + 5.0, pose_r_out=_RP4 + 15.0, sigma=2.5)

# Config 3: 64 protein/ligand pairs; protein sizes log-uniform in [1e3, 2e4] atoms (density
# 0.05 / A^3), ligand sizes uniform in [10, 200] atoms (ball radius 6 (L/50)^(1/3) A), pose
# counts log-uniform in [1e3, 2e5], translations in the 5-15 A shell of each protein, n=4096.
# One box for every pair: b = 73 A covers the largest protein (45.7 A) + 15 A + the largest
# ligand (9.5 A) + 2 A, so one quadrature and cutoff serve all pairs.
CONFIG3 = Config(
    index=3, name="cfg3-64pairs-n4096", N=0, protein_radius=0.0, protein_charge_std=0.4, L=0, ligand_radius=0.0,
    ligand_charge_std=0.4, n=4096, b=73.0, M=32, h_M=0.2335, L_s=252.87941790505607, K_long=22,
    r_cut=18.15278338984615, eps=1e-8, P=0, pose_kind="shell", pose_r_in=0.0, pose_r_out=0.0, sigma=2.5)
CONFIG3_PAIRS = 64
CONFIG3_N = (1_000, 20_000)
CONFIG3_L = (10, 200)
CONFIG3_P = (1_000, 200_000)

# Config 5 (serving): 8 resident proteins with N log-spaced over [1e3, 1e5] (density 0.05 / A^3),
# box b = ceil(R_P + 15 + R_L(200) + 2) A, grid n = next power of two >= 16384 b / b_max, M=32,
# K_long=22, eps 1e-8.  Per protein: (N, b, n, h_M, L_s, r_cut), the last three frozen from
# oracle.constants like the other configs.  Requests: Poisson arrivals at 200 / s, protein
# uniform over the 8, L uniform in [10, 200], P log-uniform in [1e4, 1e6], translations in the
# 5-15 A shell of the request's protein, vdW distance 2.5 A.
CONFIG5_PROTEINS = (
    (1000, 44.0, 8192, 0.2193, 152.4204710660612, 14.941343046913628),
    (1931, 48.0, 8192, 0.2217, 166.27687752661222, 15.463537931186579),
    (3728, 53.0, 16384, 0.2245, 183.597385602301, 16.056913646927836),
    (7197, 60.0, 16384, 0.228, 207.84609690826525, 16.833903442913364),
    (13895, 68.0, 16384, 0.2315, 235.5589098293673, 17.66806182606335),
    (26827, 77.0, 16384, 0.2351, 266.7358243656071, 18.48685992293717),
    (51795, 90.0, 16384, 0.2396, 311.7691453623979, 19.576226336846226),
    (100000, 105.0, 16384, 0.244, 363.7306695894642, 20.736774899464613),
)
CONFIG5_RATE = 200.0            # requests per second
CONFIG5_L = (10, 200)
CONFIG5_P = (10_000, 1_000_000)

CONFIGS = {1: CONFIG1, 2: CONFIG2, 3: CONFIG3, 4: CONFIG4}


@dataclass
class Workload:
    cfg: Config
    protein_positions: np.ndarray   # (N, 3)
    protein_charges: np.ndarray     # (N,)
    ligand_positions: np.ndarray    # (L, 3)
    ligand_charges: np.ndarray      # (L,)
    quats: np.ndarray               # (P, 4) (w, x, y, z)
    trans: np.ndarray               # (P, 3)


def make(cfg: Config, P: int | None = None, **overrides) -> Workload:
    """Seeded inputs for ``cfg``; ``P`` keeps the first P poses of the full pose stream."""
    if overrides:
        cfg = replace(cfg, **overrides)
    c = cfg.index
    prot = gen.ball_points(gen.rng(c, 1), cfg.N, cfg.protein_radius)
    z = gen.charges(gen.rng(c, 2), cfg.N, cfg.protein_charge_std, net_zero=True)
    lig = gen.ball_points(gen.rng(c, 3), cfg.L, cfg.ligand_radius)
    zeta = gen.charges(gen.rng(c, 4), cfg.L, cfg.ligand_charge_std, net_zero=False)
    q = gen.unit_quaternions(gen.rng(c, 5), cfg.P)
    if cfg.pose_kind == "sphere":
        t = gen.sphere_translations(gen.rng(c, 6), cfg.P, cfg.pose_r_in)
    else:
        t = gen.shell_translations(gen.rng(c, 6), cfg.P, cfg.pose_r_in, cfg.pose_r_out)
    if P is not None:
        q, t = q[:P].copy(), t[:P].copy()
    return Workload(cfg, prot, z, lig, zeta, q, t)


def make_pairs(pairs: int = CONFIG3_PAIRS, pose_scale: float = 1.0) -> list:
    """Config 3 workload: `pairs` Workloads with their own protein, ligand and pose count.

    Sizes and counts come from stream 7; pair i draws its atoms, charges and poses from
    streams 1-6 with item index i.  pose_scale shrinks every pose count (tests)."""
    cfg = CONFIG3
    g = gen.rng(3, 7)
    Ns = np.exp(g.uniform(np.log(CONFIG3_N[0]), np.log(CONFIG3_N[1]), pairs)).astype(int)
    Ls = g.integers(CONFIG3_L[0], CONFIG3_L[1] + 1, pairs)
    Ps = np.exp(g.uniform(np.log(CONFIG3_P[0]), np.log(CONFIG3_P[1]), pairs)).astype(int)
    out = []
    for i in range(pairs):
        N, L = int(Ns[i]), int(Ls[i])
        P = max(1, int(Ps[i] * pose_scale))
        rp = gen.protein_radius(N, 0.05)
        rl = 6.0 * (L / 50.0) ** (1.0 / 3.0)
        c = replace(cfg, N=N, protein_radius=rp, L=L, ligand_radius=rl, P=P, pose_r_in=rp + 5.0,
                    pose_r_out=rp + 15.0, name=f"cfg3-pair{i}")
        prot = gen.ball_points(gen.rng(3, 1, i), N, rp)
        z = gen.charges(gen.rng(3, 2, i), N, cfg.protein_charge_std, net_zero=True)
        lig = gen.ball_points(gen.rng(3, 3, i), L, rl)
        zeta = gen.charges(gen.rng(3, 4, i), L, cfg.ligand_charge_std, net_zero=False)
        q = gen.unit_quaternions(gen.rng(3, 5, i), P)
        t = gen.shell_translations(gen.rng(3, 6, i), P, c.pose_r_in, c.pose_r_out)
        out.append(Workload(c, prot, z, lig, zeta, q, t))
    return out


def config5_protein(i: int) -> Config:
    """Config of resident protein i (0..7) of the serving workload (no poses of its own)."""
    N, b, n, h_M, L_s, r_cut = CONFIG5_PROTEINS[i]
    rp = gen.protein_radius(N, 0.05)
    return Config(index=5, name=f"cfg5-protein{i}-N{N}-n{n}", N=N, protein_radius=rp, protein_charge_std=0.4, L=0,
                  ligand_radius=0.0, ligand_charge_std=0.4, n=n, b=b, M=32, h_M=h_M, L_s=L_s, K_long=22,
                  r_cut=r_cut, eps=1e-8, P=0, pose_kind="shell", pose_r_in=rp + 5.0, pose_r_out=rp + 15.0, sigma=2.5)


def make_serving_proteins(count: int = 8) -> list:
    """The resident proteins of config 5: (Config, positions, charges); protein i uses item i of streams 1-2."""
    out = []
    for i in range(count):
        c = config5_protein(i)
        pos = gen.ball_points(gen.rng(5, 1, i), c.N, c.protein_radius)
        z = gen.charges(gen.rng(5, 2, i), c.N, c.protein_charge_std, net_zero=True)
        out.append((c, pos, z))
    return out


@dataclass
class ServingRequest:
    index: int
    arrival: float                  # seconds after the start of the trace
    protein: int
    ligand_positions: np.ndarray    # (L, 3)
    ligand_charges: np.ndarray      # (L,)
    quats: np.ndarray               # (P, 4)
    trans: np.ndarray               # (P, 3)
    sigma: float = 2.5


def make_serving_trace(count: int, rate: float = CONFIG5_RATE, proteins: int = 8, pose_scale: float = 1.0,
                       first: int = 0, seed_offset: int = 0) -> list:
    """Requests `first`..`first+count-1` of the config-5 stream (arrivals rescaled to `rate`).

    Sizes come from stream 7 and inter-arrival gaps (unit rate, divided by `rate`) from stream 8,
    both drawn for the whole prefix so that a request is the same whatever `count` is; request j
    draws its ligand and poses from streams 3-6 with item j.  `seed_offset` selects an
    independent trace (rate sweeps); `pose_scale` shrinks every pose count (tests)."""
    total = first + count
    g7 = gen.rng(5 + 100 * seed_offset, 7)
    prot = g7.integers(0, proteins, total)
    Ls = g7.integers(CONFIG5_L[0], CONFIG5_L[1] + 1, total)
    Ps = np.exp(g7.uniform(np.log(CONFIG5_P[0]), np.log(CONFIG5_P[1]), total)).astype(int)
    gaps = gen.rng(5 + 100 * seed_offset, 8).exponential(1.0, total)
    arr = np.cumsum(gaps) / rate
    out = []
    for j in range(first, total):
        c = config5_protein(int(prot[j]))
        L = int(Ls[j])
        P = max(1, int(Ps[j] * pose_scale))
        item = j + 1_000_000 * seed_offset
        lig = gen.ball_points(gen.rng(5, 3, item), L, 6.0 * (L / 50.0) ** (1.0 / 3.0))
        zeta = gen.charges(gen.rng(5, 4, item), L, 0.4, net_zero=False)
        q = gen.unit_quaternions(gen.rng(5, 5, item), P)
        t = gen.shell_translations(gen.rng(5, 6, item), P, c.pose_r_in, c.pose_r_out)
        out.append(ServingRequest(j, float(arr[j]), int(prot[j]), lig, zeta, q, t))
    return out
