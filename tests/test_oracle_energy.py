"""Pins of the molecule's own energy from its RS tensor (Prop. 3.2, eqs. 3.8-3.9)."""
import numpy as np
import pytest

from oracle import constants, energy, rhosvd, score, sinc, tensor
from workloads import generators as gen

M, H_M, L_S = 24, 0.2622, 83.13843876330611
N_GRID, B_BOX = 128, 24.0


def _cluster(seed, count=40, radius=8.0, snap=False, min_sep=gen.MIN_SEPARATION):
    pos = gen.ball_points(gen.rng(seed, 1), count, radius, min_sep)
    z = gen.charges(gen.rng(seed, 2), count, 0.5, True)
    if snap:
        h, X0, inv_h, nodes = tensor.grid(N_GRID, B_BOX)
        pos = nodes[np.rint((pos - X0) * inv_h).astype(int)]
    return pos, z


def _pair_sum(pos, z, t, w):
    """1/2 sum_{j != m} z_j z_m sum_k w_k exp(-t_k^2 d^2), directly over the pairs."""
    D2 = score.pair_d2(pos, pos)
    j, m = np.nonzero(~np.eye(len(z), dtype=bool))
    g = np.exp(-np.outer(D2[j, m], t * t)) @ w
    return 0.5 * float(np.sum(z[j] * z[m] * g))


@pytest.mark.parametrize("K", [8, 12])
def test_self_term_removal_is_exact_on_nodes(K):
    """Atoms on grid nodes and the uncompressed tensor (eq. 2.6): trilinear evaluation returns the
    node values, and removing z_j sum_k w_k leaves exactly the long-range sum over distinct pairs."""
    pos, z = _cluster(80, snap=True)
    T, W = sinc.sinc_table(M, H_M, L_S)
    (tl, wl), (ts, ws) = sinc.split(T, W, K)
    F = rhosvd.uncompressed_factors(z, pos, tl, wl, N_GRID, B_BOX)
    E_long, E_short = energy.self_energy(F, N_GRID, B_BOX, pos, z, wl, ts, ws, 1e9)
    ref_long = _pair_sum(pos, z, tl, wl)
    assert E_long == pytest.approx(ref_long, rel=1e-12, abs=1e-14)
    assert E_short == pytest.approx(_pair_sum(pos, z, ts, ws), rel=1e-12, abs=1e-14)


def test_whole_energy_is_coulomb_within_the_quadrature_error():
    pos, z = _cluster(81, snap=True)
    T, W = sinc.sinc_table(M, H_M, L_S)
    (tl, wl), (ts, ws) = sinc.split(T, W, 12)
    F = rhosvd.uncompressed_factors(z, pos, tl, wl, N_GRID, B_BOX)
    E_long, E_short = energy.self_energy(F, N_GRID, B_BOX, pos, z, wl, ts, ws, 1e9)
    D = np.sqrt(score.pair_d2(pos, pos))
    off = ~np.eye(len(z), dtype=bool)
    eq = sinc.max_rel_error(M, H_M, L_S, float(np.min(D[off])), float(np.max(D[off])))
    bound = 0.5 * float(np.sum((np.abs(np.outer(z, z)) / np.where(off, D, np.inf)))) * eq
    assert abs(E_long + E_short - energy.coulomb(pos, z)) <= bound


def test_sigma_separable_needs_only_the_long_range_part():
    """Prop. 3.2's claim: when the short-range Gaussians end below the smallest pair distance,
    the long-range part alone gives the energy."""
    pos, z = _cluster(82, radius=12.0, snap=True, min_sep=3.0)
    D = np.sqrt(score.pair_d2(pos, pos))
    dmin = float(np.min(D[~np.eye(len(z), dtype=bool)]))
    T, W = sinc.sinc_table(M, H_M, L_S)
    K = next(k for k in range(M + 1) if constants.short_cutoff(M, H_M, L_S, k) < dmin)
    r_cut = constants.short_cutoff(M, H_M, L_S, K)
    (tl, wl), (ts, ws) = sinc.split(T, W, K)
    F = rhosvd.uncompressed_factors(z, pos, tl, wl, N_GRID, B_BOX)
    E_long, E_short = energy.self_energy(F, N_GRID, B_BOX, pos, z, wl, ts, ws, r_cut)
    assert E_short == 0.0 and K < M + 1
    eq = sinc.max_rel_error(M, H_M, L_S, dmin, float(np.max(D)))
    off = ~np.eye(len(z), dtype=bool)
    bound = 0.5 * float(np.sum(np.abs(np.outer(z, z)) / np.where(off, D, np.inf))) * eq + 1e-15
    assert abs(E_long - energy.coulomb(pos, z)) <= bound


def test_off_grid_energy_converges_second_order():
    """Atoms off the grid, RHOSVD tensor: the trilinear interpolation error of the long-range
    potential at the atoms falls about fourfold per halving of h, and the energy error stays
    within sum_j |z_j| times it."""
    pos, z = _cluster(83)
    T, W = sinc.sinc_table(M, H_M, L_S)
    (tl, wl), (ts, ws) = sinc.split(T, W, 12)
    r_cut = constants.short_cutoff(M, H_M, L_S, 12)
    exact_long = _pair_sum(pos, z, tl, wl)
    exact_pot = tensor.long_range_continuous(z, pos, tl, wl, pos)
    errs = []
    for n in (64, 128, 256):
        _, can = rhosvd.build(z, pos, tl, wl, n, B_BOX, 1e-12)
        E_long, E_short = energy.self_energy(can.F, n, B_BOX, pos, z, wl, ts, ws, r_cut)
        v = score.long_range(can.F, n, B_BOX, pos)[0]
        errs.append(float(np.max(np.abs(v - exact_pot))))
        assert abs(E_long - exact_long) <= 0.5 * float(np.sum(np.abs(z))) * errs[-1] + 1e-13
        assert E_short == pytest.approx(_pair_sum(pos, z, ts, ws), rel=1e-12)
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
