"""Pins of the oracle's snapped build: the shift-and-window transform of eq. 2.5, in which every
charge is moved to its nearest grid point and the reference tensor of a single charge, held on a
twice larger grid, is shifted there and restricted to the computational grid.

  * charges already on grid points: the shifted reference equals the collocated (or, with cell
    averages, the Galerkin) columns at the true positions;
  * snapping moves every coordinate by at most h/2 to a node;
  * the energy of the snapped tensor is the direct Coulomb energy of the snapped charges up to the
    second-order interpolation error, so against the true positions it errs to first order in h:
    the error halves with every doubling of the grid, as in Table 3.2's error column.
"""
import math

import numpy as np

from oracle import constants, direct, rhosvd, score, sinc, tensor


def _quadrature(b, M=24, K=12):
    L_s = constants.scale_length(b)
    h_M = constants.optimal_step(M, b)
    t, w = sinc.sinc_table(M, h_M, L_s)
    (tl, wl), (ts, ws) = sinc.split(t, w, K)
    return tl, wl, ts, ws, constants.short_cutoff(M, h_M, L_s, K)


def test_snapping_moves_to_the_nearest_node():
    n, b = 64, 8.0
    h, X0, _, nodes = tensor.grid(n, b)
    g = np.random.default_rng(5)
    x = g.uniform(X0, X0 + (n - 1) * h, 2000)
    j = tensor.snap_to_nodes(x, n, b)
    assert np.all(np.abs(nodes[j] - x) <= 0.5 * h * (1 + 1e-12))
    assert np.array_equal(tensor.snap_to_nodes(nodes, n, b), np.arange(n))      # nodes stay
    assert tensor.snap_to_nodes(np.array([-1e3, 1e3]), n, b).tolist() == [0, n - 1]   # clipped to the grid


def test_shift_and_window_equals_collocation_on_nodes():
    n, b = 48, 8.0
    tl, _, _, _, _ = _quadrature(b)
    _, _, _, nodes = tensor.grid(n, b)
    g = np.random.default_rng(6)
    coord = nodes[g.integers(0, n, 40)]
    h = (2.0 * b) / n
    for gal in (False, True):
        a = tensor.shifted_columns(coord, tl, n, b, galerkin=gal)
        if gal:
            c = tensor.galerkin_columns(coord, tl, nodes, h)
        else:
            c = tensor.factor_columns(coord, tl, nodes)
        assert a.shape == c.shape == (n, 40, tl.size)
        # equal up to the rounding of the Gaussian's argument ((i - j) h against X_i - X_j)
        assert np.max(np.abs(a - c)) <= 1e-13


def test_off_node_charges_take_the_columns_of_their_node():
    n, b = 40, 8.0
    tl, _, _, _, _ = _quadrature(b)
    _, _, _, nodes = tensor.grid(n, b)
    x = np.array([nodes[7] + 0.3 * (nodes[1] - nodes[0]), nodes[20] - 0.49 * (nodes[1] - nodes[0])])
    a = tensor.shifted_columns(x, tl, n, b)
    c = tensor.factor_columns(nodes[[7, 20]], tl, nodes)
    assert np.max(np.abs(a - c)) <= 1e-13


def test_snapped_energy_is_first_order_like_table_3_2():
    """Two charges 3 a.u. apart (the caption's setting; charge product -1/sqrt(2)), the source
    at a fixed fraction 0.3 of a cell off its node on every axis, so snapping moves it by -0.3 h
    per axis at every n: the energy error against the true positions halves per grid doubling,
    while against the snapped positions it is the small second-order interpolation error."""
    b = 8.0
    tl, wl, ts, ws, r_cut = _quadrature(b)
    zeta = -1.0 / math.sqrt(2.0)
    d = np.full(3, math.sqrt(3.0))                       # 3 a.u. along the diagonal
    errs, errs_snap = [], []
    for n in (32, 64, 128, 256):
        h, _, _, nodes = tensor.grid(n, b)
        src = np.full(3, nodes[n // 2 - 1] + 0.3 * h)     # node n/2 - 1 is the origin; 0.3 h off it
        src = src[None, :]
        lig = src + d[None, :]
        _, can = rhosvd.build(np.ones(1), src, tl, wl, n, b, 1e-12, snapped=True)
        out = score.score(can.F, n, b, src, np.ones(1), ts, ws, r_cut, np.array([zeta]), np.zeros((1, 3)),
                          np.array([[1.0, 0.0, 0.0, 0.0]]), lig, 0.5)
        E = out["E"][0]
        # the short-range part is exact at the true distance; only the long-range part is snapped
        e_true = direct.energies(src, np.ones(1), np.array([zeta]), np.zeros((1, 3)),
                                 np.array([[1.0, 0.0, 0.0, 0.0]]), lig)[0]
        snapped = tensor.snapped_positions(src, n, b)
        assert np.allclose(snapped - src, -0.3 * h, rtol=0, atol=1e-12)
        # reference for the snapped long range: direct long-range Gaussians from the snapped charge
        # plus the short range at the true distance
        el_snap = zeta * tensor.long_range_continuous(np.ones(1), snapped, tl, wl, lig)[0]
        es_true = zeta * tensor.long_range_continuous(np.ones(1), src, ts, ws, lig)[0]
        errs.append(abs(E - e_true))
        errs_snap.append(abs(E - (el_snap + es_true)))
    ratios = [a / c for a, c in zip(errs, errs[1:])]
    assert all(1.8 <= q <= 2.2 for q in ratios), (errs, ratios)          # first order, like Table 3.2
    # against the snapped charge: second order (the trilinear interpolation), a small part of the above
    assert all(a / c >= 3.5 for a, c in zip(errs_snap, errs_snap[1:])), errs_snap
    assert all(es < 0.1 * e for es, e in zip(errs_snap, errs)), (errs_snap, errs)


def test_snapped_rhosvd_within_its_bound():
    n, b = 32, 8.0
    tl, wl, _, _, _ = _quadrature(b)
    g = np.random.default_rng(7)
    pos = g.uniform(-3.0, 3.0, size=(25, 3))
    z = g.normal(0.0, 0.4, 25)
    z -= z.mean()
    tk, can = rhosvd.build(z, pos, tl, wl, n, b, 1e-8, snapped=True)
    idx = g.integers(0, n, size=(400, 3))
    T0 = tensor.long_range_at_nodes(z, tensor.snapped_positions(pos, n, b), tl, wl, n, b, idx)
    Tc = np.sum(can.F[0][idx[:, 0]] * can.F[1][idx[:, 1]] * can.F[2][idx[:, 2]], axis=1)
    assert np.max(np.abs(Tc - T0)) <= tk.bound + can.dropped_fro + 1e-13
    assert np.max(np.abs(Tc - T0)) <= 1e-6 * np.max(np.abs(T0))
