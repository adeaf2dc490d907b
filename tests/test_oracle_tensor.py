"""Pins of the oracle's grid, separable factors and RHOSVD (eqs. 2.1-2.6, Algorithm TEP)."""
import math

import numpy as np
import pytest

from oracle import rhosvd, sinc, tensor
from workloads import generators as gen

M, H_M, L_S, K = 24, 0.2622, 83.13843876330611, 12
T, W = sinc.sinc_table(M, H_M, L_S)
TL, WL = T[:K], W[:K]


def _protein(N, radius=6.0, seed=7):
    pos = gen.ball_points(gen.rng(seed, 1), N, radius)
    z = gen.charges(gen.rng(seed, 2), N, 0.3, True)
    return pos, z


def test_grid_nodes_and_origin():
    h, X0, inv_h, nodes = tensor.grid(64, 8.0)
    assert h == 0.25 and X0 == -7.75 and inv_h == 4.0
    assert nodes[0] == X0 and nodes[-1] == 8.0
    assert nodes[64 // 2 - 1] == 0.0     # the paper's node n/2 (1-based) is the origin


def test_separable_factors_equal_3d_gaussian_sum():
    """Each Gaussian exp(-t^2|x|^2) is the product of three 1-D factors (eq. 2.2)."""
    pos, z = _protein(15)
    n, b = 20, 8.0
    F = rhosvd.uncompressed_factors(z, pos, TL, WL, n, b)
    T0 = tensor.materialize_canonical(*F)
    _, _, _, X = tensor.grid(n, b)
    gx, gy, gz = np.meshgrid(X, X, X, indexing="ij")
    pts = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    direct = np.zeros(pts.shape[0])
    for m in range(pos.shape[0]):
        r2 = np.sum((pts - pos[m]) ** 2, axis=1)
        direct += z[m] * np.exp(-np.outer(r2, TL * TL)) @ WL
    scale = np.sum(np.abs(z)) * WL.sum()
    assert np.max(np.abs(T0.ravel() - direct)) <= 1e-14 * scale
    idx = np.array([[0, 0, 0], [3, 7, 11], [19, 19, 19], [10, 0, 5]])
    at = tensor.long_range_at_nodes(z, pos, TL, WL, n, b, idx)
    assert np.allclose(at, T0[idx[:, 0], idx[:, 1], idx[:, 2]], rtol=0, atol=1e-14 * scale)


def test_integer_h_joint_shift():
    """Shifting the protein by whole mesh steps shifts the tensor by whole indices."""
    pos, z = _protein(12)
    n, b = 32, 8.0
    h = 2 * b / n
    s = np.array([2, -3, 1])
    idx = np.array([[10, 10, 10], [12, 15, 9], [5, 20, 14], [16, 16, 16]])
    a = tensor.long_range_at_nodes(z, pos, TL, WL, n, b, idx)
    bb = tensor.long_range_at_nodes(z, pos + s * h, TL, WL, n, b, idx + s)
    assert np.allclose(a, bb, rtol=0, atol=1e-13 * np.sum(np.abs(z)) * WL.sum())


def test_rhosvd_error_within_bound_and_t2c_exact_tail():
    pos, z = _protein(30)
    n, b, eps = 24, 8.0, 1e-6
    T0 = tensor.materialize_canonical(*rhosvd.uncompressed_factors(z, pos, TL, WL, n, b))
    tk, can = rhosvd.build(z, pos, TL, WL, n, b, eps)
    Tt = np.einsum("abc,ia,jb,kc->ijk", tk.core, tk.U[0], tk.U[1], tk.U[2], optimize=True)
    err_t = np.linalg.norm((T0 - Tt).ravel())
    assert err_t <= tk.bound
    assert tk.bound < 1e-4 * np.linalg.norm(T0.ravel())
    Tc = tensor.materialize_canonical(*can.F)
    # Tucker -> canonical drops exactly the small slice singular values (orthonormal U_d)
    assert abs(np.linalg.norm((Tt - Tc).ravel()) - can.dropped_fro) <= 1e-12 * np.linalg.norm(T0.ravel())
    for d in range(3):
        assert np.allclose(tk.U[d].T @ tk.U[d], np.eye(tk.ranks[d]), atol=1e-12)


def test_rhosvd_no_truncation_is_exact():
    pos, z = _protein(6)
    n, b = 16, 8.0
    T0 = tensor.materialize_canonical(*rhosvd.uncompressed_factors(z, pos, TL, WL, n, b))
    tk, can = rhosvd.build(z, pos, TL, WL, n, b, 0.0)
    Tc = tensor.materialize_canonical(*can.F)
    assert np.max(np.abs(T0 - Tc)) <= 1e-13 * np.max(np.abs(T0))


def test_tucker_ranks_match_hosvd_of_unfoldings():
    """RHOSVD's subspaces hold the HOSVD subspaces of the materialised tensor."""
    pos, z = _protein(25)
    n, b, eps = 24, 8.0, 1e-8
    T0 = tensor.materialize_canonical(*rhosvd.uncompressed_factors(z, pos, TL, WL, n, b))
    tk = rhosvd.rhosvd(z, pos, TL, WL, n, b, eps)
    for d in range(3):
        unf = np.moveaxis(T0, d, 0).reshape(n, -1)
        Uh, sh, _ = np.linalg.svd(unf, full_matrices=False)
        r = int(np.count_nonzero(sh >= 1e-6 * sh[0]))
        # leading HOSVD vectors lie in span(U_d) up to the truncation level
        resid = Uh[:, :r] - tk.U[d] @ (tk.U[d].T @ Uh[:, :r])
        assert np.linalg.norm(resid, 2) < 1e-3


@pytest.mark.slow
def test_rank_nearly_independent_of_cluster_size():
    """Thm 2.2: the Tucker rank of the long-range sum barely grows with the number of particles."""
    ranks = []
    Rs = []
    for N in (25, 100, 400):
        pos = gen.ball_points(gen.rng(99, 1), N, 12.0)
        z = gen.charges(gen.rng(99, 2), N, 0.3, True)
        tk = rhosvd.rhosvd(z, pos, TL, WL, 128, 24.0, 1e-8)
        ranks.append(max(tk.ranks))
        Rs.append(rhosvd.tucker_to_canonical(tk, 1e-8).R)
    assert max(ranks) <= min(ranks) + 2
    assert max(Rs) <= 1.25 * min(Rs)


def test_galerkin_columns_are_cell_averages():
    """Eq. 2.1's piecewise-constant projection as cell averages: against adaptive quadrature of
    the Gaussian over each cell, for wide, narrow and constant (t = 0) terms, centres on and off
    the cell and far out in the tail."""
    from scipy.integrate import quad
    n, b = 64, 8.0
    h, _, _, nodes = tensor.grid(n, b)
    t_long = np.array([0.0, 1e-4, 0.03, 0.4, 2.5, 9.0])
    coord = np.array([0.0, 0.1234, -3.3, 7.9])
    G = tensor.galerkin_columns(coord, t_long, nodes, h)
    for j in (0, 5, 31, 32, 40, 63):
        for m, x in enumerate(coord):
            for k, t in enumerate(t_long):
                f = lambda s: math.exp(-(t * (s - x)) ** 2)  # noqa: E731
                ref = quad(f, nodes[j] - h / 2, nodes[j] + h / 2, epsabs=0.0, epsrel=1e-13, limit=200)[0] / h
                assert G[j, m, k] == pytest.approx(ref, rel=1e-10, abs=1e-300)


def test_galerkin_minus_collocation_is_second_order():
    """The cell average exceeds the node value by f''(X) h^2 / 24 + O(h^4): halving h quarters the
    difference, and the leading term matches."""
    t = np.array([0.3])
    x = np.array([0.37])
    diffs = []
    for n in (32, 64, 128):
        h, _, _, nodes = tensor.grid(n, 8.0)
        g = tensor.galerkin_columns(x, t, nodes, h)[:, 0, 0]
        c = tensor.factor_columns(x, t, nodes)[:, 0, 0]
        a = t[0] * (nodes - x[0])
        lead = (4.0 * a * a - 2.0) * np.exp(-a * a) * (t[0] * h) ** 2 / 24.0
        assert np.max(np.abs(g - c - lead)) <= 0.1 * np.max(np.abs(lead)) + 1e-15
        diffs.append(np.max(np.abs(g - c)))
    assert 3.5 < diffs[0] / diffs[1] < 4.5 and 3.5 < diffs[1] / diffs[2] < 4.5


def test_galerkin_build_within_the_rhosvd_bound():
    """RHOSVD of the Galerkin side matrices: the canonical tensor against the uncompressed
    Galerkin sum at sampled nodes, within the bound of the truncation."""
    n, b = 64, 12.0
    pos = gen.ball_points(gen.rng(90, 1), 30, 6.0)
    z = gen.charges(gen.rng(90, 2), 30, 0.3, True)
    tk, can = rhosvd.build(z, pos, TL, WL, n, b, 1e-8, galerkin=True)
    h, _, _, nodes = tensor.grid(n, b)
    G = [tensor.galerkin_columns(pos[:, d], TL, nodes, h) for d in range(3)]     # (n, N, K)
    idx = np.random.default_rng(4).integers(0, n, size=(400, 3))
    exact = np.einsum("m,k,qmk,qmk,qmk->q", z, WL, G[0][idx[:, 0]], G[1][idx[:, 1]], G[2][idx[:, 2]])
    approx = np.sum(can.F[0][idx[:, 0]] * can.F[1][idx[:, 1]] * can.F[2][idx[:, 2]], axis=1)
    assert np.max(np.abs(approx - exact)) <= tk.bound + can.dropped_fro
    # and it differs from the collocated build by the O(h^2) cell-average correction only
    _, col = rhosvd.build(z, pos, TL, WL, n, b, 1e-8)
    colv = np.sum(col.F[0][idx[:, 0]] * col.F[1][idx[:, 1]] * col.F[2][idx[:, 2]], axis=1)
    assert 0 < np.max(np.abs(approx - colv)) <= 0.05 * np.max(np.abs(colv))
