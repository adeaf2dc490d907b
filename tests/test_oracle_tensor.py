"""Pins of the oracle's grid, separable factors and RHOSVD (eqs. 2.1-2.6, Algorithm TEP)."""
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
