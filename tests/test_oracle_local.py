"""Pins of the restricted and recompressed long-range tensor (Sec. 3.3, schemes (B)/(C), Table 3.1)."""
import numpy as np
import pytest

from oracle import local, rhosvd, score, sinc, tensor
from workloads import generators as gen

M, H_M, L_S, K = 24, 0.2622, 83.13843876330611, 12
T, W = sinc.sinc_table(M, H_M, L_S)
TL, WL = T[:K], W[:K]
N_GRID, B_BOX = 128, 24.0
CENTRE = np.array([17.0, 3.0, -2.0])     # a site next to the cluster (radius 12 A)


@pytest.fixture(scope="module")
def glob():
    pos = gen.ball_points(gen.rng(7, 1), 200, 12.0)
    z = gen.charges(gen.rng(7, 2), 200, 0.3, True)
    tk, can = rhosvd.build(z, pos, TL, WL, N_GRID, B_BOX, 1e-8)
    return pos, z, can


def _points(lo, hi, count, seed):
    return np.random.default_rng(seed).uniform(lo, hi, size=(count, 3))


def test_restriction_is_exact(glob):
    _, _, can = glob
    lo, hi = CENTRE - 5.0, CENTRE + 5.0
    r = local.restrict(can.F, N_GRID, B_BOX, lo, hi)
    # node for node, the restricted factors are the global rows
    for d in range(3):
        i_lo, i_hi = r.rows[d]
        assert np.array_equal(r.F[d], can.F[d][i_lo:i_hi + 1])
        _, _, _, nodes = tensor.grid(N_GRID, B_BOX)
        assert r.X0s[d] == nodes[i_lo] and r.ns[d] == i_hi - i_lo + 1
    # and inside the sub-box it evaluates like the global tensor (rounding of s = (y - X0) / h aside)
    y = _points(lo, hi, 500, 1)
    v_glob, ins_g, *_ = score.long_range(can.F, N_GRID, B_BOX, y)
    v_loc, ins_l, *_ = score.long_range(r.F, N_GRID, B_BOX, y, grid_spec=r.grid_spec)
    assert ins_g.all() and ins_l.all()
    assert np.max(np.abs(v_loc - v_glob)) <= 1e-13 * np.max(np.abs(v_glob))


def test_recompression_without_truncation_is_exact(glob):
    _, _, can = glob
    r = local.restrict(can.F, N_GRID, B_BOX, CENTRE - 3.0, CENTRE + 3.0)
    tk, rc = local.recompress(r.F, 1e-15)
    A = tensor.materialize_canonical(*r.F)
    B = tensor.materialize_canonical(*rc.F)
    assert np.max(np.abs(A - B)) <= 1e-12 * np.max(np.abs(A))


@pytest.mark.parametrize("half", [3.0, 8.0])
def test_recompression_error_within_the_rhosvd_bound(glob, half):
    _, _, can = glob
    r = local.restrict(can.F, N_GRID, B_BOX, CENTRE - half, CENTRE + half)
    tk, rc = local.recompress(r.F, 1e-8)
    A = tensor.materialize_canonical(*r.F)
    B = tensor.materialize_canonical(*rc.F)
    err = float(np.sqrt(np.sum((A - B) ** 2)))
    assert err <= tk.bound + rc.dropped_fro
    assert err <= 1e-5 * float(np.sqrt(np.sum(A * A)))


def test_local_rank_is_much_smaller_than_global(glob):
    """Table 3.1: the rank of the potential restricted to a small box next to the cluster is a
    fraction of the global RS rank, and grows with the box."""
    _, _, can = glob
    Rs = []
    for half in (3.0, 5.0, 8.0):
        r = local.restrict(can.F, N_GRID, B_BOX, CENTRE - half, CENTRE + half)
        Rs.append(local.recompress(r.F, 1e-8)[1].R)
    assert Rs[0] < Rs[1] < Rs[2] < can.R
    assert Rs[0] * 3 < can.R


def test_scoring_in_the_box_matches_the_global_tensor(glob):
    pos, z, can = glob
    half = 8.0
    r = local.restrict(can.F, N_GRID, B_BOX, CENTRE - half, CENTRE + half)
    tk, rc = local.recompress(r.F, 1e-8)
    (_, _), (ts, ws) = sinc.split(T, W, K)
    r_cut = 43.836027469049675
    lig = gen.ball_points(gen.rng(8, 3), 12, 4.0)
    zeta = gen.charges(gen.rng(8, 4), 12, 0.3, False)
    q = gen.unit_quaternions(gen.rng(8, 5), 64)
    t = CENTRE[None, :] + gen.sphere_translations(gen.rng(8, 6), 64, 2.0)   # within 2 A of the site
    ref = score.score(can.F, N_GRID, B_BOX, pos, z, ts, ws, r_cut, zeta, lig, q, t, 2.5)
    loc = score.score(rc.F, N_GRID, B_BOX, pos, z, ts, ws, r_cut, zeta, lig, q, t, 2.5, grid_spec=r.grid_spec)
    assert np.all(loc["flags"] & 2)
    assert np.array_equal(loc["flags"], ref["flags"]) and np.array_equal(loc["counts"], ref["counts"])
    # each lerped value is a convex combination of node values: the pointwise error is at most
    # the largest node error, which the Frobenius bound covers
    bound = np.sum(np.abs(zeta)) * (tk.bound + rc.dropped_fro)
    assert np.max(np.abs(loc["E"] - ref["E"])) <= bound



def test_complex_of_two_molecules_is_the_sum():
    """Eq. 5.1: a ligand scored against a complex gets the sum of its energies against each
    molecule (long range by linearity, short range and counts over the union of the atoms);
    add-and-compress keeps the sum within the RHOSVD bound."""
    pa = gen.ball_points(gen.rng(11, 1), 120, 9.0) + np.array([-9.0, 0.0, 0.0])
    pb = gen.ball_points(gen.rng(12, 1), 90, 8.0) + np.array([9.0, 2.0, 0.0])
    za = gen.charges(gen.rng(11, 2), 120, 0.3, True)
    zb = gen.charges(gen.rng(12, 2), 90, 0.3, True)
    _, ca = rhosvd.build(za, pa, TL, WL, N_GRID, B_BOX, 1e-8)
    _, cb = rhosvd.build(zb, pb, TL, WL, N_GRID, B_BOX, 1e-8)
    Fsum, (tk, cc) = local.combine([ca.F, cb.F], 1e-8)
    assert Fsum[0].shape[1] == ca.R + cb.R and cc.R < ca.R + cb.R
    idx = np.random.default_rng(2).integers(0, N_GRID, size=(3000, 3))
    at = lambda F: np.sum(F[0][idx[:, 0]] * F[1][idx[:, 1]] * F[2][idx[:, 2]], axis=1)  # noqa: E731
    exact = at(ca.F) + at(cb.F)
    assert np.max(np.abs(at(Fsum) - exact)) <= 1e-14 * np.max(np.abs(exact))
    assert np.max(np.abs(at(cc.F) - exact)) <= tk.bound + cc.dropped_fro
    # energies: complex = molecule A + molecule B (long range to the truncation, the rest exactly)
    (_, _), (ts, ws) = sinc.split(T, W, K)
    r_cut = 43.836027469049675
    lig = gen.ball_points(gen.rng(13, 3), 10, 3.5)
    zeta = gen.charges(gen.rng(13, 4), 10, 0.3, False)
    q = gen.unit_quaternions(gen.rng(13, 5), 32)
    t = np.array([0.0, 14.0, 0.0])[None, :] + gen.sphere_translations(gen.rng(13, 6), 32, 2.0)
    ea = score.score(ca.F, N_GRID, B_BOX, pa, za, ts, ws, r_cut, zeta, lig, q, t, 2.5)
    eb = score.score(cb.F, N_GRID, B_BOX, pb, zb, ts, ws, r_cut, zeta, lig, q, t, 2.5)
    ec = score.score(cc.F, N_GRID, B_BOX, np.vstack([pa, pb]), np.concatenate([za, zb]), ts, ws, r_cut, zeta, lig,
                     q, t, 2.5)
    assert np.array_equal(ec["counts"], ea["counts"] + eb["counts"])
    assert np.array_equal(ec["flags"] & 1, (ea["flags"] & 1) & (eb["flags"] & 1))
    bound = np.sum(np.abs(zeta)) * (tk.bound + cc.dropped_fro) + 1e-12
    assert np.max(np.abs(ec["E"] - (ea["E"] + eb["E"]))) <= bound
