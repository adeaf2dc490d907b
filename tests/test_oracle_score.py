"""Pins of the oracle's scoring: pose transform, trilinear long-range evaluation,
short-range sum, energy, vdW flag, counts and gradients."""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator
from scipy.spatial.transform import Rotation

from oracle import constants, direct, rhosvd, score, sinc, tensor
from workloads import generators as gen

M, H_M, L_S = 24, 0.2622, 83.13843876330611
T, W = sinc.sinc_table(M, H_M, L_S)


class Small:
    """A small system: 40-atom protein, 6-atom ligand, box [-16,16]^3."""

    def __init__(self, n=128, K_long=16, eps=1e-10, P=24, seed=11, uncompressed=False):
        self.n, self.b, self.K = n, 16.0, K_long
        self.pos = gen.ball_points(gen.rng(seed, 1), 40, 5.0)
        self.z = gen.charges(gen.rng(seed, 2), 40, 0.3, True)
        self.lig = gen.ball_points(gen.rng(seed, 3), 6, 2.5)
        self.zeta = gen.charges(gen.rng(seed, 4), 6, 0.3, False)
        self.q = gen.unit_quaternions(gen.rng(seed, 5), P)
        self.t = gen.sphere_translations(gen.rng(seed, 6), P, 9.0)
        (self.tl, self.wl), (self.ts, self.ws) = sinc.split(T, W, K_long)
        self.rc = constants.short_cutoff(M, H_M, L_S, K_long) if K_long <= M else 0.0
        if K_long == 0:
            self.F = [np.zeros((n, 0))] * 3
        elif uncompressed:
            self.F = rhosvd.uncompressed_factors(self.z, self.pos, self.tl, self.wl, n, self.b)
        else:
            self.F = rhosvd.build(self.z, self.pos, self.tl, self.wl, n, self.b, eps)[1].F

    def score(self, q=None, t=None, grad=False, rc=None, sigma=2.5):
        return score.score(self.F, self.n, self.b, self.pos, self.z, self.ts, self.ws,
                           self.rc if rc is None else rc, self.zeta, self.lig,
                           self.q if q is None else q, self.t if t is None else t, sigma, want_grad=grad)

    def direct(self, q=None, t=None, grad=False):
        return direct.energies(self.pos, self.z, self.zeta, self.lig,
                               self.q if q is None else q, self.t if t is None else t, want_grad=grad)


def test_rotation_matrix_is_a_rotation_and_matches_scipy():
    q = gen.unit_quaternions(gen.rng(5, 5), 200)
    R = score.rotation_matrix(q)
    eye = np.einsum("pji,pjk->pik", R, R)
    assert np.max(np.abs(eye - np.eye(3))) < 4e-16 * 8
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-14)
    ref = Rotation.from_quat(np.stack([q[:, 1], q[:, 2], q[:, 3], q[:, 0]], axis=1)).as_matrix()
    assert np.max(np.abs(R - ref)) < 1e-15 * 4
    assert np.array_equal(score.rotation_matrix(-q), R)          # q and -q: identical, bit for bit


def test_axis_angle_rotation_matches_rodrigues():
    axis = np.array([1.0, -2.0, 0.5]) / np.linalg.norm([1.0, -2.0, 0.5])
    ang = 0.7
    q = np.array([[math.cos(ang / 2), *(math.sin(ang / 2) * axis)]])
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    rod = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    assert np.max(np.abs(score.rotation_matrix(q)[0] - rod)) < 1e-15 * 4


def test_ligand_frame_centre():
    lig = gen.ball_points(gen.rng(3, 3), 50, 6.0) + np.array([1.0, -2.0, 3.0])
    c, u = score.ligand_frame(lig)
    assert np.allclose(c, lig.mean(axis=0), rtol=0, atol=1e-14)
    assert np.max(np.abs(u.sum(axis=0))) < 1e-12


def test_trilinear_matches_regular_grid_interpolator():
    """Per-mode lerp of factor rows == trilinear interpolation of the materialised tensor."""
    n, b = 20, 5.0
    g = np.random.default_rng(0)
    F = [g.normal(size=(n, 7)) for _ in range(3)]
    full = tensor.materialize_canonical(*F)
    _, _, _, X = tensor.grid(n, b)
    interp = RegularGridInterpolator((X, X, X), full, method="linear")
    pts = g.uniform(X[0], X[-1], size=(500, 3))
    pts[:5] = [X[0], X[0], X[0]], [X[-1], X[-1], X[-1]], [X[3], X[7], X[-1]], [X[0], 0.1, X[-1]], [0, 0, 0]
    val, inside, scale, _, _ = score.long_range(F, n, b, pts)
    assert inside.all()
    assert np.max(np.abs(val - interp(pts))) <= 1e-13 * np.max(scale)
    out = np.array([[X[0] - 1e-9, 0, 0], [0, X[-1] + 1e-9, 0], [0, 0, 1e9], [np.nan, 0, 0]])
    val, inside, _, _, _ = score.long_range(F, n, b, out)
    assert not inside.any() and np.isnan(val).all()


def test_short_only_energy_equals_gaussian_sum_coulomb():
    """With every term short-range and an unbounded cutoff, E is the Gaussian-sum Coulomb energy,
    within the quadrature error (3.2e-8 relative per pair for 1 A <= r <= L_s) of the direct sum."""
    s = Small(K_long=0)
    out = s.score(rc=1e6)
    Ed = s.direct()
    _, u = score.ligand_frame(s.lig)
    y = score.transform(s.q, s.t, u)
    for p in range(len(Ed)):
        D = np.sqrt(score.pair_d2(y[p], s.pos))
        assert D.min() >= 1.0
        absum = np.sum(np.abs(s.zeta[:, None] * s.z[None, :]) / D)
        assert abs(out["E"][p] - Ed[p]) <= 3.2e-8 * absum
    assert np.all(out["counts"] == 40 * 6)


def test_all_long_range_has_no_short_part():
    s = Small(K_long=M + 1, eps=1e-12)
    out = s.score()
    assert np.allclose(out["E"], out["E_long"], rtol=0, atol=0)
    assert s.rc == 0.0 and np.all(out["counts"] == 0)


def test_long_range_interpolation_converges_second_order():
    """Trilinear evaluation of the collocated long-range tensor: O(h^2) error vs the continuous sum."""
    pos = gen.ball_points(gen.rng(21, 1), 10, 4.0)
    z = gen.charges(gen.rng(21, 2), 10, 0.3, True)
    tl, wl = T[:12], W[:12]
    g = np.random.default_rng(1)
    pts = g.uniform(-6, 6, size=(400, 3))
    exact = tensor.long_range_continuous(z, pos, tl, wl, pts)
    errs = []
    for n in (32, 64, 128):
        F = rhosvd.uncompressed_factors(z, pos, tl, wl, n, 8.0)
        val = score.long_range(F, n, 8.0, pts)[0]
        errs.append(np.max(np.abs(val - exact)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0


def _brute_flags(pos, y, rc2, sig2):
    cnt, mind = 0, math.inf
    for yl in y:
        for xm in pos:
            a, b_, c = yl[0] - xm[0], yl[1] - xm[1], yl[2] - xm[2]
            d2 = (a * a + b_ * b_) + c * c
            cnt += d2 < rc2
            mind = min(mind, d2)
    return cnt, mind


def test_counts_and_vdw_flag_brute_force():
    s = Small(P=16)
    # pull half of the poses in so that some violate the vdW distance
    t = s.t.copy()
    t[::2] *= 0.55
    out = s.score(t=t)
    _, u = score.ligand_frame(s.lig)
    y = score.transform(s.q, t, u)
    rc2, sig2 = s.rc * s.rc, 2.5 * 2.5
    n_rej = 0
    for p in range(len(t)):
        cnt, mind = _brute_flags(s.pos, y[p], rc2, sig2)
        assert out["counts"][p] == cnt
        acc = bool(out["flags"][p] & score.FLAG_ACCEPT)
        assert out["flags"][p] & score.FLAG_IN_DOMAIN
        assert acc == (mind >= sig2)
        n_rej += not acc
    assert 0 < n_rej < len(t)


def test_invalid_and_out_of_domain_poses():
    s = Small(P=4)
    q = s.q.copy()
    t = s.t.copy()
    q[1] *= 1.0 + 1e-9                  # not a unit quaternion
    t[2] = [100.0, 0.0, 0.0]           # ligand outside the grid
    q[3, 0] = np.nan
    out = s.score(q=q, t=t)
    assert out["flags"][1] == score.FLAG_INVALID and np.isnan(out["E"][1])
    assert out["flags"][3] == score.FLAG_INVALID and np.isnan(out["E"][3])
    assert out["flags"][2] == 0 and np.isnan(out["E"][2])
    assert out["flags"][0] & score.FLAG_IN_DOMAIN and np.isfinite(out["E"][0])


def test_energy_close_to_direct_coulomb():
    s = Small(n=256, eps=1e-10)
    out = s.score()
    Ed = s.direct()
    assert np.all(out["flags"] == 3)
    err = np.abs(out["E"] - Ed)
    # interpolation error of the n=256 grid (h=0.125 A) dominates: ~7e-5 of max|E|
    assert np.max(err) < 1.5e-4 * np.max(np.abs(Ed))


def _rigid(x, Rm, shift):
    return x @ Rm.T + shift


@pytest.mark.slow
def test_joint_rigid_motion_invariance():
    """Moving protein and ligand together leaves E_direct unchanged and the RS energy unchanged
    within twice its own approximation error."""
    s = Small(n=128, eps=1e-10, P=12)
    Rm = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    shift = np.array([0.37, -0.81, 0.55])
    E1, Ed1 = s.score()["E"], s.direct()
    qm = Rotation.from_matrix(Rm).as_quat()              # (x, y, z, w)
    qm = np.array([qm[3], qm[0], qm[1], qm[2]])
    # new ligand orientation: R' = Rm R(q)  -> q' = qm (x) q
    w1, v1 = qm[0], qm[1:]
    w2, v2 = s.q[:, 0], s.q[:, 1:]
    q2 = np.concatenate([(w1 * w2 - v2 @ v1)[:, None],
                         w1 * v2 + w2[:, None] * v1[None, :] + np.cross(v1[None, :], v2)], axis=1)
    t2 = _rigid(s.t, Rm, shift)
    s2 = Small(n=128, eps=1e-10, P=12)
    s2.pos = _rigid(s.pos, Rm, shift)
    s2.F = rhosvd.build(s2.z, s2.pos, s2.tl, s2.wl, s2.n, s2.b, 1e-10)[1].F
    E2, Ed2 = s2.score(q=q2, t=t2)["E"], s2.direct(q=q2, t=t2)
    assert np.max(np.abs(Ed1 - Ed2)) < 1e-12 * np.max(np.abs(Ed1))
    rs_err = max(np.max(np.abs(E1 - Ed1)), np.max(np.abs(E2 - Ed2)))
    assert np.max(np.abs(E1 - E2)) <= 2 * rs_err


def _quat_mul(a, b):
    w1, v1 = a[0], a[1:]
    w2, v2 = b[0], b[1:]
    return np.concatenate([[w1 * w2 - v1 @ v2], w1 * v2 + w2 * v1 + np.cross(v1, v2)])


def _straddles(s, q, t, hfd):
    """True if a +-hfd move of any atom coordinate crosses a grid node (derivative jump)."""
    _, X0, inv_h, _ = tensor.grid(s.n, s.b)
    _, u = score.ligand_frame(s.lig)
    y = score.transform(q[None], t[None], u)[0]
    s_lo = np.floor((y - hfd * 1.5 - X0) * inv_h)
    s_hi = np.floor((y + hfd * 1.5 - X0) * inv_h)
    return bool(np.any(s_lo != s_hi))


@pytest.mark.slow
def test_gradient_matches_central_differences_and_direct_forces():
    s = Small(n=128, eps=1e-10, P=10)
    out = s.score(grad=True)
    _, Gd = s.direct(grad=True)
    hfd = 1e-5
    checked = 0
    for p in range(len(s.q)):
        if _straddles(s, s.q[p], s.t[p], 8 * hfd):
            continue
        fd = np.zeros(6)
        for i in range(3):
            e = np.zeros(3)
            e[i] = hfd
            Ep = s.score(q=s.q[p:p + 1], t=(s.t[p] + e)[None])["E"][0]
            Em = s.score(q=s.q[p:p + 1], t=(s.t[p] - e)[None])["E"][0]
            fd[i] = (Ep - Em) / (2 * hfd)
            dq = np.concatenate([[math.cos(hfd / 2)], math.sin(hfd / 2) * np.eye(3)[i]])
            qp = _quat_mul(dq, s.q[p])
            qm = _quat_mul(np.concatenate([[math.cos(hfd / 2)], -math.sin(hfd / 2) * np.eye(3)[i]]), s.q[p])
            Ep = s.score(q=qp[None], t=s.t[p:p + 1])["E"][0]
            Em = s.score(q=qm[None], t=s.t[p:p + 1])["E"][0]
            fd[3 + i] = (Ep - Em) / (2 * hfd)
        g = out["grads"][p]
        assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(g)) + 1e-9
        checked += 1
    assert checked >= 5


@pytest.mark.slow
def test_gradient_approaches_direct_forces_first_order():
    """The exact derivative of the trilinear interpolant is first-order accurate in h: the error
    against the direct Coulomb rigid-body gradient (force formula of Sec. 3.3) halves per doubling of n."""
    errs = []
    for n in (128, 256):
        s = Small(n=n, eps=1e-10, P=10)
        g = s.score(grad=True)["grads"]
        _, Gd = s.direct(grad=True)
        errs.append(np.max(np.abs(g - Gd)) / np.max(np.abs(Gd)))
    assert errs[1] < 0.05
    assert 1.5 < errs[0] / errs[1] < 3.0


def test_uncompressed_interpolant_equals_canonical_evaluation():
    """The corner-value form of the T0 interpolant equals the per-mode lerp of T0's own factors."""
    s = Small(n=48, uncompressed=True, P=6)
    out_f = s.score(grad=True)
    out_u = score.score_uncompressed(s.z, s.pos, s.tl, s.wl, s.n, s.b, s.ts, s.ws, s.rc, s.zeta, s.lig,
                                     s.q, s.t, 2.5, want_grad=True)
    assert np.array_equal(out_f["flags"], out_u["flags"])
    assert np.array_equal(out_f["counts"], out_u["counts"])
    assert np.allclose(out_u["E"], out_f["E"], rtol=0, atol=1e-12 * np.max(out_f["scale"]))
    assert np.allclose(out_u["grads"], out_f["grads"], rtol=0, atol=1e-11 * np.max(out_f["grad_scale"]))
