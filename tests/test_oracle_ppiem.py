"""Pins of the posing search (Algorithm PPIEM, steps A2-A7)."""
import math

import numpy as np
import pytest

from oracle import ppiem, rhosvd, score, sinc
from workloads import angles, generators as gen

SIGMA = 2.5


def _min_dist(lig, q, t, atoms):
    _, ul = score.ligand_frame(lig)
    y = score.transform(np.atleast_2d(q), np.atleast_2d(t), ul)[0]
    return math.sqrt(float(np.min(score.pair_d2(y, atoms))))


def test_contact_radius_closed_form():
    """One protein atom, one ligand atom: rho* = u.d + sqrt(sigma^2 - |d_perp|^2) with d the atom's
    offset from the centre; a ray passing farther than sigma from the atom never touches it."""
    centre = np.zeros(3)
    atom = np.array([[7.0, 1.5, -0.5]])
    lig = np.array([[0.0, 0.0, 0.0]])
    q = np.array([[1.0, 0.0, 0.0, 0.0]])
    dirs = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    rho = ppiem.contact_radius(lig, q, dirs, centre, atom, SIGMA)
    d = atom[0] - centre
    perp2 = d[1] ** 2 + d[2] ** 2
    assert rho[0, 0] == pytest.approx(d[0] + math.sqrt(SIGMA ** 2 - perp2), rel=1e-15)
    assert rho[1, 0] == -np.inf   # distance from the y-axis ray: sqrt(49 + 0.25) > sigma


def test_contact_is_first_touch_from_outside():
    """On a random cluster: just outside rho* the pose keeps sigma, just inside it does not, and a
    scan of larger radii never comes closer than sigma."""
    atoms = gen.ball_points(gen.rng(70, 1), 150, 10.0)
    lig = gen.ball_points(gen.rng(70, 3), 9, 3.0)
    quats = gen.unit_quaternions(gen.rng(70, 5), 5)
    dirs = angles.orbit_sphere(7)
    xP = ppiem.geometric_centre(atoms)
    rho = ppiem.contact_radius(lig, quats, dirs, xP, atoms, SIGMA)
    assert np.all(np.isfinite(rho)) and np.all(rho > 0)
    for i, u in enumerate(dirs):
        for k, q in enumerate(quats):
            r = rho[i, k]
            assert _min_dist(lig, q, xP + (r + 1e-9) * u, atoms) >= SIGMA
            assert _min_dist(lig, q, xP + (r - 1e-9) * u, atoms) < SIGMA
            assert abs(_min_dist(lig, q, xP + r * u, atoms) - SIGMA) < 1e-9
            for extra in np.linspace(0.01, 25.0, 60):
                assert _min_dist(lig, q, xP + (r + extra) * u, atoms) >= SIGMA


def test_contact_by_scan():
    """A descending scan of the radius stops within one step of rho*."""
    atoms = gen.ball_points(gen.rng(71, 1), 80, 8.0)
    lig = gen.ball_points(gen.rng(71, 3), 6, 2.5)
    q = gen.unit_quaternions(gen.rng(71, 5), 1)
    u = angles.orbit_sphere(3)[1:2]
    xP = ppiem.geometric_centre(atoms)
    rho = ppiem.contact_radius(lig, q, u, xP, atoms, SIGMA)[0, 0]
    step = 1e-3
    r = 40.0
    while _min_dist(lig, q[0], xP + r * u[0], atoms) >= SIGMA:
        r -= step
    assert r <= rho <= r + step


def test_orbit_minima_on_a_ring():
    """Step A6 on a hand-made 6 x 3 array: per-orbit minima over accepted orientations, then the
    ring's local minima (ties count as minima on both sides)."""
    E = np.array([[3.0, 4.0, 9.0],
                  [5.0, 1.0, 2.0],
                  [2.0, 7.0, 8.0],
                  [6.0, 5.0, 9.0],
                  [0.5, 0.0, 3.0],     # the 0.0 pose is rejected below
                  [4.0, 4.0, 6.0]])
    flags = np.ones((6, 3), dtype=np.uint8)
    flags[4, 1] = 2                    # in domain, not accepted
    off, idx = angles.ring_neighbours(6)
    best, bestE, is_min = ppiem.orbit_minima(E, flags, 6, 3, off, idx)
    assert list(best) == [0, 1, 0, 1, 0, 0]
    assert list(bestE) == [3.0, 1.0, 2.0, 5.0, 0.5, 4.0]
    assert list(is_min) == [False, True, False, False, True, False]
    # ties: both equal neighbours are minima
    E2 = np.array([[1.0], [1.0], [2.0], [3.0]])
    off, idx = angles.ring_neighbours(4)
    _, _, m2 = ppiem.orbit_minima(E2, np.ones((4, 1), np.uint8), 4, 1, off, idx)
    assert list(m2) == [True, True, False, False]
    # an orbit position with no accepted pose is never a minimum and does not block others
    f3 = np.ones((4, 1), np.uint8)
    f3[0] = 0
    b3, e3, m3 = ppiem.orbit_minima(E2, f3, 4, 1, off, idx)
    assert b3[0] == -1 and e3[0] == np.inf and list(m3) == [False, True, False, False]


def test_sphere_neighbours_of_the_octahedron():
    d = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=float)
    off, idx = angles.sphere_neighbours(d, 4)
    for i in range(6):
        nb = set(idx[off[i]:off[i + 1]].tolist())
        anti = i ^ 1
        assert nb == set(range(6)) - {i, anti}


def test_a_dipole_turns_its_negative_end_to_a_positive_protein():
    """Steps A2-A7 end to end on a case with a known answer: a single positive protein charge and
    a two-atom dipole ligand spun in the plane.  At every orbit position the lowest energy is the
    orientation pointing the negative end at the protein, with Coulomb's energy at contact."""
    n, b = 128, 24.0
    M, h_M, L_s, K = 24, 0.2622, 83.13843876330611, 12
    T, W = sinc.sinc_table(M, h_M, L_s)
    (tl, wl), (ts, ws) = sinc.split(T, W, K)
    atoms = np.array([[0.0, 0.0, 0.0]])
    z = np.array([1.0])
    _, can = rhosvd.build(z, atoms, tl, wl, n, b, 1e-10)
    lig = np.array([[-1.5, 0.0, 0.0], [1.5, 0.0, 0.0]])
    zeta = np.array([-0.5, 0.5])                 # the atom at -x is negative
    dirs = angles.orbit_ring(12)
    quats = angles.spins(12)                     # spins about z: the dipole turns in the plane
    off, idx = angles.ring_neighbours(12)
    r_cut = 43.836027469049675
    out = ppiem.ppiem(can.F, n, b, atoms, z, ts, ws, r_cut, zeta, lig, dirs, quats, SIGMA, 1e-6, off, idx)
    # contact: the dipole touches at sigma with one of its atoms
    for i in range(12):
        for k in range(12):
            assert abs(_min_dist(lig, quats[k], out["trans"][i * 12 + k], atoms) - SIGMA) < 1e-5
    # best orientation at orbit angle phi_i points the negative end (-x in the ligand frame) at
    # the protein, i.e. rotates -x onto -u_i: spin angle = phi_i, index i
    assert list(out["best"]) == list(range(12))
    E = out["result"]["E"].reshape(12, 12)
    assert np.all(out["best_energy"] < 0)
    # Coulomb's law at contact: the negative atom sigma away, the positive one sigma + 3 A; the
    # interpolation of the grid (h = 0.375 A) leaves a few 1e-6
    exact = -0.5 / SIGMA + 0.5 / (SIGMA + 3.0)
    assert np.allclose(out["best_energy"], exact, rtol=1e-4)
    assert out["minima"][0][0] == np.min(out["best_energy"])
    # the worst orientation is the opposite one (positive end in)
    assert list(np.argmax(E, axis=1)) == [(i + 6) % 12 for i in range(12)]
