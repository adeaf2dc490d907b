"""GPU tests of the posing search (Algorithm PPIEM, steps A2-A7) against the oracle.

Contact radii are FP64 roots computed in a different operation order on each side, so they
are compared to 1e-9 A (the root of a pair hit at a grazing angle loses digits to the square
root; the first contact is a head-on hit in practice, and the property checks below do not
depend on the tolerance).  Integer outputs of step A6 are compared bit for bit on the same
energies; energies at the contact poses are checked at the usual parity bar.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import assert_parity, oracle_factors, oracle_score, sinc_parts  # noqa: E402
from oracle import ppiem as oppiem, score as oscore  # noqa: E402
from workloads import angles, configs, generators as gen  # noqa: E402

pytestmark = pytest.mark.gpu
RHO_TOL = 1e-9


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2510_26611_amd as rs
    from paper_2510_26611_amd import ppiem
    ctx = rs.Context(0)
    cfg = configs.CONFIG1
    wl = configs.make(cfg, P=1)
    _, can = oracle_factors(cfg, wl)
    t = rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges, wl.protein_positions)
    yield rs, ppiem, torch, ctx, cfg, wl, can.F, t
    t.free()
    ctx.close()


def _min_dist(lig, q, tr, atoms):
    _, ul = oscore.ligand_frame(lig)
    y = oscore.transform(np.atleast_2d(q), np.atleast_2d(tr), ul)[0]
    return float(np.sqrt(np.min(oscore.pair_d2(y, atoms))))


def test_centre_is_the_geometric_centre(env):
    rs, ppiem, torch, ctx, cfg, wl, F, t = env
    assert np.array_equal(ppiem.tensor_centre(t), oppiem.geometric_centre(wl.protein_positions))


@pytest.mark.parametrize("grid", ["sphere", "ring"])
def test_contact_radii_match_oracle(env, grid):
    rs, ppiem, torch, ctx, cfg, wl, F, t = env
    if grid == "sphere":
        dirs, quats = angles.orbit_sphere(40), angles.orientations(6, 4)
    else:
        dirs, quats = angles.orbit_ring(12), angles.spins(12)
    cp = ppiem.contact_poses(ctx, t, wl.ligand_positions, dirs, quats, cfg.sigma, gap=1e-6)
    torch.cuda.synchronize()
    rho = cp["rho"].cpu().numpy()
    xP = oppiem.geometric_centre(wl.protein_positions)
    ref = oppiem.contact_radius(wl.ligand_positions, quats, dirs, xP, wl.protein_positions, cfg.sigma)
    err = np.max(np.abs(rho - ref))
    print(f"{grid}: {rho.size} contact radii in [{rho.min():.3f}, {rho.max():.3f}] A, max |gpu - oracle| {err:.2e}")
    assert np.all(np.isfinite(rho)) and err <= RHO_TOL
    U, Q = rho.shape
    pq, pt = cp["quats"].cpu().numpy(), cp["trans"].cpu().numpy()
    assert np.array_equal(pq, np.broadcast_to(quats[None], (U, Q, 4)).reshape(-1, 4))
    _, t_ref = oppiem.contact_poses(quats, dirs, xP, rho, 1e-6)
    assert np.max(np.abs(pt - t_ref)) <= 1e-12 * (1.0 + np.max(np.abs(t_ref)))
    # first contact, checked with the oracle's own distances at the device's radii
    for o in np.random.default_rng(1).choice(U * Q, size=40, replace=False):
        u, q = divmod(int(o), Q)
        d_out = _min_dist(wl.ligand_positions, quats[q], pt[o], wl.protein_positions)
        d_in = _min_dist(wl.ligand_positions, quats[q], xP + (rho[u, q] - 1e-7) * dirs[u], wl.protein_positions)
        assert d_out >= cfg.sigma > d_in


def test_contact_edge_cases(env):
    """A line that misses the protein (-inf, NaN translation, an invalid pose for the scorer), an
    invalid quaternion (NaN), and a ligand of more than 256 atoms (several threads per atom loop)."""
    rs, ppiem, torch, ctx, cfg, wl, F, t = env
    xP = oppiem.geometric_centre(wl.protein_positions)
    far = xP + np.array([0.0, 0.0, 30.0])
    dirs = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0]])
    quats = np.array([[1.0, 0.0, 0.0, 0.0], [0.5, 0.5, 0.5, 0.5], [1.0, 1e-3, 0.0, 0.0]])
    cp = ppiem.contact_poses(ctx, t, wl.ligand_positions, dirs, quats, cfg.sigma, centre=far)
    rho = cp["rho"].cpu().numpy()
    ref = oppiem.contact_radius(wl.ligand_positions, quats[:2], dirs, far, wl.protein_positions, cfg.sigma)
    assert np.all(rho[0, :2] == -np.inf) and np.all(ref[0] == -np.inf)
    assert np.max(np.abs(rho[1, :2] - ref[1])) <= RHO_TOL
    assert np.all(np.isnan(rho[:, 2]))
    pt = cp["trans"].cpu().numpy().reshape(2, 3, 3)
    assert np.all(np.isnan(pt[0, :2])) and np.all(np.isnan(pt[:, 2])) and np.all(np.isfinite(pt[1, :2]))
    res = rs.score_poses(ctx, t, torch.from_numpy(wl.ligand_charges).cuda(),
                         torch.from_numpy(wl.ligand_positions).cuda(), cp["quats"], cp["trans"], cfg.sigma)
    fl = res["flags"].cpu().numpy().reshape(2, 3)
    assert np.all(fl[0, :2] & 4) and np.all(fl[:, 2] & 4) and not np.any(fl[1, :2] & 4)
    # a 300-atom ligand
    big = gen.ball_points(gen.rng(72, 3), 300, 9.0)
    d2, q2 = angles.orbit_sphere(6), angles.orientations(2, 2)
    cp2 = ppiem.contact_poses(ctx, t, big, d2, q2, cfg.sigma)
    ref2 = oppiem.contact_radius(big, q2, d2, xP, wl.protein_positions, cfg.sigma)
    assert np.max(np.abs(cp2["rho"].cpu().numpy() - ref2)) <= RHO_TOL
    with pytest.raises(rs.RsdError):
        ppiem.contact_poses(ctx, t, wl.ligand_positions, dirs, quats, 0.0)
    with pytest.raises(rs.RsdError):
        ppiem.contact_poses(ctx, t, wl.ligand_positions, dirs, quats, cfg.sigma, gap=-1.0)


def test_orbit_minima_bitwise(env):
    """Step A6 on the same energies: the device's argmins and minimum flags equal the oracle's,
    including rejected poses, ties and an orbit position with nothing accepted."""
    rs, ppiem, torch, ctx, cfg, wl, F, t = env
    for U, Q, graph in ((12, 12, "ring"), (300, 70, "sphere")):
        g = np.random.default_rng(U)
        E = np.round(g.standard_normal(U * Q), 1)       # many exact ties
        fl = (g.random(U * Q) < 0.8).astype(np.uint8) | 2
        fl[:Q] = 2                                        # orbit 0: nothing accepted
        off, idx = angles.ring_neighbours(U) if graph == "ring" else angles.sphere_neighbours(angles.orbit_sphere(U))
        m = ppiem.orbit_minima(ctx, E, fl, U, Q, off, idx)
        b, e, im = oppiem.orbit_minima(E, fl, U, Q, off, idx)
        assert np.array_equal(m["best_rotation"].cpu().numpy(), b)
        assert np.array_equal(m["best_energy"].cpu().numpy(), e)
        assert np.array_equal(m["is_minimum"].cpu().numpy().astype(bool), im)


@pytest.mark.parametrize("grid", ["ring", "sphere"])
def test_search_end_to_end(env, grid):
    """Steps A2-A7: energies of the device's contact poses at parity with the oracle scoring the
    same poses; per-orbit best energies against the oracle's own search; the minima agree
    wherever the oracle's decision is not a near-tie."""
    rs, ppiem, torch, ctx, cfg, wl, F, t = env
    if grid == "ring":
        dirs, quats = angles.orbit_ring(12), angles.spins(12)
        off, idx = angles.ring_neighbours(12)
    else:
        dirs, quats = angles.orbit_sphere(60), angles.orientations(8, 6)
        off, idx = angles.sphere_neighbours(dirs)
    out = ppiem.ppiem(ctx, t, wl.ligand_charges, wl.ligand_positions, dirs, quats, cfg.sigma, off, idx)
    res = {k: v.cpu().numpy() for k, v in out["result"].items()}
    pq, pt = out["contact"]["quats"].cpu().numpy(), out["contact"]["trans"].cpu().numpy()
    ref_same = oracle_score(cfg, wl, F, pq, pt)
    assert_parity(res, ref_same, label=f"contact poses ({grid})")
    assert np.all(res["flags"] & 1)
    _, (ts, ws) = sinc_parts(cfg)
    o = oppiem.ppiem(F, cfg.n, cfg.b, wl.protein_positions, wl.protein_charges, ts, ws, cfg.r_cut,
                     wl.ligand_charges, wl.ligand_positions, dirs, quats, cfg.sigma, 1e-6, off, idx)
    be = out["orbit"]["best_energy"].cpu().numpy()
    scale = np.max(np.abs(o["best_energy"]))
    assert np.max(np.abs(be - o["best_energy"])) <= 1e-8 * scale
    im = out["orbit"]["is_minimum"].cpu().numpy().astype(bool)
    margin = np.array([min([abs(o["best_energy"][u] - o["best_energy"][v]) for v in idx[off[u]:off[u + 1]]] or [1.0])
                       for u in range(len(dirs))])
    clear = margin > 1e-7 * scale
    assert np.array_equal(im[clear], o["is_minimum"][clear])
    print(f"{grid}: {len(out['minima'])} minima (oracle {len(o['minima'])}); lowest {out['minima'][0][0]:.6f} at orbit "
          f"{out['minima'][0][1]} rotation {out['minima'][0][2]} (oracle {o['minima'][0]})")
    assert out["minima"][0][0] == pytest.approx(o["minima"][0][0], rel=1e-8)


@pytest.mark.timeout(600)
def test_cfg2_search_full_size_sampled(env):
    """The bench's search (5,000-atom protein, 50-atom ligand, 4,096 orbit directions x 256
    orientations, the same launch): contact radii of sampled entries against the oracle."""
    rs, ppiem, torch, ctx, cfg, wl, F, t = env
    c2 = configs.CONFIG2
    w2 = configs.make(c2, P=1)
    tg = rs.build_rs_tensor(ctx, w2.protein_charges, w2.protein_positions, c2.n, c2.b, rs.Sinc.from_config(c2))
    dirs, quats = angles.orbit_sphere(4096), angles.orientations(32, 8)
    cp = ppiem.contact_poses(ctx, tg, w2.ligand_positions, dirs, quats, c2.sigma)
    rho = cp["rho"].cpu().numpy()
    xP = oppiem.geometric_centre(w2.protein_positions)
    g = np.random.default_rng(9)
    us, qs = g.choice(4096, size=24, replace=False), g.choice(256, size=6, replace=False)
    ref = oppiem.contact_radius(w2.ligand_positions, quats[qs], dirs[us], xP, w2.protein_positions, c2.sigma)
    err = np.max(np.abs(rho[np.ix_(us, qs)] - ref))
    print(f"cfg2 search: rho in [{rho.min():.2f}, {rho.max():.2f}] A; sampled max |gpu - oracle| {err:.2e}")
    assert np.all(np.isfinite(rho)) and err <= RHO_TOL
    tg.free()
