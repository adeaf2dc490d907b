"""GPU tests of rsd_tensor_restrict (Sec. 3.3, scheme (C)): the long-range tensor restricted
to a sub-box and rank-reduced, against the oracle's restriction and recompression.

Two independent rank reductions agree only to the truncation level, so the device result is
compared with the exact restricted tensor (materialised on the sub-grid) and the bound is
calibrated by the oracle's own recompression error.  Scoring with the device's local tensor
is then checked at the usual parity bar against the oracle evaluating the same factors.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import assert_parity, oracle_factors, sinc_parts  # noqa: E402
from oracle import local as olocal, score as oscore, tensor as otensor  # noqa: E402
from workloads import configs, generators as gen  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2510_26611_amd as rs
    ctx = rs.Context(0)
    cfg = configs.CONFIG1
    wl = configs.make(cfg)
    _, can = oracle_factors(cfg, wl)
    t = rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges, wl.protein_positions)
    yield rs, torch, ctx, cfg, wl, can.F, t
    t.free()
    ctx.close()


def _local_factors(tl, grid):
    F = tl.export()
    return [F[d][:grid["rows"][d]] for d in range(3)]


@pytest.mark.parametrize("half", [4.0, 7.0])
def test_restriction_matches_oracle(env, half):
    rs, torch, ctx, cfg, wl, F, t = env
    site = np.array([18.0, 0.0, 0.0])
    lo, hi = site - half, site + half
    tl = t.restrict(lo, hi, 1e-8)
    g = tl.grid()
    ref = olocal.restrict(F, cfg.n, cfg.b, lo, hi)
    # the same rows, origins bit for bit
    assert tuple(g["rows"]) == tuple(int(x) for x in ref.ns)
    assert np.array_equal(np.array(g["X0"]), ref.X0s)
    tk, rc = olocal.recompress(ref.F, 1e-8)
    A = otensor.materialize_canonical(*ref.F)
    err_o = float(np.sqrt(np.sum((otensor.materialize_canonical(*rc.F) - A) ** 2)))
    Fg = _local_factors(tl, g)
    err_g = float(np.sqrt(np.sum((otensor.materialize_canonical(*Fg) - A) ** 2)))
    norm = float(np.sqrt(np.sum(A * A)))
    q = tl.query()
    print(f"half {half}: rows {g['rows']} | R local gpu {q['R']} ranks {q['ranks']} | oracle {rc.R} {tk.ranks} | "
          f"global R {t.query()['R']} | ||err|| gpu {err_g:.3e} oracle {err_o:.3e} (||T|| {norm:.3e})")
    assert err_g <= 10.0 * max(err_o, 1e-8 * norm)
    assert q["R"] < t.query()["R"]
    tl.free()


def test_scoring_with_the_local_tensor_at_parity(env):
    rs, torch, ctx, cfg, wl, F, t = env
    site = np.array([18.0, 0.0, 0.0])
    tl = t.restrict(site - 7.0, site + 7.0, 1e-8)
    g = tl.grid()
    Fg = _local_factors(tl, g)
    P = 600
    q = gen.unit_quaternions(gen.rng(44, 5), P)
    tr = site[None, :] + gen.sphere_translations(gen.rng(44, 6), P, 2.0) * gen.rng(44, 7).random((P, 1))
    tr[:5] = site + np.array([[4.0, 0, 0], [0, 4.0, 0], [0, 0, 4.0], [-3.5, 0, 0], [0, -3.5, 3.0]])  # some leave the box
    _, (ts, ws) = sinc_parts(cfg)
    spec = (np.array(g["X0"]), 1.0 / g["h"], np.array(g["rows"]))
    ref = oscore.score(Fg, cfg.n, cfg.b, wl.protein_positions, wl.protein_charges, ts, ws, cfg.r_cut,
                       wl.ligand_charges, wl.ligand_positions, q, tr, cfg.sigma, grid_spec=spec)
    assert np.any(ref["flags"] & 2) and not np.all(ref["flags"] & 2)
    for mode in (1, 2):
        ctx.set_option("score_mode", mode)
        out = rs.score_poses(ctx, tl, wl.ligand_charges, wl.ligand_positions, q, tr, cfg.sigma, energies_long=True)
        assert_parity(out, ref, label=f"local tensor, mode {mode}")
    ctx.set_option("score_mode", 0)
    # against the global tensor: same flags where both are in domain, energies within the truncation
    glob = rs.score_poses(ctx, t, wl.ligand_charges, wl.ligand_positions, q, tr, cfg.sigma)
    ok = (ref["flags"] & 2) != 0
    assert np.array_equal(glob["flags"][ok], out["flags"][ok]) and np.array_equal(glob["counts"], out["counts"])
    assert np.max(np.abs(glob["E"][ok] - out["E"][ok])) <= 1e-6 * np.max(np.abs(glob["E"][ok]))
    tl.free()


def test_batch_with_a_local_tensor_equals_alone(env):
    rs, torch, ctx, cfg, wl, F, t = env
    site = np.array([18.0, 0.0, 0.0])
    tl = t.restrict(site - 7.0, site + 7.0, 1e-8)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    P = 700
    q = gen.unit_quaternions(gen.rng(45, 5), P)
    tr = site[None, :] + gen.sphere_translations(gen.rng(45, 6), P, 1.5)
    reqs = [dict(tensor=tl, lig_charges=d(wl.ligand_charges), lig_positions=d(wl.ligand_positions), quats=d(q),
                 trans=d(tr), vdw_min=cfg.sigma),
            dict(tensor=t, lig_charges=d(wl.ligand_charges), lig_positions=d(wl.ligand_positions), quats=d(q),
                 trans=d(tr), vdw_min=cfg.sigma)]
    b = rs.Batch(ctx, reqs)
    b.run()
    torch.cuda.synchronize()
    ctx.set_option("score_mode", 2)
    for r, out in zip(reqs, b.outputs()):
        alone = rs.score_poses(ctx, r["tensor"], r["lig_charges"], r["lig_positions"], r["quats"], r["trans"],
                               r["vdw_min"])
        torch.cuda.synchronize()
        for k in ("E", "flags", "counts"):
            assert np.array_equal(out[k].cpu().numpy(), alone[k].cpu().numpy(), equal_nan=True), k
    ctx.set_option("score_mode", 0)
    b.free()
    tl.free()


def test_restrict_argument_errors(env):
    rs, torch, ctx, cfg, wl, F, t = env
    site = np.array([18.0, 0.0, 0.0])
    for lo, hi, eps in ((site + 1, site - 1, 1e-8), (site - 1, site + 1, 0.0), (site - 1, site + 1, 1.0),
                        (site + 100, site + 101, 1e-8), (site - 1, site + np.array([1, np.nan, 1]), 1e-8)):
        with pytest.raises(rs.RsdError) as e:
            t.restrict(lo, hi, eps)
        assert e.value.code == -1
    tl = t.restrict(site - 3, site + 3, 1e-8)
    with pytest.raises(rs.RsdError) as e:
        tl.save("/tmp/never_written.rsd")
    assert e.value.code == -5
    tl.free()


@pytest.mark.timeout(600)
def test_cfg2_site_restriction_full_size(env):
    """The 5,000-atom protein built on the device, restricted to a 16 A box at a site in the pose
    shell: the local tensor against the oracle's restriction of the same global factors."""
    rs, torch, ctx, cfg, wl, F, t = env
    c2 = configs.CONFIG2
    w2 = configs.make(c2, P=1)
    tg = rs.build_rs_tensor(ctx, w2.protein_charges, w2.protein_positions, c2.n, c2.b, rs.Sinc.from_config(c2))
    site = np.array([c2.pose_r_in + 5.0, 0.0, 0.0])
    tl = tg.restrict(site - 8.0, site + 8.0, 1e-8)
    g = tl.grid()
    Fglob = tg.export()
    ref = olocal.restrict(Fglob, c2.n, c2.b, site - 8.0, site + 8.0)
    assert tuple(g["rows"]) == tuple(int(x) for x in ref.ns)
    tk, rc = olocal.recompress(ref.F, 1e-8)
    idx = np.random.default_rng(3).integers(0, np.array(g["rows"]), size=(4000, 3))
    T_ex = np.sum(ref.F[0][idx[:, 0]] * ref.F[1][idx[:, 1]] * ref.F[2][idx[:, 2]], axis=1)
    Fg = _local_factors(tl, g)
    T_g = np.sum(Fg[0][idx[:, 0]] * Fg[1][idx[:, 1]] * Fg[2][idx[:, 2]], axis=1)
    T_o = np.sum(rc.F[0][idx[:, 0]] * rc.F[1][idx[:, 1]] * rc.F[2][idx[:, 2]], axis=1)
    err_g, err_o = np.max(np.abs(T_g - T_ex)), np.max(np.abs(T_o - T_ex))
    print(f"cfg2 site box: rows {g['rows']} R local gpu {tl.query()['R']} oracle {rc.R} global {tg.query()['R']} | "
          f"max err gpu {err_g:.3e} oracle {err_o:.3e} max|T| {np.max(np.abs(T_ex)):.3e}")
    assert err_g <= 10.0 * max(err_o, 1e-8 * np.max(np.abs(T_ex)))
    assert tl.query()["R"] * 4 < tg.query()["R"]
    tl.free()
    tg.free()


@pytest.mark.parametrize("qr_solver,svd_solver", [(1, 0), (0, 3), (1, 3)])
@pytest.mark.parametrize("half", [4.0, 7.0])
def test_restriction_solver_paths(env, half, qr_solver, svd_solver):
    """The rank reduction's other solver paths, which the default one falls back to: rocSOLVER's
    Householder QR for the bases (option qr_solver 1, taken when a Cholesky pass loses rank) and
    rocSOLVER's gesvdj for the k x k SVD (svd_solver 3, taken for k > 96).  Each gives the
    oracle's ranks and stays within the oracle-calibrated bound of the exact restricted tensor,
    for the direct route (8 A box, 87 rows) and the randomized range (14 A box)."""
    rs, torch, ctx, cfg, wl, F, t = env
    site = np.array([18.0, 0.0, 0.0])
    lo, hi = site - half, site + half
    ref = olocal.restrict(F, cfg.n, cfg.b, lo, hi)
    tk, rc = olocal.recompress(ref.F, 1e-8)
    A = otensor.materialize_canonical(*ref.F)
    err_o = float(np.sqrt(np.sum((otensor.materialize_canonical(*rc.F) - A) ** 2)))
    norm = float(np.sqrt(np.sum(A * A)))
    ctx.set_option("qr_solver", qr_solver)
    ctx.set_option("svd_solver", svd_solver)
    try:
        tl = t.restrict(lo, hi, 1e-8)
    finally:
        ctx.set_option("qr_solver", 0)
        ctx.set_option("svd_solver", 0)
    g = tl.grid()
    q = tl.query()
    err_g = float(np.sqrt(np.sum((otensor.materialize_canonical(*_local_factors(tl, g)) - A) ** 2)))
    print(f"half {half} qr {qr_solver} svd {svd_solver}: R {q['R']} ranks {q['ranks']} | oracle {rc.R} {tk.ranks} | "
          f"||err|| gpu {err_g:.3e} oracle {err_o:.3e}")
    assert tuple(q["ranks"]) == tuple(tk.ranks)
    assert err_g <= 10.0 * max(err_o, 1e-8 * norm)
    tl.free()


def test_restriction_of_a_restriction(env):
    """A local tensor restricted again keeps the source's mesh: the same rows and origins as the
    direct restriction of the global tensor to the inner box, and the same values to the
    truncation level."""
    rs, torch, ctx, cfg, wl, F, t = env
    site = np.array([18.0, 0.0, 0.0])
    outer = t.restrict(site - 7.0, site + 7.0, 1e-10)
    inner = outer.restrict(site - 3.0, site + 3.0, 1e-8)
    direct = t.restrict(site - 3.0, site + 3.0, 1e-8)
    g_i, g_d = inner.grid(), direct.grid()
    assert g_i["h"] == t.grid()["h"] == outer.grid()["h"]
    assert g_i["rows"] == g_d["rows"] and np.array_equal(np.array(g_i["X0"]), np.array(g_d["X0"]))
    ref = olocal.restrict(F, cfg.n, cfg.b, site - 3.0, site + 3.0)
    rows = np.array(g_i["rows"])
    idx = np.random.default_rng(4).integers(0, rows, size=(4000, 3))
    at = lambda G: np.sum(G[0][idx[:, 0]] * G[1][idx[:, 1]] * G[2][idx[:, 2]], axis=1)  # noqa: E731
    exact = at(ref.F)
    e_i = np.max(np.abs(at(_local_factors(inner, g_i)) - exact))
    e_d = np.max(np.abs(at(_local_factors(direct, g_d)) - exact))
    print(f"inner of outer: R {inner.query()['R']} err {e_i:.3e} | direct R {direct.query()['R']} err {e_d:.3e}")
    assert e_i <= 10.0 * max(e_d, 1e-8 * np.max(np.abs(exact)))
    for x in (outer, inner, direct):
        x.free()
