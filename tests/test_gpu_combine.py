"""GPU tests of rsd_tensor_combine: the potential of a complex of molecules (eq. 5.1) by
add-and-compress (Algorithm TEP, step 4), against the oracle's concatenation and recompression.

As for the restriction, two independent rank reductions agree only to the truncation level:
the device's combined tensor is compared with the exact sum of the sources (their factors side
by side) at sampled grid nodes, with the bound calibrated by the oracle's own recompression of
the same factors.  Scoring with the combined tensor is then checked at the usual parity bar
against the oracle evaluating the device's factors with the union of the atoms.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import assert_parity, sinc_parts  # noqa: E402
from oracle import local as olocal, score as oscore  # noqa: E402
from workloads import configs, generators as gen  # noqa: E402

pytestmark = pytest.mark.gpu

CENTRES = (np.array([-10.0, 0.0, 0.0]), np.array([10.0, 3.0, 0.0]), np.array([0.0, -4.0, 11.0]))
SITE = np.array([0.0, 8.0, 0.0])


def _molecule(k, count, radius):
    pos = gen.ball_points(gen.rng(60 + k, 1), count, radius) + CENTRES[k]
    z = gen.charges(gen.rng(60 + k, 2), count, 0.3, True)
    return z, pos


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2510_26611_amd as rs
    ctx = rs.Context(0)
    cfg = configs.CONFIG1
    wl = configs.make(cfg, P=1)
    mols = [_molecule(0, 120, 8.0), _molecule(1, 90, 7.0), _molecule(2, 60, 6.0)]
    ts = [rs.build_rs_tensor(ctx, z, p, cfg.n, cfg.b, rs.Sinc.from_config(cfg)) for z, p in mols]
    yield rs, torch, ctx, cfg, wl, mols, ts
    for t in ts:
        t.free()
    ctx.close()


def _at(F, idx):
    return np.sum(F[0][idx[:, 0]] * F[1][idx[:, 1]] * F[2][idx[:, 2]], axis=1)


@pytest.mark.parametrize("count", [1, 2, 3])
def test_combined_tensor_matches_oracle(env, count):
    rs, torch, ctx, cfg, wl, mols, ts = env
    tc = rs.tensor_combine(ctx, ts[:count], 1e-8)
    Fs = [t.export() for t in ts[:count]]
    Fsum, (tk, rc) = olocal.combine(Fs, 1e-8)
    idx = np.random.default_rng(5).integers(0, cfg.n, size=(20000, 3))
    exact = _at(Fsum, idx)
    err_g = np.max(np.abs(_at(tc.export(), idx) - exact))
    err_o = np.max(np.abs(_at(rc.F, idx) - exact))
    q = tc.query()
    Rs = [t.query()["R"] for t in ts[:count]]
    print(f"{count} molecules: R sources {Rs} -> gpu {q['R']} ranks {q['ranks']} | oracle {rc.R} {tk.ranks} | "
          f"max err gpu {err_g:.3e} oracle {err_o:.3e} max|T| {np.max(np.abs(exact)):.3e}")
    assert err_g <= 10.0 * max(err_o, 1e-9 * np.max(np.abs(exact)))
    assert abs(q["R"] - rc.R) <= 2
    if count > 1:
        assert q["R"] < sum(Rs)
    g = tc.grid()
    assert g["rows"] == (cfg.n,) * 3 and g["h"] == ts[0].grid()["h"]
    tc.free()


def test_scoring_against_the_complex(env):
    """Eq. 5.1: the ligand's energy against the complex at parity with the oracle (union of the
    atoms, the device's combined factors), and equal to the sum over the molecules up to the
    truncation; counts add up and a clash with any molecule clears the vdW flag."""
    rs, torch, ctx, cfg, wl, mols, ts = env
    tc = rs.tensor_combine(ctx, ts, 1e-8)
    P = 500
    q = gen.unit_quaternions(gen.rng(61, 5), P)
    tr = SITE[None, :] + gen.sphere_translations(gen.rng(61, 6), P, 3.0) * gen.rng(61, 7).random((P, 1))
    z_all = np.concatenate([m[0] for m in mols])
    p_all = np.vstack([m[1] for m in mols])
    _, (tsh, wsh) = sinc_parts(cfg)
    F = tc.export()
    ref = oscore.score(F, cfg.n, cfg.b, p_all, z_all, tsh, wsh, cfg.r_cut, wl.ligand_charges, wl.ligand_positions,
                       q, tr, cfg.sigma)
    assert np.any((ref["flags"] & 1) == 0) and np.any(ref["flags"] & 1)
    for mode in (1, 2):
        ctx.set_option("score_mode", mode)
        out = rs.score_poses(ctx, tc, wl.ligand_charges, wl.ligand_positions, q, tr, cfg.sigma)
        assert_parity(out, ref, label=f"complex, mode {mode}")
    ctx.set_option("score_mode", 0)
    parts = [rs.score_poses(ctx, t, wl.ligand_charges, wl.ligand_positions, q, tr, cfg.sigma) for t in ts]
    assert np.array_equal(out["counts"], sum(p["counts"] for p in parts))
    acc = np.ones(P, dtype=bool)
    for p in parts:
        acc &= (p["flags"] & 1) != 0
    assert np.array_equal((out["flags"] & 1) != 0, acc)
    Esum = sum(p["E"] for p in parts)
    scale = np.max(np.abs(Esum))
    print(f"complex vs sum of molecules: max |dE| {np.max(np.abs(out['E'] - Esum)):.3e} (max |E| {scale:.3e})")
    assert np.max(np.abs(out["E"] - Esum)) <= 1e-6 * scale
    tc.free()


def test_build_in_pieces_matches_the_whole(env):
    """Add-and-compress as a build option: one molecule built in three pieces and combined
    agrees with its direct build to the truncation level."""
    rs, torch, ctx, cfg, wl, mols, ts = env
    z, p = wl.protein_charges, wl.protein_positions
    whole = rs.build_rs_tensor(ctx, z, p, cfg.n, cfg.b, rs.Sinc.from_config(cfg))
    cuts = [0, 70, 140, len(z)]
    pieces = [rs.build_rs_tensor(ctx, z[a:b], p[a:b], cfg.n, cfg.b, rs.Sinc.from_config(cfg))
              for a, b in zip(cuts[:-1], cuts[1:])]
    tc = rs.tensor_combine(ctx, pieces, 1e-8)
    idx = np.random.default_rng(6).integers(0, cfg.n, size=(20000, 3))
    Tw, Tc = _at(whole.export(), idx), _at(tc.export(), idx)
    print(f"pieces R {[t.query()['R'] for t in pieces]} combined {tc.query()['R']} whole {whole.query()['R']} | "
          f"max diff {np.max(np.abs(Tw - Tc)):.3e} of {np.max(np.abs(Tw)):.3e}")
    assert np.max(np.abs(Tw - Tc)) <= 1e-6 * np.max(np.abs(Tw))
    # the short-range part sees the same atoms: scoring agrees bit for bit in flags and counts
    P = 300
    q = gen.unit_quaternions(gen.rng(62, 5), P)
    tr = gen.sphere_translations(gen.rng(62, 6), P, cfg.pose_r_in)
    a = rs.score_poses(ctx, whole, wl.ligand_charges, wl.ligand_positions, q, tr, cfg.sigma)
    b = rs.score_poses(ctx, tc, wl.ligand_charges, wl.ligand_positions, q, tr, cfg.sigma)
    assert np.array_equal(a["flags"], b["flags"]) and np.array_equal(a["counts"], b["counts"])
    assert np.max(np.abs(a["E"] - b["E"])) <= 1e-6 * np.max(np.abs(a["E"]))
    for t in pieces + [whole, tc]:
        t.free()


def test_combining_local_tensors(env):
    """Restrictions of the molecules to one box combine like global tensors."""
    rs, torch, ctx, cfg, wl, mols, ts = env
    lo, hi = SITE - 5.0, SITE + 5.0
    locs = [t.restrict(lo, hi, 1e-8) for t in ts]
    tc = rs.tensor_combine(ctx, locs, 1e-8)
    g = tc.grid()
    assert g == locs[0].grid()
    rows = np.array(g["rows"])
    Fsum, (tk, rc) = olocal.combine([[F[d][:rows[d]] for d in range(3)] for F in (t.export() for t in locs)], 1e-8)
    idx = np.random.default_rng(7).integers(0, rows, size=(5000, 3))
    exact = _at(Fsum, idx)
    Fc = [tc.export()[d][:rows[d]] for d in range(3)]
    err_g, err_o = np.max(np.abs(_at(Fc, idx) - exact)), np.max(np.abs(_at(rc.F, idx) - exact))
    print(f"local: R {[t.query()['R'] for t in locs]} -> {tc.query()['R']} (oracle {rc.R}) | err gpu {err_g:.3e} "
          f"oracle {err_o:.3e}")
    assert err_g <= 10.0 * max(err_o, 1e-9 * np.max(np.abs(exact)))
    for t in locs + [tc]:
        t.free()


def test_combine_argument_errors(env):
    rs, torch, ctx, cfg, wl, mols, ts = env
    z, p = mols[0]
    other_n = rs.build_rs_tensor(ctx, z, p, 256, cfg.b, rs.Sinc.from_config(cfg))
    sp = rs.Sinc.from_config(cfg)
    sp.K_long = sp.K_long - 1
    other_sinc = rs.build_rs_tensor(ctx, z, p, cfg.n, cfg.b, sp)
    loc = ts[0].restrict(SITE - 4.0, SITE + 4.0, 1e-8)
    for bad, code in (([ts[0], other_n], -5), ([ts[0], other_sinc], -5), ([ts[0], loc], -5)):
        with pytest.raises(rs.RsdError) as e:
            rs.tensor_combine(ctx, bad, 1e-8)
        assert e.value.code == code
    for eps in (0.0, 1.0, float("nan")):
        with pytest.raises(rs.RsdError) as e:
            rs.tensor_combine(ctx, ts[:2], eps)
        assert e.value.code == -1
    with pytest.raises(rs.RsdError) as e:
        rs.tensor_combine(ctx, [], 1e-8)
    assert e.value.code == -1
    for t in (other_n, other_sinc, loc):
        t.free()


@pytest.mark.timeout(600)
def test_cfg2_protein_in_two_halves(env):
    """The 5,000-atom protein (n = 2048, the subspace eigensolver's size range) built as two
    halves and combined, against its direct build."""
    rs, torch, ctx, cfg, wl, mols, ts = env
    c2 = configs.CONFIG2
    w2 = configs.make(c2, P=1)
    z, p = w2.protein_charges, w2.protein_positions
    sp = rs.Sinc.from_config(c2)
    whole = rs.build_rs_tensor(ctx, z, p, c2.n, c2.b, sp)
    h = len(z) // 2
    halves = [rs.build_rs_tensor(ctx, z[:h], p[:h], c2.n, c2.b, sp), rs.build_rs_tensor(ctx, z[h:], p[h:], c2.n, c2.b, sp)]
    tc = rs.tensor_combine(ctx, halves, 1e-8)
    Fs = [t.export() for t in halves]
    Fsum, (tk, rc) = olocal.combine(Fs, 1e-8)
    idx = np.random.default_rng(8).integers(0, c2.n, size=(8000, 3))
    exact = _at(Fsum, idx)
    err_g = np.max(np.abs(_at(tc.export(), idx) - exact))
    err_o = np.max(np.abs(_at(rc.F, idx) - exact))
    dw = np.max(np.abs(_at(whole.export(), idx) - exact))
    print(f"cfg2 halves: R {[t.query()['R'] for t in halves]} -> gpu {tc.query()['R']} {tc.query()['ranks']} | "
          f"oracle {rc.R} {tk.ranks} | whole {whole.query()['R']} | err gpu {err_g:.3e} oracle {err_o:.3e} "
          f"whole-vs-sum {dw:.3e} max|T| {np.max(np.abs(exact)):.3e}")
    assert err_g <= 10.0 * max(err_o, 1e-9 * np.max(np.abs(exact)))
    for t in halves + [whole, tc]:
        t.free()
