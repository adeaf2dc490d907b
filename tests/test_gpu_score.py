"""GPU parity of rsd_score_poses against the oracle on the same factors (through the C ABI).

Bar: vdW flags, in-domain flags and pair counts bit-exact; energies, long-range
energies and gradients within 1e-10 of each pose's FP64 summation-error scale.
"""
import os
import sys
import tempfile

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import assert_parity, near_threshold_poses, oracle_factors, oracle_score, sinc_parts  # noqa: E402
from oracle import score as oscore  # noqa: E402
from workloads import configs, generators as gen  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2510_26611_amd as rs
    return rs


@pytest.fixture(scope="module")
def ctx(rs):
    c = rs.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cfg1(rs, ctx):
    cfg = configs.CONFIG1
    wl = configs.make(cfg)
    tk, can = oracle_factors(cfg, wl)
    t = rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges,
                         wl.protein_positions)
    yield cfg, wl, can.F, t
    t.free()


def _run(rs, ctx, t, wl, q, tr, sigma, grad=True, device=True, mode=0):
    import torch
    ctx.set_option("score_mode", mode)
    if device:
        args = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in
                (wl.ligand_charges, wl.ligand_positions, q, tr)]
        out = rs.score_poses(ctx, t, *args, sigma, grads=grad, energies_long=True)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    return rs.score_poses(ctx, t, wl.ligand_charges, wl.ligand_positions, q, tr, sigma, grads=grad,
                          energies_long=True)


@pytest.mark.parametrize("mode", [1, 2])
def test_cfg1_parity_device_and_host_pointers(rs, ctx, cfg1, mode):
    cfg, wl, F, t = cfg1
    ref = oracle_score(cfg, wl, F, wl.quats, wl.trans, grad=True)
    gd = _run(rs, ctx, t, wl, wl.quats, wl.trans, cfg.sigma, device=True, mode=mode)
    assert_parity(gd, ref, grad=True, label="cfg1 device")
    gh = _run(rs, ctx, t, wl, wl.quats, wl.trans, cfg.sigma, device=False, mode=mode)
    assert_parity(gh, ref, grad=True, label="cfg1 host")
    for k in gd:
        assert np.array_equal(gd[k], gh[k], equal_nan=True), k
    assert np.all(ref["flags"] & 2)


@pytest.mark.parametrize("mode", [1, 2])
def test_cfg1_repeatable_bitwise(rs, ctx, cfg1, mode):
    cfg, wl, F, t = cfg1
    a = _run(rs, ctx, t, wl, wl.quats, wl.trans, cfg.sigma, mode=mode)
    b = _run(rs, ctx, t, wl, wl.quats, wl.trans, cfg.sigma, mode=mode)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("mode", [1, 2])
def test_cfg1_pose_alone_equals_pose_in_batch(rs, ctx, cfg1, mode):
    cfg, wl, F, t = cfg1
    full = _run(rs, ctx, t, wl, wl.quats, wl.trans, cfg.sigma, mode=mode)
    for p in (0, 5, 127):
        one = _run(rs, ctx, t, wl, wl.quats[p:p + 1], wl.trans[p:p + 1], cfg.sigma, mode=mode)
        for k in full:
            assert np.array_equal(one[k][0], full[k][p], equal_nan=True), (k, p)


@pytest.mark.parametrize("mode", [1, 2])
def test_cfg1_near_thresholds_and_edge_poses(rs, ctx, cfg1, mode):
    cfg, wl, F, t = cfg1
    # pull the ligand in so that it touches the protein, then pin pairs on sigma and r_cut
    tr = wl.trans * (15.5 / 18.0)
    q1, t1 = near_threshold_poses(cfg, wl, wl.quats, tr, cfg.sigma, 24)
    q2, t2 = near_threshold_poses(cfg, wl, wl.quats[24:], wl.trans[24:], 20.0, 12)
    q = np.concatenate([q1, q2, wl.quats[:6]])
    tt = np.concatenate([t1, t2, wl.trans[:6]])
    tt[-1] = [1e3, 0, 0]            # out of the grid
    tt[-2] = [23.99, 0.0, 0.0]      # partly out of the grid
    q[-3] = [0.0, 0.0, 0.0, 0.0]    # not a unit quaternion -> invalid on the device path
    q[-4, 2] = np.nan
    ref = oracle_score(cfg, wl, F, q, tt, grad=True)
    g = _run(rs, ctx, t, wl, q, tt, cfg.sigma, mode=mode)
    assert_parity(g, ref, grad=True, label="cfg1 thresholds")
    assert ref["flags"][-3] == 4 and ref["flags"][-4] == 4 and ref["flags"][-1] == 0


@pytest.mark.parametrize("grad", [False, True])
def test_spatial_pose_order_is_bitwise_input_order(rs, ctx, cfg1, grad):
    """Option pose_order: the long range taking the poses in spatial order gives, pose for pose,
    the results of input order (including invalid and out-of-grid poses)."""
    cfg, wl, F, t = cfg1
    q, tt = wl.quats.copy(), wl.trans.copy()
    tt[-1] = [1e3, 0, 0]
    q[-2] = [0.0, 0.0, 0.0, 0.0]
    tt[-3, 1] = np.nan
    out = {}
    for order in (1, 2):
        ctx.set_option("pose_order", order)
        out[order] = _run(rs, ctx, t, wl, q, tt, cfg.sigma, grad=grad, mode=2)
    ctx.set_option("pose_order", 0)
    for k in out[1]:
        assert np.array_equal(out[1][k], out[2][k], equal_nan=True), k
    assert_parity(out[1], oracle_score(cfg, wl, F, q, tt, grad=grad), grad=grad, label="spatial order")


def _morton_cells(trans, b):
    """Morton code of each translation's cell, 32 cells per axis over [-b, b) (x in bit 3k,
    y in 3k+1, z in 3k+2); NaN and out-of-box coordinates clamp to the edge cells."""
    x = (np.asarray(trans) + b) * (32.0 / (2.0 * b))
    c = np.where(x >= 31.0, 31, np.where(x > 0.0, np.floor(np.nan_to_num(x, nan=0.0)), 0)).astype(np.int64)
    code = np.zeros(len(c), dtype=np.int64)
    for bit in range(5):
        for d in range(3):
            code |= ((c[:, d] >> bit) & 1) << (3 * bit + d)
    return code


def test_pose_order_call(rs, ctx, cfg1):
    """rsd_pose_order: a permutation whose translations' Morton cells never decrease, and the
    poses gathered in that order; the flag says whether automatic scoring sorts by itself."""
    import torch
    cfg, wl, F, t = cfg1
    g = np.random.default_rng(31)
    P = 5000
    q = gen.unit_quaternions(gen.rng(31, 1), P)
    tt = g.uniform(-1.2 * cfg.b, 1.2 * cfg.b, size=(P, 3))
    tt[7] = [np.nan, 0.0, 1.0]
    tt[8] = [-np.inf, np.inf, 0.0]
    qd, td = torch.from_numpy(q).cuda(), torch.from_numpy(tt).cuda()
    for order, want in ((0, False), (1, True), (2, False)):
        ctx.set_option("pose_order", order)
        perm, q2, t2, flag = rs.pose_order(ctx, t, qd, td)
        assert flag == want
        perm = perm.cpu().numpy()
        assert np.array_equal(np.sort(perm), np.arange(P))
        assert np.array_equal(q2.cpu().numpy(), q[perm])
        assert np.array_equal(t2.cpu().numpy(), tt[perm], equal_nan=True)
        assert np.all(np.diff(_morton_cells(tt[perm], cfg.b)) >= 0)
    ctx.set_option("pose_order", 0)
    e = torch.empty((0, 4), dtype=torch.float64, device="cuda")
    perm, _, _, _ = rs.pose_order(ctx, t, e, e[:, :3])
    assert perm.numel() == 0


@pytest.mark.parametrize("mode", [1, 2])
def test_vdw_distance_beyond_the_cutoff(rs, ctx, cfg1, mode):
    """vdw_min > r_cut: the accept flag then needs the minimum over every candidate pair, not
    only over the pairs within the cutoff (a pose can be rejected with no pair counted)."""
    cfg, wl, F, _ = cfg1
    r_cut, vdw = 3.0, 4.5
    t = rs.tensor_import(ctx, F, cfg.n, cfg.b, rs.Sinc(cfg.M, cfg.h_M, cfg.L_s, cfg.K_long, r_cut, cfg.eps),
                         wl.protein_charges, wl.protein_positions)
    tr = wl.trans * (15.5 / 18.0)   # poses that touch the protein
    q1, t1 = near_threshold_poses(cfg, wl, wl.quats, tr, vdw, 24)
    q = np.concatenate([q1, wl.quats[24:64]])
    tt = np.concatenate([t1, tr[24:64]])
    _, (ts, ws) = sinc_parts(cfg)
    ref = oscore.score(F, cfg.n, cfg.b, wl.protein_positions, wl.protein_charges, ts, ws, r_cut, wl.ligand_charges,
                       wl.ligand_positions, q, tt, vdw, want_grad=True)
    g = _run(rs, ctx, t, wl, q, tt, vdw, mode=mode)
    assert_parity(g, ref, grad=True, label="vdw beyond the cutoff")
    rejected_uncounted = np.sum(((ref["flags"] & 3) == 2) & (ref["counts"] == 0))
    print(f"{len(q)} poses: accepted {int(np.sum(ref['flags'] & 1))}, rejected with no pair within r_cut "
          f"{int(rejected_uncounted)}")
    assert rejected_uncounted > 0
    t.free()


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("R", [0, 1, 63, 64, 65, 130, 257])
@pytest.mark.parametrize("L", [1, 7, 65, 200])
def test_ragged_rank_and_ligand_sizes(rs, ctx, R, L, mode):
    """Random factors (any factors are valid input) on a 96-point grid; R and L cross chunk edges."""
    g = np.random.default_rng(1000 + R * 7 + L)
    n, b = 96, 30.0
    cfg = configs.CONFIG1
    F = [g.normal(size=(n, R)) for _ in range(3)]
    pos = gen.ball_points(gen.rng(77, 1), 60, 6.0)
    z = gen.charges(gen.rng(77, 2), 60, 0.3, True)
    lig = gen.ball_points(gen.rng(77, 3), L, max(1.5, 1.2 * L ** (1 / 3)))
    zeta = gen.charges(gen.rng(77, 4), L, 0.3, False)
    P = 37
    q = gen.unit_quaternions(gen.rng(77, 5), P)
    tr = gen.sphere_translations(gen.rng(77, 6), P, 9.0)
    sinc = rs.Sinc(cfg.M, cfg.h_M, cfg.L_s, 16, 9.5, 1e-8)
    t = rs.tensor_import(ctx, F, n, b, sinc, z, pos)

    class W:
        protein_positions, protein_charges, ligand_positions, ligand_charges = pos, z, lig, zeta

    import dataclasses
    c2 = dataclasses.replace(cfg, n=n, b=b, K_long=16, r_cut=9.5)
    ref = oracle_score(c2, W, F, q, tr, grad=True)
    gpu = _run(rs, ctx, t, W, q, tr, cfg.sigma, mode=mode)
    assert_parity(gpu, ref, grad=True, label=f"R={R} L={L} mode={mode}")
    t.free()


def test_no_protein_atoms_and_empty_batch(rs, ctx):
    cfg = configs.CONFIG1
    n, b = 64, 10.0
    g = np.random.default_rng(5)
    F = [g.normal(size=(n, 10)) for _ in range(3)]
    sinc = rs.Sinc(cfg.M, cfg.h_M, cfg.L_s, 12, 5.0, 1e-8)
    t = rs.tensor_import(ctx, F, n, b, sinc, np.zeros(0), np.zeros((0, 3)))

    class W:
        protein_positions, protein_charges = np.zeros((0, 3)), np.zeros(0)
        ligand_positions = gen.ball_points(gen.rng(3, 3), 5, 2.0)
        ligand_charges = gen.charges(gen.rng(3, 4), 5, 0.3, False)

    q = gen.unit_quaternions(gen.rng(3, 5), 9)
    tr = gen.sphere_translations(gen.rng(3, 6), 9, 4.0)
    import dataclasses
    c2 = dataclasses.replace(cfg, n=n, b=b, K_long=12, r_cut=5.0)
    ref = oracle_score(c2, W, F, q, tr, grad=True)
    gpu = _run(rs, ctx, t, W, q, tr, 2.5)
    assert_parity(gpu, ref, grad=True, label="N=0")
    empty = rs.score_poses(ctx, t, W.ligand_charges, W.ligand_positions, np.zeros((0, 4)), np.zeros((0, 3)), 2.5)
    assert empty["E"].shape == (0,)


def test_save_load_roundtrip(rs, ctx, cfg1):
    cfg, wl, F, t = cfg1
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "t.rsd")
        t.save(path)
        t2 = rs.tensor_load(ctx, path)
        a = _run(rs, ctx, t, wl, wl.quats, wl.trans, cfg.sigma)
        b = _run(rs, ctx, t2, wl, wl.quats, wl.trans, cfg.sigma)
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), k
        with open(path, "r+b") as f:
            f.seek(200)
            byte = f.read(1)
            f.seek(200)
            f.write(bytes([byte[0] ^ 1]))
        with pytest.raises(rs.RsdError) as e:
            rs.tensor_load(ctx, path)
        assert e.value.code == -6
    F2 = t.export()
    for d in range(3):
        assert np.array_equal(F2[d], F[d])


def test_budget_and_argument_errors(rs, cfg1):
    cfg, wl, F, t = cfg1
    small = rs.Context(0, hbm_budget=1 << 20)
    with pytest.raises(rs.RsdError) as e:
        rs.tensor_import(small, F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges, wl.protein_positions)
    assert e.value.code == -2
    small.close()
    ctx = rs.Context(0)
    bad = wl.protein_positions.copy()
    bad[3, 1] = cfg.b + 1.0
    with pytest.raises(rs.RsdError) as e:
        rs.tensor_import(ctx, F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges, bad)
    assert e.value.code == -1
    with pytest.raises(rs.RsdError) as e:
        rs.tensor_import(ctx, F, cfg.n + 1, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges,
                         wl.protein_positions)
    assert e.value.code == -1
    q = wl.quats[:3].copy()
    q[1] *= 1.001
    with pytest.raises(rs.RsdError) as e:    # host pointers: an invalid pose is an argument error
        rs.score_poses(ctx, t, wl.ligand_charges, wl.ligand_positions, q, wl.trans[:3], cfg.sigma)
    assert e.value.code == -1
    ctx.close()


@pytest.fixture(scope="module")
def cfg2(rs, ctx):
    cfg = configs.CONFIG2
    wl = configs.make(cfg, P=4096)
    tk, can = oracle_factors(cfg, wl)
    t = rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges,
                         wl.protein_positions)
    yield cfg, wl, can.F, t
    t.free()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", [2, 1])
def test_cfg2_parity_4096_poses_and_thresholds(rs, ctx, cfg2, mode):
    cfg, wl, F, t = cfg2
    q1, t1 = near_threshold_poses(cfg, wl, wl.quats, wl.trans, cfg.sigma, 48)
    q2, t2 = near_threshold_poses(cfg, wl, wl.quats[48:], wl.trans[48:], cfg.r_cut, 48)
    q = np.concatenate([wl.quats, q1, q2])
    tr = np.concatenate([wl.trans, t1, t2])
    ref = oracle_score(cfg, wl, F, q, tr, grad=False)
    g = _run(rs, ctx, t, wl, q, tr, cfg.sigma, grad=False, mode=mode)
    worst = assert_parity(g, ref, label=f"cfg2 mode {mode}")
    print(f"cfg2 parity: worst energy error {worst:.3g} x tolerance; accept {np.mean(ref['flags'] & 1):.3f}")


def test_context_freed_before_its_tensor(rs):
    """rsd_context_free with live tensors defers the release to the last rsd_tensor_free."""
    cfg = configs.CONFIG1
    g = np.random.default_rng(9)
    n, b = 32, 10.0
    F = [g.normal(size=(n, 5)) for _ in range(3)]
    pos = gen.ball_points(gen.rng(4, 1), 10, 3.0)
    z = gen.charges(gen.rng(4, 2), 10, 0.3, True)
    c = rs.Context(0)
    t = rs.tensor_import(c, F, n, b, rs.Sinc(cfg.M, cfg.h_M, cfg.L_s, 12, 5.0, 1e-8), z, pos)
    c.close()
    with pytest.raises(rs.RsdError) as e:
        rs.score_poses(_ClosedCtx(c), t, z[:2], pos[:2],
                       gen.unit_quaternions(gen.rng(4, 5), 1), np.zeros((1, 3)), 2.5)
    assert e.value.code == -1
    t.free()


class _ClosedCtx:
    """Carries the raw handle of a context after close() to call into the library with it."""

    def __init__(self, c):
        self.handle = c._raw


def test_short_range_table_and_exponentials_agree(rs, ctx, cfg1):
    """Energy-only scoring evaluates the short-range Gaussians from the context's piecewise
    polynomial table; a context with option short_poly = 0 evaluates the exponentials.  Both
    meet the bar against the oracle, with the same flags and counts."""
    cfg, wl, F, t = cfg1
    import torch
    c0 = rs.Context(0)
    c0.set_option("short_poly", 0)
    t0 = rs.tensor_import(c0, F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges, wl.protein_positions)
    q1, t1 = near_threshold_poses(cfg, wl, wl.quats, wl.trans * (15.5 / 18.0), cfg.r_cut * 0.5, 24)
    q = np.concatenate([wl.quats, q1])
    tr = np.concatenate([wl.trans, t1])
    ref = oracle_score(cfg, wl, F, q, tr)
    for mode in (1, 2):
        a = _run(rs, ctx, t, wl, q, tr, cfg.sigma, grad=False, mode=mode)
        b = _run(rs, c0, t0, wl, q, tr, cfg.sigma, grad=False, mode=mode)
        wa = assert_parity(a, ref, label=f"table, mode {mode}")
        wb = assert_parity(b, ref, label=f"exponentials, mode {mode}")
        assert np.array_equal(a["flags"], b["flags"]) and np.array_equal(a["counts"], b["counts"])
        print(f"mode {mode}: worst error table {wa:.3g}, exponentials {wb:.3g} x tolerance")
    ctx.set_option("score_mode", 0)
    c0.set_option("score_mode", 0)
    t0.free()
    c0.close()
    torch.cuda.synchronize()
