"""GPU tests of rsd_autotune: the recorded launch shape is used by later automatic calls,
results stay at parity with the oracle, and flags/counts do not depend on the shape."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import assert_parity, oracle_factors, oracle_score  # noqa: E402
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
    q = gen.unit_quaternions(gen.rng(71, 5), 3000)
    tr = gen.sphere_translations(gen.rng(71, 6), 3000, 18.0)
    wl.quats, wl.trans = q, tr
    _, can = oracle_factors(cfg, wl)
    t = rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges,
                         wl.protein_positions)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    dev = dict(z=d(wl.ligand_charges), x=d(wl.ligand_positions), q=d(q), t=d(tr))
    yield rs, torch, ctx, cfg, wl, can.F, t, dev
    t.free()
    ctx.close()


def _score(rs, torch, ctx, t, dev, sigma, grads):
    out = rs.score_poses(ctx, t, dev["z"], dev["x"], dev["q"], dev["t"], sigma, grads=grads)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("grads", [False, True])
def test_tuned_shape_is_used_and_stays_at_parity(env, grads):
    rs, torch, ctx, cfg, wl, F, t, dev = env
    ctx.set_option("use_tuning", 0)
    before = _score(rs, torch, ctx, t, dev, cfg.sigma, grads)
    ctx.set_option("use_tuning", 1)
    rep = ctx.autotune(t, dev["z"], dev["x"], dev["q"][:2048], dev["t"][:2048], cfg.sigma, grads=grads)
    print(rep)
    assert rep["score_mode"] in (1, 2) and rep["short_waves"] in (1, 2, 4) and rep["candidates"] >= 3
    # the untuned shape is one of the candidates: the best is no slower than it (timing noise aside)
    assert 0 < rep["best_ms"] <= 1.25 * rep["default_ms"]
    if rep["score_mode"] == 2:
        assert 1 <= rep["poses_per_wave"] <= 4
    # a later automatic call launches the recorded kernels
    ctx.set_timing(True)
    after = _score(rs, torch, ctx, t, dev, cfg.sigma, grads)
    n_long = ctx.kernel_time("long")[0]
    n_fused = ctx.kernel_time("score")[0]
    ctx.set_timing(False)
    assert (n_long, n_fused) == ((1, 0) if rep["score_mode"] == 2 else (0, 1))
    # flags and counts never depend on the shape; energies are at parity either way
    assert np.array_equal(after["flags"], before["flags"]) and np.array_equal(after["counts"], before["counts"])
    ref = oracle_score(cfg, wl, F, wl.quats, wl.trans, grad=grads)
    assert_parity(after, ref, grad=grads, label=f"tuned shape {rep}")
    # with the table ignored the untuned result comes back bit for bit
    ctx.set_option("use_tuning", 0)
    again = _score(rs, torch, ctx, t, dev, cfg.sigma, grads)
    ctx.set_option("use_tuning", 1)
    for k in before:
        assert np.array_equal(again[k], before[k], equal_nan=True), k


def test_explicit_options_override_the_table(env):
    rs, torch, ctx, cfg, wl, F, t, dev = env
    ctx.autotune(t, dev["z"], dev["x"], dev["q"][:1024], dev["t"][:1024], cfg.sigma)
    for mode, kernel in ((1, "score"), (2, "long")):
        ctx.set_option("score_mode", mode)
        ctx.set_timing(True)
        _score(rs, torch, ctx, t, dev, cfg.sigma, False)
        assert ctx.kernel_time(kernel)[0] == 1
        ctx.set_timing(False)
    ctx.set_option("score_mode", 0)
    ctx.set_option("short_waves", 2)
    out = _score(rs, torch, ctx, t, dev, cfg.sigma, False)
    ctx.set_option("short_waves", 0)
    ref = oracle_score(cfg, wl, F, wl.quats, wl.trans)
    assert_parity(out, ref, label="short_waves=2")


def test_autotune_argument_errors(env):
    rs, torch, ctx, cfg, wl, F, t, dev = env
    with pytest.raises(TypeError):
        ctx.autotune(t, wl.ligand_charges, wl.ligand_positions, wl.quats, wl.trans, cfg.sigma)
    with pytest.raises(rs.RsdError) as e:
        ctx.autotune(t, dev["z"], dev["x"], dev["q"][:0], dev["t"][:0], cfg.sigma)
    assert e.value.code == -1
    with pytest.raises(rs.RsdError):
        ctx.set_option("short_waves", 3)


@pytest.mark.parametrize("grads", [False, True])
def test_short_range_on_a_second_stream_is_bitwise_the_same(env, grads):
    """Option overlap: the short-range kernel on a second stream, joined before the combine,
    gives the same bits as one stream (same kernels, same inputs), and stays at parity."""
    rs, torch, ctx, cfg, wl, F, t, dev = env
    ctx.set_option("score_mode", 2)
    try:
        ctx.set_option("overlap", 0)
        one = _score(rs, torch, ctx, t, dev, cfg.sigma, grads)
        ctx.set_option("overlap", 1)
        two = _score(rs, torch, ctx, t, dev, cfg.sigma, grads)
        again = _score(rs, torch, ctx, t, dev, cfg.sigma, grads)
    finally:
        ctx.set_option("overlap", 0)
        ctx.set_option("score_mode", 0)
    for k in one:
        assert np.array_equal(one[k], two[k], equal_nan=True), k
        assert np.array_equal(two[k], again[k], equal_nan=True), k
    assert_parity(two, oracle_score(cfg, wl, F, wl.quats, wl.trans, grad=grads), grad=grads, label="overlap")


def test_shared_mode3_columns_bitwise(env):
    """Tensors made by the canonical -> Tucker -> canonical step keep U_3: the chunk-major energy
    kernel lerps a chunk's distinct U_3 columns once per atom.  The values are the same as the
    gathered F_3 columns, so option shared_mode3 gives the same bits on and off, alone and in a
    batch, with and without gradients, for a built, a restricted and a combined tensor."""
    rs, torch, ctx, cfg, wl, F, t, dev = env
    tb = rs.build_rs_tensor(ctx, wl.protein_charges, wl.protein_positions, cfg.n, cfg.b, rs.Sinc.from_config(cfg))
    site = np.array([18.0, 0.0, 0.0])
    tl = tb.restrict(site - 8.0, site + 8.0, 1e-8)
    tc = rs.tensor_combine(ctx, [tb, tb], 1e-8)
    qs = dev["q"].clone()
    ts = dev["t"].clone()
    ts[:1500] = torch.from_numpy(site[None, :] + gen.sphere_translations(gen.rng(73, 6), 1500, 2.0)).cuda()
    ctx.set_option("score_mode", 2)
    try:
        for tt in (tb, tl, tc):
            out = {}
            for opt in (0, 1):
                ctx.set_option("shared_mode3", opt)
                o = rs.score_poses(ctx, tt, dev["z"], dev["x"], qs, ts, cfg.sigma)
                torch.cuda.synchronize()
                out[opt] = {k: v.cpu().numpy() for k, v in o.items()}
            for k in out[0]:
                assert np.array_equal(out[0][k], out[1][k], equal_nan=True), k
            b = rs.Batch(ctx, [dict(tensor=tt, lig_charges=dev["z"], lig_positions=dev["x"], quats=qs, trans=ts,
                                    vdw_min=cfg.sigma)])
            b.run()
            torch.cuda.synchronize()
            for k, v in b.outputs()[0].items():
                assert np.array_equal(v.cpu().numpy(), out[1][k], equal_nan=True), k
            b.free()
            # the adjoint path takes the mode-3 row differences from U_3 too
            outg = {}
            for opt in (0, 1):
                ctx.set_option("shared_mode3", opt)
                o = rs.score_poses(ctx, tt, dev["z"], dev["x"], qs, ts, cfg.sigma, grads=True)
                torch.cuda.synchronize()
                outg[opt] = {k: v.cpu().numpy() for k, v in o.items()}
            for k in outg[0]:
                assert np.array_equal(outg[0][k], outg[1][k], equal_nan=True), k
    finally:
        ctx.set_option("shared_mode3", 1)
        ctx.set_option("score_mode", 0)
    for tt in (tl, tc, tb):
        tt.free()


def test_gather_probe_and_layout():
    """rsd_probe_gather times the long-range gathers' pattern alone (the roofline the scoring
    kernel is reported against); rsd_tensor_layout counts the chunks that take mode 3 from U_3."""
    import torch
    assert torch.cuda.is_available()
    import paper_2510_26611_amd as rs
    ctx = rs.Context(0)
    r = rs.probe_gather(ctx, 1024, 16)
    assert r["ms"] > 0 and r["bytes"] == 8192 * 4 * 16 * 2 * 2 * 4 * 32 * 16
    assert 1e3 < r["gbs"] < 1e6
    for bad in (1000, 2, 32768):
        with pytest.raises(rs.RsdError):
            rs.probe_gather(ctx, bad, 16)
    # the 5,000-atom protein: about 26 columns per core slice, so most 64-column chunks touch at
    # most 4 slices (the 200-atom one has 7 per slice: its chunks touch 9 or more)
    cfg = configs.CONFIG2
    wl = configs.make(cfg, P=1)
    t = rs.build_rs_tensor(ctx, wl.protein_charges, wl.protein_positions, cfg.n, cfg.b, rs.Sinc.from_config(cfg))
    lay = t.layout()
    print(f"layout: {lay}")
    assert lay["nchunk"] == -(-t.query()["R"] // 64) and 0 < lay["shared_mode3"] <= lay["nchunk"]
    ti = rs.tensor_import(ctx, t.export(), cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges,
                          wl.protein_positions)
    assert ti.layout()["shared_mode3"] == 0
    t.free()
    ti.free()
    ctx.close()


def test_cell_edge_tuner_keeps_parity():
    """rsd_autotune_cells times scoring with the cell list rebuilt at edges r_cut / 3..6 and keeps
    the fastest; counts and flags are the same at every edge and energies stay at parity with the
    oracle (only the order of the short-range sum depends on the cells)."""
    import torch
    assert torch.cuda.is_available()
    import paper_2510_26611_amd as rs
    cfg = configs.CONFIG2
    wl = configs.make(cfg, P=16384)
    ctx = rs.Context(0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    t = rs.build_rs_tensor(ctx, d(wl.protein_charges), d(wl.protein_positions), cfg.n, cfg.b, rs.Sinc.from_config(cfg))
    lz, lx, q, tr = d(wl.ligand_charges), d(wl.ligand_positions), d(wl.quats), d(wl.trans)
    before = {k: v.cpu().numpy() for k, v in rs.score_poses(ctx, t, lz, lx, q, tr, cfg.sigma).items()}
    rep = ctx.autotune_cells(t, lz, lx, q, tr, cfg.sigma)
    print(f"cell tuner: {rep}")
    assert rep["div"] in (3, 4, 5, 6) and all(v > 0 for v in rep["ms"].values())
    assert rep["ms"][rep["div"]] == min(rep["ms"].values())
    after = {k: v.cpu().numpy() for k, v in rs.score_poses(ctx, t, lz, lx, q, tr, cfg.sigma).items()}
    assert np.array_equal(before["flags"], after["flags"]) and np.array_equal(before["counts"], after["counts"])
    F = t.export()
    sample = np.arange(0, 16384, 64)
    ref = oracle_score(cfg, wl, F, wl.quats[sample], wl.trans[sample])
    assert_parity({k: v[sample] for k, v in after.items()}, ref, label="after the cell tuner")
    t.free()
    ctx.close()


def test_chunks_per_item_bitwise(env):
    """A long-range work item may take several rank chunks of one pose block, forming the pose
    transforms once; each chunk's partial sums are the same arithmetic, so chunks_per_item
    1 .. 4 give the same bits, alone and in a batch, with and without gradients, with the
    mode-3 lerps from U_3 and from the gathered columns, in spatial and in input order.  The
    5,000-atom protein's tensor has 29 rank chunks, so 2, 3 and 4 leave a partial last item."""
    rs, torch, ctx, cfg, wl, F, t, dev = env
    c2 = configs.CONFIG2
    w2 = configs.make(c2, P=1)
    tb = rs.build_rs_tensor(ctx, w2.protein_charges, w2.protein_positions, c2.n, c2.b, rs.Sinc.from_config(c2))
    assert tb.layout()["nchunk"] == 29
    qs, ts = dev["q"], dev["t"]
    ctx.set_option("score_mode", 2)
    try:
        for u3 in (1, 0):
            ctx.set_option("shared_mode3", u3)
            for order in (1, 2):
                ctx.set_option("pose_order", order)
                ref = {}
                for grads in (False, True):
                    out = {}
                    for cpi in (1, 2, 3, 4):
                        ctx.set_option("chunks_per_item", cpi)
                        o = rs.score_poses(ctx, tb, dev["z"], dev["x"], qs, ts, c2.sigma, grads=grads)
                        torch.cuda.synchronize()
                        out[cpi] = {k: v.cpu().numpy() for k, v in o.items()}
                    for cpi in (2, 3, 4):
                        for k in out[1]:
                            assert np.array_equal(out[1][k], out[cpi][k], equal_nan=True), (u3, order, grads, cpi, k)
                    ref[grads] = out[1]
                ctx.set_option("chunks_per_item", 3)
                b = rs.Batch(ctx, [dict(tensor=tb, lig_charges=dev["z"], lig_positions=dev["x"], quats=qs,
                                        trans=ts, vdw_min=c2.sigma)])
                b.run()
                torch.cuda.synchronize()
                for k, v in b.outputs()[0].items():
                    if k in ref[False]:
                        assert np.array_equal(v.cpu().numpy(), ref[False][k], equal_nan=True), (u3, order, k)
                b.free()
    finally:
        for name, v in (("chunks_per_item", 0), ("shared_mode3", 1), ("pose_order", 0), ("score_mode", 0)):
            ctx.set_option(name, v)
    tb.free()


# accepted values of every context option (include/rsdock.h); one value just outside each range
_OPTION_RANGES = {
    "score_mode": ([0, 1, 2], [-1, 3]),
    "poses_per_wave": ([0, 1, 2, 3, 4], [-1, 5]),
    "eig_solver": ([0, 1, 2], [-1, 3]),
    "t2c_solver": ([0, 1, 2, 3], [-1, 4]),
    "short_waves": ([0, 1, 2, 4], [-1, 3, 8]),
    "use_tuning": ([0, 1], [-1, 2]),
    "shared_mode3": ([0, 1], [-1, 2]),
    "short_poly": ([0, 1], [-1, 2]),
    "pose_order": ([0, 1, 2], [-1, 3]),
    "chunks_per_item": ([0, 1, 2, 3, 4], [-1, 5]),
    "qr_solver": ([0, 1], [-1, 2]),
    "batch_mode": ([0, 1, 2], [-1, 3]),
    "overlap": ([0, 1], [-1, 2]),
    "factors": ([0, 1, 2, 3], [-1, 4]),
    "svd_solver": ([0, 1, 2, 3, 4], [-1, 5]),
    "gram_solver": ([0, 1, 2], [-1, 3]),
}


def test_every_option_accepts_its_range_and_rejects_the_rest():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2510_26611_amd as rs
    ctx = rs.Context(0)
    try:
        for name, (good, bad) in _OPTION_RANGES.items():
            for v in good:
                ctx.set_option(name, v)
            for v in bad:
                with pytest.raises(rs.RsdError) as e:
                    ctx.set_option(name, v)
                assert e.value.code == -1, (name, v)
            ctx.set_option(name, 0)
        for name in ("no_such_option", "", "score_mode "):
            with pytest.raises(rs.RsdError) as e:
                ctx.set_option(name, 0)
            assert e.value.code == -1, name
    finally:
        ctx.close()
