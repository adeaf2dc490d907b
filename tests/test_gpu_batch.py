"""GPU tests of rsd_batch_*: many requests per launch, alone-vs-in-the-mix identity, graph replays."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import assert_parity, oracle_factors, oracle_score  # noqa: E402
from oracle import score as oscore, sinc as osinc  # noqa: E402
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
    t1 = rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges, wl.protein_positions)
    g = np.random.default_rng(31)
    pos = gen.ball_points(gen.rng(81, 1), 60, 6.0)
    z = gen.charges(gen.rng(81, 2), 60, 0.3, True)
    sinc2 = rs.Sinc(cfg.M, cfg.h_M, cfg.L_s, 16, 9.5, 1e-8)
    F2 = [g.normal(size=(96, 257)) * 0.01 for _ in range(3)]
    t2 = rs.tensor_import(ctx, F2, 96, 30.0, sinc2, z, pos)
    t3 = rs.tensor_import(ctx, [np.zeros((96, 0))] * 3, 96, 30.0, sinc2, z, pos)
    yield rs, ctx, torch, dict(cfg=cfg, wl=wl, F=can.F, t1=t1, t2=t2, t3=t3, F2=F2, z2=z, pos2=pos, sinc2=sinc2)
    for t in (t1, t2, t3):
        t.free()
    ctx.close()


def _requests(torch, T, seed):
    """Mixed requests: three tensors, ligands of 1..600 atoms (the last needs more than 64 KB of
    LDS in the long-range kernel), 0..1000 poses."""
    specs = [("t1", 12, 128, 18.0), ("t2", 65, 1000, 9.0), ("t1", 1, 1, 12.0), ("t3", 7, 50, 9.0),
             ("t2", 200, 333, 14.0), ("t1", 12, 0, 18.0), ("t2", 13, 257, 9.0), ("t1", 30, 700, 17.0),
             ("t2", 600, 150, 16.0)]
    reqs = []
    for i, (tn, L, P, rad) in enumerate(specs):
        if tn == "t1" and L == 12:
            lig, zeta = T["wl"].ligand_positions, T["wl"].ligand_charges
        else:
            lig = gen.ball_points(gen.rng(90 + i, 3), L, max(1.5, 1.2 * L ** (1 / 3)))
            zeta = gen.charges(gen.rng(90 + i, 4), L, 0.3, False)
        q = gen.unit_quaternions(gen.rng(seed + i, 5), P)
        tr = gen.sphere_translations(gen.rng(seed + i, 6), P, rad)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
        reqs.append(dict(tensor=T[tn], lig_charges=d(zeta), lig_positions=d(lig), quats=d(q.reshape(P, 4)),
                         trans=d(tr.reshape(P, 3)), vdw_min=2.5, np_lig=lig, np_zeta=zeta, np_q=q, np_t=tr))
    return reqs


def _alone(rs, ctx, torch, r):
    ctx.set_option("score_mode", 2)
    out = rs.score_poses(ctx, r["tensor"], r["lig_charges"], r["lig_positions"], r["quats"], r["trans"], r["vdw_min"],
                         energies_long=True)
    ctx.set_option("score_mode", 0)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _mk_out(torch, P):
    return dict(E=torch.empty(P, dtype=torch.float64, device="cuda"),
                E_long=torch.empty(P, dtype=torch.float64, device="cuda"),
                flags=torch.empty(P, dtype=torch.uint8, device="cuda"),
                counts=torch.empty(P, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("order", [0, 1])
def test_batch_equals_alone_bitwise_and_oracle(env, order, mode):
    """order 1: every request's long range takes its poses in spatial order (option pose_order);
    mode 1: requests grouped into launches by LDS occupancy, 2: one persistent launch."""
    rs, ctx, torch, T = env
    ctx.set_option("pose_order", order)
    ctx.set_option("batch_mode", mode)
    reqs = _requests(torch, T, 500)
    for r in reqs:
        r["out"] = _mk_out(torch, r["quats"].shape[0])
    b = rs.Batch(ctx, reqs)
    b.run()
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        got = {k: v.cpu().numpy() for k, v in r["out"].items()}
        ref = _alone(rs, ctx, torch, r)
        for k in ("E", "E_long", "flags", "counts"):
            assert np.array_equal(got[k], ref[k], equal_nan=True), (i, k)
    # and the first request against the oracle
    r0 = reqs[0]
    cfg = T["cfg"]
    ref = oracle_score(cfg, T["wl"], T["F"], r0["np_q"], r0["np_t"])
    got = {k: v.cpu().numpy() for k, v in r0["out"].items()}
    assert_parity(got, ref, label="batch request 0")
    # the 600-atom ligand against the oracle on the random factors
    rb = reqs[-1]
    sc = T["sinc2"]
    t, w = osinc.sinc_table(sc.M, sc.h_M, sc.L_s)
    _, (ts, ws) = osinc.split(t, w, sc.K_long)
    ref = oscore.score(T["F2"], 96, 30.0, T["pos2"], T["z2"], ts, ws, sc.r_cut, rb["np_zeta"], rb["np_lig"],
                       rb["np_q"], rb["np_t"], rb["vdw_min"])
    got = {k: v.cpu().numpy() for k, v in rb["out"].items()}
    assert_parity(got, ref, label="batch request with 600 ligand atoms")
    b.free()
    ctx.set_option("pose_order", 0)
    ctx.set_option("batch_mode", 0)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("order", [0, 1])
def test_batch_graph_replays_match_eager(env, order, mode):
    rs, ctx, torch, T = env
    ctx.set_option("pose_order", order)
    ctx.set_option("batch_mode", mode)
    reqs = _requests(torch, T, 700)
    for r in reqs:
        r["out"] = _mk_out(torch, r["quats"].shape[0])
    b = rs.Batch(ctx, reqs)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    ctx.set_stream(s.cuda_stream)
    with torch.cuda.stream(s):
        b.run()                       # warm-up outside capture
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        b.run()
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        # new poses into the same buffers, eager work between replays
        for i, r in enumerate(reqs):
            P = r["quats"].shape[0]
            q = gen.unit_quaternions(gen.rng(900 + 10 * rep + i, 5), P).reshape(P, 4)
            r["quats"].copy_(torch.from_numpy(q))
        torch.cuda.synchronize()
        refs = [_alone(rs, ctx, torch, r) for r in reqs]
        graph.replay()
        torch.cuda.synchronize()
        for i, r in enumerate(reqs):
            got = {k: v.cpu().numpy() for k, v in r["out"].items()}
            for k in ("E", "E_long", "flags", "counts"):
                assert np.array_equal(got[k], refs[i][k], equal_nan=True), (rep, i, k)
    del graph
    b.free()
    ctx.set_option("pose_order", 0)
    ctx.set_option("batch_mode", 0)


def test_batch_made_before_a_smaller_one_still_runs(env):
    """Two batches whose long-range launches need more LDS than the default, the larger made
    first: running it after the second was made still works and matches the request alone."""
    rs, ctx, torch, T = env
    big, mid = _requests(torch, T, 300)[-1], None
    lig = gen.ball_points(gen.rng(95, 3), 400, 1.2 * 400 ** (1 / 3))
    zeta = gen.charges(gen.rng(95, 4), 400, 0.3, False)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    mid = dict(big, lig_charges=d(zeta), lig_positions=d(lig))
    for r in (big, mid):
        r["out"] = _mk_out(torch, r["quats"].shape[0])
    b1 = rs.Batch(ctx, [big])
    b2 = rs.Batch(ctx, [mid])
    b1.run()
    b2.run()
    torch.cuda.synchronize()
    for r in (big, mid):
        got = {k: v.cpu().numpy() for k, v in r["out"].items()}
        ref = _alone(rs, ctx, torch, r)
        for k in ("E", "E_long", "flags", "counts"):
            assert np.array_equal(got[k], ref[k], equal_nan=True), k
    b1.free()
    b2.free()


def test_batch_argument_errors(env):
    rs, ctx, torch, T = env
    reqs = _requests(torch, T, 11)[:2]
    bad = dict(reqs[0])
    bad["quats"] = reqs[0]["quats"][:0]
    bad["trans"] = reqs[0]["trans"][:0]
    b = rs.Batch(ctx, [bad])          # a request with no poses is accepted and does nothing
    b.run()
    b.free()
    with pytest.raises(rs.RsdError) as e:
        rs.Batch(ctx, [])
    assert e.value.code == -1
