"""GPU test of the continuous-batching server: mixed requests over three resident tensors
under a tight HBM budget, split into pose slices across rounds; every served result equals
the same request scored alone, and a sample of every served request matches the oracle on
the tensors' own factors."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import TOL, oracle_factors  # noqa: E402
from oracle import score as oscore, sinc as osinc  # noqa: E402
from workloads import configs, generators as gen  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
@pytest.mark.parametrize("pose_order", [0, 1, 2])
def test_server_mix_equals_alone_under_budget(pose_order):
    """Requests sliced in spatial order (pose_order 1: every request; 0: those of at least two
    minimum slices; 2: none) come back in request order."""
    import torch
    assert torch.cuda.is_available()
    import paper_2510_26611_amd as rs
    from paper_2510_26611_amd import serve

    ctx = rs.Context(0)
    cfg = configs.CONFIG1
    wl = configs.make(cfg)
    _, can = oracle_factors(cfg, wl)
    tensors = {"cfg1": rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges,
                                        wl.protein_positions)}
    pos = gen.ball_points(gen.rng(61, 1), 300, 8.0)
    z = gen.charges(gen.rng(61, 2), 300, 0.4, True)
    tensors["built"] = rs.build_rs_tensor(ctx, z, pos, 256, 30.0, rs.Sinc(cfg.M, cfg.h_M, cfg.L_s, 16, 9.5, 1e-8))
    g = np.random.default_rng(5)
    tensors["rand"] = rs.tensor_import(ctx, [g.normal(size=(96, 257)) * 0.01 for _ in range(3)], 96, 30.0,
                                       rs.Sinc(cfg.M, cfg.h_M, cfg.L_s, 16, 9.5, 1e-8), z[:60], pos[:60] * 0.7)
    radius = {"cfg1": 18.0, "built": 20.0, "rand": 9.0}
    gt = np.random.default_rng(8)
    names = list(tensors)
    trace, t = [], 0.0
    for i in range(40):
        t += gt.exponential(0.002)
        name = names[i % 3]
        L = int(gt.integers(1, 121))
        P = int(gt.integers(1, 3000))
        lig = gen.ball_points(gen.rng(5, 3, i), L, max(1.5, 1.2 * L ** (1 / 3)))
        zeta = gen.charges(gen.rng(5, 4, i), L, 0.3, False)
        q = gen.unit_quaternions(gen.rng(5, 5, i), P)
        tr = gen.sphere_translations(gen.rng(5, 6, i), P, radius[name])
        trace.append(serve.Request(i, name, zeta, lig, q, tr, 2.5, t))
    trace.append(serve.Request(99, "nope", zeta, lig, q, tr, 2.5, t))
    resident = sum(x.query()["bytes"] for x in tensors.values())
    nchunk = max(-(-x.query()["R"] // 64) for x in tensors.values())
    mean_cost = np.mean([serve.request_bytes(r) for r in trace[:40]])
    # small rounds so that requests are split into slices; room for about four requests in flight
    scratch = 2 * serve.round_scratch_bytes(2000, nchunk)
    srv = serve.Server(tensors, hbm_budget_bytes=int(resident + scratch + 4 * mean_cost), round_poses=2000,
                       min_slice=256, options=dict(pose_order=pose_order))
    stats = srv.run(trace)
    print(f"served {stats['served']} p50 {stats['latency_p50_s'] * 1e3:.2f} ms p99 {stats['latency_p99_s'] * 1e3:.2f} ms")
    assert stats["served"] == 40 and stats["rejected"] == 1
    want = {0: sum(r.P >= 512 for r in trace[:40]), 1: sum(r.P >= 2 for r in trace[:40]), 2: 0}[pose_order]
    assert srv.ordered == want and (pose_order == 2 or want > 0)
    assert trace[-1].error == serve.E_UNKNOWN_PROTEIN
    assert np.isfinite(stats["latency_p99_s"])
    ctx.set_option("score_mode", 2)
    bad = []
    for r in trace[:40]:
        alone = rs.score_poses(ctx, tensors[r.protein], r.lig_charges, r.lig_positions, r.quats, r.trans, r.vdw_min)
        for k in ("E", "flags", "counts"):
            if not np.array_equal(r.result[k], alone[k], equal_nan=True):
                diff = np.nonzero(~((r.result[k] == alone[k]) | (np.isnan(r.result[k].astype(float)) &
                                                                  np.isnan(alone[k].astype(float)))))[0]
                print(f"rid {r.rid} protein {r.protein} L {r.L} P {r.P} key {k}: {diff.size} poses differ, "
                      f"first {diff[:5]}, batch {r.result[k][diff[:3]]} alone {alone[k][diff[:3]]} "
                      f"flags {alone['flags'][diff[:3]]}")
                bad.append((r.rid, k))
    assert not bad, bad
    # served results against the oracle (PLIE, Sec. 3.4) on each tensor's own factors
    sinc16 = osinc.split(*osinc.sinc_table(cfg.M, cfg.h_M, cfg.L_s), 16)[1]
    ref_args = {"cfg1": (can.F, cfg.n, cfg.b, wl.protein_positions, wl.protein_charges,
                         *osinc.split(*osinc.sinc_table(cfg.M, cfg.h_M, cfg.L_s), cfg.K_long)[1], cfg.r_cut),
                "built": (tensors["built"].export(), 256, 30.0, pos, z, *sinc16, 9.5),
                "rand": (tensors["rand"].export(), 96, 30.0, pos[:60] * 0.7, z[:60], *sinc16, 9.5)}
    gs = np.random.default_rng(77)
    checked = 0
    for r in trace[:40]:
        sample = np.sort(gs.choice(r.P, min(r.P, 24), replace=False))
        ref = oscore.score(*ref_args[r.protein], r.lig_charges, r.lig_positions, r.quats[sample], r.trans[sample],
                           r.vdw_min)
        assert np.array_equal(r.result["flags"][sample], ref["flags"]), r.rid
        assert np.array_equal(r.result["counts"][sample], ref["counts"]), r.rid
        E = r.result["E"][sample]
        assert np.array_equal(np.isnan(E), np.isnan(ref["E"])), r.rid
        ok = ~np.isnan(ref["E"])
        assert np.all(np.abs(E[ok] - ref["E"][ok]) <= TOL * ref["scale"][ok]), r.rid
        checked += len(sample)
    print(f"{checked} served poses at parity with the oracle")
    srv.close()
    for x in tensors.values():
        x.free()
    ctx.close()
