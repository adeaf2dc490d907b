"""Full-size parity of the serving workload (config 5) on sampled outputs.

The smallest (1,000 atoms, n = 8192) and the largest (100,000 atoms, n = 16384) resident
proteins are built on the device at their real sizes. Then:
  * the tensor at sampled grid nodes is compared with the uncompressed long-range tensor T0
    of eq. 2.6, which the oracle evaluates node by node (the RHOSVD truncation is the only
    difference, so the bound is the frozen multiple P2_C of eps * max|T0| calibrated on the
    smaller workloads);
  * poses of requests drawn from the serving trace are scored in one batch (the launch
    configuration of the server) and compared with the oracle scoring the same exported
    factors: flags and counts bit-exact, energies within 1e-10 of the summation scale.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import P2_C, assert_parity, sinc_parts  # noqa: E402
from oracle import score as oscore, tensor as otensor  # noqa: E402
from workloads import configs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2510_26611_amd as rs
    ctx = rs.Context(0)
    yield rs, torch, ctx
    ctx.close()


def _requests_for(protein: int, count: int):
    """The first `count` requests of the serving trace that ask for `protein` (pose counts
    scaled down to a sample the oracle scores in seconds)."""
    out = []
    for r in configs.make_serving_trace(120, pose_scale=0.0016):
        if r.protein == protein:
            out.append(r)
            if len(out) == count:
                break
    assert len(out) == count
    return out


@pytest.mark.timeout(900)
@pytest.mark.parametrize("protein", [0, 7])
def test_serving_protein_full_size(env, protein):
    rs, torch, ctx = env
    cfg, pos, z = configs.make_serving_proteins(protein + 1)[protein]
    t = rs.build_rs_tensor(ctx, z, pos, cfg.n, cfg.b, rs.Sinc.from_config(cfg))
    q = t.query()
    print(f"protein {protein}: N={cfg.N} n={cfg.n} ranks={q['ranks']} R={q['R']}", flush=True)
    F = t.export()
    # 1. the tensor against T0 at sampled nodes inside the protein's neighbourhood and far from it
    (tl, wl), (ts, ws) = sinc_parts(cfg)
    g = np.random.default_rng(40 + protein)
    idx = g.integers(0, cfg.n, size=(600, 3))
    T0 = otensor.long_range_at_nodes(z, pos, tl, wl, cfg.n, cfg.b, idx)
    Tg = np.sum(F[0][idx[:, 0]] * F[1][idx[:, 1]] * F[2][idx[:, 2]], axis=1)
    err = np.max(np.abs(Tg - T0))
    print(f"  max|T - T0| = {err:.3e}, max|T0| = {np.max(np.abs(T0)):.3e}", flush=True)
    assert err <= P2_C * cfg.eps * np.max(np.abs(T0))
    # 2. sampled requests scored in one batch vs the oracle on the same factors
    reqs = _requests_for(protein, 2)
    for r in reqs:                                  # at most 48 poses each: the oracle loops over all atoms
        r.quats, r.trans = r.quats[:48], r.trans[:48]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    batch_reqs = [dict(tensor=t, lig_charges=d(r.ligand_charges), lig_positions=d(r.ligand_positions),
                       quats=d(r.quats), trans=d(r.trans), vdw_min=r.sigma) for r in reqs]
    b = rs.Batch(ctx, batch_reqs)
    b.run()
    torch.cuda.synchronize()
    for r, out in zip(reqs, b.outputs()):
        got = {k: v.cpu().numpy() for k, v in out.items()}
        ref = oscore.score(F, cfg.n, cfg.b, pos, z, ts, ws, cfg.r_cut, r.ligand_charges, r.ligand_positions,
                           r.quats, r.trans, r.sigma, pose_chunk=2)
        print(f"  request {r.index}: L={r.ligand_charges.size} P={r.quats.shape[0]} "
              f"accepted {int(np.sum(ref['flags'] & 1))} in domain {int(np.sum((ref['flags'] >> 1) & 1))}", flush=True)
        assert np.any(ref["flags"] & 2)
        assert_parity(got, ref, label=f"protein {protein} request {r.index}")
    b.free()
    t.free()
