"""GPU tests of rsd_self_energy (Prop. 3.2): the molecule's own energy from its tensor, against
the oracle evaluating the same factors.  Tolerance: 1e-10 of the FP64 summation scale
sum_j |z_j| (|P_l(x_j)| + |z_j| W0) for the long-range part and sum_j |z_j| sum_m |z_m| g(d) for
the short-range part (the short-range pair set is decided bit for bit on both sides)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import oracle_factors, sinc_parts  # noqa: E402
from oracle import energy as oenergy, score as oscore  # noqa: E402
from workloads import configs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2510_26611_amd as rs
    ctx = rs.Context(0)
    yield rs, ctx
    ctx.close()


def _check(cfg, wl, F, E_long, E_short):
    (tl, wlong), (ts, ws) = sinc_parts(cfg)
    ref_long, ref_short = oenergy.self_energy(F, cfg.n, cfg.b, wl.protein_positions, wl.protein_charges, wlong, ts,
                                              ws, cfg.r_cut)
    z = wl.protein_charges
    v = oscore.long_range(F, cfg.n, cfg.b, wl.protein_positions)[0]
    scale_l = float(np.sum(np.abs(z) * (np.abs(v) + np.abs(z) * np.sum(wlong))))
    D2 = oscore.pair_d2(wl.protein_positions, wl.protein_positions)
    np.fill_diagonal(D2, np.inf)
    j, m = np.nonzero(D2 < cfg.r_cut ** 2)
    g = np.exp(-np.outer(D2[j, m], ts * ts)) @ ws
    scale_s = float(np.sum(np.abs(z[j] * z[m]) * g)) + 1e-300
    coul = oenergy.coulomb(wl.protein_positions, z)
    print(f"N={len(z)}: E_long gpu {E_long:.12e} oracle {ref_long:.12e} | E_short gpu {E_short:.12e} oracle "
          f"{ref_short:.12e} | sum {E_long + E_short:.9e} vs Coulomb {coul:.9e}")
    assert abs(E_long - ref_long) <= 1e-10 * scale_l
    assert abs(E_short - ref_short) <= 1e-10 * scale_s


def test_self_energy_imported_factors(env):
    rs, ctx = env
    cfg = configs.CONFIG1
    wl = configs.make(cfg, P=1)
    _, can = oracle_factors(cfg, wl)
    t = rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges, wl.protein_positions)
    _check(cfg, wl, can.F, *t.self_energy())
    t.free()


@pytest.mark.timeout(600)
def test_self_energy_cfg2_device_build(env):
    rs, ctx = env
    cfg = configs.CONFIG2
    wl = configs.make(cfg, P=1)
    t = rs.build_rs_tensor(ctx, wl.protein_charges, wl.protein_positions, cfg.n, cfg.b, rs.Sinc.from_config(cfg))
    _check(cfg, wl, t.export(), *t.self_energy())
    t.free()


def test_self_energy_errors(env):
    rs, ctx = env
    cfg = configs.CONFIG1
    wl = configs.make(cfg, P=1)
    _, can = oracle_factors(cfg, wl)
    t = rs.tensor_import(ctx, can.F, cfg.n, cfg.b, rs.Sinc.from_config(cfg), wl.protein_charges, wl.protein_positions)
    loc = t.restrict(np.array([15.0, -3, -3]), np.array([21.0, 3, 3]), 1e-8)
    with pytest.raises(rs.RsdError) as e:
        loc.self_energy()
    assert e.value.code == -5
    loc.free()
    t.free()
