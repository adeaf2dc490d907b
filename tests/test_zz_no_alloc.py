"""GPU test of rsd_score_poses_noalloc, the allocation-free variant of rsd_score_poses: its
results equal rsd_score_poses's on the same inputs, over two calls in a row (the second one
smaller, with gradients) that share the library's static scratch, and a sample matches the
oracle on the tensor's exported factors."""
import ctypes
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import assert_parity, oracle_score  # noqa: E402
from workloads import configs  # noqa: E402

pytestmark = pytest.mark.gpu


def _outs(torch, P, grad):
    o = dict(E=torch.full((P,), -7.0, dtype=torch.float64, device="cuda"),
             E_long=torch.full((P,), -7.0, dtype=torch.float64, device="cuda"),
             flags=torch.full((P,), 255, dtype=torch.uint8, device="cuda"),
             counts=torch.full((P,), -1, dtype=torch.int32, device="cuda"))
    if grad:
        o["grads"] = torch.full((P, 6), -7.0, dtype=torch.float64, device="cuda")
    return o


@pytest.mark.timeout(600)
def test_noalloc_equals_score_poses_twice():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2510_26611_amd as rs
    from paper_2510_26611_amd import _lib

    cfg = configs.CONFIG2
    wl = configs.make(cfg, P=600_000)
    ctx = rs.Context(0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    t = rs.build_rs_tensor(ctx, to(wl.protein_charges), to(wl.protein_positions), cfg.n, cfg.b,
                           rs.Sinc.from_config(cfg))
    lz, lx = to(wl.ligand_charges), to(wl.ligand_positions)
    F = t.export()
    print(f"cfg2 tensor R={F[0].shape[1]}", flush=True)
    # call 1: 600,000 poses (more than one slice of the static scratch), energies only;
    # call 2: 20,000 other poses with gradients
    calls = [(0, 600_000, False), (300_000, 320_000, True)]
    for k, (p0, p1, grad) in enumerate(calls):
        q, tr = to(wl.quats[p0:p1]), to(wl.trans[p0:p1])
        P = p1 - p0
        ref = rs.score_poses(ctx, t, lz, lx, q, tr, cfg.sigma, grads=grad, energies_long=True)
        got = rs.score_poses_noalloc(ctx, t, lz, lx, q, tr, cfg.sigma, out=_outs(torch, P, grad))
        torch.cuda.synchronize()
        for key in ref:
            a, b = got[key].cpu().numpy(), ref[key].cpu().numpy()
            assert np.array_equal(a, b, equal_nan=True), f"call {k}: {key} differs from rsd_score_poses"
        sample = np.sort(np.random.default_rng(55 + k).choice(P, 48, replace=False))
        oref = oracle_score(cfg, wl, F, wl.quats[p0:p1][sample], wl.trans[p0:p1][sample], grad=grad)
        idx = torch.from_numpy(sample).cuda()
        assert_parity({key: v[idx].cpu().numpy() for key, v in got.items()}, oref, grad=grad,
                      label=f"noalloc call {k}")
        print(f"call {k}: {P} poses{' with gradients' if grad else ''} equal to rsd_score_poses", flush=True)
    # host arrays need staging memory: refused
    lib = _lib.lib()
    E = np.empty(4)
    fl = np.empty(4, dtype=np.uint8)
    ct = np.empty(4, dtype=np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    st = lib.rsd_score_poses_noalloc(ctx.handle, t.handle, ptr(wl.ligand_charges), ptr(wl.ligand_positions), cfg.L,
                                     ptr(wl.quats), ptr(wl.trans), 4, cfg.sigma, 0, ptr(E), None, ptr(fl), ptr(ct),
                                     None)
    assert st == _lib.RSD_E_INVALID and b"device pointers" in lib.rsd_last_error()
    t.free()
    ctx.close()
