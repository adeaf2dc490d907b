"""Shared helpers of the GPU tests: oracle references and parity assertions."""
from __future__ import annotations

import numpy as np

from oracle import rhosvd, score, sinc
from workloads import configs

TOL = 1e-10   # relative to the FP64 summation-error scale of each pose

# Build correctness where the oracle's exact-SVD compression is too costly on the host (the
# n = 4096 and n = 8192/16384 workloads): max|T_gpu - T0| <= P2_C * eps * max|T0| at sampled
# nodes.  Calibrated on the two workloads where the oracle's own compression is affordable and
# then frozen: the device builds of the 200-atom (n = 512) and 5,000-atom (n = 2048) proteins
# give max|T_gpu - T0| / (eps max|T0|) = 3.7 and 4.4 at 4,000 sampled nodes (the oracle's
# exact-SVD builds: 3.2 and 4.4); P2_C is three times the larger.
P2_C = 13.5
P2_CALIBRATION = 4.5   # what the calibration workloads must stay within for P2_C to hold


def sinc_parts(cfg):
    t, w = sinc.sinc_table(cfg.M, cfg.h_M, cfg.L_s)
    return sinc.split(t, w, cfg.K_long)


def oracle_factors(cfg, wl):
    (tl, wlong), _ = sinc_parts(cfg)
    tk, can = rhosvd.build(wl.protein_charges, wl.protein_positions, tl, wlong, cfg.n, cfg.b, cfg.eps)
    return tk, can


def oracle_score(cfg, wl, F, quats, trans, grad=False):
    _, (ts, ws) = sinc_parts(cfg)
    return score.score(F, cfg.n, cfg.b, wl.protein_positions, wl.protein_charges, ts, ws, cfg.r_cut,
                       wl.ligand_charges, wl.ligand_positions, quats, trans, cfg.sigma, want_grad=grad)


def assert_parity(gpu: dict, ref: dict, grad: bool = False, label: str = ""):
    """Flags and counts bit-exact; energies (and gradients) within TOL of the per-pose scale."""
    f_g = np.asarray(gpu["flags"])
    c_g = np.asarray(gpu["counts"])
    bad_f = np.nonzero(f_g != ref["flags"])[0]
    assert bad_f.size == 0, f"{label}: flags differ at poses {bad_f[:10]}: gpu {f_g[bad_f[:10]]} ref {ref['flags'][bad_f[:10]]}"
    bad_c = np.nonzero(c_g != ref["counts"])[0]
    assert bad_c.size == 0, f"{label}: counts differ at poses {bad_c[:10]}"
    E = np.asarray(gpu["E"])
    nan_ref = np.isnan(ref["E"])
    assert np.array_equal(np.isnan(E), nan_ref), f"{label}: NaN pattern of E differs"
    ok = ~nan_ref
    err = np.abs(E[ok] - ref["E"][ok])
    lim = TOL * ref["scale"][ok] + 1e-300
    worst = np.max(err / lim) if err.size else 0.0
    assert np.all(err <= lim), f"{label}: energy error {worst:.3g} x tolerance"
    if "E_long" in gpu:
        El = np.asarray(gpu["E_long"])
        assert np.array_equal(np.isnan(El), np.isnan(ref["E_long"]))
        e2 = np.abs(El[ok] - ref["E_long"][ok])
        assert np.all(e2 <= lim), f"{label}: long-range energy error"
    if grad:
        G = np.asarray(gpu["grads"])
        assert np.array_equal(np.isnan(G), np.isnan(ref["grads"]))
        eg = np.abs(G[ok] - ref["grads"][ok])
        glim = TOL * ref["grad_scale"][ok][:, None] + 1e-300
        assert np.all(eg <= glim), f"{label}: gradient error {np.max(eg / glim):.3g} x tolerance"
    return worst


def near_threshold_poses(cfg, wl, quats, trans, target, count, offsets=(-1e-15, 0.0, 1e-15)):
    """Move each of the first `count` poses along its closest protein-ligand pair so that the pair
    distance lands on target*(1+o); these poses decide the vdW flag (target = sigma) or a pair count
    (target = r_cut) on the last bits of d^2."""
    _, u = score.ligand_frame(wl.ligand_positions)
    qs, ts = [], []
    for p in range(count):
        y = score.transform(quats[p:p + 1], trans[p:p + 1], u)[0]
        D2 = score.pair_d2(y, wl.protein_positions)
        d = np.sqrt(D2)
        l, m = np.unravel_index(np.argmin(np.abs(d - target)), d.shape)
        vec = (y[l] - wl.protein_positions[m]) / d[l, m]
        o = offsets[p % len(offsets)]
        qs.append(quats[p])
        ts.append(trans[p] + (target * (1.0 + o) - d[l, m]) * vec)
    return np.array(qs), np.array(ts)
