"""Throughput of the RS-tensor pose scorer on one MI355X.

A step is one whole docking job of the 5,000-atom / 50-atom / n=2048 workload:
build the protein's RS tensor on the device (rank reduction + cell list), score
1,000,000 poses (transform, long-range, short-range, vdW flag, pair counts), and
free the tensor.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  `value` = poses per second of the whole job; `roofline`
is for the dominant kernel (the scoring kernel, bound by its factor-row
gathers) from HIP-event timing of its launches inside the timed steps;
`cpu_baseline` is the FP64 oracle timed on this host on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6
METRIC = "poses scored/sec at ≤1e-10 rel err vs FP64 oracle; served p50/p99 latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "long_cfg2_traffic.json")
SCORE_SRC = os.path.join(ROOT, "paper_2510_26611_amd", "csrc", "score.hip")


def _src_hash() -> str:
    with open(SCORE_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(launch_poses: int):
    """HBM bytes per scoring launch from the committed counter summary, if it was taken on this kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("score_src_sha256_16") != _src_hash() or rec.get("poses_per_launch") != launch_poses:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(cfg, wl, sample: int):
    """The oracle as it stands: its own tensor build, then scoring a bounded pose sample."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import rhosvd, score, sinc
    t, w = sinc.sinc_table(cfg.M, cfg.h_M, cfg.L_s)
    (tl, wlong), (ts, ws) = sinc.split(t, w, cfg.K_long)
    t0 = time.perf_counter()
    _, can = rhosvd.build(wl.protein_charges, wl.protein_positions, tl, wlong, cfg.n, cfg.b, cfg.eps)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    score.score(can.F, cfg.n, cfg.b, wl.protein_positions, wl.protein_charges, ts, ws, cfg.r_cut,
                wl.ligand_charges, wl.ligand_positions, wl.quats[:sample], wl.trans[:sample], cfg.sigma)
    t_score = time.perf_counter() - t0
    per_pose = t_score / sample
    job = t_build + cfg.P * per_pose
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {
        "value": cfg.P / job, "unit": "poses/s", "cores": threads, "kind": "oracle",
        "sample": (f"oracle tensor build ({t_build:.1f} s, counted once per job) + scoring of the first "
                   f"{sample} poses ({t_score:.1f} s); value = {cfg.P} poses / (build + {cfg.P} x per-pose time); "
                   f"cores = BLAS threads (the elementwise parts run on one thread)"),
        "oracle_build_s": t_build, "oracle_score_poses_per_s": 1.0 / per_pose,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--poses", type=int, default=None, help="override the pose count (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--score-mode", type=int, default=0, help="0 automatic, 1 fused per-pose, 2 chunk-major")
    ap.add_argument("--workload", default="cfg2", choices=["cfg1", "cfg2", "cfg3", "cfg4"],
                    help="cfg2 (default): one 5,000-atom protein, 1e6 poses; cfg1: 200 atoms, 128 poses; "
                         "cfg3: 64 protein/ligand pairs batched; cfg4: 10,000 atoms, 65,536 poses with gradients")
    ap.add_argument("--pairs", type=int, default=64, help="cfg3: number of protein/ligand pairs")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="only run a device copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              f"(the multi-GPU design is described but not run)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return 0

    import paper_2510_26611_amd as rs
    from workloads import configs

    if args.workload == "cfg3":
        return run_batched(args, rs, configs, torch, np, dev)
    cfg = {"cfg1": configs.CONFIG1, "cfg2": configs.CONFIG2, "cfg4": configs.CONFIG4}[args.workload]
    want_grad = args.workload == "cfg4"
    P = args.poses or cfg.P
    wl = configs.make(cfg, P=P)
    stream = torch.cuda.current_stream(dev)
    ctx = rs.Context(0, stream=stream.cuda_stream)
    ctx.set_option("score_mode", args.score_mode)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    d_z, d_x = to(wl.protein_charges), to(wl.protein_positions)
    d_lz, d_lx, d_q, d_t = to(wl.ligand_charges), to(wl.ligand_positions), to(wl.quats), to(wl.trans)
    out = dict(E=torch.empty(P, dtype=torch.float64, device=dev),
               flags=torch.empty(P, dtype=torch.uint8, device=dev),
               counts=torch.empty(P, dtype=torch.int32, device=dev))
    if want_grad:
        out["grads"] = torch.empty((P, 6), dtype=torch.float64, device=dev)
    sinc = rs.Sinc.from_config(cfg)
    torch.cuda.synchronize()

    info = {}

    def step():
        t = rs.build_rs_tensor(ctx, d_z, d_x, cfg.n, cfg.b, sinc)
        info.update(t.query())
        rs.score_poses(ctx, t, d_lz, d_lx, d_q, d_t, cfg.sigma, out=out, grads=want_grad)
        t.free()   # frees after the scoring work queued on the stream has finished

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = {k: ctx.kernel_time(k) for k in ("score", "long", "short", "combine", "ligand_prep", "cells", "gen",
                                           "gram", "eig", "project", "core", "t2c", "assemble")}
    ctx.set_timing(False)
    ms_step = wall / args.steps * 1e3
    R = info["R"]
    # dominant kernel: the long-range gather kernel (chunk-major mode) or the fused per-pose kernel
    dom_name = "long" if kt["long"][0] else "score"
    n_dom, ms_dom = kt[dom_name]
    dom_ms = ms_dom / max(n_dom, 1)
    score_ms = sum(kt[k][1] for k in ("score", "long", "short", "combine", "ligand_prep")) / args.steps
    alg_bytes = P * (48.0 * cfg.L * R + 56)           # two factor rows per mode per atom + pose inputs
    achieved = alg_bytes / (dom_ms / 1e3) / 1e9
    traffic = _traffic(P) if args.workload == "cfg2" else None
    flags = out["flags"].cpu().numpy()
    res = {
        "metric": METRIC, "value": P / (ms_step / 1e3), "unit": "poses/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "protein_atoms": cfg.N, "ligand_atoms": cfg.L, "grid_n": cfg.n,
                   "box_b_A": cfg.b, "sinc_M": cfg.M, "K_long": cfg.K_long, "rhosvd_eps": cfg.eps,
                   "poses": P, "vdw_min_A": cfg.sigma, "canonical_rank": R, "tucker_ranks": list(info["ranks"]),
                   "parallelism": "single GPU, data-parallel over poses"},
        "roofline": {"kernel": dom_name, "kernel_ms": dom_ms, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
        "breakdown": {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in kt.items() if v[0]},
        "score_only_poses_per_s": P / (score_ms / 1e3),
        "accept_fraction": float(np.mean(flags & 1)),
    }
    mf = sum(kt[k][1] for k in ("gram", "project", "core")) / args.steps
    if mf > 0:
        # flops of the three matrix-core contractions of one build (Gram: upper tiles only)
        C = cfg.N * cfg.K_long
        r1, r2, r3 = info["ranks"]
        Tn = -(-cfg.n // 64)
        gram = 3 * 2.0 * C * (Tn * (Tn + 1) / 2) * 64 * 64
        proj = 2.0 * C * cfg.n * (r1 + r2 + r3)
        core = 2.0 * C * r1 * r2 * r3
        res["build_mfma"] = {"flops_per_build": gram + proj + core, "ms_per_build": mf,
                             "achieved_tflops": (gram + proj + core) / (mf / 1e3) / 1e12,
                             "peak_tflops": FP64_MFMA_PEAK_TFS}
    if want_grad:
        res["metric"] = "poses scored/sec with energy + 6-DoF adjoint gradient at the oracle's tolerance"
    if not args.no_cpu_baseline and args.workload == "cfg2":
        res["cpu_baseline"] = cpu_baseline(cfg, wl, args.cpu_sample)
    print(json.dumps(res), flush=True)
    ctx.close()
    return 0


def run_batched(args, rs, configs, torch, np, dev) -> int:
    """64 protein/ligand pairs (n=4096): per-request calls vs one batch vs a replayed HIP graph."""
    pairs = configs.make_pairs(args.pairs)
    cfg = configs.CONFIG3
    stream = torch.cuda.current_stream(dev)
    ctx = rs.Context(0, stream=stream.cuda_stream)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    sinc = rs.Sinc.from_config(cfg)
    t0 = time.perf_counter()
    tensors, reqs = [], []
    for w in pairs:
        t = rs.build_rs_tensor(ctx, to(w.protein_charges), to(w.protein_positions), cfg.n, cfg.b, sinc)
        tensors.append(t)
        P = w.cfg.P
        reqs.append(dict(tensor=t, lig_charges=to(w.ligand_charges), lig_positions=to(w.ligand_positions),
                         quats=to(w.quats), trans=to(w.trans), vdw_min=cfg.sigma,
                         out=dict(E=torch.empty(P, dtype=torch.float64, device=dev),
                                  flags=torch.empty(P, dtype=torch.uint8, device=dev),
                                  counts=torch.empty(P, dtype=torch.int32, device=dev))))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    total = sum(w.cfg.P for w in pairs)
    Rs = [t.query()["R"] for t in tensors]
    alg = sum(48.0 * w.cfg.L * R * w.cfg.P for w, R in zip(pairs, Rs))

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) / args.steps

    def per_request():
        for r in reqs:
            rs.score_poses(ctx, r["tensor"], r["lig_charges"], r["lig_positions"], r["quats"], r["trans"],
                           r["vdw_min"], out=r["out"])

    ms_req = timed(per_request) * 1e3
    ctx.set_timing(True)
    per_request()
    kt_req = {k: ctx.kernel_time(k) for k in ("ligand_prep", "short", "long", "combine", "score")}
    ctx.set_timing(False)
    batch = rs.Batch(ctx, reqs)
    ms_batch = timed(batch.run) * 1e3
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    ctx.set_stream(s.cuda_stream)
    with torch.cuda.stream(s):
        batch.run()
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        batch.run()
    ctx.set_stream(stream.cuda_stream)
    ms_graph = timed(graph.replay) * 1e3
    ctx.set_timing(True)
    batch.run()
    kt = {k: ctx.kernel_time(k) for k in ("ligand_prep", "short", "long", "combine")}
    ctx.set_timing(False)
    long_ms = kt["long"][1]
    res = {
        "metric": METRIC, "value": total / (ms_graph / 1e3), "unit": "poses/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_graph, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"cfg3-{len(pairs)}pairs-n{cfg.n}", "pairs": len(pairs), "poses": total,
                   "protein_atoms": [int(w.cfg.N) for w in pairs], "ligand_atoms": [int(w.cfg.L) for w in pairs],
                   "canonical_ranks": Rs, "grid_n": cfg.n, "box_b_A": cfg.b,
                   "parallelism": "single GPU, all requests in one set of launches"},
        "per_request_poses_per_s": total / (ms_req / 1e3), "per_request_ms": ms_req,
        "batch_poses_per_s": total / (ms_batch / 1e3), "batch_ms": ms_batch,
        "graph_poses_per_s": total / (ms_graph / 1e3), "graph_ms": ms_graph,
        "roofline": {"kernel": "long", "kernel_ms": long_ms, "bound": "hbm", "achieved": alg / (long_ms / 1e3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / (long_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None},
        "breakdown": {k: {"launches": v[0], "ms": v[1]} for k, v in kt.items()},
        "per_request_breakdown": {k: {"launches": v[0], "ms": v[1]} for k, v in kt_req.items() if v[0]},
        "tensor_build_s_total": build_s,
    }
    print(json.dumps(res), flush=True)
    del graph
    batch.free()
    for t in tensors:
        t.free()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
