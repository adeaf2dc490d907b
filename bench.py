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


# The source the counters measured: the pose-transform helpers, the long-range kernel and the
# single-call launch sequence around it (which decides the pose order the kernel reads in).
KERNEL_REGIONS = (("// Rotation matrix of q = (w, x, y, z)", "// Two columns of one chunk for one atom"),
                  ("struct LongParams {", "// E = sum_c part[c]"),
                  ("rsd_status launch_score(Context* ctx", "\n}\n"))


def _src_hash() -> str:
    """Hash of the scoring source regions that define the long-range kernel."""
    with open(SCORE_SRC, encoding="utf-8") as f:
        text = f.read()
    parts = [text[text.index(a):text.index(b, text.index(a))] for a, b in KERNEL_REGIONS]
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


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


def gather_roofline(rs, ctx, t, dom_name: str, dom_ms: float, P: int, L: int, R: int, traffic=None) -> dict:
    """Roofline of the dominant scoring kernel: the bytes it moves from L2 into the compute units
    against the rate of its gather pattern alone (rsd_probe_gather, measured here).  The
    chunk-major long-range kernel moves, per atom and rank chunk, rows i and i+1 of modes 1-2
    (512 bytes each) and of mode 3 unless the chunk takes its mode-3 lerps from U_3 (read as
    2 x 4 values per atom); the fused per-pose kernel moves rows i and i+1 of all three modes
    for every column (48 R bytes per atom).  The factors stay in L2, so the HBM multiple of the
    algorithmic bytes (Lemma 3.3's 48 L R per pose) is informational only."""
    lay = t.layout()
    nch, u3 = lay["nchunk"], lay["shared_mode3"]
    if dom_name == "long":
        moved = P * L * (u3 * (4 * 512 + 64) + (nch - u3) * 6 * 512)
    else:
        moved = P * L * 48.0 * R
    pn = 2048                                          # 2 MB per XCD: the L2-resident ceiling
    probe = rs.probe_gather(ctx, pn, 256)
    alg_bytes = P * (48.0 * L * R + 56)
    flops = P * L * nch * 64 * 10.0                    # per atom and column: two lerps, two products, one FMA
    achieved = moved / (dom_ms / 1e3) / 1e9
    return {"kernel": dom_name, "kernel_ms": dom_ms, "bound": "l2_gather", "achieved": achieved,
            "peak": probe["gbs"], "unit": "GB/s", "frac": achieved / probe["gbs"], "traffic": traffic,
            "bytes_per_launch": moved,
            "peak_source": (f"rsd_probe_gather on this GPU: the kernel's gather pattern alone (16-byte loads of "
                            f"rows i, i+1 of two modes per half-wavefront, {pn}-row chunks, one per XCD), "
                            f"{probe['bytes'] / 1e9:.2f} GB in {probe['ms']:.3f} ms"),
            "chunks": nch, "chunks_mode3_from_U3": u3,
            "hbm_algorithmic": {"bytes_per_launch": alg_bytes, "GB_per_s": alg_bytes / (dom_ms / 1e3) / 1e9,
                                "multiple_of_hbm_peak": alg_bytes / (dom_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                "note": "48 L R bytes per pose (Lemma 3.3's two rows per mode per atom) over the "
                                        "8 TB/s HBM peak; the factors stay in L2, so this multiple exceeds 1"},
            "fp64_valu": {"tflops": flops / (dom_ms / 1e3) / 1e12, "peak_tflops": FP64_MFMA_PEAK_TFS,
                          "frac": flops / (dom_ms / 1e3) / 1e12 / FP64_MFMA_PEAK_TFS}}


def cpu_baseline(cfg, wl, sample: int, F_gpu=None, gpu_out=None):
    """The oracle as it stands: its own tensor build (timed), then scoring of a bounded pose sample.

    With F_gpu (the factors of the tensor the timed steps scored) the sample is scored on those
    factors, and the GPU's results of the timed run (gpu_out: E, flags, counts) are checked
    against it: flags and counts bit-exact, energies within 1e-10 of the summation scale."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import rhosvd, score, sinc
    t, w = sinc.sinc_table(cfg.M, cfg.h_M, cfg.L_s)
    (tl, wlong), (ts, ws) = sinc.split(t, w, cfg.K_long)
    t0 = time.perf_counter()
    _, can = rhosvd.build(wl.protein_charges, wl.protein_positions, tl, wlong, cfg.n, cfg.b, cfg.eps)
    t_build = time.perf_counter() - t0
    F = F_gpu if F_gpu is not None else can.F
    t0 = time.perf_counter()
    ref = score.score(F, cfg.n, cfg.b, wl.protein_positions, wl.protein_charges, ts, ws, cfg.r_cut,
                      wl.ligand_charges, wl.ligand_positions, wl.quats[:sample], wl.trans[:sample], cfg.sigma)
    t_score = time.perf_counter() - t0
    per_pose = t_score / sample
    job = t_build + cfg.P * per_pose
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    res = {
        "value": cfg.P / job, "unit": "poses/s", "cores": threads, "kind": "oracle",
        "sample": (f"oracle tensor build ({t_build:.1f} s, counted once per job) + scoring of the first "
                   f"{sample} poses ({t_score:.1f} s) on the factors of the tensor the GPU scored; "
                   f"value = {cfg.P} poses / (build + {cfg.P} x per-pose time); "
                   f"cores = BLAS threads (the elementwise parts run on one thread)"),
        "oracle_build_s": t_build, "oracle_score_poses_per_s": 1.0 / per_pose,
    }
    if gpu_out is not None:
        E, flags, counts = (np.asarray(gpu_out[k][:sample]) for k in ("E", "flags", "counts"))
        ok = ~np.isnan(ref["E"])
        nan_ok = bool(np.array_equal(np.isnan(E), ~ok))
        err = np.abs(E[ok] - ref["E"][ok]) / (1e-10 * ref["scale"][ok] + 1e-300)
        res["parity"] = {"poses": sample, "flags_mismatch": int(np.sum(flags != ref["flags"])),
                         "counts_mismatch": int(np.sum(counts != ref["counts"])), "nan_pattern_equal": nan_ok,
                         "max_energy_error_over_tolerance": float(err.max()) if err.size else 0.0,
                         "tolerance": "1e-10 x per-pose summation scale"}
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--poses", type=int, default=None, help="override the pose count (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--score-mode", type=int, default=0, help="0 automatic, 1 fused per-pose, 2 chunk-major")
    ap.add_argument("--no-autotune", action="store_true", help="skip the launch-shape tuner before timing")
    ap.add_argument("--pose-order", type=int, default=0, choices=[0, 1, 2],
                    help="long range takes poses in spatial order: 0 automatic (large grids), 1 always, 2 never")
    ap.add_argument("--overlap", type=int, default=0, choices=[0, 1],
                    help="1: the short-range kernel runs on a second stream beside the long-range one")
    ap.add_argument("--tune-poses", type=int, default=16384, help="poses of the tuner's sample")
    ap.add_argument("--workload", default="cfg2", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "site", "ppiem"],
                    help="cfg2 (default): one 5,000-atom protein, 1e6 poses; cfg1: 200 atoms, 128 poses; "
                         "cfg3: 64 protein/ligand pairs batched; cfg4: 10,000 atoms, 65,536 poses with gradients; "
                         "cfg5: serving 8 resident proteins under Poisson arrivals; site: 1e6 poses at one site of "
                         "the cfg2 protein scored with the global tensor and with the tensor restricted to a box; "
                         "ppiem: the posing search over 4,096 orbit directions x 256 orientations of the cfg2 protein")
    ap.add_argument("--pairs", type=int, default=64, help="cfg3: number of protein/ligand pairs")
    ap.add_argument("--requests", type=int, default=100, help="cfg5: arrivals in the served trace")
    ap.add_argument("--rate", type=float, default=200.0, help="cfg5: offered requests per second")
    ap.add_argument("--hbm-budget-gib", type=float, default=48.0, help="cfg5: HBM for requests in flight")
    ap.add_argument("--round-poses", type=int, default=250_000, help="cfg5: poses per round, shared by the requests")
    ap.add_argument("--min-slice", type=int, default=16_384, help="cfg5: smallest pose slice of a request in a round")
    ap.add_argument("--sweep", default="0.5,0.8", help="cfg5: offered rates as fractions of capacity")
    ap.add_argument("--sweep-requests", type=int, default=200, help="cfg5: arrivals per sweep point")
    ap.add_argument("--no-serving", dest="serving", action="store_false",
                    help="cfg2: leave out the brief config-5 serving comparison of the default line")
    ap.add_argument("--serving-requests", type=int, default=60,
                    help="cfg2: arrivals per trace of the brief serving comparison")
    ap.add_argument("--serve-policy", default="small_first", choices=["share", "small_first"],
                    help="cfg5 and the brief serving comparison: how a round's poses are shared among requests")
    ap.add_argument("--dump-requests", default="", help="cfg5: write per-request times (CSV) to this file")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="only run a device copy of this many MiB (counter calibration) and exit")
    ap.add_argument("--build-only", action="store_true",
                    help="cfg1/cfg2/cfg4: time only the device build of the workload's tensor (steps builds) and exit")
    ap.add_argument("--calibrate-gather", action="store_true",
                    help="only time the long-range kernel's gather pattern alone (rsd_probe_gather) on chunks "
                         "of 512..8192 rows and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the library "
              f"scores on one device, and sharding over several is a design, not code", file=sys.stderr)
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

    if args.calibrate_gather:
        ctx = rs.Context(0)
        rows = []
        for n in (512, 1024, 2048, 4096, 8192):
            r = rs.probe_gather(ctx, n, 256)
            rows.append({"rows_per_chunk": n, "bytes_per_xcd": 2 * n * 512, **r})
        ctx.close()
        print(json.dumps({"gather_probe": rows}))
        return 0
    if args.workload == "cfg3":
        return run_batched(args, rs, configs, torch, np, dev)
    if args.workload == "cfg5":
        return run_serving(args, rs, configs, torch, np)
    if args.workload == "site":
        return run_site(args, rs, configs, torch, np, dev)
    if args.workload == "ppiem":
        return run_ppiem(args, rs, configs, torch, np, dev)
    cfg = {"cfg1": configs.CONFIG1, "cfg2": configs.CONFIG2, "cfg4": configs.CONFIG4}[args.workload]
    want_grad = args.workload == "cfg4"
    P = args.poses or cfg.P
    wl = configs.make(cfg, P=P)
    stream = torch.cuda.current_stream(dev)
    ctx = rs.Context(0, stream=stream.cuda_stream)
    ctx.set_option("score_mode", args.score_mode)
    ctx.set_option("overlap", args.overlap)
    ctx.set_option("pose_order", args.pose_order)
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

    if args.build_only:
        def one_build():
            t = rs.build_rs_tensor(ctx, d_z, d_x, cfg.n, cfg.b, sinc)
            q = t.query()
            t.free()
            return q
        for _ in range(args.warmup):
            one_build()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            q = one_build()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        print(json.dumps({"workload": cfg.name, "build_ms": ms, "builds": args.steps, "tucker_ranks": list(q["ranks"]),
                          "canonical_rank": q["R"]}), flush=True)
        ctx.close()
        return 0
    info = {}
    tune = None
    if not args.no_autotune and args.score_mode == 0:
        # launch shapes picked on a sample of this workload, kept in the context for the timed steps
        t = rs.build_rs_tensor(ctx, d_z, d_x, cfg.n, cfg.b, sinc)
        m = min(P, args.tune_poses)
        tune = ctx.autotune(t, d_lz, d_lx, d_q[:m], d_t[:m], cfg.sigma, grads=want_grad)
        tune["sample_poses"] = m
        t.free()

    def step():
        t = rs.build_rs_tensor(ctx, d_z, d_x, cfg.n, cfg.b, sinc)
        info.update(t.query())
        rs.score_poses(ctx, t, d_lz, d_lx, d_q, d_t, cfg.sigma, out=out, grads=want_grad)
        t.free()   # frees after the scoring work queued on the stream has finished

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K whole jobs, no per-launch instrumentation
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # kernel attribution: the same K jobs again with HIP events around every launch
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall_instr = time.perf_counter() - t0
    kt = {k: ctx.kernel_time(k) for k in ("score", "long", "short", "combine", "ligand_prep", "sort", "cells", "gen",
                                           "gram", "eig", "project", "core", "t2c", "assemble")}
    ctx.set_timing(False)
    ms_step = wall / args.steps * 1e3
    R = info["R"]
    # dominant kernel: the long-range gather kernel (chunk-major mode) or the fused per-pose kernel
    dom_name = "long" if kt["long"][0] else "score"
    n_dom, ms_dom = kt[dom_name]
    dom_ms = ms_dom / max(n_dom, 1)
    score_ms = sum(kt[k][1] for k in ("score", "long", "short", "combine", "ligand_prep", "sort")) / args.steps
    traffic = _traffic(P) if args.workload == "cfg2" else None
    flags = out["flags"].cpu().numpy()
    t = rs.build_rs_tensor(ctx, d_z, d_x, cfg.n, cfg.b, sinc)
    roof = gather_roofline(rs, ctx, t, dom_name, dom_ms, P, cfg.L, R, traffic)
    F_gpu = None
    if not args.no_cpu_baseline and args.workload == "cfg2":
        F_gpu = t.export()
    # the same scoring call with host arrays (PCIe upload and download inside the call)
    rs.score_poses(ctx, t, wl.ligand_charges, wl.ligand_positions, wl.quats[:4096], wl.trans[:4096], cfg.sigma,
                   grads=want_grad)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rs.score_poses(ctx, t, wl.ligand_charges, wl.ligand_positions, wl.quats, wl.trans, cfg.sigma, grads=want_grad)
    host_io_s = time.perf_counter() - t1
    t.free()
    res = {
        "metric": METRIC, "value": P / (ms_step / 1e3), "unit": "poses/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "protein_atoms": cfg.N, "ligand_atoms": cfg.L, "grid_n": cfg.n,
                   "box_b_A": cfg.b, "sinc_M": cfg.M, "K_long": cfg.K_long, "rhosvd_eps": cfg.eps,
                   "poses": P, "vdw_min_A": cfg.sigma, "canonical_rank": R, "tucker_ranks": list(info["ranks"]),
                   "parallelism": "single GPU, data-parallel over poses"},
        "roofline": roof,
        "breakdown": {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in kt.items() if v[0]},
        "ms_per_step_with_kernel_events": wall_instr / args.steps * 1e3,
        "autotune": tune, "short_range_on_second_stream": bool(args.overlap),
        "score_host_arrays_poses_per_s": P / host_io_s,
        "score_only_poses_per_s": P / (score_ms / 1e3),
        "accept_fraction": float(np.mean(flags & 1)),
    }
    mf = sum(kt[k][1] for k in ("project", "core")) / args.steps
    if mf > 0:
        # flops of the build's two matrix-core contractions (the Gram is formed from its
        # Toeplitz-times-Hankel structure on the vector units and is timed under "gram")
        C = cfg.N * cfg.K_long
        r1, r2, r3 = info["ranks"]
        proj = 2.0 * C * cfg.n * (r1 + r2 + r3)
        core = 2.0 * C * r1 * r2 * r3
        res["build_mfma"] = {"kernels": ["project", "core"], "flops_per_build": proj + core, "ms_per_build": mf,
                             "achieved_tflops": (proj + core) / (mf / 1e3) / 1e12,
                             "peak_tflops": FP64_MFMA_PEAK_TFS}
    if want_grad:
        res["metric"] = "poses scored/sec with energy + 6-DoF adjoint gradient at the oracle's tolerance"
    if not args.no_cpu_baseline and args.workload == "cfg2":
        res["cpu_baseline"] = cpu_baseline(cfg, wl, args.cpu_sample, F_gpu,
                                           {k: v.cpu().numpy() for k, v in out.items()})
    if args.serving and args.workload == "cfg2":
        ctx.close()
        ctx = None
        torch.cuda.synchronize()
        res["serving"] = serving_block(args, rs, configs, torch, np)
    print(json.dumps(res), flush=True)
    if ctx is not None:
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
    def graph_of(batch):
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
        return graph

    # the batch both ways: requests grouped into launches by LDS occupancy (batch_mode 1), and
    # one persistent launch over per-XCD work queues (batch_mode 2); each eagerly and replayed
    modes = {}
    for mode in (1, 2):
        ctx.set_option("batch_mode", mode)
        batch = rs.Batch(ctx, reqs)
        ms_b = timed(batch.run) * 1e3
        graph = graph_of(batch)
        ms_g = timed(graph.replay) * 1e3
        ctx.set_timing(True)
        batch.run()
        kt = {k: ctx.kernel_time(k) for k in ("ligand_prep", "sort", "short", "long", "fused", "combine")}
        ctx.set_timing(False)
        modes[mode] = dict(batch_ms=ms_b, graph_ms=ms_g, breakdown={k: {"launches": v[0], "ms": v[1]}
                                                                    for k, v in kt.items() if v[0]})
        del graph
        batch.free()
    ctx.set_option("batch_mode", 0)
    best = min(modes, key=lambda m: modes[m]["graph_ms"])
    ms_graph, ms_batch = modes[best]["graph_ms"], modes[best]["batch_ms"]
    kt = {k: (v["launches"], v["ms"]) for k, v in modes[1]["breakdown"].items()}
    long_ms = kt["long"][1]
    moved = 0
    for w, t in zip(pairs, tensors):
        lay = t.layout()
        moved += w.cfg.P * w.cfg.L * (lay["shared_mode3"] * (4 * 512 + 64) + (lay["nchunk"] - lay["shared_mode3"]) * 6 * 512)
    probe = rs.probe_gather(ctx, 2048, 256)
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
        "batch_mode_timed": {1: "grouped launches", 2: "one persistent launch"}[best],
        "grouped_launches": modes[1], "persistent_launch": modes[2],
        "roofline": {"kernel": "long", "kernel_ms": long_ms, "bound": "l2_gather",
                     "achieved": moved / (long_ms / 1e3) / 1e9, "peak": probe["gbs"], "unit": "GB/s",
                     "frac": moved / (long_ms / 1e3) / 1e9 / probe["gbs"], "traffic": None,
                     "bytes_per_launch": moved,
                     "peak_source": "rsd_probe_gather on this GPU (the gather pattern alone, 2048-row chunks)",
                     "hbm_algorithmic": {"bytes_per_launch": alg, "GB_per_s": alg / (long_ms / 1e3) / 1e9,
                                         "multiple_of_hbm_peak": alg / (long_ms / 1e3) / 1e9 / HBM_PEAK_GBS}},
        "breakdown": {k: {"launches": v[0], "ms": v[1]} for k, v in kt.items()},
        "per_request_breakdown": {k: {"launches": v[0], "ms": v[1]} for k, v in kt_req.items() if v[0]},
        "tensor_build_s_total": build_s,
    }
    print(json.dumps(res), flush=True)
    for t in tensors:
        t.free()
    ctx.close()
    return 0


def run_site(args, rs, configs, torch, np, dev) -> int:
    """A docking scan at one site (Sec. 3.3, schemes (B)/(C)): 1,000 translations within 2 A of a
    point 5 A outside the 5,000-atom protein, 1,000 rotations each.  Step A scores them with the
    global RS tensor; step B restricts the tensor to the 16 A box around the site (rank
    reduction included in the step) and scores them with the local tensor."""
    from workloads import generators as gen
    cfg = configs.CONFIG2
    wl = configs.make(cfg, P=1)
    T, Q = 1000, 1000
    site = np.array([cfg.pose_r_in, 0.0, 0.0])
    half = cfg.ligand_radius + 2.0
    dirs = gen.directions(gen.rng(6, 6), T)
    rad = 2.0 * np.cbrt(gen.rng(6, 7).random(T))
    centres = site[None, :] + dirs * rad[:, None]
    quats = gen.unit_quaternions(gen.rng(6, 5), T * Q)
    trans = np.repeat(centres, Q, axis=0)                        # translation-major: 1,000 rotations per site point
    P = T * Q
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    d_lz, d_lx, d_q, d_t = to(wl.ligand_charges), to(wl.ligand_positions), to(quats), to(trans)
    ctx = rs.Context(0)
    ctx.set_option("overlap", args.overlap)
    ctx.set_option("pose_order", args.pose_order)
    tg = rs.build_rs_tensor(ctx, to(wl.protein_charges), to(wl.protein_positions), cfg.n, cfg.b,
                            rs.Sinc.from_config(cfg))
    out = {k: dict(E=torch.empty(P, dtype=torch.float64, device=dev), flags=torch.empty(P, dtype=torch.uint8, device=dev),
                   counts=torch.empty(P, dtype=torch.int32, device=dev)) for k in ("global", "local")}
    m = min(P, args.tune_poses)
    tune = {"global": ctx.autotune(tg, d_lz, d_lx, d_q[:m], d_t[:m], cfg.sigma)}
    tl0 = tg.restrict(site - half, site + half, cfg.eps)
    tune["local"] = ctx.autotune(tl0, d_lz, d_lx, d_q[:m], d_t[:m], cfg.sigma)
    tl0.free()

    def step_global():
        rs.score_poses(ctx, tg, d_lz, d_lx, d_q, d_t, cfg.sigma, out=out["global"])

    info = {}

    def step_local():
        tl = tg.restrict(site - half, site + half, cfg.eps)
        info.update(tl.query())
        info["rows"] = list(tl.grid()["rows"])
        rs.score_poses(ctx, tl, d_lz, d_lx, d_q, d_t, cfg.sigma, out=out["local"])
        tl.free()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    ms_glob = timed(step_global) * 1e3
    ctx.set_timing(True)
    ms_loc = timed(step_local) * 1e3
    kt = {k: ctx.kernel_time(k) for k in ("restrict", "qr", "svd", "core", "t2c", "assemble", "cells", "long", "short",
                                          "score")}
    ctx.set_timing(False)
    fg, fl = out["global"]["flags"].cpu().numpy(), out["local"]["flags"].cpu().numpy()
    cg, cl = out["global"]["counts"].cpu().numpy(), out["local"]["counts"].cpu().numpy()
    Eg, El = out["global"]["E"].cpu().numpy(), out["local"]["E"].cpu().numpy()
    ok = (fl & 2) != 0
    Rg = tg.query()["R"]
    dom = "long" if kt["long"][0] else "score"          # chunk-major or fused, whichever the tuner chose
    long_ms = kt[dom][1] / max(kt[dom][0], 1)
    tlr = tg.restrict(site - half, site + half, cfg.eps)
    roof = gather_roofline(rs, ctx, tlr, dom, long_ms, P, cfg.L, info["R"])
    tlr.free()
    res = {
        "metric": METRIC, "value": P / (ms_loc / 1e3), "unit": "poses/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_loc, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "site-scan-cfg2-protein", "poses": P, "site_points": T, "rotations_per_point": Q,
                   "box_half_width_A": half, "canonical_rank_global": Rg, "canonical_rank_local": info["R"],
                   "local_grid_rows": info["rows"],
                   "parallelism": "single GPU, data-parallel over poses"},
        "global_tensor_poses_per_s": P / (ms_glob / 1e3), "global_ms": ms_glob,
        "local_ms_including_restriction": ms_loc,
        "restriction_kernels_ms": sum(kt[k][1] for k in ("restrict", "qr", "svd", "core", "t2c", "assemble", "cells"))
        / args.steps,
        "roofline": roof,
        "autotune": tune, "short_range_on_second_stream": bool(args.overlap),
        "in_box_fraction": float(np.mean(ok)),
        "flags_equal_in_box": bool(np.array_equal(fg[ok], fl[ok])), "counts_equal": bool(np.array_equal(cg, cl)),
        "max_abs_dE_in_box": float(np.max(np.abs(Eg[ok] - El[ok]))) if ok.any() else None,
        "max_abs_E_in_box": float(np.max(np.abs(Eg[ok]))) if ok.any() else None,
        "breakdown": {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in kt.items() if v[0]},
    }
    print(json.dumps(res), flush=True)
    tg.free()
    ctx.close()
    return 0


def run_ppiem(args, rs, configs, torch, np, dev) -> int:
    """The posing search of Algorithm PPIEM on the 5,000-atom protein: 4,096 orbit directions
    (Fibonacci sphere) x 256 orientations (32 axes x 8 spins) = 1,048,576 contact poses.  One
    step is steps A2-A6: contact radii, scoring of all contact poses, best orientation per
    orbit position and the local minima over the orbit grid (6 nearest directions); the tensor
    is the precomputed step A1 and is built once, outside the timed steps."""
    from paper_2510_26611_amd import ppiem
    from workloads import angles
    cfg = configs.CONFIG2
    wl = configs.make(cfg, P=1)
    U, QA, QS = 4096, 32, 8
    dirs, quats = angles.orbit_sphere(U), angles.orientations(QA, QS)
    Q = QA * QS
    off, idx = angles.sphere_neighbours(dirs, 6)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    d_lz, d_lx, d_dirs, d_q = to(wl.ligand_charges), to(wl.ligand_positions), to(dirs), to(quats)
    d_off, d_idx = to(off.astype(np.int32)), to(idx.astype(np.int32))
    ctx = rs.Context(0)
    ctx.set_option("overlap", args.overlap)
    ctx.set_option("pose_order", args.pose_order)
    t = rs.build_rs_tensor(ctx, to(wl.protein_charges), to(wl.protein_positions), cfg.n, cfg.b, rs.Sinc.from_config(cfg))
    centre = ppiem.tensor_centre(t)
    cp0 = ppiem.contact_poses(ctx, t, d_lx, d_dirs, d_q, cfg.sigma, centre=centre)
    m = min(U * Q, args.tune_poses)
    tune = ctx.autotune(t, d_lz, d_lx, cp0["quats"][:m], cp0["trans"][:m], cfg.sigma)
    state = {}

    def step():
        cp = ppiem.contact_poses(ctx, t, d_lx, d_dirs, d_q, cfg.sigma, centre=centre)
        res = rs.score_poses(ctx, t, d_lz, d_lx, cp["quats"], cp["trans"], cfg.sigma)
        state.update(cp=cp, res=res, mins=ppiem.orbit_minima(ctx, res["E"], res["flags"], U, Q, d_off, d_idx))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    kt = {k: ctx.kernel_time(k) for k in ("contact", "ligand_prep", "short", "long", "combine", "score", "minima")}
    ctx.set_timing(False)
    P = U * Q
    rho = state["cp"]["rho"].cpu().numpy()
    im = state["mins"]["is_minimum"].cpu().numpy().astype(bool)
    be = state["mins"]["best_energy"].cpu().numpy()
    bq = state["mins"]["best_rotation"].cpu().numpy()
    fl = state["res"]["flags"].cpu().numpy()
    order = np.argsort(be[im])
    top = [{"orbit": int(u), "rotation": int(bq[u]), "energy": float(be[u])} for u in np.nonzero(im)[0][order][:5]]
    dom = max(("long", "score", "contact"), key=lambda k: kt[k][1])   # the gather kernels; a separate short-range launch is vector ALU work
    dom_ms = kt[dom][1] / max(kt[dom][0], 1)
    R = t.query()["R"]
    if dom == "contact":
        # brute-force definition: U*Q*L*N pair roots, ~16 FP64 operations each (the cylinder
        # filter skips most of them; this counts the work the definition asks for)
        work = float(P) * cfg.L * cfg.N * 16.0
        roof = {"kernel": "contact", "kernel_ms": dom_ms, "bound": "alu", "achieved": work / (dom_ms / 1e3) / 1e12,
                "peak": 78.6, "unit": "TFLOP/s", "frac": work / (dom_ms / 1e3) / 1e12 / 78.6, "traffic": None}
    else:
        roof = gather_roofline(rs, ctx, t, dom, dom_ms, P, cfg.L, R)
    res = {
        "metric": METRIC, "value": P / (ms / 1e3), "unit": "poses/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "ppiem-search-cfg2-protein", "poses": P, "orbit_directions": U, "orientations": Q,
                   "protein_atoms": cfg.N, "ligand_atoms": cfg.L, "grid_n": cfg.n, "canonical_rank": R,
                   "parallelism": "single GPU, data-parallel over poses"},
        "roofline": roof,
        "autotune": tune, "short_range_on_second_stream": bool(args.overlap),
        "contact_ms": kt["contact"][1] / args.steps,
        "rho_range_A": [float(np.min(rho)), float(np.max(rho))],
        "accept_fraction": float(np.mean(fl & 1)),
        "orbit_minima": int(im.sum()), "lowest_minima": top,
        "breakdown": {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in kt.items() if v[0]},
    }
    print(json.dumps(res), flush=True)
    t.free()
    ctx.close()
    return 0


def _serving_setup(args, rs, configs, torch, np, note):
    """The 8 resident proteins of config 5, built on the device once; a warmed-up server."""
    from paper_2510_26611_amd import serve
    ctx = rs.Context(0)
    tensors, builds = {}, []
    for i, (c, pos, z) in enumerate(configs.make_serving_proteins()):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = rs.build_rs_tensor(ctx, z, pos, c.n, c.b, rs.Sinc.from_config(c))
        torch.cuda.synchronize()
        q = t.query()
        builds.append({"protein_atoms": c.N, "grid_n": c.n, "box_b_A": c.b, "tucker_ranks": list(q["ranks"]),
                       "canonical_rank": q["R"], "bytes": q["bytes"], "build_s": time.perf_counter() - t0})
        tensors[f"p{i}"] = t
        note(f"built protein {i}: N={c.N} n={c.n} ranks={q['ranks']} R={q['R']} "
             f"{q['bytes'] / 2**30:.2f} GiB in {builds[-1]['build_s']:.2f} s")
    resident = sum(b["bytes"] for b in builds)
    budget = int(resident + args.hbm_budget_gib * 2**30)
    srv = serve.Server(tensors, budget, round_poses=args.round_poses, min_slice=args.min_slice,
                       policy=args.serve_policy)
    warm = _requests(serve, configs.make_serving_trace(4, rate=1e6, pose_scale=0.01, seed_offset=9))
    srv.run(warm, realtime=False)
    serve.serve_plain(ctx, tensors, _requests(serve, configs.make_serving_trace(2, rate=1e6, pose_scale=0.01,
                                                                                  seed_offset=9)), realtime=False)
    torch.cuda.synchronize()
    note("warm-up done")
    return ctx, tensors, builds, budget, resident, srv


def _requests(serve, tr):
    return [serve.Request(r.index, f"p{r.protein}", r.ligand_charges, r.ligand_positions, r.quats, r.trans,
                          r.sigma, r.arrival) for r in tr]


def _served_and_plain(serve, srv, ctx, tensors, trace, note, tag, every=0):
    """The same trace through the continuous-batching server and through plain one-at-a-time
    calls (arrivals in real time for both); per-mode throughput and latency percentiles."""
    import numpy as np
    prog = (lambda m: (lambda d, n: note(f"{tag} {m}: {d}/{n} done") if d % every == 0 or d == n else None)) \
        if every else (lambda m: None)
    served = _requests(serve, trace)
    st = srv.run(served, progress=prog("served"))
    plain = _requests(serve, trace)
    sp = serve.serve_plain(ctx, tensors, plain, progress=prog("plain"))
    # served results equal the same requests scored alone (bitwise), on the three smallest
    for r in sorted(served, key=lambda r: r.P)[:3]:
        pl = next(x for x in plain if x.rid == r.rid)
        for k in ("E", "flags", "counts"):
            if not np.array_equal(r.result[k], pl.result[k], equal_nan=True):
                raise RuntimeError(f"served request {r.rid} differs from the same request alone ({k})")
    keys = ("poses_per_s", "latency_p50_s", "latency_p99_s", "latency_max_s", "queue_wait_p50_s", "wall_s",
            "served", "poses")
    note(f"{tag}: served {st['poses_per_s']:.3g} poses/s p50 {st['latency_p50_s']:.2f} s p99 "
         f"{st['latency_p99_s']:.2f} s | plain {sp['poses_per_s']:.3g} poses/s p50 {sp['latency_p50_s']:.2f} s "
         f"p99 {sp['latency_p99_s']:.2f} s")
    return {"served": {k: st[k] for k in keys}, "plain": {k: sp[k] for k in keys}}, served, plain


def serving_block(args, rs, configs, torch, np) -> dict:
    """Config 5 in brief, for the default measurement line: the same arrival traces served by
    the continuous-batching server and by plain calls, at the stated 200 req/s (far beyond
    capacity: both queue) and at half the capacity measured on the first trace."""
    from paper_2510_26611_amd import serve

    def note(msg):
        print(msg, file=sys.stderr, flush=True)

    ctx, tensors, builds, budget, resident, srv = _serving_setup(args, rs, configs, torch, np, note)
    n = args.serving_requests
    tr = configs.make_serving_trace(n, rate=args.rate)
    mean_P = float(np.mean([r.quats.shape[0] for r in tr]))
    at_rate, _, _ = _served_and_plain(serve, srv, ctx, tensors, tr, note, f"{args.rate:g} req/s")
    cap = at_rate["served"]["poses_per_s"] / mean_P
    tr2 = configs.make_serving_trace(n, rate=0.5 * cap, seed_offset=1)
    at_half, _, _ = _served_and_plain(serve, srv, ctx, tensors, tr2, note, "0.5 x capacity")
    srv.close()
    for t in tensors.values():
        t.free()
    ctx.close()
    return {"workload": f"cfg5: {len(builds)} resident proteins of 1e3-1e5 atoms (n = 8192/16384), ligands of "
                        f"10-200 atoms, 1e4-1e6 poses per request (log-uniform), Poisson arrivals",
            "arrivals_per_trace": n, "resident_bytes": resident, "hbm_budget_bytes": budget,
            "at_offered_rate": dict(offered_req_s=args.rate, mean_poses_per_request=mean_P, **at_rate),
            "capacity_req_s": cap,
            "at_half_capacity": dict(offered_req_s=0.5 * cap, **at_half),
            "policy": args.serve_policy, "round_poses": args.round_poses, "min_slice": args.min_slice,
            "latency": "arrival to the request's last results in host memory"}


def run_serving(args, rs, configs, torch, np) -> int:
    """Config 5: 8 resident proteins (1e3..1e5 atoms, n up to 16384) serving a Poisson request stream.

    Reported: served poses/s and arrival-to-result p50/p99 for the continuous-batching server and
    for plain one-request-at-a-time calls on the same trace, and the same comparison on one
    second trace replayed at fractions of the capacity measured on the first (the stated
    200 req/s is far beyond it)."""
    from paper_2510_26611_amd import serve

    def note(msg):
        print(msg, file=sys.stderr, flush=True)

    ctx, tensors, builds, budget, resident, srv = _serving_setup(args, rs, configs, torch, np, note)
    Rk = {f"p{i}": b["canonical_rank"] for i, b in enumerate(builds)}

    def alg_bytes(reqs):
        return sum(48.0 * r.L * Rk[r.protein] * r.P for r in reqs if r.state == serve.DONE)

    trace = configs.make_serving_trace(args.requests, rate=args.rate)
    mean_P = float(np.mean([r.quats.shape[0] for r in trace]))
    note(f"trace: {len(trace)} requests, {sum(r.quats.shape[0] for r in trace)} poses, offered "
         f"{args.rate * mean_P:.3g} poses/s")
    main, served_reqs, plain_reqs = _served_and_plain(serve, srv, ctx, tensors, trace, note, f"{args.rate:g} req/s",
                                                      every=max(1, args.requests // 10))
    main["served"]["alg_bytes_per_s"] = alg_bytes(served_reqs) / main["served"]["wall_s"]
    main["plain"]["alg_bytes_per_s"] = alg_bytes(plain_reqs) / main["plain"]["wall_s"]
    if args.dump_requests:
        with open(args.dump_requests, "w") as f:
            f.write("mode,rid,protein,L,P,arrival_s,admit_s,done_s\n")
            for mode, rr in (("served", served_reqs), ("plain", plain_reqs)):
                for r in rr:
                    f.write(f"{mode},{r.rid},{r.protein},{r.L},{r.P},{r.arrival:.4f},{r.t_admit:.4f},{r.t_done:.4f}\n")
    cap = main["served"]["poses_per_s"] / mean_P
    # one second trace, replayed at each offered rate: the same requests, arrival gaps rescaled
    sweep = []
    for frac in (float(x) for x in args.sweep.split(",") if x):
        rate = frac * cap
        tr = configs.make_serving_trace(args.sweep_requests, rate=rate, seed_offset=1)
        pt, _, _ = _served_and_plain(serve, srv, ctx, tensors, tr, note, f"{frac:.2f} x capacity",
                                     every=max(1, args.sweep_requests // 4))
        sweep.append(dict(offered_fraction_of_capacity=frac, offered_req_s=rate, **pt))
    res = {
        "metric": METRIC, "value": main["served"]["poses_per_s"], "unit": "poses/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": main["served"]["wall_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"cfg5-serving-{len(builds)}proteins", "requests": len(trace),
                   "offered_req_s": args.rate, "offered_poses_per_s": args.rate * mean_P,
                   "mean_poses_per_request": mean_P, "hbm_budget_bytes": budget, "resident_bytes": resident,
                   "round_poses": args.round_poses, "min_slice": args.min_slice,
                   "parallelism": "single GPU, continuous batching of pose slices, 2 streams"},
        "latency_p50_s": main["served"]["latency_p50_s"], "latency_p99_s": main["served"]["latency_p99_s"],
        "served": main["served"], "plain_per_request": main["plain"],
        "capacity_req_s": cap, "rate_sweep": sweep, "proteins": builds,
    }
    print(json.dumps(res), flush=True)
    srv.close()
    for t in tensors.values():
        t.free()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
