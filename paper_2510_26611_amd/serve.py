"""Continuous-batching request server over resident RS tensors.

Requests (protein id, ligand, poses, vdW distance) arrive over time.  Each protein's RS
tensor and cell list stay resident on the device.  The scheduler admits waiting requests in
arrival order while their device memory (inputs, outputs and the batch scratch: per-chunk
long-range partials, short-range energies, ligand frames) fits the HBM budget next to the
resident tensors; every admission round becomes one rsd_batch (all its requests scored by
one set of launches).  Rounds alternate between streams, each with its own context, so a
round's kernels overlap the previous round's on the device while the host uploads and
plans the next one.  Latency is measured from arrival to the moment a request's results are
back on the host.

The scheduler is plain Python with no device calls (unit-testable on the CPU); the executor
does the device work through the library.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import rsdock

# request states
WAITING, RUNNING, DONE, REJECTED, CANCELLED = "waiting", "running", "done", "rejected", "cancelled"

# reasons a request is rejected at submission
E_UNKNOWN_PROTEIN = -10
E_MALFORMED = -11
E_TOO_LARGE = -12


@dataclass
class Request:
    rid: int
    protein: str
    lig_charges: np.ndarray     # (L,)
    lig_positions: np.ndarray   # (L, 3)
    quats: np.ndarray           # (P, 4)
    trans: np.ndarray           # (P, 3)
    vdw_min: float
    arrival: float = 0.0        # seconds after the start of the trace
    state: str = WAITING
    error: int = 0
    t_admit: float = float("nan")
    t_done: float = float("nan")
    result: dict = field(default_factory=dict)

    @property
    def P(self) -> int:
        return int(self.quats.shape[0])

    @property
    def L(self) -> int:
        return int(self.lig_charges.shape[0])


def validate(req: Request, proteins: dict) -> int:
    """0 if the request can be served, else a rejection code."""
    if req.protein not in proteins:
        return E_UNKNOWN_PROTEIN
    try:
        ok = (req.lig_charges.ndim == 1 and req.lig_positions.shape == (req.L, 3) and 1 <= req.L <= 896
              and req.quats.ndim == 2 and req.quats.shape[1] == 4 and req.trans.shape == (req.P, 3)
              and np.isfinite(req.vdw_min) and req.vdw_min >= 0
              and np.all(np.isfinite(req.lig_charges)) and np.all(np.isfinite(req.lig_positions)))
    except (AttributeError, TypeError, ValueError):
        ok = False
    return 0 if ok else E_MALFORMED


def request_bytes(req: Request, nchunk: int) -> int:
    """Device bytes a request holds while in flight (inputs, outputs, batch scratch)."""
    P, L = req.P, req.L
    inputs = 8 * (4 * L + 7 * P)
    outputs = P * (8 + 1 + 4)
    scratch = 32 * L + 8 + 8 * P + 8 * nchunk * P + 512
    return inputs + outputs + scratch


class Scheduler:
    """FIFO admission under a byte budget, with a bound on rounds in flight and poses per round."""

    def __init__(self, budget_bytes: int, resident_bytes: int, max_rounds: int = 2, max_round_poses: int = 4_000_000):
        self.budget = int(budget_bytes)
        self.resident = int(resident_bytes)
        self.in_flight = 0
        self.max_rounds = max_rounds
        self.max_round_poses = max_round_poses
        self.rounds = 0
        self.waiting: deque = deque()

    def free_bytes(self) -> int:
        return self.budget - self.resident - self.in_flight

    def submit(self, req: Request, cost: int) -> bool:
        """Queue a request; a request that could never fit the budget is rejected."""
        if cost > self.budget - self.resident:
            req.state, req.error = REJECTED, E_TOO_LARGE
            return False
        req._cost = cost
        self.waiting.append(req)
        return True

    def cancel(self, req: Request) -> bool:
        """Cancel a waiting request (its slot goes to the next one)."""
        if req.state == WAITING and req in self.waiting:
            self.waiting.remove(req)
            req.state = CANCELLED
            return True
        return False

    def next_round(self) -> list:
        """Requests to admit now (in arrival order), or [] if none fits or too many rounds run."""
        if self.rounds >= self.max_rounds:
            return []
        take, poses, free = [], 0, self.free_bytes()
        while self.waiting:
            r = self.waiting[0]
            if r._cost > free or (take and poses + r.P > self.max_round_poses):
                break
            self.waiting.popleft()
            take.append(r)
            free -= r._cost
            poses += r.P
        if take:
            self.in_flight += sum(r._cost for r in take)
            self.rounds += 1
            for r in take:
                r.state = RUNNING
        return take

    def finish_round(self, reqs: list) -> None:
        self.in_flight -= sum(r._cost for r in reqs)
        self.rounds -= 1
        for r in reqs:
            r.state = DONE


class Server:
    """Serve a trace of requests against resident tensors on one GPU."""

    def __init__(self, tensors: dict, hbm_budget_bytes: int, streams: int = 2, max_round_poses: int = 4_000_000,
                 device: int = 0):
        import torch
        self.torch = torch
        self.tensors = tensors
        self.dev = torch.device(f"cuda:{device}")
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.ctxs = [rsdock.Context(device, stream=s.cuda_stream) for s in self.streams]
        self.nchunk = {k: -(-t.query()["R"] // 64) for k, t in tensors.items()}
        resident = sum(t.query()["bytes"] for t in tensors.values())
        self.sched = Scheduler(hbm_budget_bytes, resident, max_rounds=streams, max_round_poses=max_round_poses)

    def _launch(self, reqs: list, k: int):
        torch, dev = self.torch, self.dev
        s = self.streams[k]
        batch_reqs, keep = [], []
        with torch.cuda.stream(s):
            for r in reqs:
                host = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).pin_memory()
                        for a in (r.lig_charges, r.lig_positions, r.quats, r.trans)]
                d = [h.to(dev, non_blocking=True) for h in host]
                out = dict(E=torch.empty(r.P, dtype=torch.float64, device=dev),
                           flags=torch.empty(r.P, dtype=torch.uint8, device=dev),
                           counts=torch.empty(r.P, dtype=torch.int32, device=dev))
                batch_reqs.append(dict(tensor=self.tensors[r.protein], lig_charges=d[0], lig_positions=d[1],
                                       quats=d[2], trans=d[3], vdw_min=r.vdw_min, out=out))
                keep.append((host, d))
            b = rsdock.Batch(self.ctxs[k], batch_reqs)
            b.run()
            res = []
            for br in batch_reqs:
                o = br["out"]
                res.append({key: torch.empty(v.shape, dtype=v.dtype, pin_memory=True).copy_(v, non_blocking=True)
                            for key, v in o.items()})
            ev = torch.cuda.Event()
            ev.record(s)
        return dict(reqs=reqs, batch=b, event=ev, results=res, keep=(keep, batch_reqs), stream=k)

    def run(self, trace: list, realtime: bool = True) -> dict:
        """Serve `trace` (Requests with arrival offsets); returns latency and throughput statistics."""
        pending = deque(sorted(trace, key=lambda r: r.arrival))
        rounds = {}
        t0 = time.perf_counter()
        free_streams = deque(range(len(self.streams)))
        done_poses = 0
        while pending or self.sched.waiting or rounds:
            now = time.perf_counter() - t0
            while pending and (pending[0].arrival <= now or not realtime):
                r = pending.popleft()
                code = validate(r, self.tensors)
                if code:
                    r.state, r.error = REJECTED, code
                    continue
                self.sched.submit(r, request_bytes(r, self.nchunk[r.protein]))
            progressed = False
            for k in list(rounds):
                rd = rounds[k]
                if rd["event"].query():
                    t_done = time.perf_counter() - t0
                    for r, res in zip(rd["reqs"], rd["results"]):
                        r.result = {key: v.numpy() for key, v in res.items()}
                        r.t_done = t_done
                        done_poses += r.P
                    rd["batch"].free()
                    self.sched.finish_round(rd["reqs"])
                    free_streams.append(k)
                    del rounds[k]
                    progressed = True
            while free_streams:
                take = self.sched.next_round()
                if not take:
                    break
                k = free_streams.popleft()
                t_adm = time.perf_counter() - t0
                for r in take:
                    r.t_admit = t_adm
                rounds[k] = self._launch(take, k)
                progressed = True
            if not progressed:
                if pending and realtime and not self.sched.waiting and not rounds:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (time.perf_counter() - t0))))
                else:
                    time.sleep(0.0002)
        wall = time.perf_counter() - t0
        served = [r for r in trace if r.state == DONE]
        lat = np.array([r.t_done - r.arrival for r in served]) if served else np.zeros(0)
        return {
            "requests": len(trace), "served": len(served),
            "rejected": sum(r.state == REJECTED for r in trace),
            "poses": int(sum(r.P for r in served)), "wall_s": wall,
            "poses_per_s": sum(r.P for r in served) / wall if wall > 0 else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)) if lat.size else float("nan"),
            "latency_p99_s": float(np.percentile(lat, 99)) if lat.size else float("nan"),
            "latency_max_s": float(lat.max()) if lat.size else float("nan"),
        }

    def close(self) -> None:
        for c in self.ctxs:
            c.close()
