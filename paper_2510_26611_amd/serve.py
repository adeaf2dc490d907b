"""Continuous-batching request server over resident RS tensors.

Requests (protein id, ligand, poses, vdW distance) arrive over time.  Each protein's RS
tensor and cell list stay resident on the device.  A waiting request is admitted, in arrival
order, once its device memory (inputs and outputs) fits the HBM budget next to the resident
tensors and the scratch reserved for the rounds in flight.  Work is issued in rounds: every
round is one rsd_batch over pose slices of the admitted, unfinished requests, with a fixed
pose budget shared evenly among them (each gets at least `min_slice` poses while the budget
lasts, in admission order), or with policy "small_first" given whole to the small requests
first and then to the larger ones first come, first served.  A request that arrives while others are on the device therefore
joins the next round instead of waiting for them to finish, and a small request completes
in a round or two even behind a very large one.

Rounds alternate between streams, each with its own context: a round's uploads, host-side
planning and downloads overlap the neighbouring rounds' kernels, while an event between the
streams keeps the kernels of successive rounds in issue order (two rounds sharing the device
would only delay both).  Latency is measured from arrival to the moment the last slice of a
request is back on the host.

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

# how a round's pose budget is shared: evenly among the admitted requests ("share"), or whole
# small requests first and then the larger ones first come, first served ("small_first")
POLICIES = ("share", "small_first")

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


def request_bytes(req: Request) -> int:
    """Device bytes a request holds from admission to completion: inputs and outputs, and at
    most the spatial-order copies of its poses with their permutation and sort scratch."""
    return 8 * (4 * req.L + 7 * req.P) + req.P * (8 + 1 + 4) + req.P * (7 * 8 + 4 + 4) + 4 * 32768 + 256


def round_scratch_bytes(round_poses: int, nchunk: int, max_ligand: int = 896, slices: int = 64) -> int:
    """Batch scratch of one round of at most `round_poses` poses and `slices` slices: per-chunk
    long-range partials, short-range energies, ligand frames and the request table."""
    return 8 * round_poses * (nchunk + 1) + slices * (32 * max_ligand + 8 + 1024) + 4096


class Scheduler:
    """Admission by byte budget in arrival order, and pose slices per round shared evenly."""

    def __init__(self, budget_bytes: int, resident_bytes: int, scratch_bytes: int = 0, max_rounds: int = 2,
                 round_poses: int = 250_000, min_slice: int = 16_384, policy: str = "small_first"):
        if policy not in POLICIES:
            raise ValueError(f"policy must be one of {POLICIES}")
        self.policy = policy
        self.budget = int(budget_bytes)
        self.reserved = int(resident_bytes) + int(scratch_bytes)
        self.in_flight = 0
        self.max_rounds = max_rounds
        self.round_poses = int(round_poses)
        self.min_slice = int(min_slice)
        self.rounds = 0
        self.waiting: deque = deque()
        self.active: list = []          # admitted, not finished, in admission order

    def free_bytes(self) -> int:
        return self.budget - self.reserved - self.in_flight

    def submit(self, req: Request, cost: int) -> bool:
        """Queue a request; one that could never fit the budget is rejected."""
        if cost > self.budget - self.reserved:
            req.state, req.error = REJECTED, E_TOO_LARGE
            return False
        req._cost = cost
        self.waiting.append(req)
        return True

    def cancel(self, req: Request) -> bool:
        """Cancel a request that has not been admitted yet."""
        if req.state == WAITING and req in self.waiting:
            self.waiting.remove(req)
            req.state = CANCELLED
            return True
        return False

    def admit(self) -> list:
        """Move waiting requests that fit the budget, in arrival order, to the active set."""
        got = []
        while self.waiting and self.waiting[0]._cost <= self.free_bytes():
            r = self.waiting.popleft()
            self.in_flight += r._cost
            r.state, r._next, r._done = RUNNING, 0, 0
            self.active.append(r)
            got.append(r)
        return got

    def next_round(self) -> list:
        """Slices (request, first pose, count) for the next round, or [] if none can be issued."""
        if self.rounds >= self.max_rounds:
            return []
        live = [r for r in self.active if r._next < r.P]
        if not live:
            return []
        if self.policy == "small_first":
            return self._round_small_first(live)
        quota = max(self.min_slice, self.round_poses // len(live))
        left, take = self.round_poses, []
        for r in live:
            n = min(r.P - r._next, quota, left)
            if n <= 0:
                break
            take.append([r, n])
            left -= n
        for t in take:                  # what short requests left unused goes to the others, in order
            if left <= 0:
                break
            extra = min(t[0].P - t[0]._next - t[1], left)
            t[1] += extra
            left -= extra
        out = []
        for r, n in take:
            out.append((r, r._next, n))
            r._next += n
        self.rounds += 1
        return out

    def _round_small_first(self, live: list) -> list:
        """Policy small_first: every small request (at most 2 min_slice poses) goes whole into the
        next round, in admission order; the rest of the round goes to the larger requests first
        come, first served, so a large request is not slowed by other large ones sharing rounds."""
        small_max = 2 * self.min_slice
        order = [r for r in live if r.P <= small_max] + [r for r in live if r.P > small_max]
        left, out = self.round_poses, []
        for r in order:
            n = min(r.P - r._next, left)
            if n <= 0:
                break
            out.append((r, r._next, n))
            r._next += n
            left -= n
        self.rounds += 1
        return out

    def finish_round(self, slices: list) -> list:
        """Account a completed round; returns the requests it completed."""
        self.rounds -= 1
        done = []
        for r, _, n in slices:
            r._done += n
            if r._done == r.P:
                r.state = DONE
                self.in_flight -= r._cost
                self.active.remove(r)
                done.append(r)
        return done


def latency_stats(trace: list, wall: float) -> dict:
    """Throughput over the wall time and arrival-to-result latency percentiles of the served requests."""
    served = [r for r in trace if r.state == DONE]
    lat = np.array([r.t_done - r.arrival for r in served]) if served else np.zeros(0)
    wait = np.array([r.t_admit - r.arrival for r in served]) if served else np.zeros(0)
    poses = int(sum(r.P for r in served))
    pct = lambda a, q: float(np.percentile(a, q)) if a.size else float("nan")  # noqa: E731
    return {
        "requests": len(trace), "served": len(served),
        "rejected": sum(r.state == REJECTED for r in trace),
        "poses": poses, "wall_s": wall,
        "poses_per_s": poses / wall if wall > 0 else 0.0,
        "latency_p50_s": pct(lat, 50), "latency_p99_s": pct(lat, 99),
        "latency_max_s": float(lat.max()) if lat.size else float("nan"),
        "queue_wait_p50_s": pct(wait, 50),
    }


def serve_plain(ctx, tensors: dict, trace: list, realtime: bool = True, progress=None) -> dict:
    """The baseline the server is compared with: requests one at a time in arrival order, each
    scored by one plain rsd_score_poses call on host arrays (upload, launches, download)."""
    t0 = time.perf_counter()
    order = sorted(trace, key=lambda r: r.arrival)
    for i, r in enumerate(order):
        code = validate(r, tensors)
        if code:
            r.state, r.error = REJECTED, code
            continue
        if realtime:
            delay = r.arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
        r.t_admit = time.perf_counter() - t0
        r.result = rsdock.score_poses(ctx, tensors[r.protein], r.lig_charges, r.lig_positions, r.quats, r.trans,
                                      r.vdw_min)
        r.t_done = time.perf_counter() - t0
        r.state = DONE
        if progress is not None:
            progress(i + 1, len(order))
    return latency_stats(trace, time.perf_counter() - t0)


class Server:
    """Serve a trace of requests against resident tensors on one GPU."""

    def __init__(self, tensors: dict, hbm_budget_bytes: int, streams: int = 2, round_poses: int = 250_000,
                 min_slice: int = 16_384, device: int = 0, options: dict | None = None,
                 policy: str = "small_first"):
        import torch
        self.torch = torch
        self.tensors = tensors
        self.dev = torch.device(f"cuda:{device}")
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.ctxs = [rsdock.Context(device, stream=s.cuda_stream) for s in self.streams]
        for c in self.ctxs:
            for name, value in (options or {}).items():
                c.set_option(name, value)
        nchunk = max(-(-t.query()["R"] // 64) for t in tensors.values())
        resident = sum(t.query()["bytes"] for t in tensors.values())
        self.sched = Scheduler(hbm_budget_bytes, resident, streams * round_scratch_bytes(round_poses, nchunk),
                               max_rounds=streams, round_poses=round_poses, min_slice=min_slice, policy=policy)
        self.last_compute = None
        self.pose_order = int((options or {}).get("pose_order", 0))
        self.ordered = 0   # requests sliced in spatial order so far
        self._k = 0

    def _orders(self, r: Request) -> bool:
        """Whether a request is sliced in spatial order: option pose_order 1 always, 2 never,
        0 when it is large enough to be cut into several slices."""
        if r.P < 2 or self.pose_order == 2:
            return False
        return self.pose_order == 1 or r.P >= 2 * self.sched.min_slice

    def _upload(self, r: Request) -> None:
        """Inputs to the device and output buffers (device + pinned host) for a newly admitted request."""
        torch, dev = self.torch, self.dev
        host = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).pin_memory()
                for a in (r.lig_charges, r.lig_positions, r.quats, r.trans)]
        r._host_in = host
        r._dev = [h.to(dev, non_blocking=True) for h in host]
        r._perm = None
        if self._orders(r):
            # slices of the request in the long-range kernels' spatial order: each slice then
            # covers a compact part of the grid; results come back in that order and are put
            # back in request order on the host at the end
            perm, q, t, _ = rsdock.pose_order(self.ctxs[self._k], self.tensors[r.protein], r._dev[2], r._dev[3])
            r._dev[2], r._dev[3] = q, t
            r._perm = torch.empty(r.P, dtype=torch.int32, pin_memory=True)
            r._perm.copy_(perm, non_blocking=True)
            r._perm_dev = perm
            self.ordered += 1
        r._out = dict(E=torch.empty(r.P, dtype=torch.float64, device=dev),
                      flags=torch.empty(r.P, dtype=torch.uint8, device=dev),
                      counts=torch.empty(r.P, dtype=torch.int32, device=dev))
        r._res = {k: torch.empty(v.shape, dtype=v.dtype, pin_memory=True) for k, v in r._out.items()}

    def _launch(self, slices: list, k: int) -> dict:
        torch = self.torch
        s = self.streams[k]
        self._k = k
        with torch.cuda.stream(s):
            for r, off, _ in slices:
                if off == 0:
                    self._upload(r)
            breqs = []
            for r, off, n in slices:
                z, x, q, t = r._dev
                breqs.append(dict(tensor=self.tensors[r.protein], lig_charges=z, lig_positions=x,
                                  quats=q[off:off + n], trans=t[off:off + n], vdw_min=r.vdw_min,
                                  out={key: v[off:off + n] for key, v in r._out.items()}))
            b = rsdock.Batch(self.ctxs[k], breqs)
            if self.last_compute is not None:
                s.wait_event(self.last_compute)
            b.run()
            ce = torch.cuda.Event()
            ce.record(s)
            self.last_compute = ce
            for r, off, n in slices:
                for key, v in r._out.items():
                    r._res[key][off:off + n].copy_(v[off:off + n], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return dict(slices=slices, batch=b, event=ev)

    def run(self, trace: list, realtime: bool = True, progress=None) -> dict:
        """Serve `trace` (Requests with arrival offsets); returns latency and throughput statistics.

        `progress(done, total)` is called whenever requests complete."""
        pending = deque(sorted(trace, key=lambda r: r.arrival))
        rounds = {}
        t0 = time.perf_counter()
        free_streams = deque(range(len(self.streams)))
        finished = 0
        while pending or self.sched.waiting or self.sched.active or rounds:
            now = time.perf_counter() - t0
            while pending and (pending[0].arrival <= now or not realtime):
                r = pending.popleft()
                code = validate(r, self.tensors)
                if code:
                    r.state, r.error = REJECTED, code
                    continue
                if r.P == 0:
                    r.state, r.t_admit, r.t_done = DONE, now, now
                    r.result = dict(E=np.empty(0), flags=np.empty(0, np.uint8), counts=np.empty(0, np.int32))
                    continue
                self.sched.submit(r, request_bytes(r))
            progressed = False
            for k in list(rounds):
                rd = rounds[k]
                if rd["event"].query():
                    t_done = time.perf_counter() - t0
                    rd["batch"].free()
                    for r in self.sched.finish_round(rd["slices"]):
                        r.result = {key: v.numpy() for key, v in r._res.items()}
                        if r._perm is not None:
                            perm = r._perm.numpy()
                            for key, v in r.result.items():
                                back = np.empty_like(v)
                                back[perm] = v
                                r.result[key] = back
                        r.t_done = t_done
                        r._dev = r._out = r._host_in = r._res = r._perm = r._perm_dev = None
                        finished += 1
                        if progress is not None:
                            progress(finished, len(trace))
                    free_streams.append(k)
                    del rounds[k]
                    progressed = True
            t_adm = time.perf_counter() - t0
            for r in self.sched.admit():
                r.t_admit = t_adm
            while free_streams:
                slices = self.sched.next_round()
                if not slices:
                    break
                k = free_streams.popleft()
                rounds[k] = self._launch(slices, k)
                progressed = True
            if not progressed:
                idle = not (self.sched.waiting or self.sched.active or rounds)
                if pending and realtime and idle:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (time.perf_counter() - t0))))
                else:
                    time.sleep(0.0002)
        return latency_stats(trace, time.perf_counter() - t0)

    def close(self) -> None:
        for c in self.ctxs:
            c.close()
