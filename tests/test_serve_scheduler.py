"""CPU tests of the serving scheduler: admission by byte budget in arrival order, rejection,
cancellation, the bound on rounds in flight, and the pose slices shared by a round.  No
device is used; a simulated executor checks the latency property the slicing is for."""
import numpy as np
import pytest

from paper_2510_26611_amd import serve


def _req(rid, P=100, L=10, protein="a", arrival=0.0):
    g = np.random.default_rng(rid)
    q = g.normal(size=(P, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return serve.Request(rid, protein, g.normal(size=L), g.normal(size=(L, 3)), q, g.normal(size=(P, 3)), 2.5,
                         arrival)


def _drain(s):
    """Issue and finish rounds one at a time until nothing is active; returns the rounds issued."""
    rounds = []
    while True:
        s.admit()
        sl = s.next_round()
        if not sl:
            return rounds
        rounds.append(sl)
        s.finish_round(sl)


def test_request_bytes_and_round_scratch_grow_with_size():
    assert serve.request_bytes(_req(1, P=2000)) > serve.request_bytes(_req(0, P=1000)) > 0
    assert serve.request_bytes(_req(2, P=1000, L=100)) > serve.request_bytes(_req(3, P=1000, L=10))
    assert serve.round_scratch_bytes(1000, 20) > serve.round_scratch_bytes(1000, 2) > serve.round_scratch_bytes(10, 2)


def test_budget_exhaustion_queues_then_admits_in_order():
    reqs = [_req(i, P=1000) for i in range(5)]
    cost = serve.request_bytes(reqs[0])
    s = serve.Scheduler(budget_bytes=1000 + 500 + 2 * cost, resident_bytes=1000, scratch_bytes=500, max_rounds=8,
                        round_poses=10_000, min_slice=10)
    for r in reqs:
        assert s.submit(r, cost)
    assert [r.rid for r in s.admit()] == [0, 1]        # only two fit next to the resident and scratch bytes
    assert s.admit() == []
    assert all(r.state == serve.WAITING for r in reqs[2:])
    sl = s.next_round()
    assert [(r.rid, off, n) for r, off, n in sl] == [(0, 0, 1000), (1, 0, 1000)]
    done = s.finish_round(sl)
    assert [r.rid for r in done] == [0, 1] and all(r.state == serve.DONE for r in done)
    assert [r.rid for r in s.admit()] == [2, 3]
    assert s.free_bytes() == 0


def test_too_large_is_rejected_not_queued():
    s = serve.Scheduler(budget_bytes=10_000, resident_bytes=5_000)
    big = _req(7, P=10_000)
    assert not s.submit(big, serve.request_bytes(big))
    assert big.state == serve.REJECTED and big.error == serve.E_TOO_LARGE
    assert len(s.waiting) == 0


def test_cancel_frees_the_slot_for_the_next_request():
    reqs = [_req(i, P=500) for i in range(3)]
    cost = serve.request_bytes(reqs[0])
    s = serve.Scheduler(budget_bytes=cost, resident_bytes=0)
    for r in reqs:
        s.submit(r, cost)
    assert s.cancel(reqs[0])
    assert reqs[0].state == serve.CANCELLED
    assert [r.rid for r in s.admit()] == [1]
    assert not s.cancel(reqs[1])                       # admitted requests cannot be cancelled


def test_round_budget_is_shared_and_leftovers_redistributed():
    s = serve.Scheduler(budget_bytes=10 ** 12, resident_bytes=0, max_rounds=4, round_poses=60_000, min_slice=1_000,
                        policy="share")
    a, b, c = _req(0, P=100_000), _req(1, P=10_000), _req(2, P=300_000)
    for r in (a, b, c):
        s.submit(r, 1)
    s.admit()
    sl = s.next_round()
    # quota 20k each; b needs only 10k, the 10k it leaves go to the first request that can use them
    assert [(r.rid, off, n) for r, off, n in sl] == [(0, 0, 30_000), (1, 0, 10_000), (2, 0, 20_000)]
    assert sum(n for _, _, n in sl) == 60_000
    sl2 = s.next_round()                               # second round in flight continues where the first stopped
    assert [(r.rid, off, n) for r, off, n in sl2] == [(0, 30_000, 30_000), (2, 20_000, 30_000)]
    assert s.finish_round(sl) == [b]
    assert a.state == serve.RUNNING and c.state == serve.RUNNING


def test_every_pose_is_issued_exactly_once():
    g = np.random.default_rng(4)
    reqs = [_req(i, P=int(p)) for i, p in enumerate(g.integers(1, 50_000, 12))]
    s = serve.Scheduler(budget_bytes=10 ** 12, resident_bytes=0, round_poses=20_000, min_slice=700)
    for r in reqs:
        s.submit(r, 1)
    rounds = _drain(s)
    cover = {r.rid: np.zeros(r.P, dtype=int) for r in reqs}
    for sl in rounds:
        assert sum(n for _, _, n in sl) <= 20_000
        assert len({r.rid for r, _, _ in sl}) == len(sl)          # one slice per request per round
        for r, off, n in sl:
            assert n >= 1
            cover[r.rid][off:off + n] += 1
    assert all(np.all(c == 1) for c in cover.values())
    assert all(r.state == serve.DONE for r in reqs) and s.in_flight == 0 and s.active == []


def test_rounds_in_flight_are_bounded():
    s = serve.Scheduler(budget_bytes=10 ** 12, resident_bytes=0, max_rounds=2, round_poses=100, min_slice=10)
    for i in range(6):
        s.submit(_req(i, P=100), 1)
    s.admit()
    a, b = s.next_round(), s.next_round()
    assert a and b and s.next_round() == []            # two rounds already in flight
    s.finish_round(a)
    assert s.next_round() != []


@pytest.mark.parametrize("policy,min_slice", [("share", 1_000), ("small_first", 3_000)])
def test_small_requests_are_not_held_behind_a_large_one(policy, min_slice):
    """Simulated executor, one pose per time unit, rounds run one after another: requests
    arriving just after a huge one finish long before it; with one whole request per round
    (round budget >= the largest request, no sharing) they would wait for all of it.  Policy
    small_first takes the 5,000-pose requests (at most 2 min_slice) whole into the next round."""
    def simulate(round_poses, min_slice, policy):
        reqs = [_req(0, P=200_000, arrival=0.0)] + [_req(i, P=5_000, arrival=1.0 + i) for i in range(1, 6)]
        s = serve.Scheduler(budget_bytes=10 ** 12, resident_bytes=0, max_rounds=1, round_poses=round_poses,
                            min_slice=min_slice, policy=policy)
        t, pending = 0.0, list(reqs)
        while pending or s.active:
            for r in [r for r in pending if r.arrival <= t]:
                s.submit(r, 1)
                pending.remove(r)
            s.admit()
            sl = s.next_round()
            if not sl:
                t = pending[0].arrival
                continue
            t += sum(n for _, _, n in sl)
            for r in s.finish_round(sl):
                r.t_done = t
        return reqs

    shared = simulate(20_000, min_slice, policy)
    whole = simulate(10 ** 9, 10 ** 9, "share")
    small_shared = max(r.t_done - r.arrival for r in shared[1:])
    small_whole = min(r.t_done - r.arrival for r in whole[1:])
    # at most the round already running when they arrive plus two shared rounds
    assert small_shared <= 3 * 20_000 and small_shared < 0.3 * small_whole
    # the large request pays only for the small ones' poses
    assert shared[0].t_done <= whole[0].t_done + 5 * 5_000 + 1


def test_validate_rejects_malformed_and_unknown():
    ok = _req(0)
    assert serve.validate(ok, {"a": None}) == 0
    assert serve.validate(_req(1, protein="zz"), {"a": None}) == serve.E_UNKNOWN_PROTEIN
    bad = _req(2)
    bad.lig_positions = bad.lig_positions[:, :2]
    assert serve.validate(bad, {"a": None}) == serve.E_MALFORMED
    nan = _req(3)
    nan.lig_charges[0] = np.nan
    assert serve.validate(nan, {"a": None}) == serve.E_MALFORMED
    big = _req(4, L=900)
    assert serve.validate(big, {"a": None}) == serve.E_MALFORMED


def test_small_first_policy_takes_small_requests_whole_then_fifo():
    s = serve.Scheduler(budget_bytes=10**12, resident_bytes=0, max_rounds=8, round_poses=100_000, min_slice=1000,
                        policy="small_first")
    big1, big2, small = _req(0, P=150_000), _req(1, P=80_000), _req(2, P=1500)
    for r in (big1, big2, small):
        s.submit(r, serve.request_bytes(r))
    s.admit()
    sl = s.next_round()
    # the small request whole, then the oldest large request takes the rest of the round
    assert [(r.rid, off, n) for r, off, n in sl] == [(2, 0, 1500), (0, 0, 98_500)]
    s.finish_round(sl)
    sl = s.next_round()
    assert [(r.rid, off, n) for r, off, n in sl] == [(0, 98_500, 51_500), (1, 0, 48_500)]
    s.finish_round(sl)
    rounds = _drain(s)
    assert all(r.state == serve.DONE for r in (big1, big2, small)) and len(rounds) == 1


def test_unknown_policy_is_refused():
    import pytest
    with pytest.raises(ValueError):
        serve.Scheduler(budget_bytes=1, resident_bytes=0, policy="lottery")
