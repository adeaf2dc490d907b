"""CPU tests of the serving scheduler: admission by byte budget, FIFO order, rejection,
cancellation, and the bound on rounds in flight.  No device is used."""
import numpy as np

from paper_2510_26611_amd import serve


def _req(rid, P=100, L=10, protein="a", arrival=0.0):
    g = np.random.default_rng(rid)
    q = g.normal(size=(P, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return serve.Request(rid, protein, g.normal(size=L), g.normal(size=(L, 3)), q, g.normal(size=(P, 3)), 2.5,
                         arrival)


def test_request_bytes_grows_with_poses_and_chunks():
    r = _req(0, P=1000)
    assert serve.request_bytes(r, 10) > serve.request_bytes(r, 1) > 0
    assert serve.request_bytes(_req(1, P=2000), 10) > serve.request_bytes(r, 10)


def test_budget_exhaustion_queues_then_admits_in_order():
    reqs = [_req(i, P=1000) for i in range(5)]
    cost = serve.request_bytes(reqs[0], 4)
    s = serve.Scheduler(budget_bytes=1000 + 2 * cost, resident_bytes=1000, max_rounds=8)
    for r in reqs:
        assert s.submit(r, cost)
    first = s.next_round()
    assert [r.rid for r in first] == [0, 1]           # only two fit
    assert s.next_round() == []                       # budget exhausted: the rest wait
    assert all(r.state == serve.WAITING for r in reqs[2:])
    s.finish_round(first)
    second = s.next_round()
    assert [r.rid for r in second] == [2, 3]
    assert s.free_bytes() == 0


def test_too_large_is_rejected_not_queued():
    s = serve.Scheduler(budget_bytes=10_000, resident_bytes=5_000)
    big = _req(7, P=10_000)
    assert not s.submit(big, serve.request_bytes(big, 8))
    assert big.state == serve.REJECTED and big.error == serve.E_TOO_LARGE
    assert len(s.waiting) == 0


def test_cancel_frees_the_slot_for_the_next_request():
    reqs = [_req(i, P=500) for i in range(3)]
    cost = serve.request_bytes(reqs[0], 2)
    s = serve.Scheduler(budget_bytes=cost, resident_bytes=0)
    for r in reqs:
        s.submit(r, cost)
    assert s.cancel(reqs[0])
    assert reqs[0].state == serve.CANCELLED
    got = s.next_round()
    assert [r.rid for r in got] == [1]
    assert not s.cancel(reqs[1])                      # running requests cannot be cancelled


def test_rounds_in_flight_are_bounded_and_pose_cap_splits_rounds():
    reqs = [_req(i, P=100) for i in range(6)]
    s = serve.Scheduler(budget_bytes=10 ** 12, resident_bytes=0, max_rounds=2, max_round_poses=250)
    for r in reqs:
        s.submit(r, 1)
    a = s.next_round()
    b = s.next_round()
    assert [r.rid for r in a] == [0, 1] and [r.rid for r in b] == [2, 3]
    assert s.next_round() == []                       # two rounds already in flight
    s.finish_round(a)
    assert [r.rid for r in s.next_round()] == [4, 5]


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
