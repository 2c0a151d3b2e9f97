"""Host logic of the serving loop: admission by budget, cohorts, completion.

No GPU: the Scheduler is driven with made-up byte costs.
"""

import numpy as np
import pytest

import synth.serving as ss
from paper_2509_01180_amd.serving import BoxSpec, Request, Scheduler, latency_summary

SPECS = {32: BoxSpec(32, 16, (8, 16), 100),
         64: BoxSpec(64, 32, (8, 16, 24, 32), 1000),
         96: BoxSpec(96, 40, (8, 16, 24, 32, 40), 3000)}


def req(box, n, rid=0):
    return Request(box=box, template=0, n=n, volumes=None, starts=None, rid=rid)


def test_rejects_unservable_requests():
    s = Scheduler(SPECS, budget_bytes=100_000)
    with pytest.raises(ValueError):
        s.submit(req(48, 1))
    with pytest.raises(ValueError):
        s.submit(req(64, 0))
    with pytest.raises(ValueError):
        s.submit(req(96, 34))          # 102,000 bytes > budget even when idle
    s.submit(req(96, 33))              # fits an empty device


def test_admission_fifo_and_budget():
    s = Scheduler(SPECS, budget_bytes=10_000)
    for i, (box, n) in enumerate([(64, 4), (32, 10), (96, 2), (64, 3)]):
        s.submit(req(box, n, i))
    new = s.admit()
    # 4000 + 1000 + 6000 > 10000: the 96^3 request blocks; nothing overtakes it
    assert sorted(c.box for c in new) == [32, 64]
    assert s.used == 5000 and [r.rid for r in s.queue] == [2, 3]
    assert all(c.cursor == 0 for c in new)
    # 32^3 finishes after two ticks and frees its bytes; 64^3 needs four
    for t in range(2):
        assert s.admit() == []
        s.plan()
        done = s.advance()
    assert [c.box for c in done] == [32] and s.used == 4000
    new = s.admit()                    # 4000 + 6000 fits now, then 3000 does not
    assert [c.box for c in new] == [96] and [r.rid for r in s.queue] == [3]


def test_cohort_cap_and_single_large_request():
    s = Scheduler(SPECS, budget_bytes=10 ** 9, max_cohort=8)
    for i, n in enumerate([5, 4, 20, 1]):
        s.submit(req(32, n, i))
    c1 = s.admit()
    assert [c.n for c in c1] == [5]            # 5 + 4 > 8 stops admission
    s.advance()
    c2 = s.admit()
    assert [c.n for c in c2] == [4]            # 4 + 20 > 8
    s.advance()
    c3 = s.admit()
    assert [c.n for c in c3] == [20]           # alone it is admitted past the cap
    s.advance()
    assert [c.n for c in s.admit()] == [1]


def test_band_schedule_of_each_cohort():
    s = Scheduler(SPECS, budget_bytes=10 ** 9)
    s.submit(req(96, 1, 0))
    s.admit()
    seen = []
    for t in range(5):
        (c, band, last), = s.plan()
        seen.append((band, last))
        done = s.advance()
        assert (len(done) == 1) == (t == 4)
    assert seen == [(8, False), (16, False), (24, False), (32, False), (40, True)]
    assert not s.busy() and s.used == 0


def test_simulated_stream_properties():
    """Random arrivals: every request completes exactly once, len(bands)
    ticks after its admission; the budget is never exceeded; admission keeps
    arrival order; cohorts at one tick share their band."""
    rng = np.random.default_rng(0)
    budget = 40_000
    s = Scheduler(SPECS, budget_bytes=budget, max_cohort=64)
    boxes = list(SPECS)
    reqs = []
    for i in range(300):
        box = boxes[rng.integers(3)]
        reqs.append(req(box, int(rng.integers(1, 11)), i))
    admitted_order, admit_tick, done_tick = [], {}, {}
    i = 0
    for tick in range(2000):
        for _ in range(rng.integers(0, 4)):
            if i < len(reqs):
                s.submit(reqs[i])
                i += 1
        now = sorted(r.rid for c in s.admit() for r in c.requests)
        admitted_order += now
        admit_tick.update({rid: tick for rid in now})
        assert s.used <= budget
        bands_now = {}
        for c, band, last in s.plan():
            assert c.cursor == tick - c.tick
            bands_now.setdefault((c.box, c.tick), band)
        for c in s.advance():
            for r in c.requests:
                assert r.rid not in done_tick
                done_tick[r.rid] = tick
        if i == len(reqs) and not s.busy():
            break
    assert admitted_order == list(range(len(reqs)))
    for r in reqs:
        assert done_tick[r.rid] - admit_tick[r.rid] == len(SPECS[r.box].bands) - 1
    assert s.used == 0


def test_request_stream_recipe():
    r = ss.request_stream(200.0, 30.0, (32, 64, 96), seed=1)
    n = np.array([x.n for x in r])
    t = np.array([x.arrival for x in r])
    assert abs(len(r) / 30.0 - 200.0) < 4 * np.sqrt(200.0 / 30.0) + 1   # Poisson count
    assert n.min() >= 1 and n.max() <= 512 and abs(n.mean() - 256.5) < 15
    assert np.all(np.diff(t) > 0) and t[-1] < 30.0
    assert {x.box for x in r} == {32, 64, 96}
    assert {x.template for x in r} == set(range(8))
    # exponential gaps: coefficient of variation ~1
    g = np.diff(t)
    assert abs(g.std() / g.mean() - 1.0) < 0.1


def test_latency_summary():
    rs = [Request(box=32, template=0, n=1, volumes=None, starts=None, arrival=0.0, done=d)
          for d in np.linspace(0.001, 0.1, 100)]
    out = latency_summary(rs)
    assert out["n"] == 100 and 50 < out["p50_ms"] < 51 and out["max_ms"] == pytest.approx(100.0)
