"""The serving loop's host logic with a mock device on a simulated clock:
Poisson arrivals, HBM-footprint admission, continuous batching, latency
statistics and slot reuse."""
import math

import numpy as np
import pytest

from paper_2012_03325_amd import serve as S

RES = ((256, 256), (640, 480), (1920, 1080), (3840, 2160))


def _server(budget, s_per_px=1e-10, launch_s=20e-6, **kw):
    clock = S.SimClock()
    ex = S.MockExecutor(clock, s_per_px=s_per_px, launch_s=launch_s)
    return S.Server(ex, budget, **kw), ex, clock


def test_poisson_arrivals():
    reqs = S.poisson_arrivals(500.0, 7, 32, RES, duration=20.0)
    assert reqs == sorted(reqs, key=lambda r: r.arrival)
    assert abs(len(reqs) / 20.0 - 500.0) < 4 * math.sqrt(500.0 * 20.0) / 20.0
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 500.0) < 0.05 / 500.0
    counts = np.bincount([RES.index(r.res) for r in reqs], minlength=4)
    assert counts.min() > 0.2 * len(reqs)
    assert {r.scene for r in reqs} == set(range(32))
    again = S.poisson_arrivals(500.0, 7, 32, RES, duration=20.0)
    assert [(r.arrival, r.scene, r.res) for r in again] == [(r.arrival, r.scene, r.res) for r in reqs]
    assert len(S.poisson_arrivals(1000.0, 1, 4, RES, count=50)) == 50


def test_idle_server_latency_is_service_time():
    srv, ex, clock = _server(1 << 34, s_per_px=1e-9, launch_s=0.0)
    reqs = [S.Request(k, 0, *RES[k % 4], arrival=float(k)) for k in range(8)]
    st = srv.run(reqs, clock)
    assert st["requests"] == 8 and st["batches"] == 8
    for r in srv.finished:
        assert r.latency == pytest.approx(r.px * 1e-9, rel=1e-9)
    lat = sorted(r.px * 1e-9 for r in reqs)
    assert st["p50_ms"] == pytest.approx(1e3 * np.percentile(lat, 50))
    assert st["p99_ms"] == pytest.approx(1e3 * np.percentile(lat, 99))


def test_admission_never_exceeds_budget():
    fp = S.MockExecutor(S.SimClock()).footprint
    budget = 3 * fp((3840, 2160))
    srv, ex, clock = _server(budget, s_per_px=2e-10)
    seen = []
    alloc = ex.alloc

    def watch(res):
        seen.append(srv.pool.reserved)
        assert srv.pool.reserved <= budget
        return alloc(res)

    srv.pool._alloc = watch
    reqs = S.poisson_arrivals(2000.0, 3, 32, RES, count=600)
    st = srv.run(reqs, clock)
    assert st["requests"] == 600 and st["rejected"] == 0
    assert st["peak_reserved_bytes"] <= budget
    assert max(seen) <= budget
    # every request holds a slot from admission to completion: at any time the
    # admitted-and-unfinished requests fit the budget
    events = sorted([(r.admitted, fp(r.res)) for r in srv.finished] + [(r.done, -fp(r.res)) for r in srv.finished],
                    key=lambda e: (e[0], e[1]))
    live = 0
    for _, d in events:
        live += d
        assert live <= budget


def test_slots_are_reused():
    """With room to spare, a class never holds more slots than it had requests
    in flight at once."""
    srv, ex, clock = _server(1 << 40, s_per_px=2e-10)
    reqs = S.poisson_arrivals(2000.0, 5, 32, RES, count=600)
    st = srv.run(reqs, clock)
    assert st["requests"] == 600
    peak = 0
    for res in RES:
        events = sorted([(r.admitted, 1) for r in srv.finished if r.res == res] +
                        [(r.done, -1) for r in srv.finished if r.res == res], key=lambda e: (e[0], e[1]))
        live = best = 0
        for _, d in events:
            live += d
            best = max(best, live)
        peak += best
    assert st["slot_allocs"] <= peak < 600


def test_requests_larger_than_the_budget_are_rejected():
    fp = S.MockExecutor(S.SimClock()).footprint
    srv, ex, clock = _server(fp((1920, 1080)))
    reqs = [S.Request(0, 0, 3840, 2160, 0.0), S.Request(1, 0, 640, 480, 0.001)]
    st = srv.run(reqs, clock)
    assert st["requests"] == 1 and st["rejected"] == 1 and srv.rejected[0].rid == 0


def test_continuous_batching_admits_requests_arriving_during_a_batch():
    """One batch in flight at a time: the requests that arrive while the first
    one runs are launched together as soon as it finishes, before it drains
    anything else; admission follows arrival order."""
    srv, ex, clock = _server(1 << 34, s_per_px=1e-9, launch_s=0.0, max_inflight=1)
    first = S.Request(0, 0, 1920, 1080, 0.0)            # runs ~2.07 ms
    burst = [S.Request(k, 0, 256, 256, 1e-4 * k) for k in range(1, 11)]
    late = S.Request(11, 0, 256, 256, 0.01)
    st = srv.run([first, *burst, late], clock)
    assert st["requests"] == 12
    assert first.batch == 0
    assert {r.batch for r in burst} == {1}
    assert all(r.launched == pytest.approx(first.done) for r in burst)
    assert late.batch == 2
    order = sorted(srv.finished, key=lambda r: (r.admitted, r.rid))
    assert [r.rid for r in order] == sorted(r.rid for r in order)


def test_overlapping_batches_with_two_in_flight():
    srv, ex, clock = _server(1 << 34, s_per_px=1e-9, launch_s=0.0, max_inflight=2)
    reqs = [S.Request(k, 0, 1920, 1080, 1e-4 * k) for k in range(6)]
    srv.run(reqs, clock)
    # the second batch is launched while the first is still running
    b0 = [r for r in reqs if r.batch == 0]
    b1 = [r for r in reqs if r.batch == 1]
    assert b1 and b1[0].launched < b0[0].done


def test_batch_limits():
    srv, ex, clock = _server(1 << 36, max_batch_views=4, max_batch_px=2_500_000, max_inflight=1)
    reqs = [S.Request(k, 0, 640, 480, 0.0) for k in range(10)] + \
           [S.Request(10 + k, 0, 1920, 1080, 0.0) for k in range(3)]
    st = srv.run(reqs, clock)
    assert st["requests"] == 13
    for b in range(st["batches"]):
        members = [r for r in srv.finished if r.batch == b]
        assert 1 <= len(members) <= 4
        assert len(members) == 1 or sum(r.px for r in members) <= 2_500_000


def test_idle_slots_of_other_resolutions_are_released():
    fp = S.MockExecutor(S.SimClock()).footprint
    srv, ex, clock = _server(fp((3840, 2160)), max_inflight=1)
    reqs = [S.Request(k, 0, *RES[k % 4], arrival=0.01 * k) for k in range(12)]
    st = srv.run(reqs, clock)
    assert st["requests"] == 12
    assert ex.live_slots <= 4 and srv.pool.reserved <= fp((3840, 2160))


def test_warm_up_then_reset_keeps_slots_and_drops_stats():
    """An untimed warm-up pass leaves idle slots that the timed requests reuse;
    reset_stats makes the statistics cover the timed requests only."""
    srv, ex, clock = _server(1 << 40, s_per_px=2e-10)
    warm = [S.Request(-1 - i, i, *RES[i % 4], arrival=0.0) for i in range(8)]
    srv.run(warm, clock)
    allocs = srv.pool.allocs
    assert allocs > 0
    srv.reset_stats()
    assert srv.stats()["requests"] == 0
    reqs = [S.Request(k, k % 32, *RES[k % 4], arrival=1.0 + 0.01 * k) for k in range(12)]
    st = srv.run(reqs, clock)
    assert st["requests"] == 12 and st["batches"] == 12
    assert sorted(r.rid for r in srv.finished) == list(range(12))
    assert srv.pool.allocs == allocs  # every timed request found an idle slot of its size
