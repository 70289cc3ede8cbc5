"""The schedule autotuner's search and cache as host logic on the CPU: a
stand-in batch whose render time is a known function of the schedule."""
import json
import types

import pytest

from paper_2012_03325_amd import autotune as A
from paper_2012_03325_amd import epb as E


class _FakeBatch:
    """Views of a few sizes; ``build`` records the schedule; the 'time' of a
    schedule is a separable bowl with its minimum at ``best`` plus ``extra``."""

    def __init__(self, best, extra=None, sizes=((64, 48), (640, 480)), invalid=(), gives_up=()):
        self.dviews = [types.SimpleNamespace(W=w, H=h, gdtype=0, ao_dtype=0, hdr_dtype=0,
                                             ssao_params=types.SimpleNamespace(n_samples=16, blur=1), lights=[1])
                       for w, h in sizes]
        self.schedule = E.epb_schedule(0, 0, 0, 0)
        self.best = best
        self.extra = extra or {}
        self.invalid, self.gives_up = set(invalid), set(gives_up)
        self.builds = 0

    def _key(self, s):
        d = A._as_dict(s)
        return tuple(d[k] for k in A.ORDER)

    def build(self, s):
        if self._key(s) in self.invalid:
            raise E.EpbError("epb_batch_build", E.EPB_ERR_DTYPE)
        self.schedule = s
        self.builds += 1

    def status(self):
        return E.EPB_ERR_TIMEOUT if self._key(self.schedule) in self.gives_up else E.EPB_OK

    def time(self, batch, reps):
        d = A._as_dict(self.schedule)
        t = 10.0 + sum((A.SPACE[k].index(d[k]) - A.SPACE[k].index(self.best[k])) ** 2 for k in A.ORDER)
        return t + self.extra.get(tuple(d[k] for k in A.ORDER), 0.0)


def test_coordinate_descent_finds_the_separable_minimum_and_leaves_it_built():
    A._cache.clear()
    best = dict(blocks_per_cu=4, shade_tile=2, ssao_tile=1, ssao_batch=1, persistent=16, fuse_bloom=1)
    b = _FakeBatch(best)
    sched, trace = A.tune(b, reps=1, passes=2, use_cache=False, timer=b.time, device="test")
    assert A._as_dict(sched) == best
    assert A._as_dict(b.schedule) == best  # the batch is left built with the pick
    # no schedule is timed twice, and the search stays far below the full grid (5*3*3*2*5*2 = 900)
    keys = [tuple(t["schedule"][k] for k in A.ORDER) for t in trace]
    assert len(keys) == len(set(keys)) and len(keys) < 30


def test_schedules_a_batch_cannot_take_or_that_give_up_are_skipped():
    """A schedule the batch rejects (persistent with mixed storage) or whose
    persistent render reports a wait that gave up is never picked."""
    A._cache.clear()
    best = dict(blocks_per_cu=0, shade_tile=0, ssao_tile=0, ssao_batch=0, persistent=64, fuse_bloom=0)
    b = _FakeBatch(best, invalid={(0, 0, 0, 0, 64, 0)}, gives_up={(0, 0, 0, 0, 16, 0)})
    sched, trace = A.tune(b, reps=1, passes=2, use_cache=False, timer=b.time, device="test")
    assert A._as_dict(sched)["persistent"] not in (16, 64)
    assert all(t["ms"] is None and t["rejected"] for t in trace if t["schedule"]["persistent"] in (16, 64))


def test_second_pass_escapes_a_coupled_valley():
    """A slower cell on the first pass's path is avoided by the second pass."""
    A._cache.clear()
    best = dict(blocks_per_cu=0, shade_tile=1, ssao_tile=1, ssao_batch=0, persistent=0, fuse_bloom=0)
    b = _FakeBatch(best, extra={(0, 1, 0, 0, 0, 0): 5.0})  # stepping to shade_tile 1 alone looks worse
    s1, _ = A.tune(b, reps=1, passes=1, use_cache=False, timer=b.time, device="test")
    s2, _ = A.tune(b, reps=1, passes=3, use_cache=False, timer=b.time, device="test")
    assert A._as_dict(s1) != best  # one pass stops short
    assert A._as_dict(s2) == best
    assert b.time(b, 1) <= 10.0 + 1e-12


def test_cache_hit_skips_timing_and_survives_a_restart(tmp_path):
    A._cache.clear()
    path = str(tmp_path / "sched.json")
    best = dict(blocks_per_cu=2, shade_tile=0, ssao_tile=1, ssao_batch=0, persistent=256, fuse_bloom=1)
    b = _FakeBatch(best)
    A.tune(b, reps=1, use_cache=True, cache_path=path, timer=b.time, device="test")
    saved = json.load(open(path))
    assert list(saved.values()) == [best]
    A._cache.clear()  # a new process: the file repopulates the table
    c = _FakeBatch(best)

    def never(batch, reps):
        raise AssertionError("timed despite a cached schedule")

    sched, trace = A.tune(c, reps=1, use_cache=True, cache_path=path, timer=never, device="test")
    assert A._as_dict(sched) == best and trace[0]["cached"] and c.builds == 1
    # another device or another mix of view sizes is another entry
    d = _FakeBatch(best, sizes=((64, 48),))
    with pytest.raises(AssertionError):
        A.tune(d, reps=1, use_cache=True, cache_path=path, timer=never, device="test")
