"""The batched launch's autotuner on the CPU: its candidate grids, the
refinement round over the candidates close to the fastest, the near-tie rule
and the cache, with a stand-in batch object and simulated replay times (the
tuner's only GPU calls, the HIP-event timing and the device key, are
replaced)."""

import numpy as np
import pytest

from paper_1610_04124_amd import autotune


class FakeHandle:
    s, D = 5, 128


class FakeBatch:
    """Records the configuration set before each capture; `gmax[waves]` is
    the resident maximum for each waves-per-column setting."""

    def __init__(self, gmax, ntasks):
        self.gmax, self.ntasks = gmax, ntasks
        self.w, self.c, self.g = 1, 1, 0
        self.captured = None
        self.captures = 0

    def set_waves(self, w):
        self.w = w

    def set_columns(self, c):
        self.c = c

    def set_workgroups(self, g):
        self.g = g

    def waves(self):
        return self.w

    def columns(self):
        return self.c if self.w == 1 else 1

    def info(self):
        return (self.g or self.gmax[self.w]), self.ntasks

    def capture(self, items, stream):
        self.captured = (self.columns(), self.w, self.g or self.gmax[self.w])
        self.captures += 1

    def replay(self, stream):
        pass


def items():
    return [(FakeHandle(), np.zeros((440, 1024), np.float32), None)]


@pytest.fixture
def timed(monkeypatch):
    """Replaces the timing: `first` gives the milliseconds of the first timing
    of each configuration, `later` those of every later one (the refinement)."""
    state = {"first": {}, "later": {}, "seen": set(), "calls": []}

    def fake_time_all(run, stream, replays):
        b = run.__closure__[0].cell_contents          # the lambda's batch
        key = b.captured
        state["calls"].append(key)
        table = state["later"] if key in state["seen"] else state["first"]
        state["seen"].add(key)
        return [table.get(key, 10.0)] * replays

    monkeypatch.setattr(autotune, "_time_all", fake_time_all)
    monkeypatch.setattr(autotune, "device_key", lambda: "fake-device")
    return state


def test_candidates_cover_fractions_and_whole_rounds():
    c = autotune.candidates(4096, 13056)
    assert 4096 in c and 2048 in c and 3584 in c
    assert 3264 in c                       # 13056 tasks in 4 whole rounds
    assert all(g <= 4096 for g in c) and c == sorted(c)
    assert autotune.candidates(10, 3) == sorted(set(autotune.candidates(10, 3)))


def test_refinement_overturns_a_noisy_first_sweep(timed):
    b = FakeBatch({1: 4096, 2: 2048, 4: 1024}, 13056)
    # first sweep: 3264 looks fastest; 4096 is 0.3 % slower (inside 1.5 %)
    timed["first"] = {(1, 1, 3264): 1.383, (1, 1, 4096): 1.387}
    # timed again, 4096 is the faster by 1 %
    timed["later"] = {(1, 1, 3264): 1.400, (1, 1, 4096): 1.386}
    rec = autotune.tune(b, items(), None, replays=3, cache_path=None, waves=(1,))
    assert (rec["waves"], rec["workgroups"]) == (1, 4096)
    assert b.captured == (1, 1, 4096)
    assert set(rec["refined"]) == {"w1/g3264", "w1/g4096"}
    assert rec["tried"]["w1/g3264"] == pytest.approx(1.383)
    # only the two close candidates were timed again, three blocks each
    again = [k for k in timed["calls"][len(rec["tried"]):]]
    assert sorted(set(again)) == [(1, 1, 3264), (1, 1, 4096)] and len(again) == 6


def test_near_ties_go_to_fewer_waves_and_workgroups(timed):
    b = FakeBatch({1: 4096, 2: 2048, 4: 1024}, 13056)
    timed["first"] = {(1, 1, 3584): 1.000, (1, 1, 4096): 0.999, (1, 2, 2048): 1.001}
    timed["later"] = {(1, 1, 3584): 1.0010, (1, 1, 4096): 0.9990, (1, 2, 2048): 1.0000}
    rec = autotune.tune(b, items(), None, replays=3, cache_path=None, waves=(1, 2))
    # all three within 0.25 % of the fastest after the refinement: one wave
    # per column first, then the fewest workgroups
    assert (rec["columns"], rec["waves"], rec["workgroups"]) == (1, 1, 3584)


def test_a_clear_winner_is_not_timed_again(timed):
    b = FakeBatch({1: 4096}, 13056)
    timed["first"] = {(1, 1, 4096): 1.0}
    rec = autotune.tune(b, items(), None, replays=3, cache_path=None, waves=(1,))
    assert rec["workgroups"] == 4096
    assert len(timed["calls"]) == len(rec["tried"])   # no second round


def test_cache_applies_the_stored_choice_without_timing(timed, tmp_path):
    path = str(tmp_path / "tune.json")
    b = FakeBatch({1: 4096}, 13056)
    timed["first"] = {(1, 1, 3072): 0.9}
    rec = autotune.tune(b, items(), None, replays=3, cache_path=path, waves=(1,))
    assert rec["workgroups"] == 3072 and not rec["cached"]
    n = len(timed["calls"])
    b2 = FakeBatch({1: 4096}, 13056)
    rec2 = autotune.tune(b2, items(), None, replays=3, cache_path=path, waves=(1,))
    assert rec2["cached"] and rec2["workgroups"] == 3072
    assert b2.captured == (1, 1, 3072) and len(timed["calls"]) == n
