"""Host logic of the autotuner's coordinate search (no GPU)."""
import pytest

from paper_2007_15432_amd.autotune import search


def fake_measure(calls):
    def measure(p, k):
        calls.append((dict(p), dict(k)))
        ms = (p["n_group_max"] - 96) ** 2 / 100 + (p["n_leaf_max"] - 16) ** 2 / 10
        ms += {1: 3.0, 2: 2.0, 4: 1.0, 8: 1.5}[k["force_unroll"]] + (0.0 if k["force_split"] else 5.0)
        ms += abs(k.get("waves_per_cu", 32) - 16) / 16 + abs(k["walk_waves_per_cu"] - 4) / 8
        return ms, 1000
    return measure


def test_search_finds_the_coordinate_minimum():
    calls = []
    r = search(fake_measure(calls))
    assert r.params == dict(n_group_max=96, n_leaf_max=16)
    assert r.kernel["force_unroll"] == 4 and r.kernel["force_split"] == 1 and r.kernel["waves_per_cu"] == 16
    assert r.kernel["walk_waves_per_cu"] == 4
    assert r.ms == min(t.ms for t in r.trials)
    assert {t.stage for t in r.trials} == {1, 2, 3}
    assert len(calls) == len(r.trials)


def test_search_respects_group_cap():
    calls = []
    r = search(fake_measure(calls), group_cap=64)
    assert all(p["n_group_max"] <= 64 for p, _ in calls)
    assert r.params["n_group_max"] == 64


def test_search_rejects_empty_space():
    with pytest.raises(ValueError):
        search(fake_measure([]), group_cap=32)


def test_stage_two_keeps_stage_one_winner_if_better():
    # every launch shape slower than the default: the stage-1 trial wins
    def measure(p, k):
        base = 1.0 if (k["force_unroll"] == 4 and k.get("waves_per_cu") == 32 and k["force_split"] == 1) else 2.0
        return base + (0 if p["n_group_max"] == 128 else 1), 10
    r = search(measure)
    assert r.kernel["force_unroll"] == 4 and r.kernel["waves_per_cu"] == 32 and r.params["n_group_max"] == 128
