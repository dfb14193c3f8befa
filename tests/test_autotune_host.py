"""Autotuner bookkeeping on the host (timings replaced by a stand-in): the
choice rule with its margin, and the cache round trip through the JSON file."""

import importlib

import pytest


@pytest.fixture
def tuner(lib, tmp_path, monkeypatch):
    from paper_2202_11945_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    monkeypatch.setattr(autotune, "signature", lambda ctxs, iters: "dev|iters%d|shape" % iters)
    monkeypatch.setattr(autotune, "admissible", lambda ctxs, candidates=autotune.CANDIDATES: [32, 64, 128])
    return autotune


def fake_times(table):
    calls = []

    def time_plan(ctxs, iters, tuning, steps=10, warmup=3):
        calls.append((tuning["dwt_resident"], tuning["pt_rows"]))
        return table[(tuning["dwt_resident"], tuning["pt_rows"])]
    return time_plan, calls


def test_clear_winner_is_taken_and_cached(tuner, monkeypatch):
    table = {(r, p): 1000.0 for r in (32, 64, 128) for p in (4, 8)}
    table[(64, 4)] = 900.0
    tp, calls = fake_times(table)
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None], 4)
    assert (rec["dwt_resident"], rec["pt_rows"], rec["cached"]) == (64, 4, False)
    assert len(calls) == 6
    # a fresh module state reads the same file: no timing at all
    calls.clear()
    again = tuner.tune([None], 4)
    assert again["cached"] and (again["dwt_resident"], again["pt_rows"]) == (64, 4) and not calls


def test_near_tie_keeps_the_default(tuner, monkeypatch):
    table = {(r, p): 1000.0 for r in (32, 64, 128) for p in (4, 8)}
    table[(64, 4)] = 995.0  # 0.5 % faster: within the margin
    tp, _ = fake_times(table)
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None], 4, use_cache=False)
    assert (rec["dwt_resident"], rec["pt_rows"]) == (128, 4)
