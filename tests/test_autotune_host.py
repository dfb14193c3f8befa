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
    monkeypatch.setattr(autotune, "split_allowed", lambda ctxs, res: False)
    monkeypatch.setattr(autotune, "fusable", lambda ctxs, res: False)
    return autotune


def fake_times(table, streams=None, quarters=None, pt_split=None, fuse=None):
    """Stand-in timer: table[(R, rows)] for one stream, streams[s] for s > 1,
    quarters for the resident inverse levels in four workgroups per layer,
    pt_split for the propagation adjoint's split sensor lists (default: the
    same as unsplit)."""
    calls = []

    def time_plan(ctxs, iters, tuning, steps=10, warmup=3):
        ns = tuning.get("streams", 1)
        calls.append((tuning["dwt_resident"], tuning["pt_rows"], ns))
        if ns > 1:
            return streams[ns]
        if tuning.get("res_split", 0) == 4:
            return quarters
        if tuning.get("glob_fuse", 0) == 1 and fuse is not None:
            return fuse[tuning["dwt_resident"]]
        if tuning.get("pt_split", 0) == 1 and pt_split is not None:
            return pt_split
        return table[(tuning["dwt_resident"], tuning["pt_rows"])]
    return time_plan, calls


def test_clear_winner_is_taken_and_cached(tuner, monkeypatch):
    table = {(r, p): 1000.0 for r in (32, 64, 128) for p in (4, 8)}
    table[(64, 4)] = 900.0
    tp, calls = fake_times(table)
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None], 4)
    assert (rec["dwt_resident"], rec["pt_rows"], rec["cached"]) == (64, 4, False)
    assert len(calls) == 7 and rec["pt_split"] == 0
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


def test_streams_are_tuned_after_the_shapes(tuner, monkeypatch):
    table = {(r, p): 1000.0 for r in (32, 64, 128) for p in (4, 8)}
    # a clear gain from two streams is taken, for the best shapes only
    tp, calls = fake_times(table, {2: 900.0})
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None, None], 4, use_cache=False)
    assert (rec["dwt_resident"], rec["pt_rows"], rec["streams"]) == (128, 4, 2)
    assert calls[-1] == (128, 4, 2) and len(calls) == 8
    assert rec["streams_us"] == {"1": 1000.0, "2": 900.0}
    # a near tie keeps one stream; a single problem is not split at all
    tp, _ = fake_times(table, {2: 995.0})
    monkeypatch.setattr(tuner, "time_plan", tp)
    assert tuner.tune([None, None], 4, use_cache=False)["streams"] == 1
    tp, calls = fake_times(table)
    monkeypatch.setattr(tuner, "time_plan", tp)
    assert tuner.tune([None], 4, use_cache=False)["streams"] == 1 and len(calls) == 7


def test_cache_key_follows_geometry_and_sources(lib, monkeypatch):
    # a cached choice must not survive a change of sensor geometry (which
    # sets the propagation adjoint's paths) or of the kernel sources
    from types import SimpleNamespace
    from paper_2202_11945_amd import autotune
    from synthetic import get_config

    def key(cfg):
        return autotune.signature([SimpleNamespace(cfg=cfg, device=0)], 4, device_name="dev")

    base = key(get_config("small"))
    assert base == key(get_config("small"))
    moved = get_config("small")
    moved["wfs"][0]["theta"] = (moved["wfs"][0]["theta"][0] + 1e-6, moved["wfs"][0]["theta"][1])
    higher = get_config("small")
    higher["layers"][1]["h"] += 100.0
    assert len({base, key(moved), key(higher)}) == 3
    monkeypatch.setattr(autotune, "source_hash", lambda: "0" * 16)
    assert key(get_config("small")) != base


def test_resident_split_is_tuned_for_the_best_shape(tuner, monkeypatch):
    # one workgroup per layer is the default; four are kept only when
    # clearly faster, and the streams are then timed with that choice
    monkeypatch.setattr(tuner, "split_allowed", lambda ctxs, res: True)
    table = {(r, p): 1000.0 for r in (32, 64, 128) for p in (4, 8)}
    tp, calls = fake_times(table, {2: 2000.0}, quarters=900.0)
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None, None], 4, use_cache=False)
    assert rec["res_split"] == 4 and rec["split_us"] == {"0": 1000.0, "4": 900.0} and rec["streams"] == 1
    tp, _ = fake_times(table, {2: 2000.0}, quarters=995.0)
    monkeypatch.setattr(tuner, "time_plan", tp)
    assert tuner.tune([None, None], 4, use_cache=False)["res_split"] == 0


def test_split_sensor_lists_are_tuned_for_the_best_shape(tuner, monkeypatch):
    # split propagation-adjoint tiles (4 rows per thread) are kept only when
    # clearly faster than the best unsplit shape; the streams then use them
    table = {(r, p): 1000.0 for r in (32, 64, 128) for p in (4, 8)}
    table[(64, 8)] = 950.0
    tp, calls = fake_times(table, {2: 2000.0}, pt_split=900.0)
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None, None], 4, use_cache=False)
    assert (rec["dwt_resident"], rec["pt_rows"], rec["pt_split"]) == (64, 4, 1)
    assert rec["pt_split_us"] == {"0": 950.0, "1": 900.0} and calls[6] == (64, 4, 1)
    tp, _ = fake_times(table, {2: 2000.0}, pt_split=940.0)  # 1 % faster: within the margin
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None, None], 4, use_cache=False)
    assert (rec["dwt_resident"], rec["pt_rows"], rec["pt_split"]) == (64, 8, 0)


def test_fused_global_levels_are_tuned_per_resident_side(tuner, monkeypatch):
    # fusion is timed at every resident side where a layer has two or more
    # global levels (here 32 and 64), with the shapes chosen so far, and the
    # fastest is kept when clearly faster
    monkeypatch.setattr(tuner, "fusable", lambda ctxs, res: res < 128)
    table = {(r, p): 1000.0 for r in (32, 64, 128) for p in (4, 8)}
    tp, calls = fake_times(table, {2: 2000.0}, fuse={32: 950.0, 64: 900.0})
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None, None], 4, use_cache=False)
    assert (rec["dwt_resident"], rec["glob_fuse"]) == (64, 1)
    assert rec["glob_fuse_us"] == {"32": 950.0, "64": 900.0}
    tp, _ = fake_times(table, {2: 2000.0}, fuse={32: 990.0, 64: 995.0})  # within the margin
    monkeypatch.setattr(tuner, "time_plan", tp)
    rec = tuner.tune([None, None], 4, use_cache=False)
    assert (rec["dwt_resident"], rec["glob_fuse"]) == (128, 0)
