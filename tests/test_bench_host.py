"""bench.py's host-side contract (no GPU): the multi-GPU refusal, the
algorithmic bytes the roofline divides by, and the rule that a measured
traffic figure is reported only for the kernel sources and launch shapes it
was taken on."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synthetic import get_config  # noqa: E402


def _maory_bytes(res=128):
    cfg = get_config("maory_like")
    n_cor = sum((w["n_subap"] + 1) ** 2 for w in cfg["wfs"])
    return cfg, bench.algorithmic_bytes(cfg, 53736, n_cor, res)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_of_the_maory_like_problem():
    cfg, alg = _maory_bytes()
    assert set(alg) == set(bench.STAGES)
    n_c = sum(l["n"] ** 2 for l in cfg["layers"])
    assert n_c == 98304
    # P_T reads every corner value once and writes every node once (FP32)
    assert alg["P_T"] == 4 * (39393 + n_c) == 550788
    # the update reads p, q, x, r, J^{-1} and writes x, r
    assert alg["UPDATE"] == 4 * 7 * n_c
    # the sensor stages count the active subapertures' slopes (sum 2 |M_g|), not the dense grids
    assert alg["P_GAMMA"] == 4 * (n_c + 53736)
    assert alg["GAMMA_T"] == 4 * (53736 + 39393)
    assert all(v > 0 for v in alg.values())
    # resident side 128: only the 256 x 256 layer's top level is global
    assert alg["IDWT_GLOB"] == 4 * 17 * 128 ** 2 and alg["IDWT_RES"] == 4 * 5 * 3 * 128 ** 2
    # resident side 64: the 128 x 128 layers' top level and two of the 256 layer's go global
    _, alg64 = _maory_bytes(64)
    assert alg64["IDWT_GLOB"] == 4 * 17 * (3 * 64 ** 2 + 128 ** 2)
    assert alg64["FDWT_GLOB"] == 4 * 11 * (3 * 64 ** 2 + 128 ** 2)
    assert alg64["IDWT_RES"] == 4 * 5 * 3 * 64 ** 2


def test_active_slope_count_of_the_maory_like_problem(lib):
    ctx = lib.Context(get_config("maory_like"), device=-1)
    assert ctx.n_slopes == 53736


def test_pool_frames_stay_adjacent_in_time():
    seq = [bench.pool_index(i, 8) for i in range(40)]
    assert seq[:16] == [0, 1, 2, 3, 4, 5, 6, 7, 6, 5, 4, 3, 2, 1, 0, 1]
    assert all(abs(a - b) == 1 for a, b in zip(seq, seq[1:]))
    assert [bench.pool_index(i, 1) for i in range(3)] == [0, 0, 0]


def test_traffic_only_for_matching_sources_and_shapes():
    prof = os.path.join(ROOT, "profiles", "stages_maory_like_b32_bytes.md")
    if not os.path.exists(prof):
        pytest.skip("no committed traffic summary")
    tune = {"dwt_resident": 128, "pt_rows": 4}
    rows = [l.split() for l in open(prof) if l.split()[:1] == ["TRAFFIC"]]
    assert {r[1] for r in rows} == set(bench.STAGES)
    got = bench.measured_traffic("P_T", 32, tune)
    expected = [float(r[3]) for r in rows if r[1] == "P_T" and r[5] == "128/4/0/0/0"]
    # the summary is taken on the committed kernel sources: then it is reported
    assert got is None or [got] == expected
    # other launch shapes or batch sizes never borrow it
    assert bench.measured_traffic("P_T", 32, {"dwt_resident": 64, "pt_rows": 8}) is None
    assert bench.measured_traffic("P_T", 32, dict(tune, pt_split=1)) is None
    assert bench.measured_traffic("P_T", 32, dict(tune, glob_fuse=1)) is None
    assert bench.measured_traffic("P_T", 48, tune) is None


def test_whole_path_bytes_and_launch_count():
    # B_frame = B_rhs + iters (B_apply + B_vec) + B_out for the MAORY-like
    # frame at 4 iterations, the 9-layer frame at 20 and the paper's MAORY at
    # 2 (42.7 MB, 616 MB, 7.8 MB), from the operator counts N_c, sum V, sum S
    assert bench.path_bytes(98304, 39393, 53736, 4) == 4 * (2 * 53736 + 2 * 39393 + 7 * 98304) + 4 * (
        4 * (6 * 98304 + 4 * 39393 + 2 * 53736) + 4 * 15 * 98304) + 4 * 5 * 98304
    assert round(bench.path_bytes(98304, 39393, 53736, 4) / 1e6, 1) == 42.7
    assert round(bench.path_bytes(344064, 39366, 53712, 20) / 1e6) == 616
    assert round(bench.path_bytes(24576, 33777, 46056, 2) / 1e6, 1) == 7.8
    cfg = get_config("maory_like")
    assert bench.corner_count(cfg) == 39393
    # one frame of one MAORY-like problem: 39 launches with resident side 128
    # (the count the single-frame kernel trace shows), 49 with 64
    assert bench.launches_per_frame(cfg, 128, 4) == 39
    assert bench.launches_per_frame(cfg, 64, 4) == 49
    # fused global levels: the 256 x 256 layer's two global levels are one launch
    assert bench.launches_per_frame(cfg, 64, 4, fuse=True) == 39
    assert bench.launches_per_frame(cfg, 32, 4, fuse=True) == 49
