"""Launch-shape tuning: every admissible resident transform side gives the
oracle's frames (the tolerances of the parity suite), on single contexts
and on a mixed batch, and the autotuner picks an admissible side and caches
it."""

import numpy as np
import pytest

from oracle.operators import System
from oracle.solver import State, frame
from synthetic import get_config, random_vector
from synthetic.configs import batch_mix
from test_gpu_configs import check_frames
from parity import check_blocks
from test_gpu_parity import FRAME_ETOL, LAYER_TOL, OP_TOL, synth_slopes, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,res", [("small", 32), ("mid", 32), ("maory_like", 32), ("maory_like", 64),
                                      ("small", {"pt_rows": 8}), ("maory_like", {"dwt_resident": 64, "pt_rows": 8}),
                                      ("small_fit", {"pt_rows": 8}), ("maory_like", {"res_split": 1}),
                                      ("small", {"res_split": 1}), ("maory_like", {"dwt_resident": 64, "res_split": 4}),
                                      ("mid", {"dwt_resident": 32, "res_split": 4}),
                                      ("maory_like", {"pt_split": 1}), ("small_fit", {"pt_split": 1}),
                                      ("mid", {"dwt_resident": 32, "pt_split": 1}),
                                      ("paper_maory", {"pt_split": 1}),
                                      ("maory_like", {"dwt_resident": 64, "glob_fuse": 1}),
                                      ("maory_like", {"dwt_resident": 32, "glob_fuse": 1, "pt_split": 1}),
                                      ("mid", {"dwt_resident": 32, "glob_fuse": 1}),
                                      ("paper_maory", {"dwt_resident": 32, "glob_fuse": 1}),
                                      ("maory_like", {"dwt_resident": 64, "glob_fuse": 1, "res_split": 4})])
def test_frame_parity_with_resident_side(gpu_lib, systems, name, res):
    import torch
    S = systems(name)
    print("\n[gpu-tune]", name, "resident", res, flush=True)
    ctx = gpu_lib.Context(get_config(name), device=0, tuning=res)
    x = random_vector(S.geom.n_coeff, 300, len(str(res)))
    check_blocks(to_host(ctx.apply_M(to_dev(x))), S.apply_M(x), S.geom.layer_off, OP_TOL, "M x layer")
    st = torch.zeros(ctx.n_state, device="cuda")
    lay = torch.empty(ctx.n_coeff, device="cuda")
    s = synth_slopes(S, 0)
    ctx.reconstruct(to_dev(s), st, lay, iters=S.cfg["iters"])
    _, ref = frame(S, State(S.geom.n_coeff, S.geom.n_coeff), s.astype(np.float64))
    check_blocks(to_host(lay), ref, S.geom.layer_off, LAYER_TOL, "layers", FRAME_ETOL)
    ctx.close()


@pytest.mark.parametrize("tuning", [32, {"dwt_resident": 64, "pt_split": 1}, {"dwt_resident": 32, "glob_fuse": 1}])
def test_tuned_mixed_batch(gpu_lib, tuning):
    import torch
    cfgs = batch_mix(1, 1, 4)
    systems = [System(c) for c in cfgs]
    ctxs = [gpu_lib.Context(c, device=0) for c in cfgs]
    print("\n[gpu-tune] mixed batch, tuning", tuning, flush=True)
    batch = gpu_lib.Batch(ctxs, tuning=tuning)
    slopes = [to_dev(synth_slopes(S, k)) for k, S in enumerate(systems)]
    states = [torch.zeros(c.n_state, device="cuda") for c in ctxs]
    lays = [torch.empty(c.n_coeff, device="cuda") for c in ctxs]
    # frame 1 from the zero state, frame 2 warm-started from the GPU's own state;
    # each compared with the oracle's frame from the same (FP32) state
    def run():
        batch.reconstruct(slopes, states, lays, iters=6, use_graph=True)

    check_frames(systems, slopes, states, lays, run)
    check_frames(systems, slopes, states, lays, run)
    batch.close()


@pytest.mark.parametrize("use_graph", [True, False])
def test_streams_split_matches_one_stream_bitwise(gpu_lib, use_graph):
    # uneven batch (2 MAORY-like + 3 VLT-like) in 2 and 4 parts against one
    # part: every frame's state and layers bitwise equal; a copy queued on the
    # caller's stream right after the call sees the finished frame (join)
    import torch
    cfgs = batch_mix(2, 3, 9)
    systems = [System(c) for c in cfgs]
    ctxs = [gpu_lib.Context(c, device=0) for c in cfgs]
    slopes = [to_dev(synth_slopes(S, k)) for k, S in enumerate(systems)]
    one = gpu_lib.Batch(ctxs)
    for streams in (2, 4):
        print("\n[gpu-tune] streams", streams, "graph", use_graph, flush=True)
        split = gpu_lib.Batch(ctxs, tuning={"streams": streams})
        st1 = [torch.zeros(c.n_state, device="cuda") for c in ctxs]
        st2 = [torch.zeros(c.n_state, device="cuda") for c in ctxs]
        l1 = [torch.empty(c.n_coeff, device="cuda") for c in ctxs]
        l2 = [torch.full((c.n_coeff,), float("nan"), device="cuda") for c in ctxs]
        for f in range(3):
            one.reconstruct(slopes, st1, l1, iters=6, use_graph=use_graph)
            split.reconstruct(slopes, st2, l2, iters=6, use_graph=use_graph)
            snap = [t.clone() for t in l2]
            torch.cuda.synchronize()
            for k in range(len(ctxs)):
                assert torch.equal(st1[k], st2[k]), (streams, f, k)
                assert torch.equal(l1[k], l2[k]), (streams, f, k)
                assert torch.equal(snap[k], l1[k]), (streams, f, k)
        split.close()
    one.close()


def test_resident_side_below_coarse_block_is_rejected(gpu_lib):
    cfg = get_config("tiny")
    for l in cfg["layers"]:
        l["n"], l["levels"] = 128, 1  # coarsest block 64 x 64
    cfg["domain_side"] = 64.0
    ctx = gpu_lib.Context(cfg, device=0)
    with pytest.raises(gpu_lib.FewhaError) as e:
        gpu_lib.Batch([ctx], tuning=32)
    assert e.value.status == -1
    ctx.close()


def test_autotuner_picks_admissible_side_and_caches(gpu_lib, tmp_path, monkeypatch):
    from paper_2202_11945_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    ctx = gpu_lib.Context(get_config("small"), device=0)
    print("\n[gpu-tune] autotuner on 4 small problems", flush=True)
    rec = autotune.tune([ctx] * 4, 4, steps=3)
    assert rec["dwt_resident"] in autotune.admissible([ctx]) and not rec["cached"]
    assert set(rec["us"]) == {"%d/%d" % (r, p) for r in autotune.admissible([ctx]) for p in autotune.PT_ROWS}
    assert rec["pt_rows"] in autotune.PT_ROWS
    again = autotune.tune([ctx] * 4, 4, steps=3)
    assert again["cached"] and again["dwt_resident"] == rec["dwt_resident"]
