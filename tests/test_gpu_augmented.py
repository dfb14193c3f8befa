"""GPU parity of the augmented PCG (Sec. 3.3; Algorithm 1's augPCG line)
against the oracle: a frame that reuses the previous frame's search
directions, from the GPU's own state, including the directions the frame
hands on; and a batch mixing augmented and plain problems against single
contexts, bitwise."""

import numpy as np
import pytest

from oracle.operators import System
from oracle.solver import State, frame
from parity import check_blocks
from synthetic import get_config
from test_gpu_parity import FRAME_ETOL, LAYER_TOL, OP_TOL, synth_slopes, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,keep,iters,tuning", [("small", 2, 2, None), ("small", 4, 4, None),
                                                    ("maory_like", 4, 4, None),
                                                    ("maory_like", 2, 2, {"dwt_resident": 64, "pt_split": 1,
                                                                          "glob_fuse": 1})])
def test_augmented_frames(gpu_lib, name, keep, iters, tuning):
    # the last case in the single-frame launch shapes (fused global levels,
    # split propagation-adjoint tiles), whose transform kernels form the
    # augmented directions' inverse transforms too
    import torch
    print("\n[gpu-aug]", name, keep, iters, tuning, flush=True)
    cfg = get_config(name, augment=keep, iters=iters)
    S = System(cfg)
    ctx = gpu_lib.Context(cfg, device=0, tuning=tuning)
    n = S.geom.n_coeff
    assert ctx.n_state == 5 * n + 2 * keep * n + 4
    st = torch.zeros(ctx.n_state, device="cuda")
    lay = torch.empty(n, device="cuda")
    for k in range(3):  # frame 0 has no directions (plain PCG); 1 and 2 reuse them
        before = to_host(st)
        s = synth_slopes(S, k)
        ctx.reconstruct(to_dev(s), st, lay, iters=iters)
        got = State.unpack(to_host(st), n, n, keep)
        ref_st, ref_phi = frame(S, State.unpack(before, n, n, keep), s.astype(np.float64), iters=iters)
        o = S.geom.layer_off
        tag = "frame %d" % k
        check_blocks(to_host(lay), ref_phi, o, LAYER_TOL, tag + " layers", FRAME_ETOL)
        check_blocks(got.c, ref_st.c, o, LAYER_TOL, tag + " c", FRAME_ETOL)
        check_blocks(got.r, ref_st.r, o, LAYER_TOL, tag + " r", FRAME_ETOL, scale=ref_st.b)
        assert len(got.P) == len(ref_st.P) == min(keep, iters)
        for j, (gp, rp, gq, rq) in enumerate(zip(got.P, ref_st.P, got.Q, ref_st.Q)):
            check_blocks(gp, rp, o, LAYER_TOL, tag + " P_%d" % j, FRAME_ETOL)
            check_blocks(gq, rq, o, LAYER_TOL, tag + " Q_%d" % j, FRAME_ETOL)
    ctx.close()


def test_augmented_and_plain_in_one_batch(gpu_lib):
    import torch
    cfgs = [get_config("small", augment=2, iters=4), get_config("mid"), get_config("mid", augment=4, iters=4)]
    systems = [System(c) for c in cfgs]
    ctxs = [gpu_lib.Context(c, device=0) for c in cfgs]
    singles = [torch.zeros(c.n_state, device="cuda") for c in ctxs]
    bst = [torch.zeros(c.n_state, device="cuda") for c in ctxs]
    batch = gpu_lib.Batch(ctxs)
    for f in range(3):
        slopes = [to_dev(synth_slopes(S, f + 7 * k)) for k, S in enumerate(systems)]
        for c, sl, st in zip(ctxs, slopes, singles):
            c.reconstruct(sl, st, iters=4)
        batch.reconstruct(slopes, bst, iters=4, use_graph=True)
        torch.cuda.synchronize()
        for k in range(3):
            assert torch.equal(singles[k], bst[k]), (f, k)
    batch.close()
    for c in ctxs:
        c.close()
