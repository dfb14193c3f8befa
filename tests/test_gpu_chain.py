"""Long frame sequences on the GPU: the true-residual restart against the
oracle, checkpoint and resume (500 + 500 frames in two contexts equal 1000
frames in one, bitwise), and the drift of a 1000-frame MAORY-like chain
against the oracle's chain, with and without restarts."""

import numpy as np
import pytest

from oracle.operators import System
from oracle.solver import State, frame
from parity import check_blocks
from synthetic import get_config
from test_gpu_parity import FRAME_ETOL, LAYER_TOL, _oracle_state, synth_slopes, to_dev, to_host

pytestmark = pytest.mark.gpu


def _pool(S, n=16, key=11):
    return [synth_slopes(S, k, key) for k in range(n)]


def _tri(i, n):
    k = i % (2 * n - 2)
    return k if k < n else 2 * n - 2 - k


@pytest.mark.parametrize("name", ["small", "maory_like"])
def test_true_residual_restart_frame(gpu_lib, systems, name):
    import torch
    S = systems(name)
    ctx = gpu_lib.Context(get_config(name), device=0)
    ctx.set_refresh(3)
    ctx.set_frame_count(6)  # frame 6: a restart frame
    state = _oracle_state(S, 3)
    s = synth_slopes(S, 3)
    st = to_dev(state)
    lay = torch.empty(S.geom.n_coeff, device="cuda")
    ctx.reconstruct(to_dev(s), st, lay, iters=S.cfg["iters"])
    ref_st, ref_phi = frame(S, State.unpack(state, S.geom.n_coeff, S.geom.n_coeff), s.astype(np.float64),
                            refresh=True)
    o = S.geom.layer_off
    check_blocks(to_host(lay), ref_phi, o, LAYER_TOL, "layers", FRAME_ETOL)
    g = State.unpack(to_host(st), S.geom.n_coeff, S.geom.n_coeff)
    check_blocks(g.c, ref_st.c, o, LAYER_TOL, "c", FRAME_ETOL)
    check_blocks(g.r, ref_st.r, o, LAYER_TOL, "r", FRAME_ETOL, scale=ref_st.b)
    ctx.close()


@pytest.mark.parametrize("name,extra", [("maory_like", {}), ("small", {"augment": 2, "loop": "closed", "gain": 0.5})])
def test_checkpoint_and_resume_bitwise(gpu_lib, systems, name, extra):
    # the state is the whole of a sequence's memory: saved to the host after
    # 500 frames and restored into a new context (with the frame count, which
    # sets the restart schedule), 500 more frames equal 1000 in one context
    import torch
    cfg = get_config(name, **extra)
    pool = [to_dev(s) for s in _pool(systems(name))]

    def run(ctx, st, lay, first, n):
        for i in range(first, first + n):
            ctx.reconstruct(pool[_tri(i, len(pool))], st, lay)

    a = gpu_lib.Context(cfg, device=0)
    a.set_refresh(100)
    st_a = torch.zeros(a.n_state, device="cuda")
    lay_a = torch.empty(a.n_coeff, device="cuda")
    run(a, st_a, lay_a, 0, 1000)
    b = gpu_lib.Context(cfg, device=0)
    b.set_refresh(100)
    st_b = torch.zeros(b.n_state, device="cuda")
    lay_b = torch.empty(b.n_coeff, device="cuda")
    run(b, st_b, lay_b, 0, 500)
    saved = st_b.cpu()
    b.close()
    c = gpu_lib.Context(cfg, device=0)
    c.set_refresh(100)
    c.set_frame_count(500)
    st_c = saved.cuda()
    run(c, st_c, lay_b, 500, 500)
    torch.cuda.synchronize()
    assert torch.equal(st_a, st_c) and torch.equal(lay_a, lay_b)
    a.close()
    c.close()


@pytest.mark.slow
def test_chained_drift_over_1000_frames(gpu_lib, systems):
    # A17: the FP32 GPU chain and the FP64 oracle chain from the same zero
    # state on the same 1000 frames (a 16-frame frozen-flow pool walked
    # forward and back); each GPU frame takes the GPU's own state.  Reported
    # per 100 frames, without restarts and with a true-residual restart every
    # 100 frames.
    import torch
    S = systems("maory_like")
    n = S.geom.n_coeff
    pool = _pool(S)
    dev = [to_dev(s) for s in pool]
    ctxs = {}
    for name, every in (("recurrence", 0), ("restart_100", 100)):
        c = gpu_lib.Context(get_config("maory_like"), device=0)
        c.set_refresh(every)
        ctxs[name] = (c, torch.zeros(c.n_state, device="cuda"), torch.empty(n, device="cuda"))
    st = State(n, n)
    worst = {k: 0.0 for k in ctxs}
    report = {k: [] for k in ctxs}
    o = S.geom.layer_off
    for i in range(1000):
        s = pool[_tri(i, len(pool))]
        st, phi = frame(S, st, s.astype(np.float64))
        for name, (c, sd, lay) in ctxs.items():
            c.reconstruct(dev[_tri(i, len(pool))], sd, lay)
        if i % 10 == 9:
            for name, (c, sd, lay) in ctxs.items():
                got = to_host(lay)
                e = max(np.linalg.norm(got[o[l]:o[l + 1]] - phi[o[l]:o[l + 1]]) /
                        np.linalg.norm(phi[o[l]:o[l + 1]]) for l in range(S.Lc))
                worst[name] = max(worst[name], e)
                if i % 100 == 99:
                    report[name].append(e)
    print("\n[gpu-chain] layer drift against the oracle chain every 100 frames:", report,
          "\n[gpu-chain] worst over 1000 frames:", worst, flush=True)
    # per-frame parity is 1e-4 from an identical state; the chains here carry
    # their own states for 1000 frames.  With Algorithm 1's recurrence the
    # FP32 gap between the carried and the true residual accumulates, and the
    # drift grows about linearly (measured 2.5e-4 after 100 frames, 4.9e-3
    # after 1000); a restart every 100 frames holds it at the 100-frame level
    # (4.6e-4 at worst)
    assert worst["recurrence"] <= 1e-2
    assert worst["restart_100"] <= 1e-3 and worst["restart_100"] < 0.2 * worst["recurrence"]
    for c, _, _ in ctxs.values():
        c.close()
