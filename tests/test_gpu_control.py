"""GPU parity of the closed-loop time step (Algorithm 1: pseudo-open-loop
slopes with the two-step delay, closed-loop control) and of photon-count
noise weights against the FP64 oracle, on single contexts and on a batch
that mixes open- and closed-loop problems."""

import numpy as np
import pytest

from oracle.operators import System
from oracle.solver import State, frame
from parity import check_blocks
from synthetic import get_config, random_vector
from test_gpu_parity import FRAME_ETOL, LAYER_TOL, _check_frame, _oracle_state, synth_slopes, to_dev, to_host

pytestmark = pytest.mark.gpu


def _warm_closed_state(S, key):
    """An oracle open-loop chain's state with mirror commands a^(i) and
    a^(i-1) far apart (so that taking the wrong one shows)."""
    st = State.unpack(_oracle_state(S, 2).astype(np.float64), S.geom.n_coeff, S.geom.n_coeff)
    st.a_prev = st.a * 0.7 + random_vector(S.geom.n_coeff, 60, key).astype(np.float64) * 0.05
    st.a = -0.5 * st.a
    return st.pack().astype(np.float32)


@pytest.mark.parametrize("name", ["small", "maory_like"])
def test_closed_loop_frame(gpu_lib, name):
    print("\n[gpu-control] closed loop", name, flush=True)
    cfg = get_config(name, loop="closed", gain=0.6)
    S = System(cfg)
    ctx = gpu_lib.Context(cfg, device=0)
    state = _warm_closed_state(S, 1)
    # closed-loop measurement: the atmosphere's slopes minus the mirrors' of two frames back
    n = S.geom.n_coeff
    s_cl = synth_slopes(S, 3).astype(np.float64) - S.apply_A(state[3 * n:4 * n].astype(np.float64))
    _check_frame(gpu_lib, S, ctx, state, s_cl.astype(np.float32))
    ctx.close()


def test_photon_count_frame(gpu_lib):
    cfg = get_config("small")
    for w in cfg["wfs"]:
        w["photons"] = 500.0 if w["kind"] == "lgs" else 10000.0
        w["sigma"] = w["photons"] ** -0.5  # the slope noise the synthetic data draw
    S = System(cfg)
    ctx = gpu_lib.Context(cfg, device=0)
    _check_frame(gpu_lib, S, ctx, _oracle_state(S, 2), synth_slopes(S, 2))
    ctx.close()


def test_batch_mixing_open_and_closed_loops(gpu_lib):
    # one graph over open- and closed-loop problems: each problem's frame is
    # bitwise its single context's, and matches the oracle
    import torch
    cfgs = [get_config("small", loop="closed", gain=0.5), get_config("mid"),
            get_config("small"), get_config("mid", loop="closed", gain=0.8)]
    systems = [System(c) for c in cfgs]
    ctxs = [gpu_lib.Context(c, device=0) for c in cfgs]
    states, slopes = [], []
    for k, S in enumerate(systems):
        st = _warm_closed_state(S, 10 + k)
        states.append(to_dev(st))
        slopes.append(to_dev(synth_slopes(S, 5 + k)))
    singles = [s.clone() for s in states]
    lay_s = [torch.empty(c.n_coeff, device="cuda") for c in ctxs]
    for c, sl, st, ly in zip(ctxs, slopes, singles, lay_s):
        c.reconstruct(sl, st, ly, iters=4)
    batch = gpu_lib.Batch(ctxs)
    bst = [s.clone() for s in states]
    lay_b = [torch.empty(c.n_coeff, device="cuda") for c in ctxs]
    batch.reconstruct(slopes, bst, lay_b, iters=4, use_graph=True)
    torch.cuda.synchronize()
    for k, S in enumerate(systems):
        assert torch.equal(singles[k], bst[k]) and torch.equal(lay_s[k], lay_b[k]), k
        st0 = State.unpack(to_host(states[k]), S.geom.n_coeff, S.geom.n_coeff)
        ref_st, ref_phi = frame(S, st0, to_host(slopes[k]), iters=4)
        o = S.geom.layer_off
        check_blocks(to_host(lay_b[k]), ref_phi, o, LAYER_TOL, "problem %d layers" % k, FRAME_ETOL)
        got = State.unpack(to_host(bst[k]), S.geom.n_coeff, S.geom.n_coeff)
        check_blocks(got.a, ref_st.a, o, LAYER_TOL, "problem %d a" % k, FRAME_ETOL)
        assert np.array_equal(got.a_prev, st0.a)
    batch.close()
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("loop", ["open", "closed"])
def test_streamed_frames_match_device_slopes(gpu_lib, loop):
    # slopes from pinned host memory, taken in by sensor groups as their
    # copies land (closed loop: the mirrors' slope response computed while
    # they are in flight); two frames in a row, so the second frame's copies
    # must wait for the first frame's reads of the device buffer.  Bitwise
    # the frames of fewha_reconstruct on the same slopes in device memory.
    import torch
    print("\n[gpu-control] streamed", loop, flush=True)
    cfg = get_config("maory_like", loop=loop, gain=0.6)
    ctx = gpu_lib.Context(cfg, device=0)
    state0 = to_dev(random_vector(ctx.n_state, 70, 1) * 0.1)
    host = [torch.from_numpy(random_vector(ctx.n_slopes, 71, k)).pin_memory() for k in range(2)]
    dev = [h.cuda() for h in host]

    def chain(run):
        st = state0.clone()
        lay = torch.empty(ctx.n_coeff, device="cuda")
        outs = []
        for k in range(2):
            run(k, st, lay)
            outs.append(lay.clone())
        torch.cuda.synchronize()
        return [st] + outs

    ref = chain(lambda k, st, lay: ctx.reconstruct(dev[k], st, lay, iters=4))
    for chunks in (1, 3, 9):
        got = chain(lambda k, st, lay: ctx.reconstruct_streamed(host[k], st, lay, iters=4, chunks=chunks))
        for a, b in zip(ref, got):
            assert torch.equal(a, b), (loop, chunks)
    with pytest.raises(gpu_lib.FewhaError):
        ctx.reconstruct_streamed(host[0], state0.clone(), iters=4, chunks=10)  # 9 sensors
    ctx.close()
