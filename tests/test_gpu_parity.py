"""GPU parity of every entry point of libfewha against the FP64 oracle, on
the same seeded FP32 inputs.  Tolerances: 1e-5 per operator application,
1e-4 on the reconstructed layers after a fixed number of PCG iterations,
each checked per block (sensor or layer) norm-wise, as the largest entry
error against the block's largest entry, and entry by entry against the
entry's size with the block's RMS as floor (tests/parity.py).  Structural
results (batch vs single, graph vs direct launches, repeat runs) are
compared bitwise."""

import numpy as np
import pytest

from parity import check, check_blocks

from oracle.solver import State, frame
from synthetic import frozen_flow_frames, get_config, random_vector, slope_noise

pytestmark = pytest.mark.gpu

CONFIGS = ["tiny", "small", "mid", "maory_like"]
OP_TOL = 1e-5
LAYER_TOL = 1e-4
# Entry-wise bound of the frame's outputs (layers, c, r, a), against
# |ref_i| + rms(ref) of the block.  After k FP32 PCG iterations the error
# is a sum of many rounding contributions, spread unevenly over the
# coefficients: at the norm-wise 1e-4 it reaches 4e-4 of (|ref_i| + rms) at
# single entries (9 layers, 20 iterations); 1e-3 keeps a margin over that
# and still fails a single entry off by 0.3 % of the RMS.  Norm-wise and
# max-abs stay at LAYER_TOL.
FRAME_ETOL = 1e-3


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float32))).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


_ctx_cache = {}


def ctx_for(lib, name):
    if name not in _ctx_cache:
        print("\n[gpu] building context", name, flush=True)
        _ctx_cache[name] = lib.Context(get_config(name), device=0)
    return _ctx_cache[name]


def synth_slopes(S, k, key=11):
    true = next(frozen_flow_frames(S.cfg, 1, key, first=k))
    phi = np.concatenate([p.astype(np.float64).ravel() for p in true])
    s = S.apply_A(phi)
    sig = [w["sigma"] for w in S.cfg["wfs"]]
    return (s + slope_noise(S.geom.n_slopes, sig, key, k)).astype(np.float32)


@pytest.mark.parametrize("name", CONFIGS)
def test_apply_A(gpu_lib, systems, name):
    S = systems(name)
    ctx = ctx_for(gpu_lib, name)
    x = random_vector(S.geom.n_coeff, 100, CONFIGS.index(name))
    got = to_host(ctx.apply_A(to_dev(x)))
    check_blocks(got, S.apply_A(x), S.geom.slope_off, OP_TOL, "A x %s sensor" % name)


@pytest.mark.parametrize("name", CONFIGS)
def test_apply_AT(gpu_lib, systems, name):
    S = systems(name)
    ctx = ctx_for(gpu_lib, name)
    y = random_vector(S.A.shape[0], 101, CONFIGS.index(name))
    got = to_host(ctx.apply_AT(to_dev(y)))
    check_blocks(got, S.apply_AT(y), S.geom.layer_off, OP_TOL, "A^T y %s layer" % name)


@pytest.mark.parametrize("name", CONFIGS)
def test_apply_M(gpu_lib, systems, name):
    S = systems(name)
    ctx = ctx_for(gpu_lib, name)
    c = random_vector(S.geom.n_coeff, 102, CONFIGS.index(name))
    got = to_host(ctx.apply_M(to_dev(c)))
    ref = S.apply_M(c)
    check(got, ref, OP_TOL, "M c %s" % name)
    # per layer as well (a small layer must not hide behind a big one)
    check_blocks(got, ref, S.geom.layer_off, OP_TOL, "M c %s layer" % name)


@pytest.mark.parametrize("name", CONFIGS)
def test_rhs(gpu_lib, systems, name):
    S = systems(name)
    ctx = ctx_for(gpu_lib, name)
    s = synth_slopes(S, 0)
    got = to_host(ctx.rhs(to_dev(s)))
    check_blocks(got, S.rhs(s), S.geom.layer_off, OP_TOL, "b %s layer" % name)


def _oracle_state(S, n_frames):
    """Oracle-only warm-start chain; returns the FP32-rounded state after it."""
    st = State(S.geom.n_coeff, S.geom.n_coeff)
    for k in range(n_frames):
        st, _ = frame(S, st, synth_slopes(S, k).astype(np.float64))
    return st.pack().astype(np.float32)


def _check_frame(gpu_lib, S, ctx, state32, s32, iters=None, c_etol=FRAME_ETOL):
    import torch
    iters = S.cfg["iters"] if iters is None else iters
    st_dev = to_dev(state32)
    lay = torch.empty(S.geom.n_coeff, device="cuda", dtype=torch.float32)
    dm = torch.empty(S.geom.n_coeff, device="cuda", dtype=torch.float32)
    ctx.reconstruct(to_dev(s32), st_dev, lay, dm, iters=iters)
    got_state, got_lay, got_dm = to_host(st_dev), to_host(lay), to_host(dm)
    ref_st, ref_phi = frame(S, State.unpack(state32, S.geom.n_coeff, S.geom.n_coeff),
                            s32.astype(np.float64), iters=iters)
    o = S.geom.layer_off
    check_blocks(got_lay, ref_phi, o, LAYER_TOL, "layers", FRAME_ETOL)
    g = State.unpack(got_state, S.geom.n_coeff, S.geom.n_coeff)
    check_blocks(g.c, ref_st.c, o, LAYER_TOL, "c", c_etol)
    check_blocks(g.b, ref_st.b, o, OP_TOL, "b")
    # the recurrence residual: its FP32 rounding error scales with the size of
    # the right-hand side it is a difference of (b - M c), not with its own
    # size, which shrinks with every iteration (attainable accuracy of CG)
    check_blocks(g.r, ref_st.r, o, LAYER_TOL, "r", FRAME_ETOL, scale=ref_st.b)
    check_blocks(g.a, ref_st.a, o, LAYER_TOL, "a", FRAME_ETOL)
    n = S.geom.n_coeff
    assert np.array_equal(g.a_prev, state32[4 * n:5 * n].astype(np.float64))  # a_prev <- a
    assert np.array_equal(got_dm.astype(np.float32), g.a.astype(np.float32))
    return g


@pytest.mark.parametrize("name", CONFIGS)
def test_reconstruct_first_frame(gpu_lib, systems, name):
    S = systems(name)
    ctx = ctx_for(gpu_lib, name)
    state = np.zeros(5 * S.geom.n_coeff, dtype=np.float32)
    _check_frame(gpu_lib, S, ctx, state, synth_slopes(S, 0))


@pytest.mark.parametrize("name", ["small", "mid", "maory_like"])
def test_reconstruct_warm_frame(gpu_lib, systems, name):
    # identical input state for both sides: the oracle's own chain, rounded to FP32
    S = systems(name)
    ctx = ctx_for(gpu_lib, name)
    state = _oracle_state(S, 3)
    _check_frame(gpu_lib, S, ctx, state, synth_slopes(S, 3))


def test_reconstruct_gain_and_iterations(gpu_lib, systems):
    cfg = get_config("small", gain=0.6)
    from oracle.operators import System
    S = System(cfg)
    ctx = gpu_lib.Context(cfg, device=0)
    state = _oracle_state(systems("small"), 2)
    for iters in (0, 1, 7):
        _check_frame(gpu_lib, S, ctx, state, synth_slopes(S, 2), iters=iters)


def test_zero_input_gives_zero(gpu_lib, systems):
    S = systems("small")
    ctx = ctx_for(gpu_lib, "small")
    import torch
    st = torch.zeros(5 * S.geom.n_coeff, device="cuda")
    s = torch.zeros(S.A.shape[0], device="cuda")
    ctx.reconstruct(s, st, iters=4)
    assert float(torch.abs(st).max()) == 0.0


def test_nonfinite_slopes_report_a_breakdown(gpu_lib):
    # NaN slopes (a dead sensor) make rho non-finite: the PCG step sets the
    # context's breakdown flag, the next call returns FEWHA_ENUMERIC without
    # running, and the call after it runs normally
    import torch
    ctx = gpu_lib.Context(get_config("small"), device=0)
    st = torch.zeros(ctx.n_state, device="cuda")
    ctx.reconstruct(torch.full((ctx.n_slopes,), float("nan"), device="cuda"), st, iters=2)
    torch.cuda.synchronize()
    zs = torch.zeros(ctx.n_slopes, device="cuda")
    st2 = torch.full((ctx.n_state,), 5.0, device="cuda")
    with pytest.raises(gpu_lib.FewhaError) as e:
        ctx.reconstruct(zs, st2, iters=2)
    assert e.value.status == -6
    torch.cuda.synchronize()
    assert float(st2.min()) == 5.0 and float(st2.max()) == 5.0  # nothing ran
    st2.zero_()
    ctx.reconstruct(zs, st2, iters=2)
    torch.cuda.synchronize()
    assert float(st2.abs().max()) == 0.0
    # a batch reports it the same way
    ok = gpu_lib.Context(get_config("small"), device=0)
    b = gpu_lib.Batch([ok, ctx])
    sts = [torch.zeros(ctx.n_state, device="cuda") for _ in range(2)]
    b.reconstruct([zs, torch.full_like(zs, float("nan"))], sts, iters=2, use_graph=False)
    torch.cuda.synchronize()
    with pytest.raises(gpu_lib.FewhaError) as e:
        b.reconstruct([zs, zs], sts, iters=2, use_graph=False)
    assert e.value.status == -6 and "problem 1" in str(e.value)
    b.reconstruct([zs, zs], [s.zero_() for s in sts], iters=2, use_graph=False)
    torch.cuda.synchronize()
    assert all(float(s.abs().max()) == 0.0 for s in sts)
    b.close()
    ok.close()
    ctx.close()


def test_chain_drift(gpu_lib, systems):
    # GPU-only warm-start chain vs the oracle's chain from the same zero state
    S = systems("small")
    ctx = ctx_for(gpu_lib, "small")
    import torch
    st_dev = torch.zeros(5 * S.geom.n_coeff, device="cuda")
    lay = torch.empty(S.geom.n_coeff, device="cuda")
    st = State(S.geom.n_coeff, S.geom.n_coeff)
    worst = 0.0
    for k in range(10):
        s = synth_slopes(S, k)
        ctx.reconstruct(to_dev(s), st_dev, lay, iters=S.cfg["iters"])
        st, phi = frame(S, st, s.astype(np.float64))
        worst = max(worst, rel(to_host(lay), phi))
    print("\n[gpu] chained drift over 10 frames:", worst)
    assert worst <= 1e-3


def test_apply_M_symmetric_on_gpu(gpu_lib, systems):
    S = systems("small")
    ctx = ctx_for(gpu_lib, "small")
    u = random_vector(S.geom.n_coeff, 103, 0)
    v = random_vector(S.geom.n_coeff, 104, 0)
    Mu = to_host(ctx.apply_M(to_dev(u)))
    Mv = to_host(ctx.apply_M(to_dev(v)))
    a, b = Mu @ v, u @ Mv
    assert abs(a - b) <= 1e-5 * np.linalg.norm(Mu) * np.linalg.norm(v)


def _batch_inputs(lib, systems, names):
    import torch
    ctxs, slopes, states = [], [], []
    for k, nm in enumerate(names):
        S = systems(nm)
        ctxs.append(lib.Context(get_config(nm), device=0))
        slopes.append(to_dev(synth_slopes(S, k)))
        states.append(to_dev(_oracle_state(S, 1) if k % 2 else np.zeros(5 * S.geom.n_coeff, np.float32)))
    return ctxs, slopes, states


def test_batch_matches_single_bitwise(gpu_lib, systems):
    import torch
    names = ["small", "tiny", "mid", "small"]
    ctxs, slopes, states = _batch_inputs(gpu_lib, systems, names)
    singles = [s.clone() for s in states]
    lay_single = [torch.empty(c.n_coeff, device="cuda") for c in ctxs]
    for c, s, st, ly in zip(ctxs, slopes, singles, lay_single):
        c.reconstruct(s, st, ly, iters=4)
    batch = gpu_lib.Batch(ctxs)
    bst = [s.clone() for s in states]
    lay_b = [torch.empty(c.n_coeff, device="cuda") for c in ctxs]
    batch.reconstruct(slopes, bst, lay_b, iters=4, use_graph=False)
    torch.cuda.synchronize()
    for a, b in zip(singles, bst):
        assert torch.equal(a, b)
    for a, b in zip(lay_single, lay_b):
        assert torch.equal(a, b)


def test_timed_launch_matches_single_bitwise(gpu_lib, systems):
    # the launch bench.py times: 32 MAORY-like problems in one batch, resident
    # side 128, 4 node rows per thread, one graph replay per frame; every
    # problem's state and layers equal its own single-context frame (those
    # are checked against the oracle above)
    import torch
    S = systems("maory_like")
    ctxs = [gpu_lib.Context(get_config("maory_like"), device=0) for _ in range(32)]
    slopes = [to_dev(synth_slopes(S, k)) for k in range(32)]
    states = [torch.zeros(5 * S.geom.n_coeff, device="cuda") for _ in range(32)]
    singles = [s.clone() for s in states]
    lay_single = [torch.empty(S.geom.n_coeff, device="cuda") for _ in range(32)]
    for c, s, st, ly in zip(ctxs, slopes, singles, lay_single):
        c.reconstruct(s, st, ly, iters=4)
    batch = gpu_lib.Batch(ctxs, tuning={"dwt_resident": 128, "pt_rows": 4})
    try:
        bst = [s.clone() for s in states]
        lay_b = [torch.empty(S.geom.n_coeff, device="cuda") for _ in range(32)]
        batch.reconstruct(slopes, bst, lay_b, iters=4, use_graph=True)
        torch.cuda.synchronize()
        for k in range(32):
            assert torch.equal(singles[k], bst[k]), k
            assert torch.equal(lay_single[k], lay_b[k]), k
    finally:
        batch.close()
        for c in ctxs:
            c.close()


def test_graph_replay_matches_direct_bitwise(gpu_lib, systems):
    import torch
    names = ["small", "mid"]
    ctxs, slopes, states = _batch_inputs(gpu_lib, systems, names)
    batch = gpu_lib.Batch(ctxs)
    direct = [s.clone() for s in states]
    graph = [s.clone() for s in states]
    for rep in range(3):  # several frames: replays after the first reuse the graph
        batch.reconstruct(slopes, direct, iters=4, use_graph=False)
        torch.cuda.synchronize()
        batch.reconstruct(slopes, graph, iters=4, use_graph=True)
        torch.cuda.synchronize()
        for a, b in zip(direct, graph):
            assert torch.equal(a, b), rep


def test_repeat_runs_bitwise(gpu_lib, systems):
    import torch
    S = systems("maory_like")
    ctx = ctx_for(gpu_lib, "maory_like")
    s = to_dev(synth_slopes(S, 5))
    outs = []
    for _ in range(2):
        st = torch.zeros(5 * S.geom.n_coeff, device="cuda")
        ctx.reconstruct(s, st, iters=4)
        outs.append(st)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
