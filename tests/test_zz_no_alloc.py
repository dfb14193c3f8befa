"""The allocation-free frame entry point (fewha_reconstruct_noalloc) against
fewha_reconstruct: the same kernels on work buffers in the library's static
device scratch, so every output must be bitwise that of the existing entry
point.  Two calls in a row share the scratch, the second on a smaller
problem (its contents then are what the first call left)."""

import numpy as np
import pytest

from synthetic import get_config
from test_gpu_parity import _oracle_state, synth_slopes, to_dev

pytestmark = pytest.mark.gpu


def _frame(ctx, fn, s, state0, iters):
    import torch
    st = state0.clone()
    lay = torch.full((ctx.n_coeff,), 3.0, device="cuda")
    dm = torch.full((ctx.n_act,), 3.0, device="cuda")
    fn(s, st, lay, dm, iters=iters)
    torch.cuda.synchronize()
    return st, lay, dm


def test_noalloc_frames_match_reconstruct(gpu_lib, systems):
    import torch
    ctxs = []
    try:
        for k, name in enumerate(("maory_like", "small")):  # the second call's problem is smaller
            print("\n[gpu-noalloc]", name, flush=True)
            S = systems(name)
            ctx = gpu_lib.Context(get_config(name), device=0)
            ctxs.append(ctx)
            s = to_dev(synth_slopes(S, 4 + k))
            state0 = to_dev(_oracle_state(S, 2))  # a warm state: every part of the frame is exercised
            iters = S.cfg["iters"]
            ref = _frame(ctx, ctx.reconstruct, s, state0, iters)
            got = _frame(ctx, ctx.reconstruct_noalloc, s, state0, iters)
            for a, b, what in zip(ref, got, ("state", "layers", "dm")):
                assert torch.equal(a, b), (name, what)
            assert float(got[1].abs().max()) > 0.0
    finally:
        for c in ctxs:
            c.close()


def test_noalloc_refuses_the_fitting_step(gpu_lib):
    import torch
    ctx = gpu_lib.Context(get_config("small_fit"), device=0)
    try:
        with pytest.raises(gpu_lib.FewhaError) as e:
            ctx.reconstruct_noalloc(torch.zeros(ctx.n_slopes, device="cuda"),
                                    torch.zeros(ctx.n_state, device="cuda"))
        assert e.value.status == -1
    finally:
        ctx.close()
