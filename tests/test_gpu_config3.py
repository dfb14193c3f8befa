"""The batched workload as specified: one graph replay holds 64 independent
reconstructions, 32 MAORY-like and 32 VLT-like, each with its own seeded
Cn2 profile, r0 and noise sigma, 6 PCG iterations, launch shapes from the
autotuner.  Every problem's frame is bitwise its single context's frame,
and two of each family are checked against the FP64 oracle."""

import numpy as np
import pytest

from oracle.operators import System
from oracle.solver import State, frame
from parity import check_blocks
from synthetic import frozen_flow_frames, slope_noise
from synthetic.configs import batch_mix
from test_gpu_parity import FRAME_ETOL, LAYER_TOL, to_dev, to_host

pytestmark = pytest.mark.gpu

CHECKED = (0, 1, 32, 33)  # two MAORY-like, two VLT-like members


def _unit_noise(cfg):
    u = dict(cfg)
    u["wfs"] = [dict(w, sigma=1.0) for w in cfg["wfs"]]
    return u


def _member_system(cfg, unit_dd):
    """Oracle system of one member.  Its exact Jacobi diagonal comes from its
    family's data diagonal at unit noise: every sensor of a member has the
    same diagonal noise sigma, and C_hat^{-1} = (I - T) sigma^{-2} (I - T)
    (or sigma^{-2} I) is linear in sigma^{-2}, so the data part of J is the
    unit-noise one over sigma^2 (exact up to rounding); this saves the
    20 s per MAORY-like member that the data diagonal takes."""
    assert cfg["noise"]["alpha_eta"] == 0.0 and len({w["sigma"] for w in cfg["wfs"]}) == 1
    S = System(cfg)
    pr = cfg["prior"]
    S._J = unit_dd / cfg["wfs"][0]["sigma"] ** 2 + pr["alpha"] * np.maximum(S.D, pr["tau"])
    return S


def test_batch_of_64_uneven_problems(gpu_lib):
    import torch
    from paper_2202_11945_amd import autotune
    cfgs = batch_mix(32, 32, 3)
    print("\n[gpu-config3] oracle families", flush=True)
    fam = {k: System(_unit_noise(cfgs[k])) for k in (0, 32)}  # A depends on the geometry only
    unit_dd = {k: fam[k].data_diagonal() for k in fam}
    slopes = []
    for k, cfg in enumerate(cfgs):
        F = fam[0 if k < 32 else 32]
        true = next(frozen_flow_frames(cfg, 1, 90, k))
        phi = np.concatenate([p.astype(np.float64).ravel() for p in true])
        s = F.apply_A(phi) + slope_noise(F.geom.n_slopes, [w["sigma"] for w in cfg["wfs"]], 90, k)
        slopes.append(to_dev(s.astype(np.float32)))
    print("[gpu-config3] contexts and autotuner", flush=True)
    ctxs = [gpu_lib.Context(c, device=0) for c in cfgs]
    tune = autotune.tune(ctxs, 6)
    print("[gpu-config3] tuning", tune, flush=True)
    batch = gpu_lib.Batch(ctxs, tuning=tune)
    states = [torch.zeros(c.n_state, device="cuda") for c in ctxs]
    lays = [torch.empty(c.n_coeff, device="cuda") for c in ctxs]
    batch.reconstruct(slopes, states, lays, iters=6, use_graph=True)  # frame 1 from zero
    torch.cuda.synchronize()
    before = [s.clone() for s in states]
    batch.reconstruct(slopes, states, lays, iters=6, use_graph=True)  # frame 2, warm
    torch.cuda.synchronize()
    print("[gpu-config3] single contexts", flush=True)
    # single contexts with the batch's launch shapes (other shapes sum in
    # another order and are checked against the oracle on their own)
    shapes = {k: tune[k] for k in ("dwt_resident", "pt_rows", "res_split")}
    for k, cfg in enumerate(cfgs):
        c = gpu_lib.Context(cfg, device=0, tuning=shapes)
        st = before[k].clone()
        ly = torch.empty(c.n_coeff, device="cuda")
        c.reconstruct(slopes[k], st, ly, iters=6)
        torch.cuda.synchronize()
        assert torch.equal(st, states[k]) and torch.equal(ly, lays[k]), k
        c.close()
    for k in CHECKED:
        print("[gpu-config3] oracle member", k, flush=True)
        S = _member_system(cfgs[k], unit_dd[0 if k < 32 else 32])
        st0 = State.unpack(to_host(before[k]), S.geom.n_coeff, S.geom.n_coeff)
        ref_st, ref_phi = frame(S, st0, to_host(slopes[k]), iters=6)
        o = S.geom.layer_off
        check_blocks(to_host(lays[k]), ref_phi, o, LAYER_TOL, "member %d layers" % k, FRAME_ETOL)
        got = State.unpack(to_host(states[k]), S.geom.n_coeff, S.geom.n_coeff)
        check_blocks(got.c, ref_st.c, o, LAYER_TOL, "member %d c" % k, FRAME_ETOL)
    batch.close()
    for c in ctxs:
        c.close()
