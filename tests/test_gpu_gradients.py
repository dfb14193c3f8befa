"""GPU parity of the converged solve, W^{-1} / W^{-T} and the implicit
backward against the FP64 oracle.

* W^{-1}, W^{-T}: <= 1e-5 relative per application.
* Solve (mixed-precision refinement: FP32 PCG corrections driven by an FP64
  residual): the GPU solution against the dense Cholesky solution (8 m
  system) and, at MAORY-like size, the oracle's residual of the GPU solution.
* param_grads on the oracle's exact c* and lambda: <= 1e-4 of each
  component's scale (FP32 operators, FP64 reductions).
* The loss gradient through torch.autograd: the stored central differences
  of the FP64 oracle, |g - g_FD| <= 1e-3 max(|g_FD|, 1e-2 max|g_FD|).
"""

import json
import os
import sys

import numpy as np
import pytest

from oracle.gradients import (Science, exact_solve, implicit_gradient, implicit_terms, sensor_derivatives)
from oracle.operators import System
from synthetic import get_config, random_vector

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_gradients import frames_for  # noqa: E402

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
RTOL = 1e-6


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def scaled_err(g, ref, floor=1e-2):
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), floor * np.abs(ref).max())
    return np.abs(g - ref) / scale


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float32))).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def step(msg):
    print("\n[gpu-grad]", msg, flush=True)


_ctx = {}


def ctx_for(lib, name):
    if name not in _ctx:
        step("context " + name)
        _ctx[name] = lib.Context(get_config(name), device=0)
    return _ctx[name]


@pytest.fixture(scope="module")
def small_case():
    cfg, cfg_true, frames = frames_for("grad_small", 4)
    S = System(cfg)
    return cfg, cfg_true, frames, S


@pytest.mark.parametrize("name", ["grad_small", "maory_like"])
def test_winv_and_winvT(gpu_lib, systems, name):
    S = systems(name)
    ctx = ctx_for(gpu_lib, name)
    x = random_vector(S.geom.n_coeff, 500)
    step("W^-1 / W^-T " + name)
    from parity import check_blocks
    o = S.geom.layer_off
    check_blocks(to_host(ctx.apply_Winv(to_dev(x))), S.W_inv(x), o, OP_TOL, "W^-1 x layer")
    check_blocks(to_host(ctx.apply_WinvT(to_dev(x))), S.W_invT(x), o, OP_TOL, "W^-T x layer")


@pytest.mark.parametrize("side", [0, 16])
def test_solve_matches_cholesky_past_the_dot_ring(gpu_lib, small_case, side):
    # side 0: Jacobi PCG, past the 256-iteration ring of inner-product slots;
    # side 16: with the coarse-level correction (fewer iterations)
    cfg, _, frames, S = small_case
    ctx = gpu_lib.Context(cfg, device=0)
    ctx.set_solve_coarse(side)
    b = S.rhs(frames[0][0]).astype(np.float32).astype(np.float64)
    step("solve grad_small rtol 1e-10, coarse side %d" % side)
    x, it, r = ctx.solve(to_dev(b), rtol=1e-10, max_iters=40000)
    got = to_host(x)
    ref = exact_solve(S, b)
    print("iterations", it, "residual ratio", r, "rel error vs Cholesky", rel(got, ref),
          "oracle residual", rel(S.apply_M(got), b))
    assert r <= 1e-10 and rel(got, ref) <= 1e-6
    if side == 0:
        assert it > 256
    ctx.close()


def test_coarse_correction_cuts_iterations(gpu_lib):
    # MAORY-like MAP and adjoint solves with Jacobi alone and with the
    # coarse-level correction (two frames of one context, so the batch's two
    # instances share the set-up): both reach the tolerance, agree with each
    # other, and the correction needs far fewer iterations
    import torch
    cfg, _, frames = frames_for("grad_maory", 2)
    ctx = gpu_lib.Context(cfg, device=0)
    batch = gpu_lib.Batch([ctx, ctx])
    s = [to_dev(f[0]) for f in frames]
    g = [to_dev(random_vector(ctx.n_coeff, 520, k) * 1e-3) for k in range(2)]
    out = {}
    for side in (0, 16):
        batch.set_solve_coarse(side)
        step("MAORY-like solves, coarse side %d" % side)
        c, it, r = batch.solve_map(slopes=s, rtol=RTOL, max_iters=50000)
        lam, it2, r2 = batch.solve_map(g_layers=g, rtol=RTOL, max_iters=50000)
        print("side", side, "forward", it, r, "adjoint", it2, r2)
        assert r <= RTOL and r2 <= RTOL
        out[side] = (c, lam, it, it2)
    # both solutions through the oracle's FP64 residual (the float
    # solutions, rounding included), as in the MAORY-like solve test.  The
    # adjoint solution of a white-noise g has large fine-scale coefficients,
    # and its rounding to float alone leaves an FP64 residual of about 2e-4
    # with either preconditioner (the iterate before rounding met RTOL): the
    # correction must do as well as Jacobi there
    S = System(cfg)
    res = {}
    for side in (0, 16):
        for k in range(2):
            bf = S.rhs(frames[k][0])
            ba = S.W_invT(to_host(g[k]))
            res[side, k] = (rel(S.apply_M(to_host(out[side][0][k])), bf),
                            rel(S.apply_M(to_host(out[side][1][k])), ba))
            print("side", side, "frame", k, "oracle residuals", res[side, k])
    for k in range(2):
        assert res[0, k][0] <= 1e-5 and res[16, k][0] <= 1e-5
        assert res[16, k][1] <= max(2.0 * res[0, k][1], 1e-5)
    assert out[16][2] <= 0.6 * out[0][2] and out[16][3] <= 0.6 * out[0][3]
    batch.close()
    ctx.close()
    torch.cuda.synchronize()


def test_solve_refused_with_augmentation(gpu_lib):
    from synthetic import get_config
    ctx = gpu_lib.Context(get_config("small", augment=2), device=0)
    import torch
    with pytest.raises(gpu_lib.FewhaError) as e:
        ctx.solve(torch.ones(ctx.n_coeff, device="cuda"), rtol=1e-3)
    assert e.value.status == -4
    ctx.close()


def test_solve_zero_rhs(gpu_lib):
    import torch
    ctx = ctx_for(gpu_lib, "grad_small")
    step("solve zero rhs")
    x = torch.full((ctx.n_coeff,), 7.0, device="cuda")
    x, it, r = ctx.solve(torch.zeros(ctx.n_coeff, device="cuda"), x=x, rtol=RTOL)
    assert it == 0 and r == 0.0 and not to_host(x).any()


def test_param_grads_on_exact_pieces(gpu_lib, small_case):
    cfg, cfg_true, frames, S = small_case
    ctx = ctx_for(gpu_lib, "grad_small")
    dA = sensor_derivatives(S)
    _, _, _, pieces = implicit_gradient(cfg, frames[:1], cfg_true)
    c, lam = pieces[0][0], pieces[0][1]
    c32 = c.astype(np.float32).astype(np.float64)
    l32 = lam.astype(np.float32).astype(np.float64)
    s = frames[0][0]
    ra, rg, rh = implicit_terms(S, dA, s, c32, l32)
    ref = np.concatenate([[ra], rg, rh])
    step("param_grads grad_small")
    got = to_host(ctx.param_grads(to_dev(s), to_dev(c32), to_dev(l32)))
    err = scaled_err(got, ref)
    print("gpu", got, "\noracle", ref, "\nscaled error", err)
    assert err.max() <= 1e-4


def test_param_grads_batch_matches_single_bitwise(gpu_lib, small_case):
    cfg, _, frames, S = small_case
    ctx = ctx_for(gpu_lib, "grad_small")
    batch = gpu_lib.Batch([ctx, ctx, ctx])
    s = [to_dev(f[0]) for f in frames[:3]]
    c = [to_dev(random_vector(S.geom.n_coeff, 510, k)) for k in range(3)]
    lam = [to_dev(random_vector(S.geom.n_coeff, 511, k)) for k in range(3)]
    step("param_grads batch vs single")
    gb = [to_host(g) for g in batch.param_grads(s, c, lam)]
    for k in range(3):
        assert np.array_equal(gb[k], to_host(ctx.param_grads(s[k], c[k], lam[k])))
    batch.close()


def test_loss_gradient_matches_finite_differences(gpu_lib, small_case):
    import torch
    from paper_2202_11945_amd.autograd import FrameBatch, MAPLayers, param_vector
    from science_loss import ScienceLoss
    cfg, cfg_true, frames, S = small_case
    with open(os.path.join(HERE, "golden", "gradients_grad_small.json")) as f:
        gold = json.load(f)
    assert gold["frames"] == len(frames)
    fd = np.concatenate([[gold["fd"]["alpha"]], gold["fd"]["cn2"], gold["fd"]["h"]])
    step("autograd grad_small, %d frames" % len(frames))
    fb = FrameBatch(cfg, len(frames))
    sci = Science(cfg)
    truth = torch.stack([torch.stack([torch.tensor(np.asarray(Pt @ phi_t)[sci.mask])
                                      for Pt, _ in sci.project(cfg_true)]) for _, phi_t in frames]).cuda()
    params = param_vector(cfg).requires_grad_(True)
    slopes = torch.stack([to_dev(s) for s, _ in frames])
    phi = MAPLayers.apply(params, slopes, fb, 1e-9, 100000)
    L = len(cfg["layers"])
    heights = params[1 + L:].cuda()
    loss = ScienceLoss(cfg, "cuda")(phi, heights, truth)
    loss.backward()
    got = params.grad.numpy()
    err = scaled_err(got, fd)
    print("gpu", got, "\nfd ", fd, "\nscaled error", err)
    assert err.max() <= 1e-3
    fb.close()


def test_maory_solve_and_param_grads(gpu_lib):
    import torch
    cfg, cfg_true, frames = frames_for("grad_maory", 2)
    S = System(cfg)
    step("MAORY-like solves and param_grads, 2 frames")
    ctx = gpu_lib.Context(cfg, device=0)
    batch = gpu_lib.Batch([ctx, ctx])
    s = [to_dev(f[0]) for f in frames]
    c, it, r = batch.solve_map(slopes=s, rtol=RTOL, max_iters=50000)
    print("forward iterations", it, "ratio", r)
    assert r <= RTOL
    # the oracle's residual of the GPU solution (FP64 right-hand side)
    for k in range(2):
        bh = S.rhs(frames[k][0])
        res = rel(S.apply_M(to_host(c[k])), bh)
        print("frame", k, "oracle relative residual", res)
        assert res <= 1e-5
    g = [to_dev(random_vector(S.geom.n_coeff, 520, k) * 1e-3) for k in range(2)]
    lam, it2, r2 = batch.solve_map(g_layers=g, rtol=RTOL, max_iters=50000)
    print("adjoint iterations", it2, "ratio", r2)
    assert r2 <= RTOL
    grads = batch.param_grads(s, c, lam)
    dA = sensor_derivatives(S)
    for k in range(2):
        ra, rg, rh = implicit_terms(S, dA, frames[k][0], to_host(c[k]), to_host(lam[k]))
        err = scaled_err(to_host(grads[k]), np.concatenate([[ra], rg, rh]))
        print("frame", k, "scaled error", err)
        assert err.max() <= 1e-4
    batch.close()
    ctx.close()
    torch.cuda.synchronize()


def test_solve_map_matches_exact_map_solution(gpu_lib, small_case):
    cfg, _, frames, S = small_case
    ctx = ctx_for(gpu_lib, "grad_small")
    step("solve_map grad_small")
    s = frames[1][0]
    x, it, r = ctx.solve_map(slopes=to_dev(s), rtol=1e-10, max_iters=40000)
    ref = exact_solve(S, S.rhs(s))
    print("iterations", it, "ratio", r, "rel error", rel(to_host(x), ref))
    assert r <= 1e-10 and rel(to_host(x), ref) <= 1e-6
    g = random_vector(S.geom.n_coeff, 530)
    lam, it, r = ctx.solve_map(g_layers=to_dev(g), rtol=1e-10, max_iters=40000)
    ref = exact_solve(S, S.W_invT(g))
    print("adjoint iterations", it, "ratio", r, "rel error", rel(to_host(lam), ref))
    assert r <= 1e-10 and rel(to_host(lam), ref) <= 1e-6


def test_param_grads_refuses_stencil_outside_layer(gpu_lib):
    # an NGS whose first corner column lands exactly on node 0 of the upper
    # layer (-4 m + 4096 m * -2^-10 + 8 m = 0): the forward footprint fits, the
    # derivative on that grid line would need node -1
    cfg = get_config("tiny")
    cfg["wfs"][0]["theta"] = (-2.0 ** -10, 0.0)
    cfg["layers"][1]["h"] = 4096.0
    ctx = gpu_lib.Context(cfg, device=0)
    n = ctx.n_coeff
    step("param_grads EGEOM")
    with pytest.raises(gpu_lib.FewhaError) as e:
        ctx.param_grads(to_dev(np.zeros(ctx.n_slopes)), to_dev(np.zeros(n)), to_dev(np.zeros(n)))
    assert e.value.status == -5
    ctx.close()


@pytest.mark.parametrize("res", [128, 32, {"dwt_resident": 32, "glob_fuse": 1}])
def test_transforms_at_the_largest_layer_side(gpu_lib, res):
    # one 2048 x 2048 layer (the largest side the library takes), 8 levels:
    # with resident side 128 four global levels (2048 .. 256), with 32 six;
    # W^{-1} = delta^{-1} W^T and W^{-T} = delta^{-1} W (A7) against the
    # oracle's dense-matrix transforms, element by element
    from oracle.wavelet import daubechies_filter, dwt2, idwt2
    from parity import check_blocks
    cfg = get_config("tiny")
    cfg["layers"] = [{"h": 0.0, "n": 2048, "levels": 8, "cn2": 1.0}]
    step("W^-1 / W^-T at 2048 x 2048, tuning %s" % res)
    ctx = gpu_lib.Context(cfg, device=0, tuning=res)
    n = 2048
    delta = cfg["domain_side"] / n
    h = daubechies_filter(3)
    c = random_vector(n * n, 540)
    ref = idwt2(c.reshape(n, n), 8, h).ravel() / delta
    check_blocks(to_host(ctx.apply_Winv(to_dev(c))), ref, [0, n * n], OP_TOL, "W^-1 c (2048)")
    ref = dwt2(c.reshape(n, n), 8, h).ravel() / delta
    check_blocks(to_host(ctx.apply_WinvT(to_dev(c))), ref, [0, n * n], OP_TOL, "W^-T phi (2048)")
    ctx.close()
