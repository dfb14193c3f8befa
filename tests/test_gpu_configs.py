"""GPU parity on the remaining workload shapes: 2x2 spot-elongation noise
blocks, the paper's own MAORY geometry (sensors sampling two layers finer
than their spacing), the VLT-like geometry, 9 layers with 256x256 grids and
20 iterations, and a batch of independent problems of uneven sizes with
their own priors and noise levels."""

import numpy as np
import pytest

from oracle.operators import System
from oracle.solver import State, frame
from synthetic import get_config, random_vector
from synthetic.configs import batch_mix

from parity import check_blocks
from test_gpu_parity import FRAME_ETOL, LAYER_TOL, OP_TOL, _check_frame, synth_slopes, to_dev, to_host

pytestmark = pytest.mark.gpu

_sys = {}


def system(name, cfg):
    if name not in _sys:
        _sys[name] = (System(cfg), None)
    return _sys[name][0]


def _ops(gpu_lib, S, cfg, key):
    ctx = gpu_lib.Context(cfg, device=0)
    x = random_vector(S.geom.n_coeff, 200, key)
    o, so = S.geom.layer_off, S.geom.slope_off
    check_blocks(to_host(ctx.apply_A(to_dev(x))), S.apply_A(x), so, OP_TOL, "A x sensor")
    y = random_vector(S.A.shape[0], 201, key)
    check_blocks(to_host(ctx.apply_AT(to_dev(y))), S.apply_AT(y), o, OP_TOL, "A^T y layer")
    check_blocks(to_host(ctx.apply_M(to_dev(x))), S.apply_M(x), o, OP_TOL, "M x layer")
    s = synth_slopes(S, 0)
    check_blocks(to_host(ctx.rhs(to_dev(s))), S.rhs(s), o, OP_TOL, "b layer")
    return ctx


def _irregular_masks(cfg, key):
    """Configured masks with holes on every LGS: the annulus minus a random
    fifth of its subapertures, a whole row, a gap that leaves a row two runs,
    and rows whose active span starts or ends at the sensor adjoint's
    32-column tile edge (a tile window's halo column)."""
    from oracle.geometry import subap_mask
    rng = np.random.default_rng(key)
    for w in cfg["wfs"]:
        if w["kind"] != "lgs":
            continue
        N = w["n_subap"]
        m = subap_mask(cfg["D"], N, cfg["obstruction"]) & (rng.random((N, N)) > 0.2)
        m[N // 3, :] = False
        m[N // 2, 5:N // 2] = False
        m[N // 4, :31] = False
        m[N // 4 + 1, 33:] = False
        m[N // 4 + 2, :32] = False
        m[N // 4 + 3, 32:] = False
        w["mask"] = m.astype(np.uint8)


def test_irregular_masks(gpu_lib):
    # the sensor stages' row-span slope layout and the adjoint tiles' row
    # tables on masks with holes, split rows and spans at tile edges
    cfg = get_config("maory_like")
    _irregular_masks(cfg, 7)
    S = system("maory_like_holes", cfg)
    assert S.geom.n_active[0] < 4476 * 0.85
    ctx = _ops(gpu_lib, S, cfg, 9)
    _check_frame(gpu_lib, S, ctx, np.zeros(5 * S.geom.n_coeff, np.float32), synth_slopes(S, 0))


def test_elongated_block_noise(gpu_lib):
    cfg = get_config("small")
    cfg["noise"]["alpha_eta"] = 0.6
    S = system("small_elong", cfg)
    ctx = _ops(gpu_lib, S, cfg, 1)
    _check_frame(gpu_lib, S, ctx, np.zeros(5 * S.geom.n_coeff, np.float32), synth_slopes(S, 0))


def test_paper_maory_geometry(gpu_lib):
    # the paper's runs take 2 (augmented) and 4 iterations per frame: both,
    # the second a warm frame from the first one's state
    cfg = get_config("paper_maory")
    S = system("paper_maory", cfg)
    ctx = _ops(gpu_lib, S, cfg, 2)
    g = _check_frame(gpu_lib, S, ctx, np.zeros(5 * S.geom.n_coeff, np.float32), synth_slopes(S, 0), iters=2)
    _check_frame(gpu_lib, S, ctx, g.pack().astype(np.float32), synth_slopes(S, 1), iters=4)


def test_vlt_like_geometry(gpu_lib):
    cfg = get_config("vlt_like")
    S = system("vlt_like", cfg)
    ctx = _ops(gpu_lib, S, cfg, 3)
    _check_frame(gpu_lib, S, ctx, np.zeros(5 * S.geom.n_coeff, np.float32), synth_slopes(S, 0))


def _many_ngs(n):
    """The 8 m two-layer system with n NGS on three rings, alternately 2x2
    (3x3 corners) and 4x4 subapertures: every sensor meets every
    propagation-adjoint tile, so a tile's sensor list holds all n."""
    import math
    from synthetic.configs import ARCSEC, _ngs
    cfg = get_config("tiny")
    cfg["wfs"] = []
    for k in range(n):
        r, az = (10.0 + 15.0 * (k % 3)) * ARCSEC, 2.0 * math.pi * k / n
        cfg["wfs"].append(_ngs((r * math.cos(az), r * math.sin(az)), 2 if k % 2 == 0 else 4, 0.1))
    return cfg


def test_forty_sensors_per_tile(gpu_lib):
    cfg = _many_ngs(40)
    S = system("many_ngs_40", cfg)
    ctx = _ops(gpu_lib, S, cfg, 5)
    _check_frame(gpu_lib, S, ctx, np.zeros(5 * S.geom.n_coeff, np.float32), synth_slopes(S, 0))


def test_more_than_63_sensors_per_tile_is_refused(gpu_lib):
    with pytest.raises(gpu_lib.FewhaError) as e:
        gpu_lib.Context(_many_ngs(70), device=0)
    assert e.value.status == -1


def _small_grids(levels0):
    """Coarse layers (8 x 8 with `levels0` levels, 16 x 16) under three NGS of
    4 x 4, 5 x 5 and 10 x 10 subapertures: corner grids smaller than the
    propagation adjoint's 6- or 9-row band, K = 3 sensors whose band records
    fall back to dense sums near the grid edges, and a pair sampling a layer
    finer than 2/3 of its spacing (general gather)."""
    from synthetic.configs import ARCSEC, _ngs
    cfg = get_config("tiny")
    cfg["layers"] = [{"h": 0.0, "n": 8, "levels": levels0, "cn2": 0.8},
                     {"h": 6000.0, "n": 16, "levels": 2, "cn2": 0.2}]
    cfg["wfs"] = [_ngs((0.0, 0.0), 4, 0.1), _ngs((20 * ARCSEC, -10 * ARCSEC), 5, 0.1),
                  _ngs((-15 * ARCSEC, 25 * ARCSEC), 10, 0.1)]
    return cfg


def test_small_grids_and_single_node_coarse_block(gpu_lib):
    # operators down to a 1 x 1 coarsest block (synthesis lines of half
    # length 1); the frame on a 2 x 2 one: a 1 x 1 coarsest coefficient is
    # the layer's piston, which no slope sees, so its Jacobi entry is the
    # prior's alone (1.7e-4 against about 10 for the rest) and ten FP32
    # iterations amplify rounding in that one mode beyond the frame tolerance
    cfg = _small_grids(3)
    _ops(gpu_lib, system("small_grids_3", cfg), cfg, 6)
    cfg = _small_grids(2)
    S = system("small_grids_2", cfg)
    ctx = _ops(gpu_lib, S, cfg, 7)
    _check_frame(gpu_lib, S, ctx, np.zeros(5 * S.geom.n_coeff, np.float32), synth_slopes(S, 0))


def _fine_sensors():
    """Two 32 x 32 layers (0.5 m spacing) under NGS of 16, 28, 36, 44 and 52
    subapertures over 8 m: corner spacings of 1.0, 0.57, 0.44, 0.36 and 0.31
    node spacings, i.e. K = 2, 4, 5 and 6 corners per node (dense band
    records of up to 15 rows, also at the grid edges) and one pair finer than
    1/3 (general gather); off-axis, so the corners sit between nodes."""
    from synthetic.configs import ARCSEC, _ngs
    cfg = get_config("tiny")
    cfg["wfs"] = [_ngs((0.0, 0.0), 16, 0.1), _ngs((20 * ARCSEC, -10 * ARCSEC), 28, 0.1),
                  _ngs((-15 * ARCSEC, 25 * ARCSEC), 36, 0.1), _ngs((5 * ARCSEC, 30 * ARCSEC), 44, 0.1),
                  _ngs((-25 * ARCSEC, -5 * ARCSEC), 52, 0.1)]
    return cfg


def test_fine_sensors_wide_bands(gpu_lib):
    cfg = _fine_sensors()
    S = system("fine_sensors", cfg)
    ctx = _ops(gpu_lib, S, cfg, 8)
    _check_frame(gpu_lib, S, ctx, np.zeros(5 * S.geom.n_coeff, np.float32), synth_slopes(S, 0))


def test_large_nine_layers_with_elongation(gpu_lib):
    # the frame with F = I (the fitted frame of this system is covered with the fitting tests)
    cfg = get_config("large")
    cfg.pop("dms")
    cfg.pop("fit")
    S = system("large", cfg)
    ctx = _ops(gpu_lib, S, cfg, 4)
    # 20 FP32 iterations on 9 layers: the coarse wavelet coefficients of the
    # high layers, weakly determined by the slopes (the smallest eigenvalues
    # of M), carry the largest FP32-against-FP64 iterate differences (up to
    # 1.5e-3 of |c_i| + rms at single coefficients, 5e-5 norm-wise); the
    # layers W^{-1} c stay within the frame bounds
    _check_frame(gpu_lib, S, ctx, np.zeros(5 * S.geom.n_coeff, np.float32), synth_slopes(S, 0), c_etol=3e-3)


def check_frames(systems, slopes, states, lays, run_frame, iters=6):
    """Runs one more batched frame and checks every problem's layers against
    the oracle's frame started from the GPU's state before it."""
    import torch
    before = [to_host(st).astype(np.float32) for st in states]
    run_frame()
    torch.cuda.synchronize()
    for k, S in enumerate(systems):
        st = State.unpack(before[k], S.geom.n_coeff, S.geom.n_coeff)
        _, phi = frame(S, st, to_host(slopes[k]), iters=iters)
        check_blocks(to_host(lays[k]), phi, S.geom.layer_off, LAYER_TOL, "problem %d layer" % k, FRAME_ETOL)


def test_uneven_batch_against_oracle(gpu_lib):
    import torch
    cfgs = batch_mix(1, 2, 9)
    systems = [System(c) for c in cfgs]
    ctxs = [gpu_lib.Context(c, device=0) for c in cfgs]
    batch = gpu_lib.Batch(ctxs)
    slopes = [to_dev(synth_slopes(S, k)) for k, S in enumerate(systems)]
    states = [torch.zeros(c.n_state, device="cuda") for c in ctxs]
    lays = [torch.empty(c.n_coeff, device="cuda") for c in ctxs]
    # frame 1 from the zero state, frame 2 warm-started from the GPU's own state;
    # each compared with the oracle's frame from the same (FP32) state
    def run():
        batch.reconstruct(slopes, states, lays, iters=6, use_graph=True)

    check_frames(systems, slopes, states, lays, run)
    check_frames(systems, slopes, states, lays, run)
