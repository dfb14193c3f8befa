"""Pins of the gradient oracle: the derivative of the bilinear sampling
against finite differences (off and on grid lines), the implicit gradient
against the stored central differences of the loss, and the torch loss used
by the GPU tests against the oracle's loss terms."""

import json
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.gradients import (Science, exact_solve, frame_terms, implicit_gradient, sample_matrices,
                              sensor_derivatives)
from oracle.operators import System, propagation_matrix
from synthetic import ARCSEC, get_config, random_vector

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_gradients import frames_for  # noqa: E402


def a23_ok(g, ref):
    """|g - g_FD| <= 1e-3 max(|g_FD|, 1e-2 max|g_FD|) per component."""
    ref = np.atleast_1d(np.asarray(ref, dtype=float))
    g = np.atleast_1d(np.asarray(g, dtype=float))
    scale = np.maximum(np.abs(ref), 1e-2 * np.abs(ref).max())
    return np.all(np.abs(g - ref) <= 1e-3 * scale), np.abs(g - ref) / scale


def _layer(h, n=32):
    return {"h": h, "n": n, "levels": 3, "cn2": 0.3}


def test_sampling_equals_propagation_off_grid():
    D, N, L = 8.0, 20, 12.8
    th = (13.0 * ARCSEC, -7.0 * ARCSEC)
    layer = _layer(3777.0)
    wfs = {"kind": "lgs", "n_subap": N, "theta": th, "H": 90000.0}
    scale = 1 - layer["h"] / 90000.0
    S, _ = sample_matrices(D, N, th, layer, L, scale, (np.zeros(N + 1), np.zeros(N + 1)))
    assert abs(S - propagation_matrix(D, wfs, layer, L)).max() < 1e-12


def _fd_matrix(D, N, th, layer, L, H, eps):
    def at(h):
        l2 = dict(layer, h=h)
        sc = 1 - h / H if H else 1.0
        return sample_matrices(D, N, th, l2, L, sc, (np.zeros(N + 1), np.zeros(N + 1)))[0]
    return at(layer["h"] + eps), at(layer["h"]), at(layer["h"] - eps)


@pytest.mark.parametrize("H", [90000.0, None])
def test_height_derivative_matches_fd_off_grid(H):
    D, N, L = 8.0, 20, 12.8
    th = (21.0 * ARCSEC, 9.0 * ARCSEC)
    layer = _layer(5123.0)
    x = -0.5 * D + np.arange(N + 1) * (D / N)
    delta = L / layer["n"]
    sc = 1 - layer["h"] / H if H else 1.0
    dt = lambda a: ((-x / H if H else np.zeros_like(x)) + th[a]) / delta  # noqa: E731
    _, dS = sample_matrices(D, N, th, layer, L, sc, (dt(0), dt(1)))
    up, _, dn = _fd_matrix(D, N, th, layer, L, H, 1e-3)
    v = random_vector(layer["n"] ** 2, 400).astype(np.float64)
    fd = (up @ v - dn @ v) / 2e-3
    assert np.abs(dS @ v - fd).max() <= 1e-7 * np.abs(fd).max()


def test_height_derivative_on_grid_lines_is_the_one_sided_mean():
    # ground layer: every corner sits on a node (corner pitch = node spacing)
    D, N, L = 8.0, 20, 12.8
    th = (17.0 * ARCSEC, -11.0 * ARCSEC)
    layer = _layer(0.0)
    delta = L / layer["n"]
    dt = (np.full(N + 1, th[0] / delta), np.full(N + 1, th[1] / delta))
    _, dS = sample_matrices(D, N, th, layer, L, 1.0, dt)
    up, mid, dn = _fd_matrix(D, N, th, layer, L, None, 1e-4)
    v = random_vector(layer["n"] ** 2, 401).astype(np.float64)
    right = (up @ v - mid @ v) / 1e-4
    left = (mid @ v - dn @ v) / 1e-4
    assert np.abs(right - left).max() > 1e-3 * np.abs(right).max()  # a real kink
    assert np.abs(dS @ v - 0.5 * (right + left)).max() <= 1e-6 * np.abs(right).max()


def test_sensor_derivative_matches_fd_of_A():
    cfg = get_config("grad_small")
    S = System(cfg)
    dA = sensor_derivatives(S)
    o = S.geom.layer_off
    phi = random_vector(S.geom.n_coeff, 402).astype(np.float64)
    for l in (1, 2):
        out = []
        for sgn in (1, -1):
            c2 = get_config("grad_small")
            c2["layers"][l]["h"] += sgn * 0.01
            out.append(System(c2).apply_A(phi))
        fd = (out[0] - out[1]) / 0.02
        got = dA[l] @ phi[o[l]:o[l + 1]]
        assert np.abs(got - fd).max() <= 1e-6 * np.abs(fd).max()


@pytest.fixture(scope="module")
def grad_small():
    cfg, cfg_true, frames = frames_for("grad_small", 4)
    with open(os.path.join(HERE, "golden", "gradients_grad_small.json")) as f:
        gold = json.load(f)
    return cfg, cfg_true, frames, gold


def test_implicit_gradient_matches_finite_differences(grad_small):
    cfg, cfg_true, frames, gold = grad_small
    ga, gg, gh, _ = implicit_gradient(cfg, frames, cfg_true)
    fd = np.concatenate([[gold["fd"]["alpha"]], gold["fd"]["cn2"], gold["fd"]["h"]])
    ok, err = a23_ok(np.concatenate([[ga], gg, gh]), fd)
    assert ok, err


def test_torch_loss_matches_oracle_terms(grad_small):
    torch = pytest.importorskip("torch")
    from science_loss import ScienceLoss
    cfg, cfg_true, frames, _ = grad_small
    S = System(cfg)
    sci = Science(cfg)
    proj = sci.project(cfg)
    proj_t = sci.project(cfg_true)
    s, phi_t = frames[0]
    phi = S.W_inv(exact_solve(S, S.rhs(s)))
    loss, g_phi, g_h = frame_terms(sci, proj, proj_t, phi, phi_t, S.geom.layer_off)
    tl = ScienceLoss(cfg, "cpu")
    h = torch.tensor([l["h"] for l in cfg["layers"]], dtype=torch.float64, requires_grad=True)
    ph = torch.tensor(phi[None, :], requires_grad=True)
    truth = torch.stack([torch.tensor(np.asarray(Pt @ phi_t)[sci.mask]) for Pt, _ in proj_t])[None]
    val = tl(ph, h, truth)
    val.backward()
    assert abs(val.item() - loss) <= 1e-12 * loss
    assert np.abs(ph.grad.numpy()[0] - g_phi).max() <= 1e-10 * np.abs(g_phi).max()
    assert np.abs(h.grad.numpy() - g_h).max() <= 1e-9 * np.abs(g_h).max()
