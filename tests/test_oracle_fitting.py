"""Pins of the oracle's DM fitting (Sec. 4.1: more layers than DMs make the
fitting an additional minimisation; formulation parity unpinned, the solver
pinned against a direct solve)."""

import numpy as np
import pytest

from oracle.fitting import Fitting, dm_matrix, fit_pupil_mask, frame_fitted
from oracle.operators import System
from oracle.solver import State
from synthetic import get_config, random_vector


@pytest.fixture(scope="module")
def fit():
    return Fitting(get_config("small_fit"))


def test_pupil_corner_mask_hand_count():
    # 4x4 subapertures on D = 4: the 12 active ones cover all 25 corners but the 4 outer
    m = fit_pupil_mask(4.0, 4, 0.0)
    assert m.sum() == 21
    assert not m[0, 0] and not m[4, 4] and m[2, 2]


def test_dm_interpolation_reproduces_affine_commands():
    dm = {"h": 4000.0, "n_act": 13, "pitch": 0.8}
    B = dm_matrix(8.0, 20, (1e-5, -2e-5), dm)
    q = (np.arange(13) - 6) * 0.8
    X, Y = np.meshgrid(q, q)
    a = 0.3 + 0.2 * X - 0.7 * Y
    x = -4.0 + np.arange(21) * 0.4
    Xc, Yc = np.meshgrid(x + 4000.0 * 1e-5, x - 4000.0 * 2e-5)
    assert np.allclose(B @ a.ravel(), (0.3 + 0.2 * Xc - 0.7 * Yc).ravel(), atol=1e-12)


def test_normal_operator_symmetric_positive(fit):
    H = fit.H.toarray()
    assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() > 0.0


def test_cg_reaches_direct_least_squares(fit):
    phi = random_vector(sum(l["n"] ** 2 for l in fit.cfg["layers"]), 300, 0).astype(np.float64)
    ref = np.linalg.solve(fit.H.toarray(), fit.rhs(phi))
    # actuators outside every footprint only see eps: kappa ~ 1e7, so many iterations
    a = fit.solve(phi, iters=6000)
    assert np.linalg.norm(a - ref) <= 1e-8 * np.linalg.norm(ref)
    # the direct solution minimises sum_k |B_k a - P_k phi|^2 + eps |a|^2: gradient zero
    g = sum(B.T @ (B @ ref - P @ phi) for B, P in zip(fit.B, fit.P)) + fit.eps * ref
    assert np.linalg.norm(g) <= 1e-9 * np.linalg.norm(fit.rhs(phi))


def test_fitted_time_step_uses_fit(fit):
    cfg = fit.cfg
    S = System(cfg)
    st = State(S.geom.n_coeff, fit.n_act)
    s = random_vector(S.A.shape[0], 301, 0).astype(np.float64) * 0.1
    new, phi = frame_fitted(S, fit, st, s)
    assert np.allclose(new.a, fit.solve(phi))
    assert new.a.shape == (fit.n_act,)
