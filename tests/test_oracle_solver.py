"""Pins of the oracle's PCG and time step (Sec. 3.3-3.4, Algorithm 1 open
loop): convergence to a dense Cholesky solve, M-conjugacy of the search
directions, the warm-restart residual identity, gain control."""

import numpy as np
import scipy.linalg as sla

from oracle.solver import State, frame, pcg, pcg_to_tolerance
from synthetic import frozen_flow_frames, slope_noise


def _slopes(S, k):
    phi = frozen_flow_frames(S.cfg, 1, 7, first=k)
    true = np.concatenate([p.astype(np.float64).ravel() for p in next(phi)])
    s = S.apply_A(true)
    sig = [w["sigma"] for w in S.cfg["wfs"]]
    return s + slope_noise(S.geom.n_slopes, sig, 7, k).astype(np.float64)


def test_pcg_reaches_cholesky_solution(systems):
    S = systems("tiny")
    M = S.dense_M()
    b = S.rhs(_slopes(S, 0))
    ref = sla.cho_solve(sla.cho_factor(M), b)
    # the preconditioned system is ill-conditioned (kappa ~ 1e5): a few
    # thousand iterations reach the direct solve
    x, r, _ = pcg(lambda p: M @ p, np.zeros_like(b), b, S.preconditioner(), 3500)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    x2, it = pcg_to_tolerance(S.apply_M, b, S.preconditioner(), rtol=1e-14, max_iters=20000)
    assert np.linalg.norm(x2 - ref) <= 1e-10 * np.linalg.norm(ref)


def test_search_directions_M_conjugate(systems):
    S = systems("small")
    M = S.dense_M()
    b = S.rhs(_slopes(S, 0))
    dirs = []
    pcg(S.apply_M, np.zeros_like(b), b, S.preconditioner(), 6, record=dirs)
    P = np.stack(dirs, 1)
    G = P.T @ M @ P
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() <= 1e-9 * np.abs(np.diag(G)).max()


def test_error_decreases_in_M_norm(systems):
    S = systems("tiny")
    M = S.dense_M()
    b = S.rhs(_slopes(S, 0))
    ref = sla.cho_solve(sla.cho_factor(M), b)
    errs = []
    for k in range(8):
        x, _, _ = pcg(S.apply_M, np.zeros_like(b), b, S.preconditioner(), k)
        e = x - ref
        errs.append(e @ M @ e)
    assert all(b2 < a2 for a2, b2 in zip(errs[:-1], errs[1:]))


def test_zero_iterations_is_identity(systems):
    S = systems("tiny")
    b = S.rhs(_slopes(S, 0))
    x0 = np.arange(len(b), dtype=float)
    x, r, _ = pcg(S.apply_M, x0, b, S.preconditioner(), 0)
    assert np.array_equal(x, x0) and np.array_equal(r, b)


def test_warm_restart_residual_identity(systems):
    # r0 = (b^(i+1) - b^(i)) + r^(i) equals b^(i+1) - M c^(i) when r^(i) is the
    # exact residual of the previous step (Algorithm 1, residual line)
    S = systems("small")
    st = State(S.geom.n_coeff, S.geom.n_coeff)
    for k in range(4):
        st, _ = frame(S, st, _slopes(S, k))
        true_r = st.b - S.apply_M(st.c)
        assert np.linalg.norm(st.r - true_r) <= 1e-10 * np.linalg.norm(st.b)


def test_first_frame_from_zero_state(systems):
    S = systems("tiny")
    s = _slopes(S, 0)
    st0 = State(S.geom.n_coeff, S.geom.n_coeff)
    st1, phi = frame(S, st0, s)
    b = S.rhs(s)
    x, r, _ = pcg(S.apply_M, np.zeros_like(b), b, S.preconditioner(), S.cfg["iters"])
    assert np.allclose(st1.c, x) and np.allclose(st1.r, r) and np.allclose(st1.b, b)
    assert np.allclose(phi, S.W_inv(x))
    assert np.allclose(st1.a, phi)  # gain 1, F = I


def test_gain_blend_and_history(systems):
    S = systems("tiny")
    st = State(S.geom.n_coeff, S.geom.n_coeff)
    st.a = np.ones(S.geom.n_coeff)
    st2, phi = frame(S, st, _slopes(S, 0), gain=0.25)
    assert np.allclose(st2.a, 0.75 * 1.0 + 0.25 * phi)
    assert np.array_equal(st2.a_prev, st.a)
    v = st2.pack()
    st3 = State.unpack(v, S.geom.n_coeff, S.geom.n_coeff)
    assert np.array_equal(st3.pack(), v)


def test_pcg_stops_at_an_exact_solution():
    # M diagonal with power-of-two entries and J = diag(M): the first step is
    # exact (z = M^{-1} r, alpha = 1, x1 = M^{-1} b, r1 = 0 with no rounding),
    # so the later steps meet p = 0, p^T M p = 0 and rho = 0; CG must keep the
    # exact solution M^{-1} b rather than divide 0 by 0
    d = 2.0 ** np.arange(-3, 5)
    b = np.linspace(-1.0, 2.0, len(d))
    x, r, hist = pcg(lambda v: d * v, np.zeros_like(b), b, d, 4)
    assert np.array_equal(x, b / d)
    assert np.array_equal(r, np.zeros_like(b))
    assert hist[1] == (0.0, 0.0) and all(np.isfinite(v).all() for v in (x, r))


def test_zero_right_hand_side_gives_zero(systems):
    # M c = 0 has the unique solution c = 0 (M is positive definite): a frame
    # with zero slopes from the zero state stays exactly zero
    S = systems("small")
    st = State(S.geom.n_coeff, S.geom.n_coeff)
    st1, phi = frame(S, st, np.zeros(S.A.shape[0]), iters=4)
    assert not np.any(st1.pack()) and not np.any(phi)


def test_true_residual_restart_agrees_with_the_recurrence(systems):
    # Algorithm 1's r0 = (b^(i+1) - b^(i)) + r^(i) equals b^(i+1) - M c^(i) when
    # r^(i) is the previous step's residual: a restarted step is the same step
    S = systems("small")
    st = State(S.geom.n_coeff, S.geom.n_coeff)
    for k in range(3):
        st, _ = frame(S, st, _slopes(S, k))
    a, pa = frame(S, st, _slopes(S, 3))
    b, pb = frame(S, st, _slopes(S, 3), refresh=True)
    for u, v in ((a.c, b.c), (a.r, b.r), (pa, pb)):
        assert np.linalg.norm(u - v) <= 1e-9 * np.linalg.norm(u)
