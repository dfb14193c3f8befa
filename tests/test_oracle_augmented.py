"""Pins of the oracle's augmented (deflated) PCG (Sec. 3.3; Algorithm 1's
augPCG line; Saad, Yeung, Erhel & Guyomarc'h 2000): the plain PCG without
directions, the orthogonality the projection maintains, convergence to the
dense Cholesky solution, the small factorisation with dropped directions,
and fewer-iteration accuracy on a frozen-flow sequence."""

import numpy as np
import scipy.linalg

from oracle.augmented import aug_pcg, factor, solve
from oracle.operators import System
from oracle.solver import State, frame, pcg
from synthetic import frozen_flow_frames, get_config, random_vector, slope_noise


def _slopes(S, k, key=21):
    true = next(frozen_flow_frames(S.cfg, 1, key, first=k))
    phi = np.concatenate([p.astype(np.float64).ravel() for p in true])
    return S.apply_A(phi) + slope_noise(S.geom.n_slopes, [w["sigma"] for w in S.cfg["wfs"]], key, k)


def _directions(S, b, n):
    """The search directions of a plain PCG run on b and their images."""
    rec = []
    pcg(S.apply_M, np.zeros_like(b), b, S.preconditioner(), n, record=rec)
    return rec, [S.apply_M(p) for p in rec]


def test_without_directions_it_is_the_plain_pcg(systems):
    S = systems("small")
    b = S.rhs(_slopes(S, 0))
    x0 = random_vector(len(b), 50).astype(np.float64) * 0.01
    r0 = b - S.apply_M(x0)
    x1, r1, h1 = pcg(S.apply_M, x0, r0, S.preconditioner(), 5)
    x2, r2, P, Q, h2 = aug_pcg(S.apply_M, x0, r0, S.preconditioner(), 5, [], [], 3)
    assert np.array_equal(x1, x2) and np.array_equal(r1, r2) and h1 == h2
    assert len(P) == 3 and all(np.array_equal(S.apply_M(p), q) for p, q in zip(P, Q))


def test_projection_keeps_residuals_orthogonal_to_the_directions(systems):
    # W^T r_j = 0 from the projected start on, and every new direction is
    # A-conjugate to W: (A W)^T p_j = 0 (deflated CG invariants)
    S = systems("small")
    P, Q = _directions(S, S.rhs(_slopes(S, 0)), 4)
    b = S.rhs(_slopes(S, 1))
    rec = []
    x, r, _, _, _ = aug_pcg(S.apply_M, np.zeros_like(b), b, S.preconditioner(), 4, P, Q, 4, record=rec)
    W = np.stack(P, axis=1)
    scale_r = np.linalg.norm(W, axis=0) * np.linalg.norm(b)
    for Wr, AWp in rec:
        assert np.all(np.abs(Wr) <= 1e-10 * scale_r)
    for _, AWp in rec:
        assert np.all(np.abs(AWp) <= 1e-9 * np.linalg.norm(np.stack(Q, axis=1), axis=0) * np.linalg.norm(b))
    # the recurrence residual is the true one
    assert np.linalg.norm(r - (b - S.apply_M(x))) <= 1e-10 * np.linalg.norm(b)


def test_converges_to_the_cholesky_solution(systems):
    S = systems("tiny")
    M = S.dense_M()
    P, Q = _directions(S, S.rhs(_slopes(S, 0)), 4)
    b = S.rhs(_slopes(S, 1))
    ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(M), b)
    x, r, _, _, _ = aug_pcg(S.apply_M, np.zeros_like(b), b, S.preconditioner(), 3000, P, Q, 4)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_small_factorisation_with_dropped_directions():
    g = np.random.default_rng(3)
    B = g.standard_normal((6, 4))
    G = B.T @ B + 0.1 * np.eye(4)
    L, keep = factor(G)
    assert keep.all() and np.allclose(L, np.linalg.cholesky(G), rtol=1e-14, atol=1e-14)
    v = g.standard_normal(4)
    assert np.allclose(solve(L, keep, v), np.linalg.solve(G, v), rtol=1e-12, atol=0)
    # a zero direction (an exactly converged previous step) is dropped; the
    # others solve their own block
    G2 = G.copy()
    G2[2, :] = 0.0
    G2[:, 2] = 0.0
    L2, keep2 = factor(G2)
    assert list(keep2) == [True, True, False, True]
    y = solve(L2, keep2, v)
    idx = [0, 1, 3]
    assert y[2] == 0.0 and np.allclose(y[idx], np.linalg.solve(G2[np.ix_(idx, idx)], v[idx]), rtol=1e-12)


def test_fewer_iterations_on_a_frozen_flow_sequence(systems):
    # Sec. 3.3: reusing the previous step's directions lowers the error after
    # a fixed small number of iterations; 2 warm-started iterations per frame
    # on 12 consecutive frames, error in the M-norm against the exact MAP
    # solution of each frame
    S = systems("small")
    Sa = System(get_config("small", augment=2))
    J = S.preconditioner()
    Sa._J = J  # the same system: the same preconditioner
    n = S.geom.n_coeff
    chol = scipy.linalg.cho_factor(S.dense_M())  # M does not change between frames
    plain, aug = State(n, n), State(n, n, 2)
    ep, ea = [], []
    for k in range(12):
        s = _slopes(S, k)
        cstar = scipy.linalg.cho_solve(chol, S.rhs(s))
        plain, _ = frame(S, plain, s, iters=2)
        aug, _ = frame(Sa, aug, s, iters=2)
        err = lambda c: np.sqrt((c - cstar) @ S.apply_M(c - cstar)) / np.sqrt(cstar @ S.apply_M(cstar))
        ep.append(err(plain.c))
        ea.append(err(aug.c))
    print("\nM-norm error, plain:", np.round(ep, 4), "\naugmented:", np.round(ea, 4))
    assert np.mean(ea[3:]) < np.mean(ep[3:])
    # the state carries the step's directions for the next one
    assert len(aug.P) == 2 and np.allclose(S.apply_M(aug.P[1]), aug.Q[1], rtol=1e-12)
    v = aug.pack()
    assert len(v) == 5 * n + 4 * n + 4 and v[-4] == 2.0
    back = State.unpack(v, n, n, 2)
    assert all(np.array_equal(a, b2) for a, b2 in zip(back.P + back.Q, aug.P + aug.Q))
