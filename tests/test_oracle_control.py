"""Pins of the oracle's closed-loop time step (Algorithm 1, pseudo-open-loop
line with the two-step delay and the closed-loop control line) and of the
photon-count noise model (eq. NGS-noise, eq. LGS-noise)."""

import numpy as np

from oracle.operators import System, noise_variance
from oracle.solver import State, frame, pcg_to_tolerance
from synthetic import frozen_flow_frames, get_config, random_vector, slope_noise


def _truth(S, k, key=31):
    true = next(frozen_flow_frames(S.cfg, 1, key, first=k))
    return np.concatenate([p.astype(np.float64).ravel() for p in true])


def _noisy(S, phi, k, key=31):
    sig = [w["sigma"] for w in S.cfg["wfs"]]
    return S.apply_A(phi) + slope_noise(S.geom.n_slopes, sig, key, k)


def test_pseudo_open_loop_reproduces_the_open_loop_step(systems):
    # a closed-loop sensor sees the atmosphere minus the mirrors' shape of two
    # frames back, s_cl = s - A a^(i-1); adding the mirrors' response back
    # gives the open-loop slopes, so c, b and r of the step are those of the
    # open-loop step on s (the commands a^(i) must not enter: they are set
    # far from a^(i-1) here)
    S_open = systems("small")
    S_cl = System(get_config("small", loop="closed", gain=0.6))
    n = S_open.geom.n_coeff
    st = State(n, n)
    st.c = random_vector(n, 40, 0).astype(np.float64) * 0.1
    st.b = random_vector(n, 40, 1).astype(np.float64)
    st.r = random_vector(n, 40, 2).astype(np.float64) * 0.01
    st.a_prev = _truth(S_open, 0) * 0.8
    st.a = -2.0 * st.a_prev + 1.0
    s = _noisy(S_open, _truth(S_open, 1), 1)
    o, phi_o = frame(S_open, st, s)
    c, phi_c = frame(S_cl, st, s - S_open.apply_A(st.a_prev))
    for u, v in ((o.c, c.c), (o.b, c.b), (o.r, c.r), (phi_o, phi_c)):
        assert np.linalg.norm(u - v) <= 1e-12 * np.linalg.norm(u)
    assert np.array_equal(c.a_prev, st.a)


def test_closed_loop_integrator_with_two_step_delay(systems):
    # static atmosphere, no noise, solves converged every frame: the
    # pseudo-open-loop reconstruction is the same a* = W^{-1} M^{-1} b(A phi)
    # every frame, so the command error e_i = a^(i) - a* obeys the recurrence
    # of the delayed integrator e_{i+1} = e_i - gain e_{i-1} (from a = a_prev
    # = 0: e_{-1} = e_0 = -a*), which decays with |lambda|^2 = gain and
    # oscillates for gain > 1/4 (a controller on a^(i) instead of a^(i-1)
    # would decay monotonically by 1 - gain)
    S = System(get_config("tiny", loop="closed", gain=0.5))
    n = S.geom.n_coeff
    phi = _truth(S, 0)
    b = S.rhs(S.apply_A(phi))
    xs, _ = pcg_to_tolerance(S.apply_M, b, S.preconditioner(), rtol=1e-13)
    a_star = S.W_inv(xs)
    st = State(n, n)
    e_prev, e = -a_star, -a_star
    for i in range(12):
        s_cl = S.apply_A(phi) - S.apply_A(st.a_prev)
        st, _ = frame(S, st, s_cl, iters=3000 if i == 0 else 60)
        e_prev, e = e, e - 0.5 * e_prev
        assert np.linalg.norm((st.a - a_star) - e) <= 1e-6 * np.linalg.norm(a_star), i
    assert np.linalg.norm(st.a - a_star) <= 0.05 * np.linalg.norm(a_star)


def test_photon_count_noise_model():
    # sigma^2 = 1/n_photons for NGS and LGS (eq. NGS-noise, eq. LGS-noise): the
    # paper's highflux (10000 photons per subaperture and frame) and lowflux
    # (500) settings
    assert noise_variance({"photons": 10000, "sigma": 9.0}) == 1e-4
    assert noise_variance({"photons": 500, "sigma": 9.0}) == 1.0 / 500
    assert noise_variance({"sigma": 0.1}) == 0.1 ** 2
    cfg = get_config("tiny")
    cfg["wfs"][0]["photons"] = 500
    S = System(cfg)
    y = random_vector(S.geom.n_slopes[0], 41).astype(np.float64)
    assert np.allclose(S.apply_Chat_inv(y), 500.0 * y, rtol=1e-15, atol=0)
