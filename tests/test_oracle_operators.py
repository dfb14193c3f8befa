"""Pins of the oracle's operators: Shack-Hartmann Gamma and propagation P
(Sec. 2), noise weighting with tip/tilt removal (eq. NGS-noise, eq. LGS-noise,
Sec. 3.2), prior D and system M, J (eq. fewha, eq. M, eq. precond)."""

import numpy as np
import pytest

from oracle.geometry import corners_1d, subap_mask
from oracle.operators import (GeometryError, System, gamma_matrix, noise_blocks,
                              propagation_matrix, tt_vectors)
from synthetic import ARCSEC, get_config


def test_mask_hand_counts():
    # 4x4 subapertures on D = 4: centres at +-0.5, +-1.5; the four corner
    # subapertures (r = 2.12 > 2) are outside the pupil
    assert subap_mask(4.0, 4, 0.0).sum() == 12
    # obstruction area 1/4 -> r_in = 1: the four central ones (r = 0.71) go
    assert subap_mask(4.0, 4, 0.25).sum() == 8
    m = subap_mask(39.0, 80, 0.11)
    assert m.sum() == 4476
    assert np.array_equal(m, m.T) and np.array_equal(m, m[::-1]) and np.array_equal(m, m[:, ::-1])


def test_configured_mask_selects_subapertures():
    # a sensor's configured mask replaces the annulus rule (the set M_g of
    # Sec. 2): the annulus itself as a mask gives the same A, and a mask with
    # subapertures removed gives exactly the rows of the kept ones, in the
    # same row-major order, for s^x and s^y
    base = get_config("small")
    S0 = System(base)
    N = base["wfs"][0]["n_subap"]
    ann = subap_mask(base["D"], N, base["obstruction"])
    same = get_config("small")
    same["wfs"][0]["mask"] = ann.astype(np.uint8)
    assert (System(same).A != S0.A).nnz == 0
    m = ann.copy()
    m[3, :] = False          # a whole row
    m[10, 2:9] = False       # a gap: the row keeps two runs
    m[[5, 7, 14], [12, 4, 9]] = False
    cut = get_config("small")
    cut["wfs"][0]["mask"] = m.astype(np.uint8)
    S1 = System(cut)
    nM0, nM1 = int(ann.sum()), int(m.sum())
    assert S1.geom.n_active[0] == nM1 and S1.geom.slope_off[1] == 2 * nM1
    keep = m[ann]  # kept subapertures among the annulus's, row-major
    A0 = S0.A.tocsr()[:2 * nM0].toarray()
    A1 = S1.A.tocsr()[:2 * nM1].toarray()
    assert np.array_equal(A1[:nM1], A0[:nM0][keep])
    assert np.array_equal(A1[nM1:], A0[nM0:][keep])
    # the other sensors are untouched
    assert (S1.A.tocsr()[2 * nM1:] != S0.A.tocsr()[2 * nM0:]).nnz == 0


def _corner_field(N, D, f):
    x = corners_1d(D, N)
    X, Y = np.meshgrid(x, x)  # X along columns j, Y along rows i
    return f(X, Y).ravel()


def test_gamma_annihilates_piston():
    mask = subap_mask(8.0, 16, 0.11)
    G = gamma_matrix(16, mask)
    assert np.abs(G @ np.ones(17 * 17)).max() == 0.0


def test_gamma_tilt_exact():
    # a x + b y sampled at the corners gives s^x = a d, s^y = b d on every
    # active subaperture (this fixes the s^y stencil reading)
    D, N = 8.0, 16
    d = D / N
    mask = subap_mask(D, N, 0.11)
    G = gamma_matrix(N, mask)
    a, b = 0.37, -1.3
    s = G @ _corner_field(N, D, lambda X, Y: a * X + b * Y)
    nM = int(mask.sum())
    assert np.allclose(s[:nM], a * d, atol=1e-13)
    assert np.allclose(s[nM:], b * d, atol=1e-13)


def test_gamma_saddle_is_slope_average():
    # v = x y: the average over a subaperture of dv/dx = y is the centre's y
    D, N = 4.0, 4
    d = D / N
    mask = np.ones((N, N), dtype=bool)
    s = gamma_matrix(N, mask) @ _corner_field(N, D, lambda X, Y: X * Y)
    c = -0.5 * D + (np.arange(N) + 0.5) * d
    Xc, Yc = np.meshgrid(c, c)
    assert np.allclose(s[:N * N], (Yc * d).ravel())
    assert np.allclose(s[N * N:], (Xc * d).ravel())


def _layer_field(n, L, f):
    delta = L / n
    x = -0.5 * L + np.arange(n) * delta
    X, Y = np.meshgrid(x, x)
    return f(X, Y).ravel()


@pytest.mark.parametrize("kind,h", [("ngs", 0.0), ("ngs", 6000.0), ("lgs", 4000.0), ("lgs", 12700.0)])
def test_propagation_reproduces_affine_fields(kind, h):
    D, N, L, n = 8.0, 16, 16.0, 64
    w = {"kind": kind, "n_subap": N, "theta": (20 * ARCSEC, -35 * ARCSEC), "H": 90000.0}
    P = propagation_matrix(D, w, {"h": h, "n": n}, L)
    c0, cx, cy = 0.2, 0.7, -0.4
    v = P @ _layer_field(n, L, lambda X, Y: c0 + cx * X + cy * Y)
    s = 1.0 - h / 90000.0 if kind == "lgs" else 1.0
    x = corners_1d(D, N)
    X, Y = np.meshgrid(x, x)
    U = s * X + h * w["theta"][0]
    V = s * Y + h * w["theta"][1]
    assert np.allclose(v, (c0 + cx * U + cy * V).ravel(), atol=1e-12)
    assert np.allclose(P.sum(axis=1), 1.0)


def test_ngs_ground_layer_is_sampling():
    # d = delta and the corners on the layer grid: one weight 1 per row
    D, N, L, n = 8.0, 16, 16.0, 32
    w = {"kind": "ngs", "n_subap": N, "theta": (0.0, 0.0), "H": None}
    P = propagation_matrix(D, w, {"h": 0.0, "n": n}, L).toarray()
    assert np.allclose(P.max(axis=1), 1.0)
    assert np.allclose((P > 1e-12).sum(axis=1), 1)
    # corner (i, j) sits on node (8 + i, 8 + j)
    assert P[0 * 17 + 0, 8 * 32 + 8] == pytest.approx(1.0)
    assert P[16 * 17 + 3, 24 * 32 + 11] == pytest.approx(1.0)


def test_footprint_outside_domain_raises():
    w = {"kind": "ngs", "n_subap": 16, "theta": (200 * ARCSEC, 0.0), "H": None}
    with pytest.raises(GeometryError):
        propagation_matrix(8.0, w, {"h": 12000.0, "n": 32}, 16.0)


def test_cone_factor_on_layer_tilt(systems):
    # a layer tilt a*X at altitude h seen by an LGS gives s^x = a (1 - h/H) d
    S = systems("small")
    l = 2
    h = S.cfg["layers"][l]["h"]
    a = 0.9
    phi = [np.zeros(n * n) for n in S.geom.layer_n]
    phi[l] = _layer_field(S.geom.layer_n[l], S.geom.L, lambda X, Y: a * X)
    s = S.apply_A(np.concatenate(phi))
    for gi, w in enumerate(S.cfg["wfs"]):
        sg = S.split_slopes(s)[gi]
        nM = len(sg) // 2
        d = S.cfg["D"] / w["n_subap"]
        scale = 1.0 - h / w["H"] if w["kind"] == "lgs" else 1.0
        assert np.allclose(sg[:nM], a * scale * d, atol=1e-12)
        assert np.allclose(sg[nM:], 0.0, atol=1e-12)


def test_adjoint_pairs(systems):
    S = systems("small")
    rng = np.random.default_rng(1)
    x = rng.standard_normal(S.geom.n_coeff)
    y = rng.standard_normal(S.A.shape[0])
    assert abs(S.apply_A(x) @ y - x @ S.apply_AT(y)) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(y) * 10
    c = rng.standard_normal(S.geom.n_coeff)
    phi = rng.standard_normal(S.geom.n_coeff)
    lhs = S.W_inv(c) @ phi
    rhs = c @ S.W_invT(phi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-10
    u, v = rng.standard_normal(S.A.shape[0]), rng.standard_normal(S.A.shape[0])
    assert abs(S.apply_Chat_inv(u) @ v - u @ S.apply_Chat_inv(v)) < 1e-9


def test_W_inv_is_scaled_inverse(systems):
    S = systems("small")
    rng = np.random.default_rng(2)
    c = rng.standard_normal(S.geom.n_coeff)
    phi = S.W_inv(c)
    # W_l^{-1} = W^T / delta_l and W^{-T} = W / delta_l, so W^{-T}(W^{-1} c) = c / delta^2
    d2 = np.concatenate([np.full(n * n, dl * dl) for n, dl in zip(S.geom.layer_n, S.geom.delta)])
    assert np.allclose(S.W_invT(phi) * d2, c, atol=1e-12)


def test_tip_tilt_removed(systems):
    S = systems("small")
    for gi, on in enumerate(S.tt):
        nM = S.geom.n_active[gi]
        tx, ty = tt_vectors(nM)
        Ch = S.Chat_inv_matrix(gi)
        if on:
            assert np.abs(Ch @ tx).max() < 1e-10
            assert np.abs(Ch @ ty).max() < 1e-10
        assert np.allclose(Ch, Ch.T)
        assert np.linalg.eigvalsh(Ch).min() > -1e-9


def test_elongated_noise_blocks_sherman_morrison():
    cfg = get_config("small")
    cfg["noise"]["alpha_eta"] = 0.7
    S = System(cfg)
    g = 0
    C = noise_blocks(cfg, S.geom, g)
    sig2 = cfg["wfs"][g]["sigma"] ** 2
    # beta from the definition: FWHM/H^2 (midpoint - launch)
    D, N = cfg["D"], cfg["wfs"][g]["n_subap"]
    c = -0.5 * D + (np.arange(N) + 0.5) * (D / N)
    X, Y = np.meshgrid(c, c)
    m = S.geom.masks[g]
    w = cfg["wfs"][g]
    k = cfg["noise"]["na_fwhm"] / w["H"] ** 2
    beta = np.stack([k * (X[m] - w["launch"][0]), k * (Y[m] - w["launch"][1])], axis=1)
    kap = cfg["noise"]["alpha_eta"] ** 2 / cfg["noise"]["spot_fwhm"] ** 2
    # Sherman-Morrison: (s2 (I + kap b b^T))^{-1} = (I - kap b b^T / (1 + kap |b|^2)) / s2
    bb = np.einsum("ki,kj->kij", beta, beta)
    sm = (np.eye(2)[None] - kap * bb / (1.0 + kap * np.sum(beta * beta, axis=1))[:, None, None]) / sig2
    Ci = S.Cinv[g].toarray()
    nM = m.sum()
    got = np.stack([np.stack([np.diag(Ci[:nM, :nM]), np.diag(Ci[:nM, nM:])], 1),
                    np.stack([np.diag(Ci[nM:, :nM]), np.diag(Ci[nM:, nM:])], 1)], 1)
    assert np.allclose(got, sm, rtol=1e-12)
    assert np.allclose(np.linalg.inv(C), sm, rtol=1e-12)
    # the elongation stretches the covariance along beta only
    assert np.allclose(np.einsum("kij,kj->ki", C, beta),
                       sig2 * (1.0 + kap * np.sum(beta * beta, 1))[:, None] * beta)


def _prior_psd(f, r0, L0):
    # the oracle's spectrum at one frequency: a 2 x 2 layer with one level has
    # every coefficient at f = 1 / domain side, and D = 1 / psd there
    from oracle.operators import prior_diagonal
    cfg = {"layers": [{"n": 2, "levels": 1, "cn2": 1.0, "h": 0.0}],
           "prior": {"r0": r0, "L0": L0, "alpha": 1.0, "tau": 0.0}, "domain_side": 1.0 / f}
    return 1.0 / prior_diagonal(cfg, 0)[0]


def test_prior_scale_gives_the_kolmogorov_structure_function():
    # The absolute scale of the prior: the oracle's spectrum, sampled at many
    # level frequencies and integrated into the phase structure function
    # D(r) = 4 pi int (1 - J0(2 pi f r)) psd(f) f df, gives the Kolmogorov
    # 6.88 (r / r0)^(5/3) for r << L0 (a textbook constant, not the oracle's
    # formula): this pins the spectral constant and frequencies in cycles per
    # metre (an angular frequency would be off by (2 pi)^(5/3)).
    from scipy.special import j0
    r0 = 0.15
    f = np.logspace(-7, 5, 6001)
    psd = np.array([_prior_psd(x, r0, 1e6) for x in f])
    lnf = np.log(f)
    for r in (0.02, 0.05, 0.1):
        D = np.trapezoid(4 * np.pi * (1 - j0(2 * np.pi * f * r)) * psd * f * f, lnf)
        assert abs(D / (6.88 * (r / r0) ** (5.0 / 3.0)) - 1.0) < 5e-3


def test_prior_outer_scale_gives_the_von_karman_variance():
    # The L0 term: the phase variance int psd 2 pi f df of the oracle's
    # spectrum is the von Karman 0.0863 (L0 / r0)^(5/3) (textbook), for
    # outer scales from 10 to 100 m
    r0 = 0.157
    f = np.logspace(-7, 5, 6001)
    lnf = np.log(f)
    for L0 in (10.0, 25.0, 100.0):
        psd = np.array([_prior_psd(x, r0, L0) for x in f])
        var = np.trapezoid(2 * np.pi * psd * f * f, lnf)
        assert abs(var / (0.0863 * (L0 / r0) ** (5.0 / 3.0)) - 1.0) < 1e-2


def test_prior_level_ratio_kolmogorov_limit(systems):
    cfg = get_config("small")
    cfg["prior"]["L0"] = 1e12
    S = System(cfg)
    from oracle.wavelet import level_index
    for l, n in enumerate(S.geom.layer_n):
        Dl = S.split_layers(S.D)[l]
        j = level_index(n, cfg["layers"][l]["levels"])
        js = sorted(set(j.ravel()))
        vals = [Dl[j == jj] for jj in js]
        for v in vals:
            assert np.allclose(v, v[0], rtol=1e-14)
        for a, b in zip(vals[:-1], vals[1:]):
            assert b[0] / a[0] == pytest.approx(2.0 ** (11.0 / 3.0), rel=1e-9)
    # a weaker layer (smaller gamma) is regularised more: D proportional to 1/gamma
    cfg2 = get_config("small")
    cfg2["layers"][0]["cn2"] *= 0.5
    S2 = System(cfg2)
    assert np.allclose(S2.split_layers(S2.D)[0], 2.0 * systems("small").split_layers(systems("small").D)[0])


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_M_dense_symmetric_spd_and_matches_apply(systems, name):
    S = systems(name)
    M = S.dense_M()
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    rng = np.random.default_rng(3)
    c = rng.standard_normal(S.geom.n_coeff)
    assert np.allclose(M @ c, S.apply_M(c), rtol=1e-11, atol=1e-11 * np.abs(M @ c).max())


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_J_equals_diag_of_dense_M(systems, name):
    S = systems(name)
    J = S.preconditioner()
    dM = np.diag(S.dense_M())
    assert np.allclose(J, dM, rtol=1e-11, atol=0)


def test_J_with_elongation_equals_diag_of_dense_M():
    cfg = get_config("small")
    cfg["noise"]["alpha_eta"] = 0.5
    S = System(cfg)
    assert np.allclose(S.preconditioner(), np.diag(S.dense_M()), rtol=1e-11, atol=0)


def test_J_tau_threshold():
    cfg = get_config("small")
    cfg["prior"]["tau"] = 5.0
    S = System(cfg)
    cfg0 = get_config("small")
    S0 = System(cfg0)
    data = S0.preconditioner() - S0.D
    assert np.allclose(S.preconditioner(), data + np.maximum(S.D, 5.0), rtol=1e-12)


def test_data_diagonal_scales_with_the_noise_variance():
    # C_hat^{-1} = (I - T) sigma^{-2} (I - T) (or sigma^{-2} I) is linear in
    # sigma^{-2}, so the data part of J scales with it when every sensor has
    # the same diagonal noise
    from oracle.operators import System
    from synthetic import get_config
    cfg = get_config("small")
    for w in cfg["wfs"]:
        w["sigma"] = 1.0
    unit = System(cfg).data_diagonal()
    for w in cfg["wfs"]:
        w["sigma"] = 0.3
    assert np.allclose(System(cfg).data_diagonal(), unit / 0.09, rtol=1e-13, atol=0)
