"""Pins of the oracle's wavelet transform (Sec. 3.1: periodic orthonormal
Daubechies-3, W orthogonal so W^{-1} = W^T)."""

import os

import numpy as np
import pytest

from oracle.wavelet import (analysis_matrix_1d, daubechies_filter, dwt2, dwt2_matrix,
                            highpass, idwt2, level_index)

GOLD = os.path.join(os.path.dirname(__file__), "golden", "db3_filter.txt")


def _golden():
    return np.array([float(x) for x in open(GOLD) if x.strip() and not x.startswith("#")])


def test_db3_matches_published_table():
    h = daubechies_filter(3)
    assert np.allclose(h, _golden(), atol=4e-15, rtol=0)


def test_db3_matches_closed_form():
    # Daubechies' closed form for N = 3 in radicals (sqrt 10, sqrt(5 + 2 sqrt 10))
    a = np.sqrt(10.0)
    b = np.sqrt(5.0 + 2.0 * a)
    ref = np.sqrt(2.0) / 32.0 * np.array([1 + a + b, 5 + a + 3 * b, 10 - 2 * a + 2 * b,
                                         10 - 2 * a - 2 * b, 5 + a - 3 * b, 1 + a - b])
    assert np.allclose(daubechies_filter(3), ref, atol=1e-14, rtol=0)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_daubechies_defining_conditions(N):
    h = daubechies_filter(N)
    L = len(h)
    assert L == 2 * N
    assert abs(h.sum() - np.sqrt(2.0)) < 1e-13
    for m in range(N):
        s = sum(h[k] * h[k + 2 * m] for k in range(L - 2 * m))
        assert abs(s - (1.0 if m == 0 else 0.0)) < 1e-13
    k = np.arange(L)
    for p in range(N):
        assert abs(np.sum((-1.0) ** k * k ** p * h)) < 1e-11


def test_db3_is_minimum_phase():
    # the extremal-phase solution front-loads the energy: every partial energy
    # sum dominates that of the other spectral factor (the reversed filter)
    h = daubechies_filter(3)
    e, er = np.cumsum(h * h), np.cumsum(h[::-1] ** 2)
    assert np.all(e[:-1] >= er[:-1] - 1e-15)
    assert e[0] > er[0]


def test_haar_special_case():
    h = daubechies_filter(1)
    assert np.allclose(h, [1 / np.sqrt(2), 1 / np.sqrt(2)])
    s = 1 / np.sqrt(2)
    ref = np.array([[s, s, 0, 0], [0, 0, s, s], [s, -s, 0, 0], [0, 0, s, -s]])
    assert np.allclose(analysis_matrix_1d(4, h), ref)


@pytest.mark.parametrize("m", [2, 4, 6, 8, 16, 64])
def test_1d_periodic_transform_orthogonal(m):
    A = analysis_matrix_1d(m, daubechies_filter(3))
    assert np.abs(A @ A.T - np.eye(m)).max() < 1e-14


@pytest.mark.parametrize("n,levels", [(16, 4), (32, 3), (32, 5)])
def test_W_orthogonal(n, levels):
    W = dwt2_matrix(n, levels, daubechies_filter(3)).toarray()
    assert np.abs(W @ W.T - np.eye(n * n)).max() < 1e-13


def test_constant_field_maps_to_LL_only():
    n, lev = 64, 5
    c = dwt2(np.full((n, n), 3.0), lev, daubechies_filter(3))
    m = n >> lev
    assert np.allclose(c[:m, :m], 3.0 * 2 ** lev, atol=1e-12)
    c[:m, :m] = 0.0
    assert np.abs(c).max() < 1e-12


def test_quadratic_details_vanish_in_interior():
    # 3 vanishing moments: level-1 details of a quadratic vanish wherever the
    # 6-tap window does not wrap around the periodic boundary
    h = daubechies_filter(3)
    n = 32
    p, q = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    x = 0.3 + 0.7 * q - 0.05 * q * q + 0.2 * p + 0.01 * p * q
    c = dwt2(x, 1, h)
    k_ok = (2 * np.arange(n // 2) + 5) < n
    # x-detail quadrant: rows [0, n/2), cols [n/2, n); interior in both axes
    d = c[: n // 2, n // 2:][np.ix_(k_ok, k_ok)]
    assert np.abs(d).max() < 1e-9
    d = c[n // 2:, n // 2:][np.ix_(k_ok, k_ok)]
    assert np.abs(d).max() < 1e-9


def test_inverse_and_matrix_forms_agree():
    h = daubechies_filter(3)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((32, 32))
    c = dwt2(x, 3, h)
    assert np.abs(idwt2(c, 3, h) - x).max() < 1e-13
    W = dwt2_matrix(32, 3, h)
    assert np.abs(W @ x.ravel() - c.ravel()).max() < 1e-13
    assert np.abs(W.T @ c.ravel() - x.ravel()).max() < 1e-13


def test_highpass_relation():
    h = daubechies_filter(3)
    g = highpass(h)
    assert abs(g.sum()) < 1e-14
    assert abs(h @ g) < 1e-14


def test_level_index_blocks():
    j = level_index(32, 3)
    assert j[0, 0] == 2 and j[3, 3] == 2       # LL block 4x4 -> j = 5 - 3
    assert j[0, 4] == 2 and j[7, 7] == 2       # coarsest detail block size 4
    assert j[0, 8] == 3 and j[15, 0] == 3      # block size 8
    assert j[16, 31] == 4 and j[31, 0] == 4    # finest block size 16
