"""Periodic orthonormal Daubechies wavelets (Sec. 3.1: periodic Daubechies-N
with N = 3, W orthogonal; the layer transform is delta_l W).

Conventions (stated readings):
* 1-D analysis of a length-m periodic signal:
      a_k = sum_i h_i x[(2k+i) mod m],   d_k = sum_i g_i x[(2k+i) mod m],
  with g_i = (-1)^i h_{L-1-i}; the output is stacked [a; d].
* 2-D level: the 1-D analysis along every row (x), then along every column
  (y), of the current top-left m x m block; Mallat layout.
"""

from math import comb

import numpy as np
import scipy.sparse as sp


def daubechies_filter(N=3):
    """Minimum-phase Daubechies lowpass filter with N vanishing moments
    (2N taps, sum = sqrt 2) by spectral factorisation of the Daubechies
    polynomial P(y) = sum_{k<N} C(N-1+k, k) y^k, y = sin^2(w/2)."""
    # P as a polynomial in y; numpy.roots wants the highest degree first
    py = [comb(N - 1 + k, k) for k in range(N)][::-1]
    yroots = np.roots(py) if N > 1 else np.array([])
    # y = (2 - z - 1/z)/4  <=>  z^2 - (2 - 4y) z + 1 = 0; keep the root with
    # |z| > 1 so that the filter's zeros in z^{-1} lie inside the unit circle
    zr = []
    for y in yroots:
        b = 2.0 - 4.0 * y
        cand = np.roots([1.0, -b, 1.0])
        zr.append(cand[np.argmax(np.abs(cand))])
    # m0(z) = ((1+z)/2)^N * prod (z - z_r)/(1 - z_r), polynomial in z, low degree first
    poly = np.array([1.0 + 0j])
    for _ in range(N):
        poly = np.convolve(poly, [0.5, 0.5])
    for z in zr:
        poly = np.convolve(poly, np.array([-z, 1.0]) / (1.0 - z))
    h = np.sqrt(2.0) * np.real(poly)
    return h


def highpass(h):
    L = len(h)
    return np.array([(-1) ** i * h[L - 1 - i] for i in range(L)])


def analysis_matrix_1d(m, h):
    """Dense m x m periodic analysis matrix, rows [a_0..a_{m/2-1}, d_0..]."""
    g = highpass(h)
    A = np.zeros((m, m))
    for k in range(m // 2):
        for i in range(len(h)):
            A[k, (2 * k + i) % m] += h[i]
            A[m // 2 + k, (2 * k + i) % m] += g[i]
    return A


def dwt2(x, levels, h):
    """Forward 2-D periodic DWT (the action of W) of an n x n array."""
    c = np.array(x, dtype=np.float64, copy=True)
    n = c.shape[0]
    m = n
    for _ in range(levels):
        A = analysis_matrix_1d(m, h)
        c[:m, :m] = A @ c[:m, :m] @ A.T
        m //= 2
    return c


def idwt2(c, levels, h):
    """Inverse 2-D periodic DWT (the action of W^T = W^{-1})."""
    x = np.array(c, dtype=np.float64, copy=True)
    n = x.shape[0]
    sizes = [n >> k for k in range(levels)][::-1]
    for m in sizes:
        A = analysis_matrix_1d(m, h)
        x[:m, :m] = A.T @ x[:m, :m] @ A
    return x


def level_matrix_2d(n, m, h):
    """Sparse n^2 x n^2 matrix of one 2-D analysis level on the top-left
    m x m block of a row-major n x n array (identity elsewhere)."""
    A = sp.csr_matrix(analysis_matrix_1d(m, h))
    K = sp.kron(A, A, format="coo")  # row-major block index r*m + c
    r_out, c_out = np.divmod(K.row, m)
    r_in, c_in = np.divmod(K.col, m)
    rows = r_out * n + c_out
    cols = r_in * n + c_in
    idx = np.arange(n * n).reshape(n, n)
    rest = idx.copy()
    rest[:m, :m] = -1
    rest = rest.ravel()
    rest = rest[rest >= 0]
    rows = np.concatenate([rows, rest])
    cols = np.concatenate([cols, rest])
    vals = np.concatenate([K.data, np.ones(len(rest))])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def dwt2_matrix(n, levels, h):
    """Explicit sparse W = W_levels ... W_1 for an n x n layer."""
    W = sp.identity(n * n, format="csr")
    m = n
    for _ in range(levels):
        W = level_matrix_2d(n, m, h) @ W
        m //= 2
    W.eliminate_zeros()
    return W.tocsr()


def level_index(n, levels):
    """Per Mallat position of an n x n array: the level exponent j with the
    coefficient's block side 2^j (detail blocks [2^j, 2^{j+1})); the coarse
    LL block gets j = log2(n) - levels."""
    J = int(round(np.log2(n)))
    jmin = J - levels
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m = np.maximum(r, c)
    j = np.full((n, n), jmin, dtype=np.int64)
    nz = m >= (1 << jmin)
    j[nz] = np.floor(np.log2(m[nz])).astype(np.int64)
    return j
