"""Explicit operators of the FEWHA system (Sec. 2, Sec. 3.1-3.3).

* Gamma_g (Sec. 2, Shack-Hartmann model): average slope of the bilinear
  wavefront over each active subaperture,
      s^x_ij = ((v_{i,j+1} - v_{i,j}) + (v_{i+1,j+1} - v_{i+1,j})) / 2
      s^y_ij = ((v_{i+1,j} - v_{i,j}) + (v_{i+1,j+1} - v_{i,j+1})) / 2
  (second term of s^y read as the symmetric partner of s^x's), stacked
  s = [s^x over the mask, row-major; s^y in the same order].
* P_g (Sec. 2, NGS and LGS propagation): v_g(x) = sum_l phi_l(c_gl x + h_l theta_g)
  with c_gl = 1 - h_l/H for a laser guide star at altitude H and 1 for a
  natural guide star; phi_l is the bilinear interpolant of the layer nodes.
* A = [Gamma_g P_gl] (eq. atmo).
* C_g (eq. NGS-noise, eq. LGS-noise): sigma^2 I (sigma^2 = 1/n_photons when
  the photon count is given), or 2x2 blocks
  sigma^2 (I + alpha_eta^2/f^2 beta beta^T) with the elongation
  beta = FWHM/H^2 (midpoint - launch) per subaperture.
* C_hat_g^{-1} = (I - T) C_g^{-1} (I - T) for laser guide stars, T the
  orthogonal projector onto t^x = (e, 0), t^y = (0, e) (Sec. 3.2).
* M = W^{-T} A^T C_hat^{-1} A W^{-1} + alpha D, b = W^{-T} A^T C_hat^{-1} s
  (eq. fewha, eq. M), with W = diag(delta_l W).
* J = diag(W^{-T} A^T C_hat^{-1} A W^{-1}) + alpha max(D, tau) (eq. precond).
"""

import numpy as np
import scipy.sparse as sp

from .geometry import Geometry, corners_1d, subap_centres
from .wavelet import daubechies_filter, dwt2, dwt2_matrix, idwt2, level_index


class GeometryError(ValueError):
    pass


def gamma_matrix(N, mask):
    """Sparse Gamma of one sensor: (2|M|) x (N+1)^2."""
    act = np.argwhere(mask)  # row-major (i, j)
    nM = len(act)
    nc = N + 1
    rows, cols, vals = [], [], []

    def put(r, i, j, v):
        rows.append(r)
        cols.append(i * nc + j)
        vals.append(v)

    for k, (i, j) in enumerate(act):
        put(k, i, j + 1, 0.5)
        put(k, i, j, -0.5)
        put(k, i + 1, j + 1, 0.5)
        put(k, i + 1, j, -0.5)
        put(nM + k, i + 1, j, 0.5)
        put(nM + k, i, j, -0.5)
        put(nM + k, i + 1, j + 1, 0.5)
        put(nM + k, i, j + 1, -0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nM, nc * nc))


def propagation_matrix(D, wfs, layer, L):
    """Sparse P_gl: (N+1)^2 x n^2, bilinear interpolation of the layer nodes
    at the sensor's corner positions traced through the layer."""
    N = wfs["n_subap"]
    n = layer["n"]
    delta = L / n
    h = layer["h"]
    scale = 1.0 - h / wfs["H"] if wfs["kind"] == "lgs" else 1.0
    x = corners_1d(D, N)
    tx = (scale * x + h * wfs["theta"][0] + 0.5 * L) / delta
    ty = (scale * x + h * wfs["theta"][1] + 0.5 * L) / delta
    qx = np.floor(tx).astype(int)
    qy = np.floor(ty).astype(int)
    if qx.min() < 0 or qy.min() < 0 or qx.max() > n - 2 or qy.max() > n - 2:
        raise GeometryError("sensor footprint leaves the layer domain")
    wx = tx - qx
    wy = ty - qy
    nc = N + 1
    rows, cols, vals = [], [], []
    for i in range(nc):
        for j in range(nc):
            r = i * nc + j
            for di, fy in ((0, 1.0 - wy[i]), (1, wy[i])):
                for dj, fx in ((0, 1.0 - wx[j]), (1, wx[j])):
                    rows.append(r)
                    cols.append((qy[i] + di) * n + (qx[j] + dj))
                    vals.append(fy * fx)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc * nc, n * n))


def noise_variance(w):
    """Variance of one slope measurement of sensor w: 1 / n_photons when the
    sensor states its photon count per subaperture and frame (eq. NGS-noise,
    eq. LGS-noise), else sigma^2."""
    if w.get("photons") is not None:
        return 1.0 / float(w["photons"])
    return float(w["sigma"]) ** 2


def noise_blocks(cfg, geom, g):
    """Per active subaperture the 2x2 covariance C_ij (rows = (x, y))."""
    w = cfg["wfs"][g]
    mask = geom.masks[g]
    s2 = noise_variance(w)
    nM = int(mask.sum())
    C = np.zeros((nM, 2, 2))
    C[:, 0, 0] = s2
    C[:, 1, 1] = s2
    ae = cfg["noise"]["alpha_eta"]
    if w["kind"] == "lgs" and ae > 0.0:
        X, Y = subap_centres(cfg["D"], w["n_subap"])
        fw = cfg["noise"]["na_fwhm"]
        H = w["H"]
        bx = fw / (H * H) * (X[mask] - w["launch"][0])
        by = fw / (H * H) * (Y[mask] - w["launch"][1])
        k = ae * ae / (cfg["noise"]["spot_fwhm"] ** 2)
        C[:, 0, 0] += s2 * k * bx * bx
        C[:, 0, 1] += s2 * k * bx * by
        C[:, 1, 0] += s2 * k * bx * by
        C[:, 1, 1] += s2 * k * by * by
    return C


def noise_inverse_matrix(cfg, geom, g):
    """Sparse C_g^{-1} (2|M| x 2|M|), blocks pairing slope k with |M| + k,
    each block inverted with numpy.linalg.inv."""
    C = noise_blocks(cfg, geom, g)
    nM = C.shape[0]
    Ci = np.linalg.inv(C)
    k = np.arange(nM)
    rows = np.concatenate([k, k, nM + k, nM + k])
    cols = np.concatenate([k, nM + k, k, nM + k])
    vals = np.concatenate([Ci[:, 0, 0], Ci[:, 0, 1], Ci[:, 1, 0], Ci[:, 1, 1]])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(2 * nM, 2 * nM))
    M.eliminate_zeros()
    return M


def tt_vectors(nM):
    tx = np.concatenate([np.ones(nM), np.zeros(nM)])
    ty = np.concatenate([np.zeros(nM), np.ones(nM)])
    return tx, ty


def prior_diagonal(cfg, l):
    """D_l over the Mallat positions of layer l: the inverse von Karman
    spectrum 0.023 gamma_l r0^{-5/3} (f^2 + L0^{-2})^{-11/6} at the level
    frequency f_j = 2^j / L (the formula is not in the paper: the spectrum is
    pinned by turbulence statistics, the level frequency is parity unpinned)."""
    layer = cfg["layers"][l]
    pr = cfg["prior"]
    j = level_index(layer["n"], layer["levels"])
    f = (2.0 ** j) / cfg["domain_side"]
    psd = 0.023 * layer["cn2"] * pr["r0"] ** (-5.0 / 3.0) * (f * f + pr["L0"] ** -2.0) ** (-11.0 / 6.0)
    return (1.0 / psd).ravel()


class System:
    """The FEWHA system of one configuration in float64."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.geom = Geometry(cfg)
        g = self.geom
        self.h = daubechies_filter(3)
        self.G = len(cfg["wfs"])
        self.Lc = len(cfg["layers"])
        self.Gam = [gamma_matrix(w["n_subap"], m) for w, m in zip(cfg["wfs"], g.masks)]
        self.P = [[propagation_matrix(cfg["D"], w, l, g.L) for l in cfg["layers"]] for w in cfg["wfs"]]
        self.A_blocks = [[(self.Gam[gi] @ self.P[gi][li]).tocsr() for li in range(self.Lc)]
                         for gi in range(self.G)]
        self.A = sp.bmat(self.A_blocks, format="csr")
        self.Cinv = [noise_inverse_matrix(cfg, g, gi) for gi in range(self.G)]
        self.tt = [cfg["wfs"][gi]["kind"] == "lgs" and cfg["wfs"][gi]["tt_removal"] for gi in range(self.G)]
        self.D = np.concatenate([prior_diagonal(cfg, l) for l in range(self.Lc)])
        self._J = None

    # ---- building blocks ------------------------------------------------
    def split_layers(self, v):
        o = self.geom.layer_off
        return [v[o[l]:o[l + 1]].reshape(n, n) for l, n in enumerate(self.geom.layer_n)]

    def split_slopes(self, s):
        o = self.geom.slope_off
        return [s[o[g]:o[g + 1]] for g in range(self.G)]

    def apply_A(self, phi):
        """s = A phi (finite-element layer domain -> slopes)."""
        return self.A @ np.asarray(phi, dtype=np.float64)

    def apply_AT(self, s):
        return self.A.T @ np.asarray(s, dtype=np.float64)

    def apply_Chat_inv(self, s):
        """C_hat^{-1} s, block by block: (I-T) C^{-1} (I-T) for LGS with tip/tilt
        removal, C^{-1} otherwise."""
        out = []
        for gi, sg in enumerate(self.split_slopes(np.asarray(s, dtype=np.float64))):
            if self.tt[gi]:
                nM = len(sg) // 2
                tx, ty = tt_vectors(nM)
                y = sg - tx * (tx @ sg) / nM - ty * (ty @ sg) / nM
                y = self.Cinv[gi] @ y
                y = y - tx * (tx @ y) / nM - ty * (ty @ y) / nM
            else:
                y = self.Cinv[gi] @ sg
            out.append(y)
        return np.concatenate(out)

    def W_inv(self, c):
        """phi_l = delta_l^{-1} W^T c_l for every layer."""
        out = []
        for l, cl in enumerate(self.split_layers(np.asarray(c, dtype=np.float64))):
            lev = self.cfg["layers"][l]["levels"]
            out.append((idwt2(cl, lev, self.h) / self.geom.delta[l]).ravel())
        return np.concatenate(out)

    def W_invT(self, phi):
        """c_l = delta_l^{-1} W phi_l for every layer (the action of W^{-T})."""
        out = []
        for l, pl in enumerate(self.split_layers(np.asarray(phi, dtype=np.float64))):
            lev = self.cfg["layers"][l]["levels"]
            out.append((dwt2(pl, lev, self.h) / self.geom.delta[l]).ravel())
        return np.concatenate(out)

    # ---- system -----------------------------------------------------------
    def apply_M(self, c):
        alpha = self.cfg["prior"]["alpha"]
        phi = self.W_inv(c)
        y = self.apply_Chat_inv(self.apply_A(phi))
        return self.W_invT(self.apply_AT(y)) + alpha * self.D * np.asarray(c, dtype=np.float64)

    def rhs(self, s):
        return self.W_invT(self.apply_AT(self.apply_Chat_inv(s)))

    def Chat_inv_matrix(self, gi):
        """Dense-free C_hat_g^{-1} as a sparse matrix plus rank-2 terms, returned
        as a dense matrix (small sensors only)."""
        Ci = self.Cinv[gi].toarray()
        if not self.tt[gi]:
            return Ci
        nM = Ci.shape[0] // 2
        tx, ty = tt_vectors(nM)
        T = (np.outer(tx, tx) + np.outer(ty, ty)) / nM
        I = np.eye(2 * nM)
        return (I - T) @ Ci @ (I - T)

    def dense_M(self):
        """Explicit M (small configurations only)."""
        n = self.geom.n_coeff
        Winv = np.zeros((n, n))
        o = self.geom.layer_off
        for l, nl in enumerate(self.geom.layer_n):
            Wl = dwt2_matrix(nl, self.cfg["layers"][l]["levels"], self.h).toarray()
            Winv[o[l]:o[l + 1], o[l]:o[l + 1]] = Wl.T / self.geom.delta[l]
        A = self.A.toarray()
        Ch = np.zeros((A.shape[0], A.shape[0]))
        so = self.geom.slope_off
        for gi in range(self.G):
            Ch[so[gi]:so[gi + 1], so[gi]:so[gi + 1]] = self.Chat_inv_matrix(gi)
        AW = A @ Winv
        return AW.T @ Ch @ AW + self.cfg["prior"]["alpha"] * np.diag(self.D)

    def data_diagonal(self):
        """diag(W^{-T} A^T C_hat^{-1} A W^{-1}) from explicit sparse W: for each
        layer and sensor, Z = Gamma_g P_gl W_l^T / delta_l holds in column k the
        slopes of basis function k; the diagonal is the column-wise quadratic
        form with C_hat_g^{-1} = C^{-1} - U U^T C^{-1} - C^{-1} U U^T
        + U (U^T C^{-1} U) U^T, U = [t^x t^y] / sqrt|M|."""
        out = []
        for l, nl in enumerate(self.geom.layer_n):
            Wl = dwt2_matrix(nl, self.cfg["layers"][l]["levels"], self.h)
            WT = (Wl.T / self.geom.delta[l]).tocsc()
            acc = np.zeros(nl * nl)
            for gi in range(self.G):
                Z = (self.A_blocks[gi][l] @ WT).tocsc()
                CZ = (self.Cinv[gi] @ Z).tocsc()
                acc += np.asarray(Z.multiply(CZ).sum(axis=0)).ravel()
                if self.tt[gi]:
                    nM = Z.shape[0] // 2
                    tx, ty = tt_vectors(nM)
                    U = np.stack([tx, ty], axis=1) / np.sqrt(nM)
                    UZ = np.asarray((Z.T @ U)).T          # 2 x n
                    UCZ = np.asarray((CZ.T @ U)).T        # 2 x n
                    UCU = U.T @ (self.Cinv[gi] @ U)
                    acc -= 2.0 * np.sum(UZ * UCZ, axis=0)
                    acc += np.sum(UZ * (UCU @ UZ), axis=0)
            out.append(acc)
        return np.concatenate(out)

    def preconditioner(self):
        """J of eq. (precond) (cached)."""
        if self._J is None:
            pr = self.cfg["prior"]
            self._J = self.data_diagonal() + pr["alpha"] * np.maximum(self.D, pr["tau"])
        return self._J
