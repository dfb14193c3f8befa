"""Gradients of a reconstruction-error loss with respect to the method's
parameters (alpha, the Cn2 layer weights gamma_l, the layer heights h_l),
through the exact MAP solution c* = M^{-1} b (eq. fewha).  Test
infrastructure only, like the rest of this package.  The implicit gradient is
pinned against central finite differences of the loss (the golden values in
tests/golden are written by a script that calls this package only).

Readings (the paper does not differentiate FEWHA; these are the stated
definitions of this workload):
* Loss L = (1/F) sum_frames sum_theta |Pi (P_theta(h) phi - P_theta(h_true) phi_true)|^2,
  phi = W^{-1} c*, P_theta the natural-guide-star propagation (no cone
  effect) onto the corners of the first sensor's subaperture grid, restricted
  to the corners of its active subapertures, Pi removing the mean over them,
  theta on a 5 x 5 grid of half-width cfg["science_half"] (default 60",
  a 2' field).
* At a sample position exactly on a grid line the bilinear interpolant has no
  derivative; its derivative is taken as the average of the two one-sided
  ones (what a central difference returns).
* D scales as 1/gamma_l; J does not enter the exact solution.

Implicit gradient: with lambda = M^{-1} W^{-T} dL/dphi, lambda_phi = W^{-1} lambda,
  dL/dalpha = -lambda^T D c
  dL/dgamma_l = alpha lambda_l^T D_l c_l / gamma_l
  dL/dh_l = <dA lambda_phi, C^{-1}(s - A phi)> - <C^{-1} A lambda_phi, dA phi> + dL/dh_l|explicit
with dA = dA/dh_l and C^{-1} the tip/tilt-filtered noise weighting.
"""

import copy

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fitting import fit_pupil_mask
from .geometry import corners_1d
from .operators import GeometryError, System
from synthetic import ARCSEC

TIE = 1e-9


def science_directions(cfg):
    """5 x 5 grid of directions, row-major in y then x (rad)."""
    hw = cfg.get("science_half", 60.0 * ARCSEC)
    g = [hw * k / 2.0 for k in (-2, -1, 0, 1, 2)]
    return [(x, y) for y in g for x in g]


def _axis_weights(t):
    """Cell index and fraction along one axis, with exact grid lines marked."""
    r = np.round(t)
    tie = np.abs(t - r) < TIE
    q0 = np.where(tie, r, np.floor(t)).astype(int)
    w = np.where(tie, 0.0, t - np.floor(t))
    return q0, w, tie


def sample_matrices(D, N, theta, layer, L, scale=1.0, dtdh=None):
    """Sparse bilinear sampling of one layer at the corners of an N x N grid
    traced to (scale x + h theta), and its derivative with respect to h (node
    units per metre along each axis given by dtdh = (d tx/dh, d ty/dh) per
    corner column / row)."""
    n = layer["n"]
    delta = L / n
    h = layer["h"]
    x = corners_1d(D, N)
    tx = (scale * x + h * theta[0] + 0.5 * L) / delta
    ty = (scale * x + h * theta[1] + 0.5 * L) / delta
    qx, wx, tiex = _axis_weights(tx)
    qy, wy, tiey = _axis_weights(ty)
    if min(qx.min(), qy.min()) < 1 or max(qx.max(), qy.max()) > n - 3:
        raise GeometryError("footprint too close to the layer edge for derivatives")
    nc = N + 1
    rows, cols, vals, drows, dcols, dvals = [], [], [], [], [], []
    dtx, dty = dtdh

    def put(r, p, q, v, lst):
        lst[0].append(r)
        lst[1].append(p * n + q)
        lst[2].append(v)

    F = (rows, cols, vals)
    G = (drows, dcols, dvals)
    for i in range(nc):
        for j in range(nc):
            r = i * nc + j
            for di, fy in ((0, 1.0 - wy[i]), (1, wy[i])):
                for dj, fx in ((0, 1.0 - wx[j]), (1, wx[j])):
                    put(r, qy[i] + di, qx[j] + dj, fy * fx, F)
            # d/dtx of the bilinear interpolant (average of both cells on a grid line)
            cells_x = [(qx[j] - 1, 0.5), (qx[j], 0.5)] if tiex[j] else [(qx[j], 1.0)]
            for (q, cw) in cells_x:
                for di, fy in ((0, 1.0 - wy[i]), (1, wy[i])):
                    put(r, qy[i] + di, q + 1, cw * fy * dtx[j], G)
                    put(r, qy[i] + di, q, -cw * fy * dtx[j], G)
            cells_y = [(qy[i] - 1, 0.5), (qy[i], 0.5)] if tiey[i] else [(qy[i], 1.0)]
            for (p, cw) in cells_y:
                for dj, fx in ((0, 1.0 - wx[j]), (1, wx[j])):
                    put(r, p + 1, qx[j] + dj, cw * fx * dty[i], G)
                    put(r, p, qx[j] + dj, -cw * fx * dty[i], G)
    S = sp.csr_matrix((vals, (rows, cols)), shape=(nc * nc, n * n))
    dS = sp.csr_matrix((dvals, (drows, dcols)), shape=(nc * nc, n * n))
    return S, dS


def with_params(cfg, alpha=None, cn2=None, heights=None):
    c = copy.deepcopy(cfg)
    if alpha is not None:
        c["prior"]["alpha"] = float(alpha)
    if cn2 is not None:
        for l, v in zip(c["layers"], cn2):
            l["cn2"] = float(v)
    if heights is not None:
        for l, v in zip(c["layers"], heights):
            l["h"] = float(v)
    return c


class Science:
    """Science-direction projections of the layers (for the loss)."""

    def __init__(self, cfg):
        self.D = cfg["D"]
        self.N = cfg["wfs"][0]["n_subap"]
        self.mask = fit_pupil_mask(self.D, self.N, cfg["obstruction"]).ravel()
        self.L = cfg["domain_side"]

    def project(self, cfg):
        """Per direction: (S_theta, [dS_theta/dh_l]) with S_theta the masked
        sampling of all layers (no cone effect)."""
        x = corners_1d(self.D, self.N)
        out = []
        Mk = sp.diags(self.mask.astype(float))
        for th in science_directions(cfg):
            Ss, dSs = [], []
            for layer in cfg["layers"]:
                n = layer["n"]
                delta = self.L / n
                dt = (np.full(self.N + 1, th[0] / delta), np.full(self.N + 1, th[1] / delta))
                S, dS = sample_matrices(self.D, self.N, th, layer, self.L, 1.0, dt)
                Ss.append(S)
                dSs.append(dS)
            out.append((Mk @ sp.hstack(Ss).tocsr(), [Mk @ d for d in dSs]))
        return out

    def centre(self, v):
        m = self.mask
        out = np.where(m, v, 0.0)
        out[m] -= out[m].mean()
        return out


def sensor_derivatives(system):
    """dA/dh_l as sparse matrices (slopes x layer nodes of layer l)."""
    cfg = system.cfg
    D, L = cfg["D"], cfg["domain_side"]
    out = []
    for li, layer in enumerate(cfg["layers"]):
        blocks = []
        for gi, w in enumerate(cfg["wfs"]):
            N = w["n_subap"]
            x = corners_1d(D, N)
            n = layer["n"]
            delta = L / n
            if w["kind"] == "lgs":
                scale = 1.0 - layer["h"] / w["H"]
                dtx = (-x / w["H"] + w["theta"][0]) / delta
                dty = (-x / w["H"] + w["theta"][1]) / delta
            else:
                scale = 1.0
                dtx = np.full(N + 1, w["theta"][0] / delta)
                dty = np.full(N + 1, w["theta"][1] / delta)
            _, dS = sample_matrices(D, N, w["theta"], layer, L, scale, (dtx, dty))
            blocks.append(system.Gam[gi] @ dS)
        out.append(sp.vstack(blocks).tocsr())
    return out


def exact_solve(system, b):
    """c* = M^{-1} b by dense Cholesky (small configurations; the factor is
    kept on the system)."""
    if getattr(system, "_chol", None) is None:
        system._chol = sla.cho_factor(system.dense_M())
    return sla.cho_solve(system._chol, b)


def frame_terms(sci, proj, proj_t, phi, phi_t, layer_off):
    """One frame's loss, dL/dphi and the explicit dL/dh_l (heights held in the
    science projections only)."""
    Lc = len(layer_off) - 1
    o = layer_off
    loss = 0.0
    g_phi = np.zeros_like(phi)
    g_h = np.zeros(Lc)
    for (P, dPs), (Pt, _) in zip(proj, proj_t):
        e = sci.centre(P @ phi - Pt @ phi_t)
        loss += e @ e
        g_phi += 2.0 * (P.T @ e)
        for l in range(Lc):
            g_h[l] += 2.0 * e @ (dPs[l] @ phi[o[l]:o[l + 1]])
    return loss, g_phi, g_h


def loss(cfg, frames, cfg_true):
    """L for parameters in cfg; frames = list of (slopes, phi_true) with
    phi_true on the layers of cfg_true."""
    S = System(cfg)
    sci = Science(cfg)
    proj = sci.project(cfg)
    proj_t = sci.project(cfg_true)
    tot = 0.0
    for s, phi_t in frames:
        c = exact_solve(S, S.rhs(s))
        tot += frame_terms(sci, proj, proj_t, S.W_inv(c), phi_t, S.geom.layer_off)[0]
    return tot / len(frames)


def fd_gradient(cfg, frames, cfg_true, rel_step=1e-4, h_step=0.01):
    """Central finite differences of L over (alpha, cn2, heights).  The height
    step is small because L has a kink in h wherever samples sit on grid lines
    (the ground layer): there a central difference is off by O(step)."""
    a0 = cfg["prior"]["alpha"]
    g0 = [l["cn2"] for l in cfg["layers"]]
    h0 = [l["h"] for l in cfg["layers"]]
    ga = (loss(with_params(cfg, alpha=a0 * (1 + rel_step)), frames, cfg_true)
          - loss(with_params(cfg, alpha=a0 * (1 - rel_step)), frames, cfg_true)) / (2 * a0 * rel_step)
    gg, gh = [], []
    for l in range(len(g0)):
        up, dn = list(g0), list(g0)
        up[l] *= 1 + rel_step
        dn[l] *= 1 - rel_step
        gg.append((loss(with_params(cfg, cn2=up), frames, cfg_true)
                   - loss(with_params(cfg, cn2=dn), frames, cfg_true)) / (2 * g0[l] * rel_step))
        up, dn = list(h0), list(h0)
        up[l] += h_step
        dn[l] -= h_step
        gh.append((loss(with_params(cfg, heights=up), frames, cfg_true)
                   - loss(with_params(cfg, heights=dn), frames, cfg_true)) / (2 * h_step))
    return ga, np.array(gg), np.array(gh)


def implicit_gradient(cfg, frames, cfg_true):
    """The implicit (adjoint) gradient in FP64 and per frame the pieces
    (c*, lambda, explicit dL/dh, the frame's share of the implicit g_alpha,
    g_cn2, g_h)."""
    S = System(cfg)
    sci = Science(cfg)
    proj = sci.project(cfg)
    proj_t = sci.project(cfg_true)
    dA = sensor_derivatives(S)
    Lc = S.Lc
    o = S.geom.layer_off
    ga, gg, gh = 0.0, np.zeros(Lc), np.zeros(Lc)
    pieces = []
    for s, phi_t in frames:
        c = exact_solve(S, S.rhs(s))
        phi = S.W_inv(c)
        _, g_phi, g_h_exp = frame_terms(sci, proj, proj_t, phi, phi_t, o)
        g_phi /= len(frames)
        g_h_exp /= len(frames)
        lam = exact_solve(S, S.W_invT(g_phi))
        fa, fg, fh = implicit_terms(S, dA, s, c, lam)
        ga += fa
        gg += fg
        gh += fh + g_h_exp
        pieces.append((c, lam, g_h_exp, fa, fg, fh))
    return ga, gg, gh, pieces


def implicit_terms(S, dA, s, c, lam):
    """The parameter gradient carried by c* = M^{-1} b(s) for a given adjoint
    lambda: (-lambda^T D c, alpha lambda_l^T D_l c_l / gamma_l,
    <dA_l W^{-1} lambda, C^{-1}(s - A phi)> - <C^{-1} A W^{-1} lambda, dA_l phi>)."""
    cfg = S.cfg
    o = S.geom.layer_off
    alpha = cfg["prior"]["alpha"]
    phi = S.W_inv(c)
    lam_phi = S.W_inv(lam)
    Dc = S.D * c
    ga = -(lam @ Dc)
    gg = np.array([alpha * (lam[o[l]:o[l + 1]] @ Dc[o[l]:o[l + 1]]) / cfg["layers"][l]["cn2"]
                   for l in range(S.Lc)])
    y1 = S.apply_Chat_inv(s - S.apply_A(phi))
    y2 = S.apply_Chat_inv(S.apply_A(lam_phi))
    gh = np.array([(dA[l] @ lam_phi[o[l]:o[l + 1]]) @ y1 - y2 @ (dA[l] @ phi[o[l]:o[l + 1]])
                   for l in range(S.Lc)])
    return ga, gg, gh
