"""DM fitting when the reconstruction layers do not sit at the DM altitudes
(Sec. 4.1: with more layers than DMs the fitting becomes an additional
minimisation problem; the paper does not spell it out).

Reading used here (parity of the formulation with the paper is unpinned; the
solver is pinned against a direct solve):

* Fitting pupil: the corner grid of an N_fit x N_fit sensor on the telescope
  pupil (pitch D / N_fit); the evaluation points are the corners of the
  active subapertures (annulus rule), mask M.
* In each fitting direction theta_k the wavefront of the layers is
  P_k phi = sum_l phi_l(x + h_l theta_k) (no cone effect), that of the DMs
  B_k a = sum_m a_m(x + h_m theta_k), each DM a centred grid of n_act x n_act
  actuators with bilinear influence.
* Normal equations (sum_k B_k^T M B_k + eps I) a = sum_k B_k^T M P_k phi with
  eps = eps_rel * mean(diag(sum_k B_k^T M B_k)); solved by textbook CG from
  a = 0 for a fixed number of iterations.
"""

import numpy as np
import scipy.sparse as sp

from .geometry import corners_1d, subap_mask
from .operators import GeometryError, propagation_matrix


def fit_pupil_mask(D, N, obstruction):
    """Boolean (N+1) x (N+1) mask of the corners of active subapertures."""
    m = subap_mask(D, N, obstruction)
    c = np.zeros((N + 1, N + 1), dtype=bool)
    c[:-1, :-1] |= m
    c[1:, :-1] |= m
    c[:-1, 1:] |= m
    c[1:, 1:] |= m
    return c


def dm_matrix(D, N, theta, dm):
    """Sparse (N+1)^2 x n_act^2 bilinear interpolation of one DM at the
    corners x + h theta (actuator q at (q - (n_act - 1)/2) pitch)."""
    n = dm["n_act"]
    pitch = dm["pitch"]
    h = dm["h"]
    x = corners_1d(D, N)
    tx = (x + h * theta[0]) / pitch + 0.5 * (n - 1)
    ty = (x + h * theta[1]) / pitch + 0.5 * (n - 1)
    qx = np.floor(tx).astype(int)
    qy = np.floor(ty).astype(int)
    if qx.min() < 0 or qy.min() < 0 or qx.max() > n - 2 or qy.max() > n - 2:
        raise GeometryError("fitting footprint leaves a DM")
    wx = tx - qx
    wy = ty - qy
    nc = N + 1
    rows, cols, vals = [], [], []
    for i in range(nc):
        for j in range(nc):
            for di, fy in ((0, 1.0 - wy[i]), (1, wy[i])):
                for dj, fx in ((0, 1.0 - wx[j]), (1, wx[j])):
                    rows.append(i * nc + j)
                    cols.append((qy[i] + di) * n + (qx[j] + dj))
                    vals.append(fy * fx)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc * nc, n * n))


class Fitting:
    """The fitting operators of one configuration."""

    def __init__(self, cfg):
        self.cfg = cfg
        fit = cfg["fit"]
        D = cfg["D"]
        self.N = fit.get("n_subap", cfg["wfs"][0]["n_subap"])
        self.mask = fit_pupil_mask(D, self.N, cfg["obstruction"]).ravel()
        Mk = sp.diags(self.mask.astype(float))
        ngs = lambda th: {"kind": "ngs", "n_subap": self.N, "theta": th, "H": None}
        self.P = []   # layers -> pupil corners, per direction
        self.B = []   # DMs -> pupil corners, per direction
        for th in fit["directions"]:
            self.P.append(Mk @ sp.hstack([propagation_matrix(D, ngs(th), l, cfg["domain_side"])
                                          for l in cfg["layers"]]).tocsr())
            self.B.append(Mk @ sp.hstack([dm_matrix(D, self.N, th, dm) for dm in cfg["dms"]]).tocsr())
        self.n_act = sum(dm["n_act"] ** 2 for dm in cfg["dms"])
        H = sum((B.T @ B) for B in self.B)
        self.eps = fit["eps_rel"] * float(np.mean(H.diagonal()))
        self.H = (H + self.eps * sp.identity(self.n_act)).tocsr()

    def apply_H(self, a):
        return sum(B.T @ (B @ a) for B in self.B) + self.eps * a

    def rhs(self, phi):
        return sum(B.T @ (P @ phi) for B, P in zip(self.B, self.P))

    def solve(self, phi, iters=None):
        """Textbook CG from a = 0 for a fixed number of iterations."""
        iters = self.cfg["fit"]["iters"] if iters is None else iters
        b = self.rhs(np.asarray(phi, dtype=np.float64))
        a = np.zeros(self.n_act)
        r = b.copy()
        p = r.copy()
        rho = r @ r
        for _ in range(iters):
            q = self.apply_H(p)
            pi = p @ q
            al = rho / pi if pi > 0 else 0.0
            a += al * p
            r -= al * q
            rho_new = r @ r
            p = r + (rho_new / rho if rho > 0 else 0.0) * p
            rho = rho_new
        return a


def frame_fitted(system, fitting, state, s, iters=None, gain=None):
    """Algorithm 1 time step with the fitting step: a~ = fit(W^{-1} c)."""
    from .solver import State, pcg
    cfg = system.cfg
    iters = cfg["iters"] if iters is None else iters
    gain = cfg["gain"] if gain is None else gain
    b = system.rhs(s)
    r0 = (b - state.b) + state.r
    x, r, _ = pcg(system.apply_M, state.c, r0, system.preconditioner(), iters)
    phi = system.W_inv(x)
    at = fitting.solve(phi)
    new = State(len(x), len(state.a))
    new.c, new.b, new.r = x, b, r
    new.a_prev = state.a.copy()
    new.a = (1.0 - gain) * state.a + gain * at
    return new, phi
