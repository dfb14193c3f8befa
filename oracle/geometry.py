"""Pupil, sensor and layer grids (Sec. 2 and Sec. 3.1).

* Sensor g with N subapertures per side: pitch d = D/N, corners at
  x_j = -D/2 + j d, y_i = -D/2 + i d (i, j = 0..N); subaperture (i, j) spans
  corners (i..i+1, j..j+1); rows = y, columns = x, row-major.
* Active subaperture: its centre lies in the annulus [sqrt(obs) D/2, D/2]
  (obs = obstructed area fraction), unless the sensor's configuration gives
  its own N x N mask (the set M_g of the slope model is then that mask).
* Layer l: n_l x n_l nodes on a centred square of side L; delta_l = L/n_l;
  node (p, q) at (x, y) = (-L/2 + q delta_l, -L/2 + p delta_l).
"""

import numpy as np


def corners_1d(D, N):
    return -0.5 * D + np.arange(N + 1) * (D / N)


def subap_mask(D, N, obstruction):
    """Boolean N x N mask of active subapertures."""
    d = D / N
    c = -0.5 * D + (np.arange(N) + 0.5) * d
    X, Y = np.meshgrid(c, c)  # X varies along columns (j), Y along rows (i)
    r = np.sqrt(X * X + Y * Y)
    r_in = np.sqrt(obstruction) * 0.5 * D
    return (r >= r_in) & (r <= 0.5 * D)


def subap_centres(D, N):
    d = D / N
    c = -0.5 * D + (np.arange(N) + 0.5) * d
    X, Y = np.meshgrid(c, c)
    return X, Y


def layer_spacing(cfg):
    return [cfg["domain_side"] / l["n"] for l in cfg["layers"]]


class Geometry:
    """All geometric data of one configuration."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.D = cfg["D"]
        self.masks = [np.asarray(w["mask"], dtype=bool).reshape(w["n_subap"], w["n_subap"])
                      if w.get("mask") is not None else subap_mask(self.D, w["n_subap"], cfg["obstruction"])
                      for w in cfg["wfs"]]
        self.n_active = [int(m.sum()) for m in self.masks]
        self.n_slopes = [2 * a for a in self.n_active]
        self.delta = layer_spacing(cfg)
        self.L = cfg["domain_side"]
        self.layer_n = [l["n"] for l in cfg["layers"]]
        self.n_coeff = sum(n * n for n in self.layer_n)
        self.layer_off = np.concatenate([[0], np.cumsum([n * n for n in self.layer_n])]).astype(int)
        self.slope_off = np.concatenate([[0], np.cumsum(self.n_slopes)]).astype(int)
        self.corner_n = [(w["n_subap"] + 1) ** 2 for w in cfg["wfs"]]
