"""The reconstruction-error loss of the gradient workloads, written with
torch operations so that autograd supplies dL/dphi and the loss's own
dependence on the layer heights (the science projections move with h).

L = (1/F) sum_frames sum_theta |Pi (P_theta(h) phi - y_theta)|^2 over a 5 x 5
grid of directions; P_theta samples every layer bilinearly at the corners of
the first sensor's subaperture grid (no cone effect), restricted to the
corners of active subapertures; Pi removes the mean over them; y_theta is the
same projection of the true atmosphere.  On a grid line the derivative along
that axis is the central difference (average of the one-sided ones).
"""

import numpy as np
import torch

from oracle.fitting import fit_pupil_mask
from oracle.gradients import TIE, science_directions


def _axis(t):
    r = torch.round(t.detach())
    tie = (t.detach() - r).abs() < TIE
    q = torch.where(tie, r, torch.floor(t.detach())).long()
    return q, t - q.to(t.dtype), tie


def sample(v, tx, ty):
    """Bilinear samples of the grid v (n x n) at (ty_i, tx_j) for all i, j."""
    qx, wx, tiex = _axis(tx)
    qy, wy, tiey = _axis(ty)

    def value_x(rows):
        base = v[rows][:, qx]
        right = v[rows][:, qx + 1]
        left = v[rows][:, (qx - 1).clamp(min=0)]
        sx = torch.where(tiex[None, :], 0.5 * (right - left), right - base)
        return base + wx[None, :] * sx

    v0 = value_x(qy)
    vp = value_x(qy + 1)
    vm = value_x((qy - 1).clamp(min=0))
    sy = torch.where(tiey[:, None], 0.5 * (vp - vm), vp - v0)
    return v0 + wy[:, None] * sy


class ScienceLoss:
    def __init__(self, cfg, device):
        self.cfg = cfg
        self.D = cfg["D"]
        self.N = cfg["wfs"][0]["n_subap"]
        self.L = cfg["domain_side"]
        self.mask = torch.tensor(fit_pupil_mask(self.D, self.N, cfg["obstruction"]).ravel(), device=device)
        self.x = torch.tensor(-0.5 * self.D + np.arange(self.N + 1) * (self.D / self.N), dtype=torch.float64,
                              device=device)
        self.dirs = science_directions(cfg)
        self.sizes = [l["n"] for l in cfg["layers"]]
        self.device = device

    def project(self, phi, heights):
        """(n_dirs, n_masked) projections of one frame's layers phi (N_c)."""
        out = []
        off = np.concatenate([[0], np.cumsum([n * n for n in self.sizes])])
        for th in self.dirs:
            acc = 0.0
            for l, n in enumerate(self.sizes):
                v = phi[off[l]:off[l + 1]].reshape(n, n)
                delta = self.L / n
                tx = (self.x + heights[l] * th[0] + 0.5 * self.L) / delta
                ty = (self.x + heights[l] * th[1] + 0.5 * self.L) / delta
                acc = acc + sample(v, tx, ty)
            out.append(acc.reshape(-1)[self.mask])
        return torch.stack(out)

    def __call__(self, phi, heights, truth):
        """phi (F, N_c), heights (L,) tensor, truth (F, n_dirs, n_masked)."""
        tot = 0.0
        for k in range(phi.shape[0]):
            e = self.project(phi[k].double(), heights) - truth[k]
            e = e - e.mean(dim=1, keepdim=True)
            tot = tot + (e * e).sum()
        return tot / phi.shape[0]
