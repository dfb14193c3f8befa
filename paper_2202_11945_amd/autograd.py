"""Reconstructed layers as a differentiable function of the method's
parameters (alpha, the Cn2 weights gamma_l, the layer heights h_l).

Forward, per frame: c* = M^{-1} W^{-T} A^T C_hat^{-1} s (eq. fewha, solved to
a tolerance by mixed-precision refinement), phi = W^{-1} c*.  Backward
(implicit function theorem, M symmetric): lambda = M^{-1} W^{-T} dL/dphi by a
second solve with the same operator, then the library's parameter-gradient
reductions.  Every step runs in libfewha; this module only marshals
arguments.

The parameters are baked into a context at set-up (the prior table, the
propagation tables and J depend on them), so ``params`` must hold exactly the
values the frames' context was configured with; an optimiser builds a new
``FrameBatch`` after each update.
"""

import torch

from .fewha import Batch, Context


def param_vector(cfg, device=None):
    """[alpha, gamma_1..gamma_L, h_1..h_L] of a configuration (float64)."""
    v = [cfg["prior"]["alpha"]] + [l["cn2"] for l in cfg["layers"]] + [l["h"] for l in cfg["layers"]]
    return torch.tensor(v, dtype=torch.float64, device=device)


class FrameBatch:
    """One configured problem and a batch of ``n_frames`` copies of it (one
    launch per stage over all frames)."""

    def __init__(self, cfg, n_frames, device=0):
        self.cfg = cfg
        self.ctx = Context(cfg, device)
        self.batch = Batch([self.ctx] * n_frames)
        self.n_frames = n_frames
        self.params = param_vector(cfg)

    def close(self):
        self.batch.close()
        self.ctx.close()


class MAPLayers(torch.autograd.Function):
    """phi[k] = W^{-1} M^{-1} b(s[k]) for the frames of a FrameBatch.

    apply(params, slopes, frames, rtol, max_iters) with params as returned by
    ``param_vector`` (its gradient is the output of the backward) and slopes a
    (n_frames, n_slopes) float32 device tensor; returns (n_frames, N_c)."""

    @staticmethod
    def forward(fctx, params, slopes, frames, rtol=1e-6, max_iters=1 << 20):
        if not torch.equal(params.detach().cpu(), frames.params):
            raise ValueError("params differ from the values the frames were configured with")
        if slopes.shape[0] != frames.n_frames:
            raise ValueError("expected %d frames of slopes" % frames.n_frames)
        s = [slopes[k].contiguous() for k in range(frames.n_frames)]
        c, it, rel = frames.batch.solve_map(slopes=s, rtol=rtol, max_iters=max_iters)
        phi = frames.batch.apply_Winv(c)
        fctx.frames, fctx.rtol, fctx.max_iters = frames, rtol, max_iters
        fctx.pdev = params.device
        fctx.s, fctx.c = s, c
        fctx.forward_iters, fctx.forward_rel = it, rel
        return torch.stack(phi)

    @staticmethod
    def backward(fctx, g_phi):
        frames = fctx.frames
        g = [g_phi[k].contiguous().float() for k in range(frames.n_frames)]
        lam, _, _ = frames.batch.solve_map(g_layers=g, rtol=fctx.rtol, max_iters=fctx.max_iters)
        grads = frames.batch.param_grads(fctx.s, fctx.c, lam)
        return torch.stack(grads).sum(0).to(fctx.pdev), None, None, None, None
