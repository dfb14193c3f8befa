"""GPU parity of the time step with the DM fitting step (Sec. 4.1) against
the oracle: layers and fitted DM commands after one reconstruction."""

import numpy as np
import pytest

from oracle.fitting import Fitting, frame_fitted
from oracle.operators import System
from oracle.solver import State
from synthetic import get_config

from parity import check_blocks
from test_gpu_parity import FRAME_ETOL, LAYER_TOL, synth_slopes, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["small_fit", "large"])
def test_fitted_frame(gpu_lib, name):
    import torch
    cfg = get_config(name)
    S = System(cfg)
    F = Fitting(cfg)
    ctx = gpu_lib.Context(cfg, device=0)
    assert ctx.n_act == F.n_act
    st = torch.zeros(ctx.n_state, device="cuda")
    lay = torch.empty(ctx.n_coeff, device="cuda")
    dm = torch.empty(ctx.n_act, device="cuda")
    s = synth_slopes(S, 0)
    ctx.reconstruct(to_dev(s), st, lay, dm, iters=cfg["iters"])
    ref_st, ref_phi = frame_fitted(S, F, State(S.geom.n_coeff, F.n_act), s.astype(np.float64))
    check_blocks(to_host(lay), ref_phi, S.geom.layer_off, LAYER_TOL, "layers", FRAME_ETOL)
    got = to_host(st)
    n = S.geom.n_coeff
    a = got[3 * n + F.n_act:]
    # each DM's commands at the layer tolerance
    dm_off = np.cumsum([0] + [dm["n_act"] ** 2 for dm in cfg["dms"]])
    m = check_blocks(a, ref_st.a, dm_off, LAYER_TOL, "DM", FRAME_ETOL)
    print("\n[gpu] fitted commands:", m)
    assert np.array_equal(to_host(dm), a)
    # fitted commands reproduce the layers' wavefront in the fitting directions
    # better than zero commands do
    resid = sum(np.linalg.norm(B @ a - P @ ref_phi) ** 2 for B, P in zip(F.B, F.P))
    base = sum(np.linalg.norm(P @ ref_phi) ** 2 for P in F.P)
    assert resid < base
