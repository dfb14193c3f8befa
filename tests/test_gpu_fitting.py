"""GPU parity of the time step with the DM fitting step (Sec. 4.1) against
the oracle: layers and fitted DM commands after one reconstruction."""

import numpy as np
import pytest

from oracle.fitting import Fitting, frame_fitted
from oracle.operators import System
from oracle.solver import State
from synthetic import get_config

from test_gpu_parity import LAYER_TOL, rel, synth_slopes, to_dev, to_host

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
    o = S.geom.layer_off
    got_lay = to_host(lay)
    for l in range(S.Lc):
        assert rel(got_lay[o[l]:o[l + 1]], ref_phi[o[l]:o[l + 1]]) <= LAYER_TOL, l
    got = to_host(st)
    n = S.geom.n_coeff
    a = got[3 * n + F.n_act:]
    print("\n[gpu] fitted commands rel. error:", rel(a, ref_st.a))
    assert rel(a, ref_st.a) <= 10 * LAYER_TOL
    assert np.array_equal(to_host(dm), a)
    # fitted commands reproduce the layers' wavefront in the fitting directions
    # better than zero commands do
    resid = sum(np.linalg.norm(B @ a - P @ ref_phi) ** 2 for B, P in zip(F.B, F.P))
    base = sum(np.linalg.norm(P @ ref_phi) ** 2 for P in F.P)
    assert resid < base
