"""Writes the finite-difference gradients of the reconstruction-error loss
(tests/golden/gradients_<name>.json) with the FP64 oracle only.

    python tests/golden/make_gradients.py grad_small 4

Inputs are rebuilt from seeds by ``frames_for``; the file stores the seeds,
the frame count and the central differences (alpha and Cn2 steps 1e-4
relative, height steps 0.01 m) of the loss at the exact MAP solution.
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.gradients import fd_gradient, implicit_gradient  # noqa: E402
from oracle.operators import System  # noqa: E402
from synthetic import frozen_flow_frames, get_config, slope_noise, truth_of  # noqa: E402

KEY = 23


def frames_for(name, n_frames, key=KEY):
    """(cfg, cfg_true, [(slopes float32, phi_true float64)]) of a gradient
    workload: frozen-flow screens of the true atmosphere, slopes through the
    true geometry plus seeded noise."""
    cfg = get_config(name)
    cfg_true = truth_of(cfg)
    St = System(cfg_true)
    sig = [w["sigma"] for w in cfg["wfs"]]
    out = []
    for k, scr in enumerate(frozen_flow_frames(cfg_true, n_frames, key)):
        phi_t = np.concatenate([p.astype(np.float64).ravel() for p in scr])
        s = St.apply_A(phi_t) + slope_noise(St.geom.n_slopes, sig, key, k)
        out.append((s.astype(np.float32).astype(np.float64), phi_t))
    return cfg, cfg_true, out


def main(name, n_frames):
    cfg, cfg_true, frames = frames_for(name, n_frames)
    ga, gg, gh = fd_gradient(cfg, frames, cfg_true)
    ia, ig, ih, _ = implicit_gradient(cfg, frames, cfg_true)
    rec = {"config": name, "frames": n_frames, "key": KEY,
           "steps": {"alpha_rel": 1e-4, "cn2_rel": 1e-4, "h_m": 0.01},
           "fd": {"alpha": ga, "cn2": list(gg), "h": list(gh)}}
    path = os.path.join(HERE, "gradients_%s.json" % name)
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print("fd      ", ga, gg, gh)
    print("implicit", ia, ig, ih)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]))
