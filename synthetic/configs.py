"""Workload configurations (plain data).

Each configuration is a dict:

``D`` (m), ``obstruction`` (obstructed *area* fraction of the pupil),
``wfs``: list of guide-star sensors, each
    ``kind`` ("lgs" | "ngs"), ``n_subap`` (N, the sensor has N x N
    subapertures on an (N+1) x (N+1) corner grid), ``theta`` (rad, x/y),
    ``H`` (m, LGS altitude; None for NGS), ``sigma`` (rad, slope noise std),
    ``launch`` (m, laser launch position, LGS only), ``tt_removal``;
``layers``: list of reconstruction layers ``h`` (m), ``n`` (grid side, a
    power of two), ``levels`` (wavelet decomposition depth), ``cn2``
    (fractional turbulence weight gamma);
``domain_side`` (m): side of the square layer domain, shared by all layers;
``prior``: ``alpha``, ``r0`` (m), ``L0`` (m), ``tau``;
``noise``: ``alpha_eta``, ``na_fwhm`` (m), ``spot_fwhm`` (rad);
``iters``, ``gain``; optional ``dms`` / ``fit`` for the fitting step.

The numbers follow the paper's system description (Tables 1-5 and the
asterism figure of the numerical-simulation section) where it gives them;
where it is silent the values are stated choices of this workload set.
"""

import copy
import math

ARCSEC = math.pi / (180.0 * 3600.0)


def _ring(n, radius_arcsec, az0_deg, step_deg):
    out = []
    for k in range(n):
        az = math.radians(az0_deg + k * step_deg)
        out.append((radius_arcsec * ARCSEC * math.cos(az),
                    radius_arcsec * ARCSEC * math.sin(az)))
    return out


def _lgs(theta, n_subap, sigma, D, H=90000.0):
    # laser launched from the pupil edge on the side of the guide star
    az = math.atan2(theta[1], theta[0])
    return {"kind": "lgs", "n_subap": n_subap, "theta": tuple(theta),
            "H": H, "sigma": sigma,
            "launch": (0.5 * D * math.cos(az), 0.5 * D * math.sin(az)),
            "tt_removal": True}


def _ngs(theta, n_subap, sigma):
    return {"kind": "ngs", "n_subap": n_subap, "theta": tuple(theta),
            "H": None, "sigma": sigma, "launch": (0.0, 0.0),
            "tt_removal": False}


def tiny():
    """8 m, one on-axis NGS 16x16, two 32x32 layers, 3 levels (runs in seconds)."""
    D = 8.0
    return {
        "name": "tiny",
        "D": D, "obstruction": 0.0,
        "wfs": [_ngs((0.0, 0.0), 16, 0.1)],
        "layers": [{"h": 0.0, "n": 32, "levels": 3, "cn2": 0.8},
                   {"h": 6000.0, "n": 32, "levels": 3, "cn2": 0.2}],
        "domain_side": 32 * 0.5,
        "prior": {"alpha": 1.0, "r0": 0.15, "L0": 25.0, "tau": 0.0},
        "noise": {"alpha_eta": 0.0, "na_fwhm": 11400.0, "spot_fwhm": 1.0 * ARCSEC},
        "iters": 10, "gain": 1.0,
    }


def small():
    """A reduced MAORY-like system: LGS with tip/tilt removal plus NGS, three
    layers of uneven size, central obstruction, sensor grids that do not divide
    into whole tiles."""
    D = 8.0
    lgs = [_lgs(t, 20, 0.1, D) for t in _ring(3, 40.0, 0.0, 120.0)]
    ngs = [_ngs(t, 2, 0.05) for t in _ring(2, 30.0, 60.0, 180.0)]
    return {
        "name": "small",
        "D": D, "obstruction": 0.11,
        "wfs": lgs + ngs,
        "layers": [{"h": 0.0, "n": 32, "levels": 3, "cn2": 0.6},
                   {"h": 4000.0, "n": 32, "levels": 3, "cn2": 0.25},
                   {"h": 12700.0, "n": 64, "levels": 3, "cn2": 0.15}],
        "domain_side": 32 * (D / 20),
        "prior": {"alpha": 1.0, "r0": 0.157, "L0": 25.0, "tau": 0.0},
        "noise": {"alpha_eta": 0.0, "na_fwhm": 11400.0, "spot_fwhm": 1.0 * ARCSEC},
        "iters": 4, "gain": 1.0,
    }


def mid():
    """Like ``small`` but with one 256x256 layer (two global wavelet levels on
    the GPU) and 5 decomposition levels."""
    D = 8.0
    lgs = [_lgs(t, 20, 0.1, D) for t in _ring(3, 40.0, 0.0, 120.0)]
    ngs = [_ngs(t, 2, 0.05) for t in _ring(2, 30.0, 60.0, 180.0)]
    return {
        "name": "mid",
        "D": D, "obstruction": 0.11,
        "wfs": lgs + ngs,
        "layers": [{"h": 0.0, "n": 64, "levels": 5, "cn2": 0.6},
                   {"h": 4000.0, "n": 128, "levels": 5, "cn2": 0.25},
                   {"h": 12700.0, "n": 256, "levels": 5, "cn2": 0.15}],
        "domain_side": 32 * (D / 20),
        "prior": {"alpha": 1.0, "r0": 0.157, "L0": 25.0, "tau": 0.0},
        "noise": {"alpha_eta": 0.0, "na_fwhm": 11400.0, "spot_fwhm": 1.0 * ARCSEC},
        "iters": 4, "gain": 1.0,
    }


def maory_like():
    """39 m, 6 LGS 80x80 at 90 km on a 45" ring with tip/tilt removed, 3 NGS
    2x2 on a 55" ring, layers at 0/4/12.7 km with 128/128/256 grids, D3 with 5
    levels, diagonal noise, 4 warm-started PCG iterations per frame."""
    D = 39.0
    lgs = [_lgs(t, 80, 0.1, D) for t in _ring(6, 45.0, 0.0, 60.0)]
    ngs = [_ngs(t, 2, 0.1) for t in _ring(3, 55.0, 60.0, 120.0)]
    return {
        "name": "maory_like",
        "D": D, "obstruction": 0.11,
        "wfs": lgs + ngs,
        "layers": [{"h": 0.0, "n": 128, "levels": 5, "cn2": 0.75},
                   {"h": 4000.0, "n": 128, "levels": 5, "cn2": 0.15},
                   {"h": 12700.0, "n": 256, "levels": 5, "cn2": 0.10}],
        "domain_side": 128 * (D / 80),
        "prior": {"alpha": 1.0, "r0": 0.157, "L0": 25.0, "tau": 0.0},
        "noise": {"alpha_eta": 0.0, "na_fwhm": 11400.0, "spot_fwhm": 1.0 * ARCSEC},
        "iters": 4, "gain": 1.0,
        "frame_rate": 500.0, "wind": (5.0, 20.0),
    }


def paper_maory():
    """The paper's own MAORY system: 37 m, 11 % obstruction, 6 LGS 74x74 on a
    90" diameter ring, 3 NGS 2x2 on a 110" diameter ring, layers 128/64/64 at
    0.5/1/1 m spacing, 2 PCG iterations."""
    D = 37.0
    lgs = [_lgs(t, 74, 0.1, D) for t in _ring(6, 45.0, 0.0, 60.0)]
    ngs = [_ngs(t, 2, 0.1) for t in _ring(3, 55.0, 60.0, 120.0)]
    return {
        "name": "paper_maory",
        "D": D, "obstruction": 0.11,
        "wfs": lgs + ngs,
        "layers": [{"h": 0.0, "n": 128, "levels": 5, "cn2": 0.75},
                   {"h": 4000.0, "n": 64, "levels": 5, "cn2": 0.15},
                   {"h": 12700.0, "n": 64, "levels": 5, "cn2": 0.10}],
        "domain_side": 64.0,
        "prior": {"alpha": 1.0, "r0": 0.157, "L0": 25.0, "tau": 0.0},
        "noise": {"alpha_eta": 0.0, "na_fwhm": 11400.0, "spot_fwhm": 1.0 * ARCSEC},
        "iters": 2, "gain": 1.0,
    }


def vlt_like():
    """8 m, 4 LGS 40x40 on a 30" ring, 5 layers of 64x64, 4 levels, no
    obstruction, no NGS."""
    D = 8.0
    lgs = [_lgs(t, 40, 0.1, D) for t in _ring(4, 30.0, 45.0, 90.0)]
    heights = [0.0, 2000.0, 4000.0, 8000.0, 14000.0]
    return {
        "name": "vlt_like",
        "D": D, "obstruction": 0.0,
        "wfs": lgs,
        "layers": [{"h": h, "n": 64, "levels": 4, "cn2": 0.2} for h in heights],
        "domain_side": 64 * (D / 40),
        "prior": {"alpha": 1.0, "r0": 0.15, "L0": 25.0, "tau": 0.0},
        "noise": {"alpha_eta": 0.0, "na_fwhm": 11400.0, "spot_fwhm": 1.0 * ARCSEC},
        "iters": 6, "gain": 1.0,
    }


def large():
    """9 layers from 0 to 20 km (128x128 up to 10 km, 256x256 above), 6 LGS
    80x80 with spot-elongated 2x2 block noise, 20 PCG iterations, then a
    fitting step onto 3 DMs over 9 directions."""
    D = 39.0
    cfg = maory_like()
    lgs = [_lgs(t, 80, 0.1, D) for t in _ring(6, 45.0, 0.0, 60.0)]
    heights = [2500.0 * k for k in range(9)]
    weights = [0.45, 0.12, 0.09, 0.08, 0.07, 0.06, 0.05, 0.045, 0.035]
    cfg.update({
        "name": "large",
        "wfs": lgs,
        "layers": [{"h": h, "n": (128 if h <= 10000.0 else 256), "levels": 5,
                    "cn2": w} for h, w in zip(heights, weights)],
        "noise": {"alpha_eta": 0.2, "na_fwhm": 11400.0, "spot_fwhm": 1.0 * ARCSEC},
        "iters": 20,
        "dms": [{"h": 0.0, "n_act": 83, "pitch": D / 80},
                {"h": 4000.0, "n_act": 47, "pitch": 1.0},
                {"h": 12700.0, "n_act": 47, "pitch": 1.0}],
        "fit": {"directions": [(x * ARCSEC, y * ARCSEC) for y in (-30.0, 0.0, 30.0)
                               for x in (-30.0, 0.0, 30.0)],
                "iters": 10, "eps_rel": 1e-6},
    })
    return cfg


def small_fit():
    """``small`` with a fitting step onto 3 DMs over 4 directions."""
    cfg = small()
    cfg.update({
        "name": "small_fit",
        "dms": [{"h": 0.0, "n_act": 23, "pitch": 0.4},
                {"h": 4000.0, "n_act": 13, "pitch": 0.8},
                {"h": 12700.0, "n_act": 15, "pitch": 0.8}],
        "fit": {"directions": [(x * ARCSEC, y * ARCSEC) for y in (-20.0, 20.0) for x in (-20.0, 20.0)],
                "iters": 10, "eps_rel": 1e-6},
    })
    return cfg


def grad_small():
    """``small`` with the science field of the gradient loss: a 5 x 5 grid of
    directions over +-20" (the guide-star field of this 8 m system)."""
    cfg = small()
    cfg["name"] = "grad_small"
    cfg["science_half"] = 20.0 * ARCSEC
    return cfg


def grad_maory():
    """MAORY-like geometry with the science field of the gradient loss: a
    5 x 5 grid of directions over a 2' field (+-60")."""
    cfg = maory_like()
    cfg["name"] = "grad_maory"
    cfg["science_half"] = 60.0 * ARCSEC
    return cfg


def truth_of(cfg):
    """The atmosphere that generates the data of a gradient workload: the
    reconstruction's layers moved up by 2 % (the ground layer stays) and the
    Cn2 weights tilted by +-30 % and renormalised."""
    t = copy.deepcopy(cfg)
    w = [l["cn2"] * (1.3 if k % 2 == 0 else 0.7) for k, l in enumerate(t["layers"])]
    for l, wk in zip(t["layers"], w):
        l["h"] = 1.02 * l["h"]
        l["cn2"] = wk / sum(w)
    t["name"] = cfg["name"] + "_truth"
    return t


CONFIGS = {
    "tiny": tiny,
    "small": small,
    "mid": mid,
    "maory_like": maory_like,
    "paper_maory": paper_maory,
    "vlt_like": vlt_like,
    "large": large,
    "small_fit": small_fit,
    "grad_small": grad_small,
    "grad_maory": grad_maory,
}


def get_config(name, **overrides):
    """Return a fresh copy of a named configuration with top-level overrides."""
    cfg = copy.deepcopy(CONFIGS[name]())
    for k, v in overrides.items():
        cfg[k] = v
    return cfg


def sizes(cfg):
    """Counts that depend only on the configuration data: (N_c, per-WFS
    corner counts).  Active-subaperture counts depend on the mask rule and
    are computed by each implementation."""
    n_c = sum(l["n"] ** 2 for l in cfg["layers"])
    corners = [(w["n_subap"] + 1) ** 2 for w in cfg["wfs"]]
    return n_c, corners


def batch_mix(n_maory, n_vlt, *key):
    """Independent reconstructions of uneven sizes for one batch: n_maory
    MAORY-like and n_vlt VLT-like configurations, each with its own seeded
    Cn2 profile (Dirichlet(1) weights), Fried parameter r0 ~ U[0.1, 0.2] m and
    slope noise sigma ~ U[0.05, 0.3] rad, 6 PCG iterations each."""
    import numpy as np
    from .inputs import rng
    g = rng(5, *key)
    out = []
    for k in range(n_maory + n_vlt):
        cfg = maory_like() if k < n_maory else vlt_like()
        w = g.dirichlet(np.ones(len(cfg["layers"])))
        for layer, wk in zip(cfg["layers"], w):
            layer["cn2"] = float(max(wk, 1e-3))
        cfg["prior"]["r0"] = float(g.uniform(0.1, 0.2))
        sigma = float(g.uniform(0.05, 0.3))
        for s in cfg["wfs"]:
            s["sigma"] = sigma
        cfg["iters"] = 6
        cfg["name"] = "%s_%d" % (cfg["name"], k)
        out.append(cfg)
    return out
