"""Seeded synthetic inputs: phase screens, frozen flow, slope noise and
random test vectors.  All outputs are float32 numpy arrays (the precision the
GPU path consumes); the oracle promotes them to float64.

Seeds: a master entropy, spawned by an integer key tuple with
``numpy.random.SeedSequence`` so that every (purpose, problem, layer, ...)
stream is independent and reproducible.
"""

import numpy as np

MASTER_SEED = 20220224


def rng(*key):
    """Independent generator for an integer key tuple."""
    ss = np.random.SeedSequence(entropy=MASTER_SEED, spawn_key=tuple(int(k) for k in key))
    return np.random.Generator(np.random.PCG64(ss))


def random_vector(n, *key, scale=1.0):
    """n standard-normal float32 values times ``scale``."""
    return (rng(1, *key).standard_normal(n) * scale).astype(np.float32)


def _vk_spectrum(m, spacing, r0, L0):
    """Square root of the von Karman phase PSD times the frequency step, on
    the m x m FFT grid (turbulence simulation, rad per mode)."""
    f1 = np.fft.fftfreq(m, d=spacing)
    fx, fy = np.meshgrid(f1, f1)
    f2 = fx * fx + fy * fy + 1.0 / (L0 * L0)
    psd = 0.023 * r0 ** (-5.0 / 3.0) * f2 ** (-11.0 / 6.0)
    psd[0, 0] = 0.0  # no piston
    df = 1.0 / (m * spacing)
    return np.sqrt(psd) * df


def von_karman_spectrum(n, spacing, r0, L0, *key, pad=2):
    """Complex Fourier coefficients of a periodic von Karman screen on a
    (pad*n)^2 grid; the phase screen is ``screen_from_spectrum``."""
    m = pad * n
    g = rng(2, *key)
    noise = g.standard_normal((m, m)) + 1j * g.standard_normal((m, m))
    return _vk_spectrum(m, spacing, r0, L0) * noise


def screen_from_spectrum(spec, n, shift_m=(0.0, 0.0), spacing=1.0):
    """Real phase screen (n x n crop, rows = y) of the periodic screen with
    Fourier coefficients ``spec`` translated by ``shift_m`` metres."""
    m = spec.shape[0]
    f1 = np.fft.fftfreq(m, d=spacing)
    fx, fy = np.meshgrid(f1, f1)
    ph = np.exp(-2j * np.pi * (fx * shift_m[0] + fy * shift_m[1]))
    scr = np.real(np.fft.ifft2(spec * ph)) * (m * m)
    return scr[:n, :n]


def von_karman_screen(n, spacing, r0, L0, *key):
    """One n x n von Karman screen (rad) with the given Fried parameter."""
    spec = von_karman_spectrum(n, spacing, r0, L0, *key)
    return screen_from_spectrum(spec, n, spacing=spacing).astype(np.float32)


def layer_r0(cfg, layer):
    """Fried parameter of one layer from its fractional weight gamma:
    r0_l^(-5/3) = gamma_l r0^(-5/3)."""
    return cfg["prior"]["r0"] * layer["cn2"] ** (-3.0 / 5.0)


def wind(cfg, *key):
    """Per-layer wind vectors (m/s): random direction, speed in the range."""
    lo, hi = cfg.get("wind", (5.0, 20.0))
    g = rng(3, *key)
    out = []
    for _ in cfg["layers"]:
        v = g.uniform(lo, hi)
        a = g.uniform(0.0, 2.0 * np.pi)
        out.append((v * np.cos(a), v * np.sin(a)))
    return out


def frozen_flow_frames(cfg, n_frames, *key, first=0):
    """Yield per-frame lists of true layer screens (float32, n_l x n_l each)
    moving with frozen flow at the configuration's frame rate."""
    spacing = [cfg["domain_side"] / l["n"] for l in cfg["layers"]]
    specs = [von_karman_spectrum(l["n"], dl, layer_r0(cfg, l), cfg["prior"]["L0"], *key, k)
             for k, (l, dl) in enumerate(zip(cfg["layers"], spacing))]
    winds = wind(cfg, *key)
    dt = 1.0 / cfg.get("frame_rate", 500.0)
    for f in range(first, first + n_frames):
        yield [screen_from_spectrum(sp, l["n"], (w[0] * f * dt, w[1] * f * dt), dl).astype(np.float32)
               for sp, l, w, dl in zip(specs, cfg["layers"], winds, spacing)]


def slope_noise(n_per_wfs, sigmas, *key):
    """Gaussian slope noise, sigma_g * N(0,1), concatenated over sensors."""
    g = rng(4, *key)
    return np.concatenate([(g.standard_normal(n) * s) for n, s in zip(n_per_wfs, sigmas)]).astype(np.float32)
