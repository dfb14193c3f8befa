"""Element-wise comparison of GPU results with the FP64 oracle.

Every check takes one block of a result (a layer, a sensor's slopes, a
state part) and asserts three things at one tolerance `tol`:

* norm-wise:   |g - r|_2 <= tol |r|_2
* max-abs:     max_i |g_i - r_i| <= tol max_i |r_i|
* entry-wise:  |g_i - r_i| <= etol (|r_i| + rms(r)) for every i

The norm-wise check is the reading of "relative" used for the tolerances of
the method (1e-5 per operator application, 1e-4 on the layers after a fixed
number of iterations).  It can hide one wrong entry among 10^5; the max-abs
check bounds every entry by the block's largest, and the entry-wise check,
with the block's RMS as its floor, bounds every entry by its own size (a
single coefficient off by 0.3 % of the RMS fails it where the norm-wise
check at n = 10^5 would not).  etol defaults to tol; where a block's
entries are differences of much larger terms (cancellation), a caller
states a larger etol with its reason.

Failures name the block and the worst entry (index, GPU value, oracle
value).  With FEWHA_PARITY_LOG=<file> every check's figures are appended
to that file as JSON lines.
"""

import json
import os

import numpy as np


def metrics(got, ref, scale=None):
    g = np.asarray(got, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    assert g.shape == r.shape, (g.shape, r.shape)
    sc = r if scale is None else np.asarray(scale, dtype=np.float64).ravel()
    d = np.abs(g - r)
    nr = np.linalg.norm(sc)
    mx = np.abs(sc).max() if sc.size else 0.0
    rms = nr / np.sqrt(max(sc.size, 1))
    out = {"n": int(r.size), "norm": float(np.linalg.norm(g - r) / nr) if nr > 0 else float(np.linalg.norm(g)),
           "maxabs": float(d.max() / mx) if mx > 0 else float(d.max() if d.size else 0.0)}
    if r.size:
        e = d / (np.abs(r) + rms) if rms > 0 else d
        i = int(np.argmax(e))
        out.update({"entry": float(e[i]), "worst": i, "gpu": float(g[i]), "ref": float(r[i])})
        j = int(np.argmax(d))
        out["worst_abs"] = j
    else:
        out.update({"entry": 0.0, "worst": -1, "gpu": 0.0, "ref": 0.0, "worst_abs": -1})
    return out


def _log(what, m, tol, etol):
    path = os.environ.get("FEWHA_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(dict(m, what=str(what), tol=tol, etol=etol)) + "\n")


def _eval(got, ref, tol, what, etol, scale=None):
    m = metrics(got, ref, scale)
    _log(what, m, tol, etol)
    bad = []
    if not m["norm"] <= tol:
        bad.append("norm-wise %.3e > %.1e" % (m["norm"], tol))
    if not m["maxabs"] <= tol:
        bad.append("max-abs %.3e > %.1e at entry %d" % (m["maxabs"], tol, m["worst_abs"]))
    if not m["entry"] <= etol:
        bad.append("entry-wise %.3e > %.1e at entry %d (gpu %.9g, oracle %.9g)"
                   % (m["entry"], etol, m["worst"], m["gpu"], m["ref"]))
    return m, ("%s (n = %d): %s" % (what, m["n"], "; ".join(bad)) if bad else None)


def check(got, ref, tol, what, etol=None):
    """Asserts the three bounds above on one block; returns the figures."""
    m, bad = _eval(got, ref, tol, what, tol if etol is None else etol)
    assert bad is None, bad
    return m


def check_blocks(got, ref, offsets, tol, what, etol=None, scale=None):
    """The three bounds on every block [offsets[k], offsets[k+1]) (layers,
    sensors); every block is evaluated before the assertion names the
    failing ones.  `scale` (same layout as ref) replaces ref as the size
    the bounds are relative to (its norm, largest entry and RMS)."""
    g = np.asarray(got, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    sc = None if scale is None else np.asarray(scale, dtype=np.float64).ravel()
    out, bad = [], []
    for k in range(len(offsets) - 1):
        a, b = int(offsets[k]), int(offsets[k + 1])
        m, why = _eval(g[a:b], r[a:b], tol, "%s[%d]" % (what, k), tol if etol is None else etol,
                       None if sc is None else sc[a:b])
        out.append(m)
        if why:
            bad.append(why)
    assert not bad, "\n".join(bad)
    return out
