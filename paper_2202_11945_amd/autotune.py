"""Autotuner of a plan's launch shapes.

Six tunables:

* the resident transform side R (32, 64 or 128): the resident DWT kernels
  keep every level up to R x R in one workgroup's LDS, and the levels above R
  run as tiled global passes.  A large R means few, heavy workgroups (a
  MAORY-like layer of 128 x 128 is one workgroup); a small R spreads the same
  levels over many more workgroups at the cost of one launch per extra level.
* the node rows per thread of the propagation adjoint (4 or 8): more rows
  put more independent loads in flight per thread, at more registers.
* for the best of those, the propagation adjoint's sensor lists split over
  the waves of 4-row tiles (pt_split), which shortens each wave's serial
  chain of sensors where a launch has few tiles;
* fused global levels (glob_fuse): a layer with two or more levels above
  the resident side runs its top two levels as one launch per transform,
  timed for every resident side where that applies;
* then the resident inverse levels in one workgroup per layer (the default)
  or in four (each synthesizing the lower levels itself and one quadrant of
  the top level);
* then the number of streams a batch's frame runs on
  (1 or 2 parts of the problem list, each on its own stream, so that the
  stages of one part overlap those of the other).

Which combination wins depends on the batch size, the layer sizes and the
device, so it is measured: every admissible combination builds the batch
plan, replays the captured frame graph on zero inputs, and the fastest is
kept.

Results are cached per (device, problem shapes, batch size, iterations) in
a JSON file (``FEWHA_TUNE_CACHE`` or ``lib/autotune_cache.json`` next to the
library).  Timing uses HIP events on the current torch stream.
"""

import json
import os

CANDIDATES = (32, 64, 128)
PT_ROWS = (4, 8)
STREAMS = (1, 2)
MARGIN = 0.02  # relative gain a non-default choice needs
CACHE = os.environ.get("FEWHA_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "autotune_cache.json"))


def admissible(ctxs, candidates=CANDIDATES):
    """Resident sides that hold every layer's coarsest block."""
    m0 = max(l["n"] >> l["levels"] for c in ctxs for l in c.cfg["layers"])
    return [r for r in candidates if r >= m0]


def source_hash():
    """sha256 prefix of the library's sources: a cached choice is kept only
    for the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in sorted(os.listdir(src)):
        with open(os.path.join(src, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def split_allowed(ctxs, res):
    """Whether the resident inverse levels can run in quarters (the library's
    rule): every layer has a resident side min(n, res) of at least 16 and
    at least one resident level."""
    for c in ctxs:
        for l in c.cfg["layers"]:
            R = min(l["n"], res)
            if R < 16 or R < 2 * (l["n"] >> l["levels"]):
                return False
    return True


def fusable(ctxs, res):
    """Whether some layer has two or more global levels at resident side res
    (side above 2 res), so that glob_fuse changes the plan."""
    return any(l["n"] > 2 * res for c in ctxs for l in c.cfg["layers"])


def signature(ctxs, iters, device_name=None):
    """Cache key: device name, library sources and the multiset of problem
    shapes (layer sides, levels and heights; each sensor's kind, size,
    altitude and direction, which set the propagation adjoint's paths)."""
    if device_name is None:
        import torch
        device_name = torch.cuda.get_device_name(ctxs[0].device)
    shapes = {}
    for c in ctxs:
        cfg = c.cfg
        s = "L%s|W%s|F%d" % (",".join("%dx%d@%.6g" % (l["n"], l["levels"], l["h"]) for l in cfg["layers"]),
                            ",".join("%s%d@%s:%.9g,%.9g" % (w["kind"], w["n_subap"], w["H"], w["theta"][0],
                                                            w["theta"][1]) for w in cfg["wfs"]),
                            1 if (cfg.get("dms") and cfg.get("fit")) else 0)
        shapes[s] = shapes.get(s, 0) + 1
    body = ";".join("%dx[%s]" % (n, s) for s, n in sorted(shapes.items()))
    return "%s|iters%d|%s|src%s" % (device_name, iters, body, source_hash())


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def time_plan(ctxs, iters, tuning, steps=10, warmup=3):
    """Microseconds per graph replay of one frame over the batch, for a
    tuning as accepted by Batch."""
    import torch
    from .fewha import Batch
    b = Batch(ctxs, tuning=tuning)
    try:
        dev = "cuda:%d" % ctxs[0].device
        slopes = [torch.zeros(c.n_slopes, device=dev) for c in ctxs]
        states = [torch.zeros(c.n_state, device=dev) for c in ctxs]
        for _ in range(warmup):
            b.reconstruct(slopes, states, iters=iters, use_graph=True)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            b.reconstruct(slopes, states, iters=iters, use_graph=True)
        t1.record()
        t1.synchronize()
        return 1000.0 * t0.elapsed_time(t1) / steps
    finally:
        b.close()


def tune(ctxs, iters, steps=10, use_cache=True):
    """Best launch shapes for a batch of these contexts; returns
    {"dwt_resident": R, "pt_rows": r, "pt_split": 0 or 1, "glob_fuse": 0 or 1,
     "res_split": 0 or 4, "streams": s, "us": {"R/r": us per step},
     "pt_split_us", "glob_fuse_us", "split_us",
     "streams_us": {"s": us per step}, "cached": bool}."""
    key = signature(ctxs, iters)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        rec = dict(db[key])
        rec["cached"] = True
        return rec
    us = {(r, pr): time_plan(ctxs, iters, {"dwt_resident": r, "pt_rows": pr}, steps=steps)
          for r in admissible(ctxs) for pr in PT_ROWS}
    best = min(us, key=us.get)
    # keep the default shapes unless another choice is clearly faster: near
    # ties would otherwise flip between runs on timing noise
    default = (max(admissible(ctxs)), PT_ROWS[0])
    if us[best] > (1.0 - MARGIN) * us[default]:
        best = default
    shape = {"dwt_resident": best[0], "pt_rows": best[1], "pt_split": 0}
    # the propagation adjoint's sensor lists split over the waves (4 rows
    # per thread) against the best unsplit shape
    pts_us = {0: us[best], 1: time_plan(ctxs, iters, {"dwt_resident": best[0], "pt_rows": 4, "pt_split": 1},
                                        steps=steps)}
    if pts_us[1] <= (1.0 - MARGIN) * pts_us[0]:
        shape = {"dwt_resident": best[0], "pt_rows": 4, "pt_split": 1}
    shape["glob_fuse"] = 0
    # fused global levels, at every resident side where a layer has two or
    # more global levels, with the propagation adjoint's shape just chosen
    cur = pts_us[shape["pt_split"]]
    fuse_us = {}
    for r in admissible(ctxs):
        if fusable(ctxs, r):
            fuse_us[r] = time_plan(ctxs, iters, dict(shape, dwt_resident=r, glob_fuse=1), steps=steps)
    if fuse_us:
        rf = min(fuse_us, key=fuse_us.get)
        if fuse_us[rf] <= (1.0 - MARGIN) * cur:
            shape = dict(shape, dwt_resident=rf, glob_fuse=1)
            cur = fuse_us[rf]
    # then the resident inverse levels in four workgroups per layer against
    # the default one
    split_us = {0: cur}
    if split_allowed(ctxs, shape["dwt_resident"]):
        split_us[4] = time_plan(ctxs, iters, dict(shape, res_split=4), steps=steps)
    split = min(split_us, key=split_us.get)
    if split_us[split] > (1.0 - MARGIN) * split_us[0]:
        split = 0
    sus = {1: split_us[split]}
    for ns in STREAMS[1:]:
        if ns <= len(ctxs):
            sus[ns] = time_plan(ctxs, iters, dict(shape, res_split=split, streams=ns), steps=steps)
    streams = min(sus, key=sus.get)
    if sus[streams] > (1.0 - MARGIN) * sus[1]:
        streams = 1
    rec = {"dwt_resident": shape["dwt_resident"], "pt_rows": shape["pt_rows"], "pt_split": shape["pt_split"],
           "glob_fuse": shape["glob_fuse"], "res_split": split, "streams": streams,
           "us": {"%d/%d" % k: round(t, 3) for k, t in us.items()},
           "pt_split_us": {"%d" % k: round(t, 3) for k, t in pts_us.items()},
           "glob_fuse_us": {"%d" % k: round(t, 3) for k, t in fuse_us.items()},
           "split_us": {"%d" % k: round(t, 3) for k, t in split_us.items()},
           "streams_us": {"%d" % k: round(t, 3) for k, t in sus.items()}}
    if use_cache:
        db = _load()
        db[key] = rec
        _store(db)
    rec = dict(rec)
    rec["cached"] = False
    return rec
