"""Benchmark of the FEWHA hot path on one MI355X.

Workload: MAORY-like reconstructions (39 m, 6 LGS 80x80 with tip/tilt
removal + 3 NGS 2x2, layers 128/128/256 at 0/4/12.7 km, D3 with 5 levels,
diagonal noise, 4 warm-started PCG iterations per frame).  A step advances
B independent MAORY-like frame sequences by one frame each (RHS, warm
restart, 4 PCG iterations, inverse transform and open-loop control) with
one HIP graph replay; inputs (slopes of frozen-flow von Karman screens plus
noise) are resident in HBM before timing starts.

Prints one JSON line: batched frames/s (value), single-frame latency of the
graph path and of the plain (unbatched, ungraphed) path, the dominant
kernel's roofline and the FP64 CPU oracle's rate on this host.
"""

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "maory_like"
STAGES = ["IDWT_RES", "IDWT_GLOB", "P_GAMMA", "GAMMA_T", "P_T", "FDWT_GLOB", "FDWT_RES", "UPDATE"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--batch", type=int, default=64, help="independent MAORY-like frame sequences")
    p.add_argument("--iters", type=int, default=4)
    p.add_argument("--pool", type=int, default=8, help="distinct input frames per sequence")
    p.add_argument("--latency-frames", type=int, default=1000)
    p.add_argument("--no-tune", action="store_true", help="default launch shapes instead of the autotuner's")
    p.add_argument("--grad-frames", type=int, default=16,
                   help="frames of the forward + implicit-backward leg (0 = skip)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--cpu-child", default=None, help=argparse.SUPPRESS)
    p.add_argument("--no-extra", action="store_true",
                   help="skip the legs beyond the timed workload (batched 64 uneven, large, paper MAORY, "
                        "streamed slopes, bandwidth probes)")
    return p.parse_args()


# ------------------------------------------------------------ CPU oracle leg

def cpu_child(workload, seconds):
    """Runs in a single-threaded child process: times the oracle's time step
    on consecutive frames of a workload (set-up excluded) and prints
    frames/s as JSON.  maory_like: RHS, warm restart, 4 PCG iterations, W^-1
    and control; large: 20 PCG iterations and the fitting CG."""
    import numpy as np
    from oracle.operators import System
    from oracle.solver import State, frame
    from synthetic import frozen_flow_frames, get_config, slope_noise

    cfg = get_config(workload)
    t0 = time.perf_counter()
    S = System(cfg)
    S.preconditioner()
    fit = None
    if cfg.get("fit"):
        from oracle.fitting import Fitting, frame_fitted
        fit = Fitting(cfg)
    setup = time.perf_counter() - t0
    sig = [w["sigma"] for w in cfg["wfs"]]
    st = State(S.geom.n_coeff, fit.n_act if fit else S.geom.n_coeff)
    gen = frozen_flow_frames(cfg, 10 ** 6, 77)
    n, spent = 0, 0.0
    while spent < seconds and n < 1000:
        true = next(gen)
        s = S.apply_A(np.concatenate([p.astype(np.float64).ravel() for p in true]))
        s = s + slope_noise(S.geom.n_slopes, sig, 77, n)
        t0 = time.perf_counter()
        st, _ = frame_fitted(S, fit, st, s) if fit else frame(S, st, s)
        spent += time.perf_counter() - t0
        n += 1
    print(json.dumps({"frames": n, "seconds": spent, "setup_s": setup}))


def cpu_start(workload, seconds):
    """Starts the oracle timing child (one thread) so that it runs while the
    GPU legs run on the device."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-child", workload, "--cpu-seconds",
                             str(seconds)], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def cpu_host():
    """The host CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_finish(proc, workload, iters_text):
    try:
        out, err = proc.communicate(timeout=900)
    except subprocess.TimeoutExpired:
        proc.kill()
        return None
    if proc.returncode != 0:
        sys.stderr.write(err)
        return None
    r = json.loads(out.strip().splitlines()[-1])
    model, ncore = cpu_host()
    return {"value": r["frames"] / r["seconds"], "unit": "frames/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "cores_available": ncore,
            "sample": "%d consecutive %s frames (%s) of the FP64 scipy oracle, one thread (OMP/BLAS 1), "
                      "%.1f s of CPU time, run beside the GPU legs on a core of its own; set-up (operators, exact "
                      "J%s) %.1f s, excluded" % (r["frames"], workload, iters_text, r["seconds"],
                                                 ", fitting operators" if workload == "large" else "",
                                                 r["setup_s"])}


# ------------------------------------------------------------ GPU legs

def algorithmic_bytes(cfg, n_slopes, n_corners, res=128):
    """Bytes each stage moves per problem when every operand is read once
    and every result written once (FP32), with resident transform side res.
    n_slopes counts the active subapertures' slopes (sum over sensors of
    2 |M_g|), n_corners the sensors' corner grids."""
    n_c = sum(l["n"] ** 2 for l in cfg["layers"])
    n_res = sum(min(l["n"], res) ** 2 for l in cfg["layers"])
    # global levels: output (inverse) / input (forward) sides 2 res .. n
    glob = [m for l in cfg["layers"] for m in (2 ** k for k in range(1, 16)) if res < m <= l["n"]]
    return {
        # r, J^{-1}, p_old read, p_new and the output written per coefficient
        "IDWT_RES": 4 * 5 * n_res,
        # coarse block + 3 detail quadrants x (r, J^{-1}, p_old) read, p_new and the output written
        "IDWT_GLOB": 4 * sum(17 * (m // 2) ** 2 for m in glob),
        "P_GAMMA": 4 * (n_c + n_slopes),
        "GAMMA_T": 4 * (n_slopes + n_corners),
        "P_T": 4 * (n_corners + n_c),
        # input read, coarse block written, epilogue p read and q written for 3 quadrants
        "FDWT_GLOB": 4 * sum(11 * (m // 2) ** 2 for m in glob),
        # input read, epilogue p read and q written per coefficient
        "FDWT_RES": 4 * 3 * n_res,
        # x, p, r, q, J^{-1} read, x and r written
        "UPDATE": 4 * 7 * n_c,
    }


def path_bytes(n_c, n_corners, n_slopes, iters):
    """Algorithmic bytes of one whole frame (FP32, each operator of the
    paper's factorisation reads its input once and writes its output once):
    B_frame = B_rhs + iters (B_apply + B_vec) + B_out with
      B_apply = 4 (6 N_c + 4 sum V + 2 sum S)   one application of M
      B_vec   = 4 * 15 N_c                       PCG vector work of an iteration
      B_rhs   = 4 (2 sum S + 2 sum V + 7 N_c)    right-hand side and warm restart
      B_out   = 4 * 5 N_c                        W^{-1} and the control update
    (sum V: corner values, sum S: active slopes; the DM-fitting CG of the
    9-layer system is not counted)."""
    b_apply = 4 * (6 * n_c + 4 * n_corners + 2 * n_slopes)
    b_vec = 4 * 15 * n_c
    b_rhs = 4 * (2 * n_slopes + 2 * n_corners + 7 * n_c)
    return b_rhs + iters * (b_apply + b_vec) + 4 * 5 * n_c


def path_rate(bytes_per_frame, frames_per_s, peaks):
    """A frame rate as whole-path GB/s and its fractions of the HBM peak and
    of the measured copy rates."""
    gbs = bytes_per_frame * frames_per_s / 1e9
    out = {"GBs": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS}
    if peaks:
        out["frac_of_measured_hbm_copy"] = gbs / peaks["hbm_copy_GBs"]
        out["frac_of_measured_mall_copy"] = gbs / peaks["mall_copy_GBs"]
    return out


def launches_per_frame(cfg, res, iters, fuse=False):
    """Kernel launches of one open-loop frame of one problem (plain PCG):
    slope input, sensor adjoint, propagation adjoint and forward transform
    for the right-hand side; per iteration the inverse transform, the
    propagation and sensor stages, the forward transform and the update;
    the final inverse transform.  A transform is one resident launch plus
    one launch per level of output side above the resident side res (with
    fused global levels, a layer's top two such levels are one launch)."""
    def glob(l):
        ng = sum(1 for k in range(1, 16) if res < 2 ** k <= l["n"])
        return ng - 1 if fuse and ng >= 2 else ng
    g = max(glob(l) for l in cfg["layers"])
    return 3 + (1 + g) + iters * (2 * (1 + g) + 4) + (1 + g)


def corner_count(cfg):
    return sum((w["n_subap"] + 1) ** 2 for w in cfg["wfs"])


def measured_traffic(stage, batch, tuning):
    """Bytes per launch of a stage from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when it was taken on other kernel code, another
    batch size or other launch shapes."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "fewha_internal.h", "api.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2202_11945_amd", "csrc", f), "rb").read())
    sha = h.hexdigest()[:16]
    tune = "%d/%d/%d/%d/%d" % (tuning["dwt_resident"], tuning["pt_rows"], tuning.get("res_split", 0),
                               tuning.get("pt_split", 0), tuning.get("glob_fuse", 0))
    prof = os.path.join(ROOT, "profiles", "stages_maory_like_b%d_bytes.md" % batch)
    if not os.path.exists(prof):
        return None
    for line in open(prof):
        f = line.split()
        if (len(f) == 6 and f[0] == "TRAFFIC" and f[1] == stage and int(f[2]) == batch and f[4] == sha
                and f[5] == tune):
            return float(f[3])
    return None


def pool_index(i, n):
    """Frame of an n-frame pool used at step i: forward then backward through
    the pool (0, 1, .., n-1, n-2, .., 1, 0, 1, ..), so that consecutive steps
    always use frames one frozen-flow step apart and the warm start never
    jumps across the pool."""
    if n <= 1:
        return 0
    k = i % (2 * n - 2)
    return k if k < n else 2 * n - 2 - k


def measure_peaks():
    """Achievable bandwidths of this device, measured with torch's copy and
    sum kernels: a 1 GiB copy (HBM, read + write) and a 1 GiB sum (HBM read),
    and the same on 32 MiB buffers replayed hot (a 64 MiB copy working set,
    held by the 256 MB MALL).  GB/s = bytes moved / time, HIP events."""
    import torch
    out = {}
    for name, nbytes, reps in (("hbm", 1 << 30, 20), ("mall", 32 << 20, 400)):
        n = nbytes // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty(n, device="cuda")
        for kind in ("copy", "read"):
            run = (lambda: dst.copy_(src)) if kind == "copy" else (lambda: src.sum())
            for _ in range(3):
                run()
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(reps):
                run()
            t1.record()
            t1.synchronize()
            moved = nbytes * (2 if kind == "copy" else 1)
            out["%s_%s_GBs" % (name, kind)] = moved * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
        del src, dst
    torch.cuda.empty_cache()
    return out


def problem_bytes(fw, ctx, res):
    """algorithmic_bytes of a context's configuration, with its active slope count."""
    cfg = ctx.cfg
    n_cor = sum((w["n_subap"] + 1) ** 2 for w in cfg["wfs"])
    return algorithmic_bytes(cfg, ctx.n_slopes, n_cor, res)


def stage_roofline(fw, batch, ctxs, tuning, iters, peaks, reps=50):
    """Per-stage launch times of a batch (HIP events on its stream), the
    stage with the largest share of a frame and its roofline figures."""
    stage_us = {}
    for sid, name in enumerate(STAGES):
        stage_us[name] = batch.time_stage(sid, reps=reps)
    launches = {"IDWT_RES": iters + 1, "IDWT_GLOB": iters + 1, "P_GAMMA": iters, "GAMMA_T": iters + 1,
                "P_T": iters + 1, "FDWT_GLOB": iters + 1, "FDWT_RES": iters + 1, "UPDATE": iters}
    share = {k: stage_us[k][0] * launches[k] for k in STAGES if stage_us[k][1] > 0}
    dom = max(share, key=share.get)
    per = [problem_bytes(fw, c, tuning["dwt_resident"]) for c in ctxs]
    dom_bytes = sum(b[dom] for b in per)
    us = stage_us[dom][0]
    achieved = dom_bytes / (us * 1e-6) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": dom_bytes,
            "problems_per_launch": len(ctxs), "avg_launch_us": us}
    if peaks:
        roof["frac_of_measured_hbm_copy"] = achieved / peaks["hbm_copy_GBs"]
        roof["frac_of_measured_mall_copy"] = achieved / peaks["mall_copy_GBs"]
    stage_frac = {k: (sum(b[k] for b in per) / (stage_us[k][0] * 1e-6) / 1e9) / HBM_PEAK_GBS
                  for k in STAGES if stage_us[k][1] > 0}
    return stage_us, roof, stage_frac


def config3_leg(fw, peaks, replays=1000):
    """The batched workload of uneven sizes: 64 independent reconstructions
    (32 MAORY-like, 32 VLT-like, each with its own Cn2 weights, r0 and sigma),
    6 PCG iterations, one graph replay per step, autotuned launch shapes."""
    import numpy as np
    import torch
    from paper_2202_11945_amd import autotune
    from synthetic import frozen_flow_frames, slope_noise
    from synthetic.configs import batch_mix
    cfgs = batch_mix(32, 32, 3)
    ctxs = [fw.Context(c, device=0) for c in cfgs]
    pool = []
    for k, (c, cfg) in enumerate(zip(ctxs, cfgs)):
        mask = c.get_table(fw._abi.FEWHA_TABLE_MASK)
        per, o = [], 0
        for w in cfg["wfs"]:
            per.append(2 * int(mask[o:o + w["n_subap"] ** 2].sum()))
            o += w["n_subap"] ** 2
        frames = []
        for f, true in enumerate(frozen_flow_frames(cfg, 4, 3000 + k)):
            phi = torch.from_numpy(np.concatenate([p.ravel() for p in true])).cuda()
            s = c.apply_A(phi)
            s += torch.from_numpy(slope_noise(per, [w["sigma"] for w in cfg["wfs"]], 3000 + k, f)).cuda()
            frames.append(s)
        pool.append(frames)
    tune = autotune.tune(ctxs, 6)
    batch = fw.Batch(ctxs, tuning=tune)
    states = [torch.zeros(c.n_state, device="cuda") for c in ctxs]

    def step(i):
        batch.reconstruct([pool[k][pool_index(i, 4)] for k in range(len(ctxs))], states, iters=6, use_graph=True)

    for i in range(10):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(replays):
        step(10 + i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / replays
    # the same frames as 64 sequential plain-path reconstructions
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(3):
        for k, c in enumerate(ctxs):
            c.reconstruct(pool[k][pool_index(i, 4)], states[k], iters=6)
    torch.cuda.synchronize()
    plain = 3 * len(ctxs) / (time.perf_counter() - t0)
    tb = batch if tune.get("streams", 1) == 1 else None
    out = {"workload": "64 independent reconstructions: 32 MAORY-like + 32 VLT-like (8 m, 4 LGS 40x40, 5 layers "
                       "64x64), own Cn2 / r0 / sigma each, 6 PCG iterations, one graph replay per step",
           "frames_per_s": len(ctxs) / dt, "ms_per_step": dt * 1e3, "steps": replays,
           "plain_path_frames_per_s": plain, "speedup_vs_plain": len(ctxs) / dt / plain, "tuning": tune}
    step_bytes = sum(path_bytes(c.n_coeff, corner_count(cfg), c.n_slopes, 6) for c, cfg in zip(ctxs, cfgs))
    out["path_roofline"] = dict(path_rate(step_bytes, 1.0 / dt, peaks), bytes_per_replay=step_bytes)
    if tb is None:  # stage times need the single-stream plan: time a copy built with streams = 1
        tb = fw.Batch(ctxs, tuning=dict(tune, streams=1))
        tb.reconstruct([pool[k][0] for k in range(len(ctxs))], [s.clone() for s in states], iters=6,
                       use_graph=True)
    stage_us, roof, frac = stage_roofline(fw, tb, ctxs, tune, 6, peaks)
    out["stage_us"] = {k: round(v[0], 3) for k, v in stage_us.items()}
    out["stage_hbm_frac"] = {k: round(v, 3) for k, v in frac.items()}
    out["roofline"] = roof
    if tb is not batch:
        tb.close()
    batch.close()
    for c in ctxs:
        c.close()
    return out


def config5_leg(fw, peaks, replays=5, B=32):
    """The large workload: 9 layers (0-20 km, 256 x 256 above 10 km), 6 LGS
    80x80 with 2x2 spot-elongation noise blocks, 20 PCG iterations, then the
    fitting CG onto 3 DMs over 9 directions; 32 independent frame sequences
    of the same system per graph replay."""
    import numpy as np
    import torch
    from synthetic import frozen_flow_frames, get_config
    cfg = get_config("large")
    t0 = time.time()
    ctx = fw.Context(cfg, device=0)
    setup_s = time.time() - t0
    batch = fw.Batch([ctx] * B)
    slopes = []
    for k, true in enumerate(frozen_flow_frames(cfg, 2, 5000)):
        phi = torch.from_numpy(np.concatenate([p.ravel() for p in true])).cuda()
        slopes.append(ctx.apply_A(phi))
    states = [torch.zeros(ctx.n_state, device="cuda") for _ in range(B)]
    for i in range(2):
        batch.reconstruct([slopes[(i + k) % 2] for k in range(B)], states, iters=20, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(replays):
        batch.reconstruct([slopes[(i + k) % 2] for k in range(B)], states, iters=20, use_graph=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / replays
    fb = path_bytes(ctx.n_coeff, corner_count(cfg), ctx.n_slopes, 20)
    batch.close()
    ctx.close()
    return {"workload": "9 layers (0-20 km; 128x128 up to 10 km, 256x256 above), 6 LGS 80x80 with 2x2 "
                        "elongation noise blocks, 20 PCG iterations, fitting CG (10 iterations) onto 3 DMs over "
                        "9 directions; %d sequences per graph replay" % B,
            "frames_per_s": B / dt, "ms_per_step": dt * 1e3, "steps": replays, "context_setup_s": setup_s,
            "path_roofline": dict(path_rate(fb, B / dt, peaks), bytes_per_frame=fb,
                                  note="the fitting CG's bytes are not counted")}


def latency(run, nf):
    """p50 / p99 of per-call device time (HIP events around each call on the
    current stream, synchronized after each) over frames nf/10 .. nf - 1 of
    a sequence of nf frames (the first tenth is the warm-up: frames 100..999
    of 1000 by default), and the back-to-back rate."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nf)]
    for i in range(nf):
        ev[i][0].record()
        run(i)
        ev[i][1].record()
        torch.cuda.synchronize()
    per_frame = sorted(a.elapsed_time(b) * 1e3 for a, b in ev[nf // 10:])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nf):
        run(i)
    torch.cuda.synchronize()
    return {"p50_us": per_frame[len(per_frame) // 2], "p99_us": per_frame[int(0.99 * (len(per_frame) - 1))],
            "back_to_back_us": (time.perf_counter() - t0) / nf * 1e6}


def paper_maory_leg(fw, nf=1000):
    """The paper's own MAORY system (37 m, 11 % obstruction, 6 LGS 74x74 + 3
    NGS, layers 128/64/64 at 0/4/12.7 km): single-frame latency of the graph
    path (autotuned) at 2 and 4 PCG iterations, beside the paper's 1.48 ms."""
    import numpy as np
    import torch
    from paper_2202_11945_amd import autotune
    from synthetic import frozen_flow_frames, get_config
    cfg = get_config("paper_maory")
    ctx = fw.Context(cfg, device=0)
    slopes = []
    for true in frozen_flow_frames(cfg, 4, 6000):
        phi = torch.from_numpy(np.concatenate([p.ravel() for p in true])).cuda()
        slopes.append(ctx.apply_A(phi))
    out = {"workload": "paper MAORY: 37 m, 6 LGS 74x74 + 3 NGS 2x2, layers 128/64/64, single frame, graph path",
           "paper_us_per_frame_2_iters": 1480.0}
    for iters in (2, 4):
        tune = autotune.tune([ctx], iters)
        b = fw.Batch([ctx], tuning=tune)
        st = torch.zeros(ctx.n_state, device="cuda")
        lay = torch.empty(ctx.n_coeff, device="cuda")
        lat = latency(lambda i: b.reconstruct([slopes[pool_index(i, 4)]], [st], [lay], iters=iters,
                                              use_graph=True), nf)
        fb = path_bytes(ctx.n_coeff, corner_count(cfg), ctx.n_slopes, iters)
        out["iters_%d" % iters] = dict(lat, tuning={k: tune[k] for k in ("dwt_resident", "pt_rows", "pt_split", "glob_fuse")},
                                       speedup_vs_paper=1480.0 / lat["p50_us"] if iters == 2 else None,
                                       bytes_per_frame=fb, path_GBs=fb / lat["p50_us"] / 1e3)
        b.close()
    # the paper's own setting: 2 iterations of the augmented PCG (the
    # previous frame's 2 directions), the like-for-like comparison
    ca = fw.Context(dict(cfg, augment=2), device=0)
    tune = autotune.tune([ca], 2)
    b = fw.Batch([ca], tuning=tune)
    st = torch.zeros(ca.n_state, device="cuda")
    lay = torch.empty(ca.n_coeff, device="cuda")
    lat = latency(lambda i: b.reconstruct([slopes[pool_index(i, 4)]], [st], [lay], iters=2, use_graph=True), nf)
    out["iters_2_augmented"] = dict(lat, tuning={k: tune[k] for k in ("dwt_resident", "pt_rows", "pt_split", "glob_fuse")},
                                    speedup_vs_paper=1480.0 / lat["p50_us"])
    b.close()
    ca.close()
    ctx.close()
    return out


def streamed_leg(fw, c0, pool_host, iters, nf=100):
    """Single-frame latency with the slopes in pinned host memory: the frame
    takes them in by sensor groups as their host-to-device copies land
    (1 group = copy then frame), open and closed loop; PCIe included."""
    import torch
    from synthetic import get_config
    out = {}
    st = torch.zeros(c0.n_state, device="cuda")
    lay = torch.empty(c0.n_coeff, device="cuda")
    for chunks in (1, 3, 9):
        out["open_%d_groups" % chunks] = latency(
            lambda i: c0.reconstruct_streamed(pool_host[pool_index(i, len(pool_host))], st, lay, iters=iters,
                                              chunks=chunks), nf)
    cl = fw.Context(get_config("maory_like", loop="closed", gain=0.5), device=0)
    stc = torch.zeros(cl.n_state, device="cuda")
    for chunks in (1, 3, 9):
        out["closed_%d_groups" % chunks] = latency(
            lambda i: cl.reconstruct_streamed(pool_host[pool_index(i, len(pool_host))], stc, lay, iters=iters,
                                              chunks=chunks), nf)
    cl.close()
    return out


def augmentation_leg(fw, cfg, pool_dev, n_frames=16, iters=2, keep=2, nf=100):
    """Warm-started frames at `iters` PCG iterations with and without the
    augmented PCG (Sec. 3.3), on one MAORY-like frozen-flow sequence: the
    M-norm error of c against the converged MAP solution of each frame
    (fewha_solve_map, refined to 1e-7), and the single-frame latency of both
    (graph path, autotuned launch shapes)."""
    import torch
    ctx_p = fw.Context(dict(cfg, iters=iters), device=0)
    ctx_a = fw.Context(dict(cfg, iters=iters, augment=keep), device=0)
    runs = {"plain": (ctx_p, iters), "augmented": (ctx_a, iters), "plain_%d_iterations" % (2 * iters): (ctx_p, 2 * iters)}
    st = {name: torch.zeros(c.n_state, device="cuda") for name, (c, _) in runs.items()}
    n = ctx_p.n_coeff
    err = {name: [] for name in runs}
    for k in range(n_frames):
        s = pool_dev[pool_index(k, len(pool_dev))]
        for name, (c, it) in runs.items():
            c.reconstruct(s, st[name], iters=it)
        cstar, _, _ = ctx_p.solve_map(slopes=s, rtol=1e-7, max_iters=20000)
        mstar = ctx_p.apply_M(cstar)
        norm = float(torch.dot(cstar.double(), mstar.double()))
        for name in runs:
            e = st[name][:n] - cstar
            err[name].append((float(torch.dot(e.double(), ctx_p.apply_M(e).double())) / norm) ** 0.5)
    out = {"workload": "MAORY-like, one frozen-flow sequence of %d frames, %d warm PCG iterations per frame; "
                       "augmented: the previous frame's %d directions; plain PCG also at %d iterations"
                       % (n_frames, iters, keep, 2 * iters),
           "m_norm_error_plain": err["plain"], "m_norm_error_augmented": err["augmented"],
           "mean_error_frames_4_on": {k: sum(v[4:]) / len(v[4:]) for k, v in err.items()}}
    from paper_2202_11945_amd import autotune
    for name, (c, it) in runs.items():
        b = fw.Batch([c], tuning=autotune.tune([c], it))
        s1 = torch.zeros(c.n_state, device="cuda")
        out["latency_us_" + name] = latency(lambda i: b.reconstruct([pool_dev[pool_index(i, len(pool_dev))]], [s1],
                                                                    iters=it, use_graph=True), nf)
        b.close()
    ctx_p.close()
    ctx_a.close()
    return out


def gradient_leg(fw, pool, n_frames, rtol=1e-6):
    """Forward + implicit backward of the differentiated reconstruction on
    MAORY-like geometry: n_frames frames per batch, both solves refined to
    rtol, a fixed random upstream gradient dL/dphi."""
    import torch
    from paper_2202_11945_amd.autograd import FrameBatch, MAPLayers, param_vector
    from synthetic import get_config, random_vector
    cfg = get_config("grad_maory")
    fb = FrameBatch(cfg, n_frames)
    slopes = torch.stack([pool[k % len(pool)][0] for k in range(n_frames)])
    g = torch.from_numpy(random_vector(n_frames * fb.ctx.n_coeff, 77).reshape(n_frames, -1) * 1e-3).cuda()
    params = param_vector(cfg).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi = MAPLayers.apply(params, slopes, fb, rtol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phi.backward(g)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fb.close()
    print("[bench] gradient leg: forward %.1f ms, backward %.1f ms" % ((t1 - t0) * 1e3, (t2 - t1) * 1e3),
          file=sys.stderr, flush=True)
    return {"workload": "MAORY-like geometry, %d frames per batch, forward and adjoint solves refined to a "
                        "relative residual %g" % (n_frames, rtol),
            "forward_ms": (t1 - t0) * 1e3, "backward_ms": (t2 - t1) * 1e3,
            "grad": [float(v) for v in params.grad]}


def main():
    args = parse()
    if args.cpu_child:
        cpu_child(args.cpu_child, args.cpu_seconds)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the batch of independent frame sequences is the unit that would shard across GPUs)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    # the oracle's timing runs on host cores of its own while the GPU legs run
    cpu_jobs = {} if args.no_cpu_baseline else {w: cpu_start(w, args.cpu_seconds) for w in ("maory_like", "large")}

    import numpy as np
    import torch

    import paper_2202_11945_amd as fw
    from synthetic import frozen_flow_frames, get_config, slope_noise

    dev = torch.device("cuda:0")
    cfg = get_config(WORKLOAD)
    B = args.batch
    t_setup = time.time()
    ctxs = [fw.Context(cfg, device=0) for _ in range(B)]
    c0 = ctxs[0]
    print("[bench] %d contexts set up in %.1f s" % (B, time.time() - t_setup), file=sys.stderr, flush=True)

    # ---- inputs: slopes of frozen-flow screens through A, plus noise ----
    sig = [w["sigma"] for w in cfg["wfs"]]
    mask = c0.get_table(fw._abi.FEWHA_TABLE_MASK)  # per-sensor slope counts for the noise
    per = []
    o = 0
    for w in cfg["wfs"]:
        nn = w["n_subap"] ** 2
        per.append(2 * int(mask[o:o + nn].sum()))
        o += nn
    assert sum(per) == c0.n_slopes
    pool = []
    t_in = time.time()
    for k in range(B):
        frames = []
        for f, true in enumerate(frozen_flow_frames(cfg, args.pool, 1000 + k)):
            phi = torch.from_numpy(np.concatenate([p.ravel() for p in true])).to(dev)
            s = c0.apply_A(phi)
            s += torch.from_numpy(slope_noise(per, sig, 1000 + k, f)).to(dev)
            frames.append(s)
        pool.append(frames)
    torch.cuda.synchronize()
    print("[bench] inputs generated in %.1f s" % (time.time() - t_in), file=sys.stderr, flush=True)

    # ---- launch shapes from the autotuner (cached per device and shapes) ----
    from paper_2202_11945_amd import autotune
    default = {"dwt_resident": 128, "pt_rows": 4, "streams": 1, "cached": None}
    tune_b = autotune.tune(ctxs, args.iters) if not args.no_tune else default
    tune_1 = autotune.tune([c0], args.iters) if not args.no_tune else default
    H = B // 2
    tune_h = (autotune.tune(ctxs[:H], args.iters) if not args.no_tune else default) if H >= 1 else None
    print("[bench] tuning: batch %s, half %s, single %s" % (tune_b, tune_h, tune_1), file=sys.stderr,
          flush=True)

    # ---- batched graph path: the timed workload ----
    # The B sequences run either as one batch on the bench stream, or as two
    # batches of B/2 on two streams of their own (each batch stream-ordered;
    # a half's next frame may then overlap the other half's current one).
    # Both are timed briefly first and the faster is the timed workload.
    batch = fw.Batch(ctxs, tuning=tune_b)
    states = [torch.zeros(c.n_state, device=dev) for c in ctxs]
    halves = None
    if H >= 1:
        # the two streams are the overlap: no stream parts inside a half
        tune_h = dict(tune_h, streams=1)
        halves = [(fw.Batch(ctxs[:H], tuning=tune_h), 0, H, torch.cuda.Stream()),
                  (fw.Batch(ctxs[H:], tuning=tune_h), H, B, torch.cuda.Stream())]

    def step_one(i, use_graph=True):
        batch.reconstruct([pool[k][pool_index(i, args.pool)] for k in range(B)], states, iters=args.iters,
                          use_graph=use_graph)

    def step_two(i, use_graph=True):
        for hb, k0, k1, st in halves:
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                hb.reconstruct([pool[k][pool_index(i, args.pool)] for k in range(k0, k1)], states[k0:k1],
                               iters=args.iters, use_graph=use_graph)

    def rate(run, n, first):
        for i in range(5):
            run(first + i)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(n):
            run(first + 5 + i)
        torch.cuda.synchronize()
        return B * n / (time.perf_counter() - t)

    split = {"one_batch_frames_per_s": rate(step_one, 20, 0)}
    if halves:
        split["two_halves_frames_per_s"] = rate(step_two, 20, 0)
    two = halves is not None and split["two_halves_frames_per_s"] > split["one_batch_frames_per_s"]
    split["timed"] = ("two batches of %d on two streams" % H) if two else ("one batch of %d" % B)
    print("[bench] split: %s" % split, file=sys.stderr, flush=True)
    step = step_two if two else step_one

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    value = B / dt
    print("[bench] batched graph path: %.3f ms/step, %.0f frames/s" % (dt * 1e3, value), file=sys.stderr,
          flush=True)

    # ---- same batch, direct launches (no graph) ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nd = max(10, args.steps // 4)
    for i in range(nd):
        step(i, use_graph=False)
    torch.cuda.synchronize()
    dt_nograph = (time.perf_counter() - t0) / nd

    # ---- single-frame latency: graph path (batch of one) and plain path ----
    single = fw.Batch([c0], tuning=tune_1)
    st1 = torch.zeros(c0.n_state, device=dev)
    lay1 = torch.empty(c0.n_coeff, device=dev)
    nf = args.latency_frames

    lat_graph = latency(lambda i: single.reconstruct([pool[0][pool_index(i, args.pool)]], [st1], [lay1],
                                                     iters=args.iters, use_graph=True), nf)
    lat_plain = latency(lambda i: c0.reconstruct(pool[0][pool_index(i, args.pool)], st1, lay1, iters=args.iters), nf)

    # plain path over the whole batch: B sequential unbatched, ungraphed frames
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    npl = 5
    for i in range(npl):
        for k in range(B):
            ctxs[k].reconstruct(pool[k][pool_index(i, args.pool)], states[k], iters=args.iters)
    torch.cuda.synchronize()
    plain_fps = B * npl / (time.perf_counter() - t0)

    # ---- per-stage kernel time (HIP events on the batch stream), in the
    # launch configuration of the timed step (one launch per batch) ----
    peaks = None if args.no_extra else measure_peaks()
    print("[bench] measured peaks: %s" % peaks, file=sys.stderr, flush=True)
    tb, tb_ctxs, tune_t = (halves[0][0], ctxs[:H], tune_h) if two else (batch, ctxs, tune_b)
    nb_prob = len(tb_ctxs)
    stage_us, roof, stage_frac = stage_roofline(fw, tb, tb_ctxs, tune_t, args.iters, peaks)
    dom = roof["kernel"]
    roof["traffic"] = measured_traffic(dom, nb_prob, tune_t)

    frame_b = path_bytes(c0.n_coeff, corner_count(cfg), c0.n_slopes, args.iters)
    extra = {}
    if not args.no_extra:
        pool_host = [pool[0][f].cpu().pin_memory() for f in range(args.pool)]
        for name, leg in (("augmented_pcg", lambda: augmentation_leg(fw, cfg, pool[0])),
                          ("streamed_slopes_us", lambda: streamed_leg(fw, c0, pool_host, args.iters)),
                          ("paper_maory", lambda: paper_maory_leg(fw)),
                          ("batched_uneven_64", lambda: config3_leg(fw, peaks)),
                          ("large_9_layers", lambda: config5_leg(fw, peaks))):
            t_leg = time.time()
            extra[name] = leg()
            print("[bench] %s leg: %.1f s" % (name, time.time() - t_leg), file=sys.stderr, flush=True)

    grad = None if args.grad_frames <= 0 else gradient_leg(fw, pool, args.grad_frames)

    cpu = cpu_finish(cpu_jobs["maory_like"], "MAORY-like", "RHS, warm restart, 4 PCG iterations, W^-1, control") \
        if cpu_jobs else None
    cpu5 = cpu_finish(cpu_jobs["large"], "large 9-layer", "20 PCG iterations, fitting CG onto 3 DMs") \
        if cpu_jobs else None

    out = {
        "metric": "FEWHA µs/frame and batched frames/s, MAORY-like FP32 vs plain GPU path",
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 PCG inner products and alpha/beta)",
        "data": "synthetic: frozen-flow von Karman screens (r0 0.157 m, L0 25 m, Cn2 0.75/0.15/0.10) "
                "through A plus Gaussian slope noise (sigma 0.1 rad), %d frames per sequence" % args.pool,
        "config": {"workload": "MAORY-like FEWHA: 39 m, 6 LGS 80x80 (TT removed) + 3 NGS 2x2, layers "
                               "128/128/256 at 0/4/12.7 km, D3 5 levels, %d warm PCG iterations; "
                               "%d independent sequences per step, %s, graph replays"
                               % (args.iters, B, split["timed"]),
                   "batch": B, "iters": args.iters, "n_coeff": c0.n_coeff, "n_slopes": c0.n_slopes},
        "path_roofline": {
            "accounting": "B_frame = B_rhs + iters (B_apply + B_vec) + B_out, every operator's input read once "
                          "and output written once (FP32)",
            "bytes_per_frame": frame_b,
            "batched": path_rate(frame_b, value, peaks),
            "single_frame_graph_p50": path_rate(frame_b, 1e6 / lat_graph["p50_us"], peaks),
            "launches_per_frame_single": launches_per_frame(cfg, tune_1["dwt_resident"], args.iters,
                                                            bool(tune_1.get("glob_fuse", 0)))},
        "latency_graph_us": lat_graph,
        "latency_plain_us": lat_plain,
        "batched_nograph_frames_per_s": B / dt_nograph,
        "plain_path_frames_per_s": plain_fps,
        "speedup_vs_plain": value / plain_fps,
        "tuning": {"batch": tune_b, "half_batch": tune_h, "single_frame": tune_1},
        "batch_split": split,
        "gradient": grad,
        "stage_us": {k: round(v[0], 3) for k, v in stage_us.items()},
        "stage_workgroups": {k: v[1] for k, v in stage_us.items()},
        "stage_hbm_frac": {k: round(v, 3) for k, v in stage_frac.items()},
        "measured_peaks_GBs": peaks,
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_baseline_large": cpu5,
        "paper_context": {"us_per_frame": 1480.0, "hardware": "2x Xeon E5-2630v3, 9 OpenMP threads + AVX2",
                          "workload": "paper MAORY (37 m, 6 LGS 74x74, layers 128/64/64), 2 augmented-PCG "
                                      "iterations"},
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
