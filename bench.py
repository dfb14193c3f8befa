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
    p.add_argument("--latency-frames", type=int, default=200)
    p.add_argument("--no-tune", action="store_true", help="default launch shapes instead of the autotuner's")
    p.add_argument("--grad-frames", type=int, default=16,
                   help="frames of the forward + implicit-backward leg (0 = skip)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    return p.parse_args()


# ------------------------------------------------------------ CPU oracle leg

def cpu_child(seconds):
    """Runs in a single-threaded child process: times the oracle's time step
    on MAORY-like frames (set-up excluded) and prints frames/s as JSON."""
    import numpy as np
    from oracle.operators import System
    from oracle.solver import State, frame
    from synthetic import frozen_flow_frames, get_config, slope_noise

    cfg = get_config(WORKLOAD)
    S = System(cfg)
    S.preconditioner()
    sig = [w["sigma"] for w in cfg["wfs"]]
    st = State(S.geom.n_coeff, S.geom.n_coeff)
    gen = frozen_flow_frames(cfg, 10 ** 6, 77)
    n, spent = 0, 0.0
    while spent < seconds and n < 1000:
        true = next(gen)
        s = S.apply_A(np.concatenate([p.astype(np.float64).ravel() for p in true]))
        s = s + slope_noise(S.geom.n_slopes, sig, 77, n)
        t0 = time.perf_counter()
        st, _ = frame(S, st, s)
        spent += time.perf_counter() - t0
        n += 1
    print(json.dumps({"frames": n, "seconds": spent}))


def cpu_baseline(seconds):
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", "--cpu-seconds", str(seconds)],
                         env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        sys.stderr.write(out.stderr)
        return None
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": r["frames"] / r["seconds"], "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": "%d consecutive MAORY-like frames (RHS, warm restart, %d PCG iterations, W^-1 and "
                      "control) of the FP64 scipy oracle, single-threaded, %.1f s of CPU time; set-up "
                      "(operators, exact J) excluded" % (r["frames"], 4, r["seconds"])}


# ------------------------------------------------------------ GPU legs

def algorithmic_bytes(cfg, n_slopes_dense, n_corners):
    """Bytes each stage moves per problem when every operand is read once
    and every result written once (FP32)."""
    R = 128
    n_c = sum(l["n"] ** 2 for l in cfg["layers"])
    n_res = sum(min(l["n"], R) ** 2 for l in cfg["layers"])
    glob = [l["n"] for l in cfg["layers"] if l["n"] > R]
    idwt_glob = sum(17 * (m // 2) ** 2 for n in glob for m in [n])  # one global level per layer here
    fdwt_glob = sum(11 * (n // 2) ** 2 for n in glob)
    res_in = sum(min(l["n"], R) ** 2 for l in cfg["layers"])
    return {
        "IDWT_RES": 4 * (4 * n_res + res_in),
        "IDWT_GLOB": 4 * idwt_glob,
        "P_GAMMA": 4 * (n_c + n_slopes_dense),
        "GAMMA_T": 4 * (n_slopes_dense + n_corners),
        "P_T": 4 * (n_corners + n_c),
        "FDWT_GLOB": 4 * fdwt_glob,
        "FDWT_RES": 4 * (res_in + 2 * n_res),
        "UPDATE": 4 * 7 * n_c,
    }


def measured_traffic(stage, batch, tuning):
    """Bytes per launch of a stage from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when it was taken on other kernel code, another
    batch size or other launch shapes."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "fewha_internal.h", "api.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2202_11945_amd", "csrc", f), "rb").read())
    sha = h.hexdigest()[:16]
    tune = "%d/%d" % (tuning["dwt_resident"], tuning["pt_rows"])
    prof = os.path.join(ROOT, "profiles", "stages_maory_like_b%d_bytes.md" % batch)
    if not os.path.exists(prof):
        return None
    for line in open(prof):
        f = line.split()
        if (len(f) == 6 and f[0] == "TRAFFIC" and f[1] == stage and int(f[2]) == batch and f[4] == sha
                and f[5] == tune):
            return float(f[3])
    return None


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
        cpu_child(args.cpu_seconds)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the batch of independent frame sequences is the unit that would shard across GPUs)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

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
        batch.reconstruct([pool[k][i % args.pool] for k in range(B)], states, iters=args.iters,
                          use_graph=use_graph)

    def step_two(i, use_graph=True):
        for hb, k0, k1, st in halves:
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                hb.reconstruct([pool[k][i % args.pool] for k in range(k0, k1)], states[k0:k1], iters=args.iters,
                               use_graph=use_graph)

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

    def lat(run):
        for i in range(10):
            run(i)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nf)]
        for i in range(nf):
            ev[i][0].record()
            run(i)
            ev[i][1].record()
            torch.cuda.synchronize()
        per_frame = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nf):
            run(i)
        torch.cuda.synchronize()
        return {"p50_us": per_frame[len(per_frame) // 2], "p99_us": per_frame[int(0.99 * (len(per_frame) - 1))],
                "back_to_back_us": (time.perf_counter() - t0) / nf * 1e6}

    lat_graph = lat(lambda i: single.reconstruct([pool[0][i % args.pool]], [st1], [lay1], iters=args.iters,
                                                 use_graph=True))
    lat_plain = lat(lambda i: c0.reconstruct(pool[0][i % args.pool], st1, lay1, iters=args.iters))

    # plain path over the whole batch: B sequential unbatched, ungraphed frames
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    npl = 5
    for i in range(npl):
        for k in range(B):
            ctxs[k].reconstruct(pool[k][i % args.pool], states[k], iters=args.iters)
    torch.cuda.synchronize()
    plain_fps = B * npl / (time.perf_counter() - t0)

    # ---- per-stage kernel time (HIP events on the batch stream), in the
    # launch configuration of the timed step (one launch per batch) ----
    stage_us = {}
    tb, nb_prob, tune_t = (halves[0][0], H, tune_h) if two else (batch, B, tune_b)
    for sid, name in enumerate(STAGES):
        us, wg = tb.time_stage(sid, reps=50)
        stage_us[name] = (us, wg)
    launches = {"IDWT_RES": args.iters + 1, "IDWT_GLOB": args.iters + 1, "P_GAMMA": args.iters,
                "GAMMA_T": args.iters + 1, "P_T": args.iters + 1, "FDWT_GLOB": args.iters + 1,
                "FDWT_RES": args.iters + 1, "UPDATE": args.iters}
    share = {k: stage_us[k][0] * launches[k] for k in STAGES}
    dom = max(share, key=share.get)
    n_sd = sum(2 * w["n_subap"] ** 2 for w in cfg["wfs"])
    n_cor = sum((w["n_subap"] + 1) ** 2 for w in cfg["wfs"])
    alg = algorithmic_bytes(cfg, n_sd, n_cor)
    dom_bytes = alg[dom] * nb_prob
    achieved = dom_bytes / (stage_us[dom][0] * 1e-6) / 1e9
    traffic = measured_traffic(dom, nb_prob, tune_t)

    grad = None if args.grad_frames <= 0 else gradient_leg(fw, pool, args.grad_frames)

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds)

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
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": dom_bytes, "problems_per_launch": nb_prob,
                     "avg_launch_us": stage_us[dom][0]},
        "cpu_baseline": cpu,
        "paper_context": {"us_per_frame": 1480.0, "hardware": "2x Xeon E5-2630v3, 9 OpenMP threads + AVX2",
                          "workload": "paper MAORY (37 m, 6 LGS 74x74, layers 128/64/64), 2 augmented-PCG "
                                      "iterations"},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
