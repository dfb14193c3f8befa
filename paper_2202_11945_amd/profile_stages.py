"""Stage profiler: one batched step of a workload, then every PCG-iteration
stage launched alone over the whole batch, then a plain 256 MiB device copy
whose byte counters calibrate the hardware FETCH_SIZE / WRITE_SIZE reading.

Run under rocprofv3, e.g.
  rocprofv3 --pmc FETCH_SIZE -d OUT -o fetch --output-format csv -- \
      python3 paper_2202_11945_amd/profile_stages.py --batch 64 --tuned
"""

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="maory_like")
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--iters", type=int, default=4)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--res", type=int, default=0, help="resident transform side (0 = default)")
    ap.add_argument("--pt-rows", type=int, default=0, help="node rows per thread of P^T (0 = default)")
    ap.add_argument("--split", type=int, default=0, help="resident inverse levels: 0 default, 1 or 4 workgroups")
    ap.add_argument("--pt-split", type=int, default=0, help="propagation adjoint: 1 = sensor lists split over waves")
    ap.add_argument("--glob-fuse", type=int, default=0, help="1 = a layer's top two global levels in one launch")
    ap.add_argument("--tuned", action="store_true", help="launch shapes from the autotuner (as bench.py)")
    ap.add_argument("--latency-frames", type=int, default=0,
                    help="then this many single frames of one problem (graph replays, synchronized each)")
    a = ap.parse_args()
    import torch

    import paper_2202_11945_amd as fw
    from synthetic import get_config, random_vector

    cfg = get_config(a.config)
    ctxs = [fw.Context(cfg, device=0) for _ in range(a.batch)]
    tuning = {"dwt_resident": a.res, "pt_rows": a.pt_rows, "res_split": a.split, "pt_split": a.pt_split,
              "glob_fuse": a.glob_fuse}
    if a.tuned:
        from paper_2202_11945_amd import autotune
        rec = autotune.tune(ctxs, a.iters)
        tuning = {k: rec[k] for k in ("dwt_resident", "pt_rows", "res_split", "pt_split", "glob_fuse")}
    print("tuning %d/%d/%d/%d/%d batch %d" % (tuning["dwt_resident"] or 128, tuning["pt_rows"] or 4,
                                              tuning["res_split"], tuning["pt_split"], tuning["glob_fuse"], a.batch),
          flush=True)
    batch = fw.Batch(ctxs, tuning=tuning)
    dev = torch.device("cuda:0")
    slopes = [torch.from_numpy(random_vector(ctxs[0].n_slopes, 5, k)).to(dev) for k in range(a.batch)]
    states = [torch.zeros(c.n_state, device=dev) for c in ctxs]
    for _ in range(2):
        batch.reconstruct(slopes, states, iters=a.iters, use_graph=False)
    torch.cuda.synchronize()
    for sid, name in enumerate(fw._abi.STAGES):
        us, wg = batch.time_stage(sid, reps=a.reps)
        print("stage %-10s %9.2f us  workgroups %d" % (name, us, wg), flush=True)
    if a.latency_frames > 0:
        single = fw.Batch([ctxs[0]], tuning=tuning)
        st = torch.zeros(ctxs[0].n_state, device=dev)
        for _ in range(3):
            single.reconstruct([slopes[0]], [st], iters=a.iters, use_graph=True)
        torch.cuda.synchronize()
        print("single frames start", flush=True)
        for _ in range(a.latency_frames):
            single.reconstruct([slopes[0]], [st], iters=a.iters, use_graph=True)
            torch.cuda.synchronize()
        print("single frames done", flush=True)
        single.close()
    x = torch.empty(64 * 2 ** 20, dtype=torch.float32, device=dev).fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copy 256 MiB x3 done", flush=True)


if __name__ == "__main__":
    main()
