"""Benchmark: FIFA-GP Gibbs iterations per second on one MI355X.

A step is one full Gibbs sweep (f by Algorithm 1 -> tau -> sigma_f^-2 -> length-scale
Metropolis step, including the HODLR build and both factorizations) of the large 1-D
workload: n = 2^20 sorted inputs, squared-exponential kernel, leaf 128, tol 1e-10,
ell0 = 0.02, FP64 throughout.  Inputs are synthetic (workloads.large_1d) and resident
in HBM before the timed region.

Prints one JSON line (metric, value, roofline of the dominant kernel, CPU oracle
baseline).  Only one GPU is used: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=None, help="override n (testing only)")
    ap.add_argument("--kernel", type=int, default=1,
                    help="kernel timed for the roofline: 1 leaf, 2 level reduce, 3 level update")
    return ap.parse_args()


def cpu_baseline(x, y, cfg):
    """The oracle as it stands, on the host cores: one full Gibbs sweep of the same
    workload (chain set-up untimed)."""
    from threadpoolctl import threadpool_info

    from oracle import kernels, sampler
    ch = sampler.Chain(x, y, kernels.SE, cfg["ell0"], cfg["nugget"], cfg["leaf"], cfg["tol"],
                       cfg["tau0"], cfg["sigf2_0"], cfg["seed"])
    t0 = time.perf_counter()
    ch.step()
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": 1.0 / dt, "unit": "Gibbs iters/s", "cores": threads, "kind": "oracle",
            "sample": f"one Gibbs sweep of the same n={x.size} chain (set-up untimed), "
                      f"{dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU layout is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2006_06537_amd as fg
    from workloads import LARGE_1D, large_1d, sinusoid_1d

    cfg = dict(LARGE_1D)
    if args.n:
        cfg["n"] = args.n
        x, y = sinusoid_1d(args.n, seed=cfg["seed"])
    else:
        x, y = large_1d(cfg["n"], cfg["seed"])
    dev = torch.device("cuda:0")
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    chain = fg.Chain(xt, yt, ell0=cfg["ell0"], tau0=cfg["tau0"], sigf2_0=cfg["sigf2_0"],
                     nugget=cfg["nugget"], leaf=cfg["leaf"], tol=cfg["tol"], seed=cfg["seed"])
    print(f"bench: chain ready (n={cfg['n']})", file=sys.stderr, flush=True)
    chain.step(args.warmup)
    torch.cuda.synchronize()
    print(f"bench: {args.warmup} warm-up sweeps done", file=sys.stderr, flush=True)
    timer = fg.KernelTimer(args.kernel)
    timer.start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ktime_ms, launches, kbytes = timer.stop()
    st = chain.state()
    print(f"bench: {args.steps} timed sweeps in {dt:.3f} s; status {st['status']}, "
          f"accepts {st['accepts']}, ell {st['ell']:.4g}, tau {st['tau']:.4g}",
          file=sys.stderr, flush=True)
    roof = None
    if launches > 0 and ktime_ms > 0:
        achieved = kbytes / (ktime_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": timer.name, "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None, "launches": launches,
                "avg_launch_us": 1e3 * ktime_ms / launches,
                "algorithmic_bytes_per_launch": kbytes / launches}
    out = {
        "metric": "Gibbs iters/s at n=2^20 (FP64)",
        "value": args.steps / dt,
        "unit": "Gibbs iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "large_1d: single FP64 chain, n=2^20 sorted U[0,1], 5-sinusoid y "
                               "+ N(0,0.05^2), SE kernel ell0=0.02 (100-point grid), leaf 128, "
                               "tol 1e-10, nugget 1e-6",
                   "n": cfg["n"], "leaf": cfg["leaf"], "tol": cfg["tol"], "ell0": cfg["ell0"]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(x, y, cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
