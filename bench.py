"""Benchmark: FIFA-GP Gibbs iterations per second on one MI355X.

A step is one full Gibbs sweep (f by Algorithm 1 -> tau -> sigma_f^-2 -> length-scale
Metropolis step, including the HODLR build and both factorizations) of the large 1-D
workload: n = 2^20 sorted inputs, squared-exponential kernel, leaf 128, tol 1e-10,
ell0 = 0.02, FP64 throughout.  Inputs are synthetic (workloads.large_1d) and resident
in HBM before the timed region.

Prints one JSON line (metric, value, roofline of the dominant kernel, CPU oracle
baseline).  Only one GPU is used: --gpus above 1 exits with a message.

Other workloads (--workload), each printing its own JSON line:
  batch   64 independent chains, n = 32,768 each (the large-workload generator with
          seeds 1000 + c), stepped together by gibbs_step_batch in the mode its autotuner
          picks (grouped launches, eager streams or captured graphs); value = chain sweeps
          per second over all chains.  Every mode, and the same chains stepped one after
          the other (gibbs_step), are timed beside it.
  tensor  the d = 4, n = 65,536 tensor-product surface chain; value = sweeps/s.
  copy    a plain 2 GiB FP64 copy kernel (one read, one write of 2 GiB per launch): the
          calibration run for the HBM byte counters (FETCH_SIZE, WRITE_SIZE).
  predict the large 1-D chain with predictive draws at --nstar new inputs
          (workloads.new_inputs) after every sweep (Appendix, function posterior at new
          inputs); W_1^-1 k1(X, X*) kept for up to --zcache grid points.  value = Gibbs
          iterations/s including the draws; the cached and rebuilt draw costs are
          reported beside it, with the roofline of the per-point reduction kernel.
  collapse gridded data with repeats (workloads.gridded_1d: 2^20 observations on 2^14
          grid inputs, 64 each): the chain on the collapsed data (Appendix, non-unique
          input points); value = Gibbs iterations/s, with the plain chain on the raw
          2^20 observations timed beside it.
  exact   the length-scale drawn from its exact grid conditional (gibbs_chain_create_grid:
          all 100 grid factorizations kept), n = 2^17 sinusoid inputs; value = Gibbs
          iterations/s, with the Metropolis chain on the same data beside it and the
          set-up time and device memory of the grid.
  serve   GP-regression jobs of mixed n (workloads.served_jobs) through the serving
          loop: first all at once (saturation throughput), then Poisson arrivals at
          0.7 x that rate; value = p50 latency (s), with p99 and the same arrival list
          run as a sequential FIFO of plain FP64 chains beside it.
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
    ap.add_argument("--workload", default="large_1d",
                    choices=["large_1d", "batch", "tensor", "serve", "copy", "predict",
                             "collapse", "exact"])
    ap.add_argument("--nstar", type=int, default=1024, help="predict: new inputs per draw")
    ap.add_argument("--ncomp", type=int, default=1,
                    help="tensor: additive tensor-product components (ncomp * d <= 8)")
    ap.add_argument("--zcache", type=int, default=8,
                    help="predict: grid points whose W_1^-1 k1(X, X*) is kept")
    ap.add_argument("--jobs", type=int, default=512, help="serve workload: number of jobs")
    ap.add_argument("--job-iters", type=int, default=100, help="serve workload: sweeps per job")
    ap.add_argument("--slots", type=int, default=32, help="serve workload: jobs running at once")
    ap.add_argument("--load", type=float, default=0.7, help="serve: arrival rate / saturation")
    ap.add_argument("--chains", type=int, default=64, help="batch workload: number of chains")
    ap.add_argument("--batch-mode", default="auto", choices=["auto", "grouped", "eager", "graphs"],
                    help="batch workload: one stepping mode only (profiling), or the autotuner")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: M~ factored in FP32, its solves refined by PCG to 1e-10")
    ap.add_argument("--kernel", type=int, default=0,
                    help="kernel of the roofline line: 1 leaf Cholesky, 2 level reduce, 3 level "
                         "update, 4 leaf whitening; 0 (default) = whichever of the four HBM-bound "
                         "factorization kernels (2, 3, 4) takes the most time in the timed region. "
                         "All four are timed in the same region and reported under 'kernels'")
    return ap.parse_args()


def counter_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` (all its template instances, weighted by
    their launch counts) from the committed counter summary, if the library sources are
    still the ones it was taken on (else None)."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_large_1d.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        doc = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2006_06537_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    if h.hexdigest()[:16] != doc.get("source_hash"):
        return None
    # every instance of the kernel (templated variants included), weighted by launches
    rows = [v for k, v in doc["kernels"].items()
            if k == f"fg::{kernel_name}" or k.startswith(f"fg::{kernel_name}<")]
    launches = sum(v["launches"] for v in rows)
    if not launches:
        return None
    return sum(v["traffic_bytes"] * v["launches"] for v in rows) / launches


def bench_copy(args):
    import torch
    n = (2 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    print(json.dumps({"metric": "copy bandwidth (counter calibration)", "value": 2 * 8 * n / dt / 1e9,
                      "unit": "GB/s", "bytes_read_per_launch": 8 * n,
                      "bytes_written_per_launch": 8 * n}), flush=True)


def cpu_baseline(x, y, cfg, threads=None):
    """The oracle as it stands, on the host cores: one full Gibbs sweep of the same
    workload (chain set-up untimed), with the BLAS/LAPACK pools at `threads` threads
    (None: their default, all host cores)."""
    import contextlib

    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import kernels, sampler
    ctx = threadpool_limits(threads) if threads else contextlib.nullcontext()
    with ctx:
        ch = sampler.Chain(x, y, kernels.SE, cfg["ell0"], cfg["nugget"], cfg["leaf"], cfg["tol"],
                           cfg["tau0"], cfg["sigf2_0"], cfg["seed"])
        t0 = time.perf_counter()
        ch.step()
        dt = time.perf_counter() - t0
        used = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": 1.0 / dt, "unit": "Gibbs iters/s", "cores": used, "kind": "oracle",
            "sample": f"one Gibbs sweep of the same n={x.size} chain (set-up untimed), "
                      f"{dt:.1f} s"}


def _line(metric, value, unit, args, dt, dtype, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    import torch

    import paper_2006_06537_amd as fg
    from workloads import LARGE_1D, sinusoid_1d
    cfg = dict(LARGE_1D)
    n = args.n or 32768
    dev = torch.device("cuda:0")
    prec = fg.MIXED if args.precision == "mixed" else fg.FP64

    def make():
        out = []
        for c in range(args.chains):
            x, y = sinusoid_1d(n, seed=1000 + c)
            out.append(fg.Chain(torch.tensor(x, device=dev), torch.tensor(y, device=dev),
                                ell0=cfg["ell0"], tau0=cfg["tau0"], sigf2_0=cfg["sigf2_0"],
                                nugget=cfg["nugget"], leaf=cfg["leaf"], tol=cfg["tol"],
                                seed=1000 + c, stream_id=c, precision=prec))
        return out

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    chains = make()
    print(f"bench: {args.chains} chains ready (n={n})", file=sys.stderr, flush=True)
    pname = "mixed" if prec == fg.MIXED else "FP64"
    dname = "f32+f64" if prec == fg.MIXED else "f64"
    if args.batch_mode != "auto":  # one mode alone (for a profile of that mode)
        mode, ns = {"grouped": (fg.BATCH_GROUPED, 1), "eager": (fg.BATCH_EAGER, 4),
                    "graphs": (fg.BATCH_GRAPHS, 4)}[args.batch_mode]
        fg.step_batch(chains, max(args.warmup, 1), nstreams=ns, mode=mode)
        dt = timed(lambda: fg.step_batch(chains, args.steps, nstreams=ns, mode=mode))
        bad = sum(1 for c in chains if c.state()["status"] != 0)
        _line(f"chain Gibbs iters/s, {args.chains} chains x n={n} ({pname}, {args.batch_mode})",
              args.chains * args.steps / dt, "chain Gibbs iters/s", args, dt, dname,
              {"workload": f"batch: {args.chains} independent {pname} chains, n={n} each, "
                           f"gibbs_step_batch in {args.batch_mode} mode only",
               "chains": args.chains, "n": n}, failed_chains=bad)
        return
    # the autotuner's trials (8 sweeps) first, untimed
    fg.step_batch(chains, 8, nstreams=4, mode=fg.BATCH_AUTO)
    choice = fg.batch_tuning(chains)
    print(f"bench: autotuner chose {choice}", file=sys.stderr, flush=True)
    fg.step_batch(chains, args.warmup, mode=fg.BATCH_AUTO)
    dt = timed(lambda: fg.step_batch(chains, args.steps, nstreams=4, mode=fg.BATCH_AUTO))
    print(f"bench: batched, autotuned ({choice[0]}) {dt:.3f} s", file=sys.stderr, flush=True)
    others = {}
    for name, mode, ns in [("grouped", fg.BATCH_GROUPED, 1), ("eager_4_streams", fg.BATCH_EAGER, 4),
                           ("graphs_4_streams", fg.BATCH_GRAPHS, 4)]:
        fg.step_batch(chains, 1, nstreams=ns, mode=mode)  # graph capture outside the timing
        d = timed(lambda: fg.step_batch(chains, args.steps, nstreams=ns, mode=mode))
        others[name] = args.chains * args.steps / d
        print(f"bench: batched {name} {d:.3f} s", file=sys.stderr, flush=True)

    def seq():
        for c in chains:
            c.step(args.steps)
    dt_seq = timed(seq)
    print(f"bench: sequential {dt_seq:.3f} s", file=sys.stderr, flush=True)
    st = chains[0].state()
    bad = sum(1 for c in chains if c.state()["status"] != 0)
    tot = args.chains * args.steps
    _line(f"chain Gibbs iters/s, {args.chains} chains x n={n} ({pname})", tot / dt,
          "chain Gibbs iters/s", args, dt, dname,
          {"workload": f"batch: {args.chains} independent {pname} chains, n={n} each (5-sinusoid y, "
                       "seeds 1000+c), SE kernel ell0=0.02, leaf 128, tol 1e-10; "
                       "gibbs_step_batch with the autotuned mode (grouped launches, eager on "
                       "2 or 4 streams, or captured graphs)",
           "chains": args.chains, "n": n},
          autotuned=choice[0], autotuned_streams=choice[1], modes_chain_iters_per_s=others,
          sequential_value=tot / dt_seq, failed_chains=bad, status0=st["status"],
          precision_used0=st["precision_used"], pcg_iters0=st["pcg_iters"])


def bench_tensor(args):
    import torch

    import paper_2006_06537_amd as fg
    from workloads import TENSOR_4D, tensor_surface
    T = dict(TENSOR_4D)
    n = args.n or T["n"]
    x, y = tensor_surface(T["d"], n, seed=T["seed"])
    dev = torch.device("cuda:0")
    ch = fg.TensorChain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), T["ell0"],
                        tau0=T["tau0"], beta0=T["beta0"], nugget=T["nugget"], leaf=T["leaf"],
                        tol=T["tol"], seed=T["seed"], ncomp=args.ncomp)
    ch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ch.state()
    print(f"bench: tensor status {st['status']} tau {st['tau']:.4g} beta {st['beta']:.4g} "
          f"k {st['k']}", file=sys.stderr, flush=True)
    extra = {}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info

        from oracle import kernels, tensor
        oc = tensor.TensorChain(x, y, kernels.SE, T["ell0"], T["nugget"], T["leaf"], T["tol"],
                                T["tau0"], T["beta0"], T["seed"], ncomp=args.ncomp)
        t1 = time.perf_counter()
        oc.step()
        dto = time.perf_counter() - t1
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        extra["cpu_baseline"] = {"value": 1.0 / dto, "unit": "tensor sweeps/s", "cores": threads,
                                 "kind": "oracle",
                                 "sample": f"one sweep of the same chain (set-up untimed), {dto:.1f} s"}
    comp = "" if args.ncomp == 1 else f", {args.ncomp} additive components"
    model = ("y = beta prod_h f_h(x_h) + noise" if args.ncomp == 1 else
             "y = sum_c beta_c prod_h f_ch(x_h) + noise")
    _line(f"tensor-product sweeps/s, d={T['d']} x n={n}{comp} (FP64)", args.steps / dt, "sweeps/s",
          args, dt, "f64",
          {"workload": f"tensor: {model}, d={T['d']}, n={n}, x ~ U[0,1]^d, "
                       "s(x)=sin(4x)sqrt(4x) per factor, Algorithm 1.h per factor, leaf 128, "
                       "tol 1e-10", "d": T["d"], "n": n, "ncomp": args.ncomp}, **extra)


def bench_predict(args):
    import torch

    import paper_2006_06537_amd as fg
    from workloads import LARGE_1D, large_1d, new_inputs
    cfg = dict(LARGE_1D)
    x, y = large_1d(cfg["n"], cfg["seed"])
    n, m = cfg["n"], args.nstar
    dev = torch.device("cuda:0")
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    chain = fg.Chain(xt, yt, ell0=cfg["ell0"], tau0=cfg["tau0"], sigf2_0=cfg["sigf2_0"],
                     nugget=cfg["nugget"], leaf=cfg["leaf"], tol=cfg["tol"], seed=cfg["seed"])
    chain.predict_inputs(torch.tensor(new_inputs(m), device=dev), max_grid_points=args.zcache)

    def sweep_and_draw():
        chain.step(1)
        return chain.predict()

    for _ in range(args.warmup):
        sweep_and_draw()
    torch.cuda.synchronize()
    b0 = chain.predict_stats()[1]
    print(f"bench: predict warm-up done, {b0} Z builds", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fs, mu, s2 = sweep_and_draw()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cached, builds = chain.predict_stats()
    timed_builds = builds - b0
    # one draw with Z cached, alone: events on the stream the kernels are launched on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    timer = fg.KernelTimer(fg.KID_PREDICT)
    timer.start()
    ev[0].record()
    reps = 5
    for _ in range(reps):
        chain.predict()
    ev[1].record()
    torch.cuda.synchronize()
    cached_ms = ev[0].elapsed_time(ev[1]) / reps
    ktime_ms, launches, kbytes = timer.stop()
    # one draw that builds Z (new inputs: nothing cached)
    chain.predict_inputs(torch.tensor(new_inputs(m), device=dev), max_grid_points=args.zcache)
    torch.cuda.synchronize()
    ev[0].record()
    chain.predict()
    ev[1].record()
    torch.cuda.synchronize()
    build_ms = ev[0].elapsed_time(ev[1])
    st = chain.state()
    print(f"bench: predict {args.steps} sweeps+draws in {dt:.3f} s, {timed_builds} Z builds, "
          f"cached draw {cached_ms:.2f} ms, building draw {build_ms:.1f} ms, status "
          f"{st['status']}", file=sys.stderr, flush=True)
    achieved = kbytes / (ktime_ms * 1e-3) / 1e9 if ktime_ms > 0 else None
    roof = {"bound": "hbm", "kernel": "k_predict_partial", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
            "launches": launches, "avg_launch_us": 1e3 * ktime_ms / max(launches, 1),
            "algorithmic_bytes_per_launch": kbytes / max(launches, 1)}
    extra = {"predictive_draws_per_s": m * args.steps / dt,
             "cached_draw_ms": cached_ms, "building_draw_ms": build_ms,
             "z_builds_in_timed_region": timed_builds, "grid_points_cached": cached,
             "zcache_bytes": 8 * n * m * cached}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info

        from oracle import hodlr as oh, kernels, predict, rng
        sub = 64  # new inputs in the CPU sample
        H = oh.HODLR(x, kernels.SE, cfg["ell0"], cfg["nugget"], cfg["leaf"], cfg["tol"])
        W1 = oh.Factor(H, 1.0, 0.0)
        f = W1.apply_W(rng.normals(n, 1, 1, 0, 0))
        t1 = time.perf_counter()
        predict.predict(H, W1, f, 1.0, new_inputs(m)[:sub], rng.normals(sub, 1, rng.TAG_PRED, 0, 0))
        dto = time.perf_counter() - t1
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        extra["cpu_baseline"] = {"value": sub / dto, "unit": "predictive draws/s (uncached)",
                                 "cores": threads, "kind": "oracle",
                                 "sample": f"{sub} new inputs at n={n}, oracle factor given, "
                                           f"{dto:.1f} s"}
    _line(f"Gibbs iters/s with predictive draws at {m} new inputs, n=2^20 (FP64)",
          args.steps / dt, "Gibbs iters/s", args, dt, "f64",
          {"workload": f"predict: large_1d chain (n=2^20, leaf 128, tol 1e-10, ell0 0.02) with "
                       f"one draw of f at {m} new inputs U[-0.02,1.02] after every sweep; Z "
                       f"kept for up to {args.zcache} grid points", "n": n, "nstar": m},
          roofline=roof, **extra)


def bench_collapse(args):
    import numpy as np
    import torch

    import paper_2006_06537_amd as fg
    from workloads import LARGE_1D, gridded_1d
    cfg = dict(LARGE_1D)
    x, y = gridded_1d()
    dev = torch.device("cuda:0")
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    kw = dict(ell0=cfg["ell0"], tau0=cfg["tau0"], sigf2_0=cfg["sigf2_0"], nugget=cfg["nugget"],
              leaf=cfg["leaf"], tol=cfg["tol"], seed=cfg["seed"])
    t0 = time.perf_counter()
    ch = fg.Chain(xt, yt, collapse=True, **kw)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    ch.step(args.warmup)
    torch.cuda.synchronize()
    timer = fg.KernelTimer(args.kernel or fg.KID_UPDATE)  # 0: the dominant kernel
    timer.start()
    t0 = time.perf_counter()
    ch.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ktime_ms, launches, kbytes = timer.stop()
    st = ch.state()
    print(f"bench: collapsed chain U={ch.n} of n={ch.n_obs}: {args.steps} sweeps in {dt:.3f} s, "
          f"status {st['status']}, tau {st['tau']:.4g}", file=sys.stderr, flush=True)
    # the plain chain on the raw observations (repeated inputs kept), sorted by input
    order = np.argsort(x, kind="stable")
    raw = fg.Chain(torch.tensor(x[order], device=dev), torch.tensor(y[order], device=dev), **kw)
    raw_steps = max(1, min(args.steps, 5))
    raw.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    raw.step(raw_steps)
    torch.cuda.synchronize()
    dt_raw = time.perf_counter() - t0
    rst = raw.state()
    print(f"bench: plain chain on n={x.size}: {raw_steps} sweeps in {dt_raw:.3f} s, status "
          f"{rst['status']}, tau {rst['tau']:.4g}", file=sys.stderr, flush=True)
    achieved = kbytes / (ktime_ms * 1e-3) / 1e9 if ktime_ms > 0 else None
    roof = {"bound": "hbm", "kernel": timer.name, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": None, "launches": launches,
            "avg_launch_us": 1e3 * ktime_ms / max(launches, 1)}
    extra = {"uncollapsed_iters_per_s": raw_steps / dt_raw, "uncollapsed_status": rst["status"],
             "speedup": (args.steps / dt) / (raw_steps / dt_raw), "create_s": t_create}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info

        from oracle import collapse, kernels
        oc = collapse.CollapsedChain(x, y, kernels.SE, cfg["ell0"], cfg["nugget"], cfg["leaf"],
                                     cfg["tol"], cfg["tau0"], cfg["sigf2_0"], cfg["seed"])
        t1 = time.perf_counter()
        oc.step()
        dto = time.perf_counter() - t1
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        extra["cpu_baseline"] = {"value": 1.0 / dto, "unit": "Gibbs iters/s", "cores": threads,
                                 "kind": "oracle",
                                 "sample": f"one sweep of the collapsed chain (U={ch.n}), {dto:.2f} s"}
    _line(f"Gibbs iters/s on collapsed gridded data, n={ch.n_obs} observations on U={ch.n} "
          "inputs (FP64)", args.steps / dt, "Gibbs iters/s", args, dt, "f64",
          {"workload": f"collapse: {ch.n_obs} observations on a grid of {ch.n} inputs (64 each), "
                       "5-sinusoid signal + N(0,0.2^2), SE kernel ell0=0.02, leaf 128, tol 1e-10, "
                       "nugget 1e-6", "n": ch.n_obs, "unique": ch.n},
          roofline=roof, **extra)


def bench_exact(args):
    import torch

    import paper_2006_06537_amd as fg
    from workloads import LARGE_1D, sinusoid_1d
    cfg = dict(LARGE_1D)
    n = args.n or (1 << 17)
    x, y = sinusoid_1d(n, seed=cfg["seed"])
    dev = torch.device("cuda:0")
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    kw = dict(ell0=cfg["ell0"], tau0=cfg["tau0"], sigf2_0=cfg["sigf2_0"], nugget=cfg["nugget"],
              leaf=cfg["leaf"], tol=cfg["tol"], seed=cfg["seed"])
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    ch = fg.Chain(xt, yt, exact_rho=True, **kw)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    held = free0 - torch.cuda.mem_get_info()[0]
    ch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ch.state()
    print(f"bench: grid chain n={n}: set-up {t_create:.2f} s ({held / 1e9:.1f} GB), "
          f"{args.steps} sweeps in {dt:.3f} s, k {st['k']}, moves {st['accepts']}, status "
          f"{st['status']}", file=sys.stderr, flush=True)
    # the same sweeps replayed from captured graphs (one graph per grid index)
    fg.step_batch([ch], iters=args.warmup, nstreams=1, graphs=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fg.step_batch([ch], iters=args.steps, nstreams=1, graphs=True)
    torch.cuda.synchronize()
    dt_graph = time.perf_counter() - t0
    print(f"bench: grid chain from captured graphs: {args.steps} sweeps in {dt_graph:.3f} s",
          file=sys.stderr, flush=True)
    mh = fg.Chain(xt, yt, **kw)
    mh.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mh.step(args.steps)
    torch.cuda.synchronize()
    dt_mh = time.perf_counter() - t0
    extra = {"metropolis_iters_per_s": args.steps / dt_mh, "graphs_iters_per_s": args.steps / dt_graph,
             "setup_s": t_create,
             "grid_bytes": held, "grid_points": 100, "moves": st["accepts"]}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info

        from oracle import exact_rho, kernels
        sub = 1 << 13  # the oracle's set-up (100 factorizations) at n = 2^17 runs for minutes
        xs_, ys_ = sinusoid_1d(sub, seed=cfg["seed"])
        oc = exact_rho.ExactGridChain(xs_, ys_, kernels.SE, cfg["ell0"], cfg["nugget"],
                                      cfg["leaf"], cfg["tol"], cfg["tau0"], cfg["sigf2_0"],
                                      cfg["seed"])
        t1 = time.perf_counter()
        oc.step()
        dto = time.perf_counter() - t1
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        extra["cpu_baseline"] = {"value": 1.0 / dto, "unit": "Gibbs iters/s", "cores": threads,
                                 "kind": "oracle",
                                 "sample": f"one sweep of the oracle grid chain at n={sub} "
                                           f"(set-up untimed), {dto:.2f} s"}
    _line(f"Gibbs iters/s with the exact grid conditional of the length-scale, n={n} (FP64)",
          args.steps / dt, "Gibbs iters/s", args, dt, "f64",
          {"workload": f"exact: n={n} sorted U[0,1], 5-sinusoid y + N(0,0.05^2), SE kernel "
                       "ell0=0.02, 100-point grid with every factorization kept, leaf 128, "
                       "tol 1e-10, nugget 1e-6", "n": n},
          roofline=None, **extra)


def bench_serve(args):
    import threading

    import numpy as np
    import torch

    import paper_2006_06537_amd as fg
    from workloads import served_jobs
    jobs = served_jobs(args.jobs, seed=5)
    prec = fg.MIXED if args.precision == "mixed" else fg.FP64
    budget = 160 << 30
    common = dict(leaf=128, tol=1e-10, precision=prec, want_f=False)

    def run(arrivals):
        srv = fg.Server(budget, max_active=args.slots)
        t0 = time.perf_counter()

        def feeder():
            for j, job in enumerate(jobs):
                dt = arrivals[j] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                srv.submit(job["x"], job["y"], job["ell0"], args.job_iters, seed=job["seed"],
                           stream_id=j, tau0=job["tau0"], **common)
        th = threading.Thread(target=feeder)
        th.start()
        while th.is_alive():  # progress while the arrivals are fed
            th.join(30.0)
            if th.is_alive():
                print(f"bench: arrivals in progress, {srv.stats()['outstanding']} jobs "
                      "outstanding", file=sys.stderr, flush=True)
        while True:  # progress while the last jobs run
            try:
                srv.drain(30.0)
                break
            except fg.FgError as e:
                if e.code != fg._lib.FG_ENOTCONV:
                    raise
                st_ = srv.stats()
                print(f"bench: serving, {st_['outstanding']} jobs outstanding", file=sys.stderr,
                      flush=True)
        span = time.perf_counter() - t0
        res = srv.poll(4096)
        st = srv.stats()
        srv.close()
        bad = [r for r in res if r["status"] != 0]
        for r in bad[:10]:
            j = r["id"] - 1
            print(f"bench: job {j} (n={jobs[j]['n']}, ell0={jobs[j]['ell0']:.4g}, "
                  f"tau0={jobs[j]['tau0']:.4g}) ended with status {r['status']} after "
                  f"{r['iteration']} sweeps", file=sys.stderr, flush=True)
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        return span, lat, st, len(bad)

    # saturation: every job at t = 0
    span0, lat0, st0, bad0 = run([0.0] * len(jobs))
    sat = len(jobs) / span0
    print(f"bench: saturation {sat:.3f} jobs/s ({span0:.1f} s, peak {st0['peak_bytes'] / 2**30:.1f} GiB,"
          f" {bad0} failed)", file=sys.stderr, flush=True)
    lam = args.load * sat
    gaps = np.random.default_rng(55).exponential(1.0 / lam, len(jobs))
    arrivals = np.cumsum(gaps) - gaps[0]
    span, lat, st, bad = run(list(arrivals))
    print(f"bench: served at {lam:.3f} jobs/s in {span:.1f} s, {bad} failed", file=sys.stderr,
          flush=True)
    # sequential FIFO of plain FP64 chains on the same arrivals: service times measured
    # one job at a time, queue replayed on the host
    dev = torch.device("cuda:0")
    svc, seq_bad = [], []
    for j, job in enumerate(jobs):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c = fg.Chain(torch.tensor(job["x"], device=dev), torch.tensor(job["y"], device=dev),
                     ell0=job["ell0"], tau0=job["tau0"], leaf=128, tol=1e-10, seed=job["seed"],
                     stream_id=j)
        c.step(args.job_iters)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t1)
        sst = c.state()["status"]
        if sst != 0:
            seq_bad.append(j)
            print(f"bench: sequential job {j} (n={job['n']}) ended with status {sst}",
                  file=sys.stderr, flush=True)
        del c
        if j % 64 == 63:
            print(f"bench: sequential FIFO, {j + 1} jobs timed", file=sys.stderr, flush=True)
    fin, seq_lat = 0.0, []
    for j in range(len(jobs)):
        fin = max(fin, arrivals[j]) + svc[j]
        seq_lat.append(fin - arrivals[j])
    seq_lat = np.array(seq_lat)
    q = lambda a, p: float(np.percentile(a, p))
    print(f"bench: sequential FIFO p50 {q(seq_lat, 50):.2f} s p99 {q(seq_lat, 99):.2f} s",
          file=sys.stderr, flush=True)
    ns = [j["n"] for j in jobs]
    out = {"metric": "p50 latency of served GP-regression jobs", "value": q(lat, 50), "unit": "s",
           "n_gpus": 1, "steps": args.job_iters, "warmup": 0, "ms_per_step": None,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64" if prec == fg.MIXED else "f64", "data": "synthetic",
           "config": {"workload": f"serve: {len(jobs)} jobs, n log-uniform [1e3, 2e5] (mean "
                                  f"{np.mean(ns):.0f}), 5-sinusoid y, noise U[0.02,0.2], ell0 "
                                  f"LogU[0.01,0.3], {args.job_iters} sweeps each, Poisson "
                                  f"arrivals at {args.load} x saturation; budget "
                                  f"{budget >> 30} GiB, {args.slots} slots, tau0 = 1/noise^2",
                      "jobs": len(jobs), "sweeps_per_job": args.job_iters,
                      "slots": args.slots},
           "p99": q(lat, 99), "throughput_jobs_per_s": len(jobs) / span,
           "saturation_jobs_per_s": sat, "arrival_rate": lam,
           "peak_bytes": st["peak_bytes"], "failed_jobs": bad,
           "sequential_fp64_fifo": {"p50": q(seq_lat, 50), "p99": q(seq_lat, 99),
                                    "throughput_jobs_per_s": len(jobs) / fin,
                                    "mean_service_s": float(np.mean(svc)),
                                    "failed_jobs": len(seq_bad)}}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU layout is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "tensor":
        return bench_tensor(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "predict":
        return bench_predict(args)
    if args.workload == "collapse":
        return bench_collapse(args)
    if args.workload == "exact":
        return bench_exact(args)
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
    mixed = args.precision == "mixed"
    chain = fg.Chain(xt, yt, ell0=cfg["ell0"], tau0=cfg["tau0"], sigf2_0=cfg["sigf2_0"],
                     nugget=cfg["nugget"], leaf=cfg["leaf"], tol=cfg["tol"], seed=cfg["seed"],
                     precision=fg.MIXED if mixed else fg.FP64)
    print(f"bench: chain ready (n={cfg['n']})", file=sys.stderr, flush=True)
    chain.step(args.warmup)
    torch.cuda.synchronize()
    print(f"bench: {args.warmup} warm-up sweeps done", file=sys.stderr, flush=True)
    kids = [fg.KID_LEAF, fg.KID_REDUCE, fg.KID_UPDATE, fg.KID_WHITEN]
    timer = fg.KernelTimer(kids[0], also=kids[1:])
    timer.start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timer.stop()
    per = {k: fg.KernelTimer.result(k) for k in kids}
    kid = args.kernel
    if kid == 0:  # the HBM-bound kernel with the largest total time
        kid = max([fg.KID_REDUCE, fg.KID_UPDATE, fg.KID_WHITEN], key=lambda k: per[k][0])
    ktime_ms, launches, kbytes = per[kid]
    timer = fg.KernelTimer(kid)
    st = chain.state()
    print(f"bench: {args.steps} timed sweeps in {dt:.3f} s; status {st['status']}, "
          f"accepts {st['accepts']}, ell {st['ell']:.4g}, tau {st['tau']:.4g}",
          file=sys.stderr, flush=True)
    # the same kernel once more with nothing beside it: one factorization of K~_1 alone
    iso_us = None
    if not args.n or args.n == LARGE_1D["n"]:
        K1 = fg.Hodlr(xt, cfg["ell0"], nugget=cfg["nugget"], leaf=cfg["leaf"], tol=cfg["tol"])
        torch.cuda.synchronize()
        timer.start()
        F1 = fg.Factor(K1, 1.0, 0.0)
        torch.cuda.synchronize()
        iso_ms, iso_n, iso_b = timer.stop()
        iso_us = 1e3 * iso_ms / max(iso_n, 1)
        del F1, K1
    kernels = {}
    for k, (ms_k, n_k, b_k) in per.items():
        if n_k and ms_k > 0:
            kernels[fg.KID_NAMES[k]] = {
                "total_ms": ms_k, "share_of_timed_region": ms_k / (1e3 * dt), "launches": n_k,
                "avg_launch_us": 1e3 * ms_k / n_k, "algorithmic_bytes_per_launch": b_k / n_k,
                "achieved_GBs": b_k / (ms_k * 1e-3) / 1e9,
                "frac": b_k / (ms_k * 1e-3) / 1e9 / HBM_PEAK_GBS}
    roof = None
    if launches > 0 and ktime_ms > 0:
        achieved = kbytes / (ktime_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": timer.name, "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": counter_traffic(timer.name), "launches": launches,
                "avg_launch_us": 1e3 * ktime_ms / launches,
                "algorithmic_bytes_per_launch": kbytes / launches,
                "isolated_avg_launch_us": iso_us,
                "note": "launches in the timed region share the GPU with the proposal's "
                        "build on the chain's second stream; isolated = one launch alone"}
    extra = {}
    if mixed:
        # the same chain in FP64 (itself held to the oracle at 1e-9), run to the same sweep
        ref = fg.Chain(xt, yt, ell0=cfg["ell0"], tau0=cfg["tau0"], sigf2_0=cfg["sigf2_0"],
                       nugget=cfg["nugget"], leaf=cfg["leaf"], tol=cfg["tol"], seed=cfg["seed"])
        ref.step(args.warmup + args.steps)
        a, b = chain.state(with_vectors=True), ref.state(with_vectors=True)
        fe = float(torch.linalg.norm(a["f"] - b["f"]) / torch.linalg.norm(b["f"]))
        extra["vs_fp64_path"] = {
            "sweeps": args.warmup + args.steps, "same_grid_index": a["k"] == b["k"],
            "same_accepts": a["accepts"] == b["accepts"],
            "tau_rel": abs(a["tau"] - b["tau"]) / abs(b["tau"]),
            "sigf2_rel": abs(a["sigf2"] - b["sigf2"]) / abs(b["sigf2"]), "f_rel": fe,
            "loglik_abs": abs(a["loglik"] - b["loglik"]), "pcg_iters": a["pcg_iters"],
            "pcg_relres": a["pcg_relres"], "precision_used": "mixed" if
            a["precision_used"] == fg.MIXED else "fp64 (fell back)"}
        print(f"bench: mixed vs FP64 path {extra['vs_fp64_path']}", file=sys.stderr, flush=True)
    out = {
        "metric": "Gibbs iters/s at n=2^20 (mixed)" if mixed else "Gibbs iters/s at n=2^20 (FP64)",
        "value": args.steps / dt,
        "unit": "Gibbs iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": ("large_1d: single chain, M~ with its leaf Cholesky factors "
                                "in FP32 (levels, node factors and log-det FP64), both solves "
                                "refined by PCG to 1e-10 on the FP64 HODLR, W_1 FP64;"
                                if mixed else "large_1d: single FP64 chain,") + " "
                               "n=2^20 sorted U[0,1], 5-sinusoid y "
                               "+ N(0,0.05^2), SE kernel ell0=0.02 (100-point grid), leaf 128, "
                               "tol 1e-10, nugget 1e-6",
                   "n": cfg["n"], "leaf": cfg["leaf"], "tol": cfg["tol"], "ell0": cfg["ell0"]},
        "roofline": roof,
        "kernels": kernels,
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle (all host threads)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(x, y, cfg)
        print(f"bench: oracle {out['cpu_baseline']['sample']}; now on one thread", file=sys.stderr,
              flush=True)
        out["cpu_baseline_1core"] = cpu_baseline(x, y, cfg, threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
