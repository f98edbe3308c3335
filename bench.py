#!/usr/bin/env python3
"""Benchmark of librtdetmcd on one MI355X.

Workload: RT-DetMCD fit of one dataset, n = 1,000,000 rows, p = 20, float32
input, AR(0.75) inliers with 10% cluster outliers, 64 contiguous blocks of
15,625 rows, h = 11,718 per block (seeded synthetic data).  One "step" is one
complete fit (standardisation, starts, refinement, C-steps, aggregation,
reweighting, final distances and flags) with X resident in HBM.

Prints one JSON line: rows/s fitted with the batched launch (value), the plain
per-block launch for comparison, the time of each kernel class of the fit
measured live over the timed fits with the library's HIP-event timing, the
roofline of the fit's dominant kernel, the roofline of the distance kernel on
a 10^7 x 40 input (larger than the last-level cache), and the CPU oracle timed
on a bounded sample of the same workload on one core and on every core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
FP64_TFLOPS = 78.6               # MI355X float64 peak, vector and matrix cores

N, P, BLOCKS = 1_000_000, 20, 64
HERE = os.path.dirname(os.path.abspath(__file__))

# kernel class -> (source of the kernels, bound, name of the kernel)
KERNELS = {
    "segsort": ("paper_1910_05615_amd/csrc/k_sort.hip", "hbm",
                "k_seg_lds (LDS radix sort + univariate MCD of each segment)"),
    "cstep_dist": ("paper_1910_05615_amd/csrc/k_dist.hip", "hbm",
                   "k_dist_direct (C-step distances, first step, both starts)"),
    "select": ("paper_1910_05615_amd/csrc/k_cstep.hip", "hbm",
               "k_select_reg (h-subset selection, first step)"),
    "sscp": ("paper_1910_05615_amd/csrc/k_rows.hip", "mfma",
             "k_sscp (subset sums on the float64 matrix cores, first step)"),
    "finalize": ("paper_1910_05615_amd/csrc/k_cstep.hip", "latency",
                 "k_finalize (Cholesky, inverse, condition)"),
    "final_dist": ("paper_1910_05615_amd/csrc/k_dist.hip", "hbm",
                   "k_final_dist_direct (final distances and flags)"),
}


def _sha(path):
    with open(os.path.join(HERE, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _counters(name):
    """HBM bytes per launch from a committed counter summary of the kernel, or
    None if it is missing or was taken on another version of the source."""
    try:
        with open(os.path.join(HERE, "profiles", name)) as f:
            rec = json.load(f)
        if rec.get("kernel_source_sha256") != _sha(rec["kernel_source"]):
            return None
        return rec.get("hbm_bytes_per_launch")
    except (OSError, KeyError, ValueError):
        return None


def _kernel_entry(kind, rec, peak_hbm=HBM_PEAK_GBS):
    src, bound, label = KERNELS[kind]
    n = max(rec["launches"], 1)
    t = rec["ms"] * 1e-3 / n
    e = {"kernel": label, "launches": rec["launches"], "launch_us": t * 1e6}
    if rec["bytes"] > 0 and t > 0:
        gbs = rec["bytes"] / n / t / 1e9
        e.update({"algorithmic_bytes_per_launch": rec["bytes"] / n, "GB_s": gbs,
                  "hbm_frac": gbs / peak_hbm})
    if rec["flops_useful"] > 0 and t > 0:
        e["tflops_useful"] = rec["flops_useful"] / n / t / 1e12
        e["fp64_frac_useful"] = e["tflops_useful"] / FP64_TFLOPS
        if rec["flops_exec"] > 0:
            e["tflops_executed"] = rec["flops_exec"] / n / t / 1e12
            e["fp64_frac_executed"] = e["tflops_executed"] / FP64_TFLOPS
    return e


def _roofline(kind, rec, counters_file=None):
    """roofline object of one kernel class from its live-timed records."""
    e = _kernel_entry(kind, rec)
    bound = KERNELS[kind][1]
    if bound == "mfma":
        r = {"bound": "mfma", "achieved": e["tflops_useful"], "peak": FP64_TFLOPS,
             "unit": "TFLOP/s", "frac": e["tflops_useful"] / FP64_TFLOPS,
             "executed_frac": e.get("fp64_frac_executed")}
    else:
        r = {"bound": "hbm", "achieved": e["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": e["GB_s"] / HBM_PEAK_GBS}
    r["traffic"] = _counters(counters_file) if counters_file else None
    r.update({k: v for k, v in e.items() if k not in ("GB_s", "hbm_frac")})
    return r


def _distance_roofline(R, torch, dev, reps):
    """The distance kernel of the C-step pass (float64 arithmetic on float32
    rows, one row per thread) on 10^7 x 40 rows, 1.6 GB, larger than the 256 MB
    last-level cache; timed with HIP events on the stream it is launched on."""
    n, p = 10_000_000, 40
    g = torch.Generator(device=dev).manual_seed(7)
    X = torch.randn(n, p, generator=g, device=dev, dtype=torch.float32)
    A = torch.randn(p, p, generator=g, device=dev, dtype=torch.float64)
    L = torch.linalg.cholesky(A @ A.T / p + torch.eye(p, device=dev, dtype=torch.float64))
    mu = torch.zeros(p, device=dev, dtype=torch.float64)
    d2 = torch.empty(n, device=dev, dtype=torch.float64)
    for _ in range(3):
        R.distances_into(X, mu, L, d2)
    torch.cuda.synchronize()
    # the kernel alone: HIP events around each launch on the library's stream
    # (the call also uploads its item table and forms the factor's inverse)
    R.profile(True)
    for _ in range(reps):
        R.distances_into(X, mu, L, d2)
    rec = R.profile_read()["distances"]
    R.profile(False)
    t = rec["ms"] * 1e-3 / max(rec["launches"], 1)
    byt = n * (4 * p + 8)
    fl = n * (p * (p + 1) + 3 * p)
    del X, d2
    return {"kernel": "k_dist_direct<float, 40> (distances, one factor)", "bound": "alu",
            "achieved": fl / t / 1e12, "peak": FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": fl / t / 1e12 / FP64_TFLOPS,
            "traffic": _counters("k_dist_p40_n10M_counters.json"),
            "hbm_GB_s": byt / t / 1e9, "hbm_frac": byt / t / 1e9 / HBM_PEAK_GBS,
            "launch_us": t * 1e6, "launches": rec["launches"],
            "algorithmic_bytes_per_launch": byt, "flops_per_launch": fl, "n": n, "p": p,
            "note": "float64 arithmetic: p(p+1)+3p flops per 4p+8 bytes, so at p = 40 the "
                    "float64 rate, not HBM, bounds the kernel"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_SHARES = None


def _oracle_share(k):
    """Fit share k of the CPU sample (one process per share)."""
    from threadpoolctl import threadpool_limits
    import oracle
    X, nb = _SHARES[k]
    with threadpool_limits(limits=1):
        oracle.fit(X, n_chunks=nb)
    return X.shape[0]


def _cpu_baseline(X, blocks, m, cores):
    """The oracle on the first `blocks` blocks of the data: one core (the
    serial fit), then every core with one process per share of the blocks
    (each share fitted as its own dataset: the paper's one block per thread,
    Sec. 4).  Runs before the GPU is touched (the pool forks)."""
    global _SHARES
    import concurrent.futures as cf
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    import oracle
    ns = blocks * m
    Xs = X[:ns]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.fit(Xs, n_chunks=blocks)
        t1 = time.perf_counter() - t0
    w = max(1, min(cores, blocks))
    per = [blocks // w + (1 if k < blocks % w else 0) for k in range(w)]
    _SHARES, r0 = [], 0
    for nb in per:
        _SHARES.append((Xs[r0 * m:(r0 + nb) * m], nb))
        r0 += nb
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=w, mp_context=mp.get_context("fork")) as ex:
        rows = sum(ex.map(_oracle_share, range(w)))
    tn = time.perf_counter() - t0
    return {"value": rows / tn, "unit": "rows/s", "cores": w, "kind": "oracle",
            "sample": f"first {blocks} blocks ({ns} rows, p={P}) of the same data; all cores: "
                      f"{w} processes, each fitting {per[0]} of the blocks as its own dataset "
                      f"(one block per thread as in Sec. 4), {tn:.1f} s with process start-up",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "single_core": {"value": ns / t1, "unit": "rows/s", "cores": 1,
                            "sample": f"the {blocks} blocks fitted serially, {t1:.1f} s"}}


def _other_workload(args, R, torch, synthdata, dev):
    """rows/s of the batched-uneven (512 datasets, one batched call against one
    call per dataset) or the large (10^7 x 40, 1,024 blocks, batched against
    per-block launches) workload, with the kernel times of the batched fits."""
    def clock(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    if args.workload == "batched_uneven":
        sets = synthdata.workload_batched_uneven()
        Xs = [torch.from_numpy(s.X).to(dev) for s in sets]
        rows = sum(int(X.shape[0]) for X in Xs)
        R.profile(True)
        t_b = clock(lambda: R.fit_batched(Xs), args.steps)
        prof = R.profile_read()
        R.profile(False)
        t_s = clock(lambda: [R.fit(X) for X in Xs], max(1, args.plain_steps))
        cfg = {"workload": "512 datasets, n log-uniform [2e3, 2e5], p in {5,10,20,40}, "
                           "float32, point outliers (eps in {0,.1,.2}), blocks by the omega rule",
               "datasets": len(Xs), "rows": rows}
        other = {"per_dataset_calls": {"value": rows / t_s, "unit": "rows/s",
                                       "ms_per_step": t_s * 1e3,
                                       "batched_over_per_dataset": t_s / t_b}}
        t = t_b
    else:
        ds = synthdata.workload_large_p40()
        X = torch.from_numpy(ds.X).to(dev)
        rows = int(X.shape[0])
        kw = dict(n_chunks=1024, cstep_mode="update")
        R.profile(True)
        t = clock(lambda: R.fit(X, **kw), args.steps)
        prof = R.profile_read()
        R.profile(False)
        t_p = clock(lambda: R.fit(X, launch="plain", **kw), 1)
        cfg = {"workload": "n=10,000,000 p=40 float32, random correlation (eigenvalues "
                           "U[0.1,10]), 5% N(0,25I); 1,024 blocks, update-based C-steps",
               "n": rows, "p": 40, "blocks": 1024}
        other = {"plain": {"value": rows / t_p, "unit": "rows/s", "ms_per_step": t_p * 1e3,
                           "batched_over_plain": t_p / t},
                 "cstep_distance_roofline": dict(
                     _kernel_entry("cstep_dist", prof["cstep_dist"]),
                     note="two factors per row (both starts), float64 arithmetic")}
    out = {"metric": "rows/sec fitted (RT-DetMCD), batched launch", "value": rows / t,
           "unit": "rows/s", "n_gpus": 1, "steps": args.steps, "ms_per_step": t * 1e3,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic", "config": cfg,
           "kernels": {k: _kernel_entry(k, v) for k, v in prof.items()
                       if k in KERNELS and v["launches"] > 0}}
    out.update(other)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-sample-blocks", type=int, default=64)
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="processes of the all-core oracle leg (0: every core, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-p40-distance", action="store_true")
    ap.add_argument("--workload", default="chunked_p20",
                    choices=["chunked_p20", "batched_uneven", "large_p40"],
                    help="chunked_p20 (the headline line) or one of the other workloads")
    ap.add_argument("--only-distance", action="store_true",
                    help="a 64 MiB device copy (counter calibration), then the 10^7 x 40 "
                         "distance launches only (for counter collection)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only; multi-GPU runs are not supported "
              "(the fit would shard by blocks, a design that is not implemented)",
              file=sys.stderr)
        return 2

    import numpy as np  # noqa: F401
    import synthdata

    q_m = None
    ds = None
    cpu = None
    if args.workload == "chunked_p20" and not args.only_distance:
        ds = synthdata.workload_chunked_p20(n=N, p=P)
        if not args.no_cpu_baseline:
            m = N // BLOCKS
            cores = args.cpu_cores or min(16, os.cpu_count() or 1)
            cpu = _cpu_baseline(ds.X, args.cpu_sample_blocks, m, cores)

    import torch
    import paper_1910_05615_amd as R

    dev = torch.device("cuda:0")
    if args.only_distance:
        src = torch.empty(64 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)            # plain copy of known size: 64 MiB read, 64 MiB written
        torch.cuda.synchronize()
        print(json.dumps({"p40_distance": _distance_roofline(R, torch, dev, args.kernel_reps),
                          "copy_calibration_bytes": 64 << 20}))
        return 0
    if args.workload != "chunked_p20":
        print(json.dumps(_other_workload(args, R, torch, synthdata, dev)))
        return 0
    X = torch.from_numpy(ds.X).to(dev)
    q, m, h = R.plan(N, P, 0, BLOCKS)

    # ---------------------------------------------------------------- batched fit
    def timed(profile=False, **kw):
        for _ in range(args.warmup):
            R.fit(X, n_chunks=BLOCKS, **kw)
        torch.cuda.synchronize()
        if profile:
            R.profile(True)
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(s)
        for _ in range(args.steps):
            Fk = R.fit(X, n_chunks=BLOCKS, **kw)
        e1.record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev = e0.elapsed_time(e1) * 1e-3
        prof = None
        if profile:
            prof = R.profile_read()
            R.profile(False)
        return Fk, max(wall, ev) / args.steps, prof

    # the batched launches enqueued one by one (value); the same timed fits
    # again with every kernel class timed by HIP events on the launching
    # stream (the event records cost some host time, so value comes from the
    # fits without them); the same fit with the C-step rounds replayed from
    # captured hipGraphs
    reruns0 = R.sort_reruns()
    F, t_step, _ = timed(graph=False)
    value = N / t_step
    _, t_prof, prof = timed(profile=True, graph=False)
    graph = None
    if not args.no_graph:
        Fg, t_g, _ = timed(graph=True)
        graph = {"value": N / t_g, "unit": "rows/s", "ms_per_step": t_g * 1e3,
                 "identical_to_eager": bool(torch.equal(F.hsubset, Fg.hsubset) and
                                            torch.equal(F.outlier, Fg.outlier) and
                                            torch.equal(F.sigma, Fg.sigma))}
    # the autotuned C-step loop (opts tune): the first warm-up fit times the
    # candidate distance tilings and keeps the fastest; the timed fits take it
    tuned = None
    if not args.no_tune:
        def same(Fa, Fb):
            return bool(torch.equal(F.hsubset, Fa.hsubset) and torch.equal(F.outlier, Fa.outlier)
                        and torch.equal(F.sigma, Fa.sigma) and torch.equal(F.dist, Fa.dist))
        Ft, t_t, _ = timed(graph=False, tune=True)
        tuned = {"value": N / t_t, "unit": "rows/s", "ms_per_step": t_t * 1e3,
                 "identical_to_untuned": same(Ft, F),
                 "plan": dict(zip(("p_bucket", "rows_per_distance_tile", "items_per_distance_tile",
                                   "csteps_of_last_fit"), R.tuned_plans()[-1]))}
        if not args.no_graph:
            Ftg, t_tg, _ = timed(graph=True, tune=True)
            tuned["graph"] = {"value": N / t_tg, "unit": "rows/s", "ms_per_step": t_tg * 1e3,
                              "identical_to_untuned": same(Ftg, F)}
    reruns = R.sort_reruns() - reruns0

    # ---------------------------------------------------------------- plain fit
    plain = None
    if not args.no_plain:
        Fp = R.fit(X, n_chunks=BLOCKS, launch="plain")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            Fp = R.fit(X, n_chunks=BLOCKS, launch="plain")
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) / args.plain_steps
        same = bool(torch.equal(F.hsubset, Fp.hsubset) and torch.equal(F.outlier, Fp.outlier))
        plain = {"value": N / tp, "unit": "rows/s", "ms_per_step": tp * 1e3,
                 "batched_over_plain": tp / t_step, "identical_hsubsets_and_flags": same}

    # ---------------------------------------------------------------- kernels and rooflines
    kernels = {k: _kernel_entry(k, v) for k, v in prof.items() if k in KERNELS and v["launches"]}
    fit_ms = prof["fit"]["ms"] / max(prof["fit"]["launches"], 1)
    for k, e in kernels.items():
        e["share_of_fit"] = prof[k]["ms"] / max(prof["fit"]["ms"], 1e-30)
    dominant = max(kernels, key=lambda k: prof[k]["ms"])
    roofline = _roofline(dominant, prof[dominant],
                         {"segsort": "k_seg_lds_p20_n1M_counters.json"}.get(dominant))
    roofline["share_of_fit"] = kernels[dominant]["share_of_fit"]
    p40 = None if args.no_p40_distance else _distance_roofline(R, torch, dev, args.kernel_reps)

    out = {
        "metric": "rows/sec fitted (RT-DetMCD, p=20), batched launch",
        "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "RT-DetMCD one dataset n=1,000,000 p=20 float32 input, "
                               "64 blocks of 15,625 rows, AR(0.75) with 10% cluster outliers",
                   "n": N, "p": P, "blocks": q, "m": m, "h": h, "input_dtype": "f32",
                   "launch": "batched"},
        "batched_graph": graph,
        "batched_tuned": tuned,
        "plain": plain,
        "roofline": roofline,
        "kernels": kernels,
        "fit_gpu_ms": fit_ms,
        "profiled_ms_per_step": t_prof * 1e3,
        "p40_distance": p40,
        "cpu_baseline": cpu,
        "sort_reruns": reruns,
        "fit_check": {"n_w": int(F.n_w.item()),
                      "outliers_flagged": int(F.outlier.sum().item()),
                      "blocks_valid": int((F.block_status < 3).sum().item())},
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
