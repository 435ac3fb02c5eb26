#!/usr/bin/env python3
"""Benchmark of the space-time predictor on one MI355X.

Workload: elastic waves, N = 7 (8^3 Gauss-Legendre nodes), m = 9, 65536 elements, per-node rho, lambda,
mu, Q ~ N(0, 1), dt = 0.4 h / ((2N+1) c_p). One step = one stp_run over the whole batch (every output:
q-bar, the three time-averaged fluxes and the six faces), inputs resident in HBM.

Prints ONE JSON line: element-updates/s of the headline variant (the fastest FP32-I/O variant), its
roofline position, the plain FP64 GPU predictor timed in the same run, and the FP64 CPU oracle timed on a
bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# VALU peaks from the unit counts: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz.
# FP32 without packed instructions runs at the FP64 rate (packed FP32 is not used by this build).
ALU_PEAK_TFS = {"f64": 78.6, "f32": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nelem", type=int, default=65536)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU-oracle time (bounded sample)")
    ap.add_argument("--copy-gib", type=float, default=1.0,
                    help="size of the device-to-device copy timed as the measured HBM reference (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variants", default="fp64_plain,fp32_plain,fp32_fused,bf16x3_mfma")
    return ap.parse_args()


def time_variant(name, plan, db, steps, warmup, torch):
    """Run warmup + steps launches on one stream; per-launch HIP events on that stream."""
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(warmup):
        plan.run(db.cbatch, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        plan.run(db.cbatch, stream)
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([s.elapsed_time(e) for s, e in ev])  # ms
    log(f"[bench] {name}: median {np.median(per):.3f} ms  min {per.min():.3f} ms  wall/step {wall / steps * 1e3:.3f} ms")
    return {"ms_median": float(np.median(per)), "ms_min": float(per.min()), "ms_mean": float(per.mean()),
            "wall_ms_per_step": wall / steps * 1e3}


def measured_traffic(variant, launches_bytes):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this variant,
    scaled by the counters' reading of a copy of known size; None when the kernel source has changed since
    the counters were taken (or none were taken)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path)).get(variant)
    if rec is None:
        return None, None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, "paper_2003_12787_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec["source_hash"]:
        return None, None
    t = (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0
    return t, t / launches_bytes


def copy_bandwidth(gib, torch):
    """Device-to-device copy of `gib` GiB (read + write), the measured HBM reference."""
    n = int(gib * (1 << 30)) // 4
    x = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    reps = 10
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        y.copy_(x)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    log(f"[bench] copy {gib:.2f} GiB: {ms:.3f} ms, {gbs:.0f} GB/s (read + write)")
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_read": n * 4, "bytes_written": n * 4, "ms": ms, "gbs": gbs}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (elements are independent: "
                                   "a multi-GPU run would shard them, see DESIGN.md)"}))
        sys.exit(2)
    import torch

    from paper_2003_12787_amd import runner, stp
    from paper_2003_12787_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    E = args.nelem
    log(f"[bench] generating elastic N=7 workload, {E} elements")
    b = W.c3_elastic_n7(nelem=E)
    cls = runner.class_of(b)
    results = {}
    variants = args.variants.split(",")
    specs = {
        "fp64_plain": (stp.FP64, stp.VARIANT_PLAIN),
        "fp32_plain": (stp.FP32, stp.VARIANT_PLAIN),
        "fp32_fused": (stp.FP32, stp.VARIANT_FUSED),
        "bf16x3_mfma": (stp.BF16X3, stp.VARIANT_MFMA),
    }
    for name in variants:
        prec, var = specs[name]
        plan = stp.Plan([cls], prec=prec, variant=var)
        db = runner.DeviceBatch(plan, b)
        r = time_variant(name, plan, db, args.steps, args.warmup, torch)
        bytes_el, flops_el = plan.cost(0)
        r["elements_per_s"] = E / (r["ms_median"] * 1e-3)
        r["gflops"] = flops_el * E / (r["ms_median"] * 1e-3) / 1e9
        r["hbm_gbs_algorithmic"] = bytes_el * E / (r["ms_median"] * 1e-3) / 1e9
        r["bytes_per_element"] = bytes_el
        r["flops_per_element"] = flops_el
        r["dtype"] = "f64" if prec == stp.FP64 else "f32"
        results[name] = r
        del db
        plan.close()
        torch.cuda.empty_cache()

    fp32_names = [k for k in results if results[k]["dtype"] == "f32"]
    head = max(fp32_names, key=lambda k: results[k]["elements_per_s"]) if fp32_names else variants[0]
    h = results[head]
    # roofline of the dominant (only) kernel of a step: which ceiling binds at the algorithmic counts
    t_hbm = h["bytes_per_element"] / (HBM_PEAK_GBS * 1e9)
    t_alu = h["flops_per_element"] / (ALU_PEAK_TFS[h["dtype"]] * 1e12)
    if t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": h["hbm_gbs_algorithmic"], "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": h["gflops"] / 1e3, "peak": ALU_PEAK_TFS[h["dtype"]], "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"], roof["traffic_over_algorithmic"] = measured_traffic(head, h["bytes_per_element"] * E)
    roof["kernel"] = head
    roof["hbm_frac"] = h["hbm_gbs_algorithmic"] / HBM_PEAK_GBS
    roof["alu_frac"] = h["gflops"] / 1e3 / ALU_PEAK_TFS[h["dtype"]]

    copy = None
    if args.copy_gib > 0:
        copy = copy_bandwidth(args.copy_gib, torch)

    cpu = None
    if not args.no_cpu:
        import oracle
        oracle.build()
        threads = oracle.default_threads()
        # size the sample from a short probe so that the timed run takes about --cpu-seconds
        probe = np.linspace(0, E - 1, min(E, 4 * threads)).astype(np.int64)
        t0 = time.perf_counter()
        oracle.stp(b.N, b.physics, b.Q[probe], b.dt[probe], b.h[probe], params=b.params[probe], nthreads=threads)
        rate = len(probe) / (time.perf_counter() - t0)
        k = int(min(E, max(threads, rate * args.cpu_seconds)))
        ids = np.linspace(0, E - 1, k).astype(np.int64)
        log(f"[bench] CPU oracle on {k} elements, {threads} threads")
        t0 = time.perf_counter()
        oracle.stp(b.N, b.physics, b.Q[ids], b.dt[ids], b.h[ids], params=b.params[ids], nthreads=threads)
        t = time.perf_counter() - t0
        cpu = {"value": k / t, "unit": "element-updates/s", "cores": threads, "kind": "oracle",
               "sample": f"{k} of the {E} elements (evenly spaced), FP64, {t:.1f} s"}
        log(f"[bench] CPU oracle: {k / t:.1f} el/s")

    line = {
        "metric": "STP element-updates/s + % roofline (elastic N=7) vs plain FP64; p50/p99 latency",
        "value": h["elements_per_s"],
        "unit": "element-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": h["dtype"],
        "data": "synthetic",
        "config": {"workload": "elastic waves N=7 (8^3 Gauss-Legendre nodes), m=9, per-node rho/lambda/mu, "
                               f"{E} elements, FP32 I/O", "nelem": E, "order": 7, "nquant": 9,
                   "variant": head},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": results,
        "copy_reference": copy,
        "speedup_vs_fp64_plain": (h["elements_per_s"] / results["fp64_plain"]["elements_per_s"]
                                  if "fp64_plain" in results else None),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
