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
MFMA_BF16_PEAK_TFS = 2500.0    # dense BF16 matrix-core peak
MFMA_F32_PEAK_TFS = 157.3      # dense FP32 matrix-core peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nelem", type=int, default=65536)
    ap.add_argument("--cpu-seconds", type=float, default=18.0,
                    help="target CPU-oracle time over its three timed runs (bounded sample)")
    ap.add_argument("--copy-gib", type=float, default=1.0,
                    help="size of the device-to-device copy timed as the measured HBM reference (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variants", default="fp64_plain,fp32_plain,fp32_fused,bf16x3_mfma,fp32_mfma")
    ap.add_argument("--no-hetero", action="store_true", help="skip the heterogeneous 16384-element batch")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop latency measurement")
    ap.add_argument("--serve-batches", type=int, default=10000, help="measured batches per arrival rate")
    ap.add_argument("--serve-mesh", type=int, default=131072, help="elements per resident serving mesh")
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


def time_launches(fn, steps, warmup, stream, torch):
    """Per-call HIP-event times (ms) of fn(stream) on one stream."""
    for _ in range(warmup):
        fn(stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        fn(stream)
        b.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def bench_c1(args, torch, stp, W, runner):
    """The small FP64 configuration: elastic N = 3 (4^3 nodes), 64 elements, per-node material, the plain FP64
    predictor. The whole batch is 2 MB, so a call is bound by launch latency, not by a roofline: report the
    per-call GPU time (HIP events on the stream) and the wall latency of a call plus its synchronisation, as
    p50 / p99 over many calls. Returns the outputs for the CPU leg's error check."""
    b = W.c1_elastic_n3()
    plan = stp.Plan([runner.class_of(b)], prec=stp.FP64)
    db = runner.DeviceBatch(plan, b)
    stream = torch.cuda.Stream()
    calls = 400
    ev = time_launches(lambda st: plan.run(db.cbatch, st), calls, 20, stream, torch)
    wall = np.zeros(calls)
    for i in range(calls):
        t0 = time.perf_counter()
        plan.run(db.cbatch, stream)
        stream.synchronize()
        wall[i] = time.perf_counter() - t0
    out = db.outputs()
    plan.close()
    res = {"workload": "elastic N=3 (4^3 nodes), m=9, 64 elements, per-node material, FP64 plain",
           "calls": calls, "gpu_p50_us": float(np.percentile(ev, 50) * 1e3),
           "gpu_p99_us": float(np.percentile(ev, 99) * 1e3), "wall_p50_us": float(np.percentile(wall, 50) * 1e6),
           "wall_p99_us": float(np.percentile(wall, 99) * 1e6)}
    res["elements_per_s_gpu"] = b.nelem / (res["gpu_p50_us"] * 1e-6)
    res["elements_per_s_wall"] = b.nelem / (res["wall_p50_us"] * 1e-6)
    log(f"[bench] C1 elastic N=3, 64 elements, FP64: GPU p50 {res['gpu_p50_us']:.1f} us p99 {res['gpu_p99_us']:.1f} us; "
        f"wall p50 {res['wall_p50_us']:.1f} us p99 {res['wall_p99_us']:.1f} us")
    return res, b, out


def cpu_description(threads):
    """The host CPU as /proc/cpuinfo names it, with the logical CPUs visible and the oracle's thread count."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for l in f:
                if ":" not in l:
                    if info:
                        break  # first processor only
                    continue
                k, v = (x.strip() for x in l.split(":", 1))
                if k in ("vendor_id", "model name", "cpu family", "model", "stepping", "cpu MHz", "cache size") \
                        and k not in info:
                    info[k] = v
    except OSError:
        pass
    info["logical_cpus"] = os.cpu_count()
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    info["oracle_threads"] = threads
    return info


def bench_lobatto(args, torch, stp, runner, b, ids):
    """The benchmark workload on Gauss-Lobatto nodes (the other node family of Sec. II-A): the split-BF16x3
    MFMA, FP32 MFMA and FP32 fused kernels with the plan's Lobatto tables. Returns timings and sampled outputs of
    the elements `ids` for the CPU leg."""
    E = b.nelem
    res = {"workload": "elastic N=7 benchmark workload on Gauss-Lobatto nodes (same inputs)"}
    tid = torch.from_numpy(ids).cuda()
    for name, prec, var in (("bf16x3_mfma", stp.BF16X3, stp.VARIANT_MFMA), ("fp32_mfma", stp.FP32, stp.VARIANT_MFMA),
                            ("fp32_fused", stp.FP32, stp.VARIANT_FUSED)):
        plan = stp.Plan([runner.class_of(b)], prec=prec, variant=var, nodes=stp.GAUSS_LOBATTO)
        db = runner.DeviceBatch(plan, b)
        ms = float(np.median(time_launches(lambda st: plan.run(db.cbatch, st), args.steps, args.warmup,
                                           torch.cuda.Stream(), torch)))
        res[name] = {"ms": ms, "elements_per_s": E / (ms * 1e-3),
                     "hbm_gbs_algorithmic": plan.cost(0)[0] * E / (ms * 1e-3) / 1e9,
                     "sampled": {k: v.index_select(0, tid).double().cpu().numpy()
                                 for k, v in (("qavg", db.qavg), ("favg", db.favg), ("qface", db.qface))}}
        log(f"[bench] Gauss-Lobatto {name}: {ms:.3f} ms")
        del db
        plan.close()
        torch.cuda.empty_cache()
    return res


def bench_acoustic(args, torch, stp, W, runner):
    """Acoustic plane wave, N = 5 (6^3 nodes), m = 4, 32768 elements, rho = 1, K per element: the plain
    FP64 predictor against the fused FP32 kernel (their accuracy against the oracle is a parity test)."""
    log("[bench] acoustic N=5 plane wave, 32768 elements")
    b = W.c2_acoustic_n5()
    out = {"workload": "acoustic plane wave N=5 (6^3 nodes), m=4, 32768 elements, rho=1, K~U[1,2] per element"}
    for name, prec, var in (("fp64_plain", stp.FP64, stp.VARIANT_PLAIN), ("fp32_fused", stp.FP32, stp.VARIANT_FUSED)):
        plan = stp.Plan([runner.class_of(b)], prec=prec, variant=var)
        db = runner.DeviceBatch(plan, b)
        ms = float(np.median(time_launches(lambda st: plan.run(db.cbatch, st), args.steps, args.warmup,
                                           torch.cuda.Stream(), torch)))
        bytes_el = plan.cost(0)[0]
        out[name] = {"ms": ms, "elements_per_s": b.nelem / (ms * 1e-3),
                     "hbm_gbs_algorithmic": bytes_el * b.nelem / (ms * 1e-3) / 1e9}
        log(f"[bench] acoustic {name}: {ms:.3f} ms")
        del db
        plan.close()
    torch.cuda.empty_cache()
    out["speedup_fp32_fused_vs_fp64_plain"] = out["fp64_plain"]["ms"] / out["fp32_fused"]["ms"]
    return out


def bench_full_step(args, torch, stp, W):
    """A full ADER-DG step on a periodic 64 x 32 x 32 mesh (65536 elements): elastic N = 7, per-element
    material, the split-BF16x3 predictor (stp_run) then the corrector (stp_correct), FP32."""
    nx, ny, nz = 64, 32, 32
    E, N, m = nx * ny * nz, 7, 9
    n3, n2 = (N + 1) ** 3, (N + 1) ** 2
    log(f"[bench] full step: {nx} x {ny} x {nz} mesh, elastic N=7, per-element material")
    g = torch.Generator(device="cuda")
    g.manual_seed(W.SEED0 + 60)
    Q = torch.randn(E * n3 * m, generator=g, device="cuda")
    u = torch.rand(E, 3, generator=g, device="cuda")
    par = (torch.tensor([2.0, 1.0, 1.0], device="cuda") + torch.tensor([1.0, 3.0, 2.0], device="cuda") * u).reshape(-1)
    h = 1.0 / nx
    dt = 0.2 * h / ((2 * N + 1) * W.C_MAX[W.ELASTIC])
    plan = stp.Plan([(N, m, stp.ELASTIC, stp.PARAM_PER_ELEMENT)], prec=stp.BF16X3)
    qavg = torch.empty(E * n3 * m, device="cuda")
    favg = torch.empty(3 * E * n3 * m, device="cuda")
    qface = torch.empty(E * 6 * n2 * m, device="cuda")
    Qn = torch.empty_like(Q)
    batch = plan.batch(E, Q, qavg, favg, qface, dt, h, params=par)
    stream = torch.cuda.Stream()
    t_pred = time_launches(lambda st: plan.run(batch, st), args.steps, args.warmup, stream, torch)
    t_corr = time_launches(lambda st: plan.correct((nx, ny, nz), dt, h, Q, favg, qface, Qn, params=par, stream=st),
                           args.steps, args.warmup, stream, torch)

    def step(st):
        plan.run(batch, st)
        plan.correct((nx, ny, nz), dt, h, Q, favg, qface, Qn, params=par, stream=st)

    t_step = time_launches(step, args.steps, args.warmup, stream, torch)
    plan.close()
    # algorithmic bytes: Q and favg x3 read, q_new written, and every element's face block read once (a block is
    # used by its element and by the neighbour across each face; the second use is not new HBM data)
    corr_bytes = 4.0 * (5 * n3 * m + 6 * n2 * m) * E
    ms_c = float(np.median(t_corr))
    res = {"workload": f"periodic {nx}x{ny}x{nz} mesh, elastic N=7, per-element material, split-BF16x3 predictor "
                       "+ FP32 corrector", "nelem": E,
           "ms_predictor": float(np.median(t_pred)), "ms_corrector": ms_c, "ms_step": float(np.median(t_step)),
           "element_steps_per_s": E / (float(np.median(t_step)) * 1e-3),
           "corrector_hbm_gbs_algorithmic": corr_bytes / (ms_c * 1e-3) / 1e9,
           "corrector_hbm_frac": corr_bytes / (ms_c * 1e-3) / 1e9 / HBM_PEAK_GBS}
    log(f"[bench] full step: predictor {res['ms_predictor']:.3f} ms, corrector {ms_c:.3f} ms "
        f"({res['corrector_hbm_gbs_algorithmic']:.0f} GB/s), step {res['ms_step']:.3f} ms")

    # the same mesh under a non-symmetric affine map (curvilinear elastic elements, one metric per element):
    # the paper's benchmark physics over a full step
    rng = np.random.default_rng(W.SEED0 + 61)
    G = np.linalg.inv(np.eye(3) + 0.2 * rng.standard_normal((3, 3)))
    parc = torch.cat([par.reshape(E, 3), torch.tensor(G.ravel(), device="cuda", dtype=torch.float32).expand(E, 9)],
                     dim=1).contiguous().reshape(-1)
    gmax = float(np.linalg.norm(G, axis=1).max())
    dtc = 0.2 * h / ((2 * N + 1) * W.C_MAX[W.ELASTIC] * gmax)
    plan = stp.Plan([(N, m, stp.ELASTIC_CURV, stp.PARAM_PER_ELEMENT)], prec=stp.BF16X3)
    batch = plan.batch(E, Q, qavg, favg, qface, dtc, h, params=parc)
    t_pred = time_launches(lambda st: plan.run(batch, st), args.steps, args.warmup, stream, torch)
    t_corr = time_launches(lambda st: plan.correct((nx, ny, nz), dtc, h, Q, favg, qface, Qn, params=parc, stream=st),
                           args.steps, args.warmup, stream, torch)

    def step_c(st):
        plan.run(batch, st)
        plan.correct((nx, ny, nz), dtc, h, Q, favg, qface, Qn, params=parc, stream=st)

    t_step = time_launches(step_c, args.steps, args.warmup, stream, torch)
    plan.close()
    res["curvilinear"] = {"workload": "the same mesh under a non-symmetric affine map: curvilinear elastic "
                                      "elements with one metric per element (12 parameters)",
                          "ms_predictor": float(np.median(t_pred)), "ms_corrector": float(np.median(t_corr)),
                          "ms_step": float(np.median(t_step)),
                          "element_steps_per_s": E / (float(np.median(t_step)) * 1e-3)}
    log(f"[bench] full step (affine curvilinear): predictor {res['curvilinear']['ms_predictor']:.3f} ms, corrector "
        f"{res['curvilinear']['ms_corrector']:.3f} ms, step {res['curvilinear']['ms_step']:.3f} ms")
    del Q, qavg, favg, qface, Qn
    torch.cuda.empty_cache()
    return res


def bench_curvilinear(args, torch, stp, W):
    """Elastic waves on curvilinear elements (the benchmark physics of Sec. VI: 9 wave quantities and 12
    parameters per node, material and metric terms), N = 7, the elements of a deformed 64 x 32 x 32 box,
    inputs generated on the device. The split-BF16x3 MFMA kernel and the FP32 and FP64 plain kernels (the fused
    kernel covers the Cartesian presets). Returns the timings and, for the CPU leg, the inputs and outputs of
    256 elements."""
    N, E, m = 7, args.nelem, 9
    n3, n2 = (N + 1) ** 3, (N + 1) ** 2
    log(f"[bench] curvilinear elastic N=7, {E} elements, generating on the device")
    Q, par, dt = W.curvilinear_device(N, E, W.SEED0 + 7)
    ids = np.linspace(0, E - 1, min(E, 256)).astype(np.int64)
    tid = torch.from_numpy(ids).cuda()
    res = {"workload": f"curvilinear elastic N=7, m=9 + 12 per-node parameters (rho, lambda, mu, 9 metric terms), "
                       f"{E} elements of a deformed {'x'.join(map(str, W.grid_of(E)))} box, FP32 I/O",
           "nelem": E, "check": {"ids": ids, "Q": Q.index_select(0, tid).double().cpu().numpy(),
                                  "params": par.index_select(0, tid).double().cpu().numpy(), "dt": dt}}
    for name, prec, var in (("bf16x3_mfma", stp.BF16X3, stp.VARIANT_MFMA), ("fp32_plain", stp.FP32, stp.VARIANT_PLAIN),
                            ("fp64_plain", stp.FP64, stp.VARIANT_PLAIN)):
        tdt = torch.float64 if prec == stp.FP64 else torch.float32
        plan = stp.Plan([(N, m, stp.ELASTIC_CURV, 0)], prec=prec, variant=var)
        q, p = Q.to(tdt), par.to(tdt)
        qavg = torch.empty((E, n3, m), device="cuda", dtype=tdt)
        favg = torch.empty((E, 3, n3, m), device="cuda", dtype=tdt)
        qface = torch.empty((E, 6, n2, m), device="cuda", dtype=tdt)
        batch = plan.batch(E, q, qavg, favg, qface, dt, 1.0, params=p)
        ms = float(np.median(time_launches(lambda st: plan.run(batch, st), args.steps, args.warmup,
                                           torch.cuda.Stream(), torch)))
        bytes_el, flops_el = plan.cost(0)
        res[name] = {"ms": ms, "elements_per_s": E / (ms * 1e-3),
                     "hbm_gbs_algorithmic": bytes_el * E / (ms * 1e-3) / 1e9,
                     "tflops": flops_el * E / (ms * 1e-3) / 1e12,
                     "alu_frac": flops_el * E / (ms * 1e-3) / 1e12 / ALU_PEAK_TFS["f64" if prec == stp.FP64 else "f32"],
                     "hbm_frac": bytes_el * E / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "bytes_per_element": bytes_el, "flops_per_element": flops_el,
                     "sampled": {k: v.index_select(0, tid).double().cpu().numpy()
                                 for k, v in (("qavg", qavg), ("favg", favg), ("qface", qface))}}
        log(f"[bench] curvilinear {name}: {ms:.3f} ms, {res[name]['tflops']:.1f} TFLOP/s "
            f"({100 * res[name]['alu_frac']:.1f}% of the VALU peak)")
        grid = W.grid_of(E)
        if name == "bf16x3_mfma" and grid[0] * grid[1] * grid[2] == E:
            # a full ADER-DG step on the curved periodic mesh: MFMA predictor, then the corrector with the
            # parameters at the face points, extrapolated once before the time loop (they do not change); the
            # corrector that extrapolates them at every step is timed beside it (the full step takes half the
            # predictor workloads' dt)
            Qn = torch.empty_like(q)
            dts = dt / 2
            b2 = plan.batch(E, q, qavg, favg, qface, dts, 1.0, params=p)
            st0 = torch.cuda.Stream()
            fp = torch.empty((E, 6, n2, 12), device="cuda", dtype=tdt)
            t_fp = time_launches(lambda st: plan.face_params(E, p, fp, stream=st), 3, 1, st0, torch)
            t_corr = time_launches(lambda st: plan.correct(grid, dts, 1.0, q, favg, qface, Qn, params=p, fparams=fp,
                                                           stream=st), args.steps, args.warmup, st0, torch)
            t_ext = time_launches(lambda st: plan.correct(grid, dts, 1.0, q, favg, qface, Qn, params=p, stream=st),
                                  args.steps, args.warmup, st0, torch)

            def step(st):
                plan.run(b2, st)
                plan.correct(grid, dts, 1.0, q, favg, qface, Qn, params=p, fparams=fp, stream=st)

            t_step = time_launches(step, args.steps, args.warmup, st0, torch)
            res["ader_dg_step"] = {"mesh": "x".join(map(str, grid)) + ", periodic, curved (metric per node)",
                                   "ms_corrector": float(np.median(t_corr)), "ms_step": float(np.median(t_step)),
                                   "ms_corrector_extrapolating": float(np.median(t_ext)),
                                   "ms_face_params_once": float(np.median(t_fp)),
                                   "element_steps_per_s": E / (float(np.median(t_step)) * 1e-3)}
            log(f"[bench] curvilinear full step: corrector {res['ader_dg_step']['ms_corrector']:.3f} ms "
                f"({res['ader_dg_step']['ms_corrector_extrapolating']:.3f} ms extrapolating the parameters; "
                f"{res['ader_dg_step']['ms_face_params_once']:.3f} ms once for the face parameters), step "
                f"{res['ader_dg_step']['ms_step']:.3f} ms")
            del fp
            del Qn
        del q, p, qavg, favg, qface
        plan.close()
    del Q, par
    torch.cuda.empty_cache()
    res["speedup_fp32_vs_fp64"] = res["fp64_plain"]["ms"] / res["fp32_plain"]["ms"]
    res["speedup_mfma_vs_fp32_plain"] = res["fp32_plain"]["ms"] / res["bf16x3_mfma"]["ms"]
    return res


def bench_hetero(args, torch, stp, W):
    """Mixed orders and quantity counts in one batch: 16384 generic elements, N ~ U{2..9}, m ~ U{4, 9},
    dense per-node B_d, FP32. Times the heterogeneous stp_run (eager and replayed from a captured HIP graph)
    against the same elements run as one uniform launch per class."""
    log("[bench] heterogeneous: generating 16384 generic elements on the device")
    d = W.c4_device(16384)
    E = d["nelem"]
    plan = stp.Plan(d["classes"], prec=stp.FP32, autotune=1)  # tuned (or cached) grid and tile sizes
    tuned = plan.describe()
    log(f"[bench] heterogeneous: tuned grid {tuned['hetero_grid_per_cu']}/CU, "
        f"tile LDS budget {tuned['hetero_lds_budget'] // 1024} KB")
    plan.reserve(E)
    qavg = torch.empty(d["size_q"], device="cuda")
    favg = torch.empty(3 * d["size_q"], device="cuda")
    qface = torch.empty(d["size_face"], device="cuda")
    batch = plan.batch(E, d["Q"], qavg, favg, qface, d["dt"], d["h"], B=d["B"], cls=d["cls"], off_q=d["off_q"],
                       off_coef=d["off_coef"], off_face=d["off_face"])
    stream = torch.cuda.Stream()
    eager = time_launches(lambda st: plan.run(batch, st), args.steps, args.warmup, stream, torch)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        plan.run(batch)
    graph = time_launches(lambda st: g.replay(), args.steps, 2, torch.cuda.current_stream(), torch)
    bytes_tot = sum(plan.cost(c)[0] * int(k) for c, k in enumerate(d["counts"]))
    flops_tot = sum(plan.cost(c)[1] * int(k) for c, k in enumerate(d["counts"]))
    # the same elements, one uniform plan and launch per class over its contiguous storage
    per_class, per_class_ms = [], {}
    for c, (first, k) in enumerate(d["class_ranges"]):
        if k == 0:
            continue
        up = stp.Plan([d["classes"][c]], prec=stp.FP32)
        sq, sf, sc = int(d["sizes_q"][c]), int(d["sizes_face"][c]), int(d["sizes_coef"][c])
        oq, of, oc = int(d["storage_q"][first]), int(d["storage_face"][first]), int(d["storage_coef"][first])
        ids = torch.from_numpy(d["order"][first:first + k]).cuda()
        dts, hs = d["dt"][ids].contiguous(), d["h"][ids].contiguous()
        ub = up.batch(k, d["Q"][oq:oq + k * sq], qavg[oq:oq + k * sq], favg[3 * oq:3 * (oq + k * sq)],
                      qface[of:of + k * sf], dts, hs, B=d["B"][oc:oc + k * sc])
        t = time_launches(lambda st: up.run(ub, st), max(3, args.steps // 2), 2, stream, torch)
        per_class.append(float(np.median(t)))
        per_class_ms[f"N{d['classes'][c][0]}m{d['classes'][c][1]}"] = per_class[-1]
        up.close()
    del g
    plan.close()
    ms = float(np.median(eager))
    res = {"workload": f"{E} generic elements, N ~ U{{2..9}}, m ~ U{{4,9}}, dense per-node B_d, FP32, "
                       f"{len(d['classes'])} classes",
           "ms_eager": ms, "ms_graph": float(np.median(graph)), "elements_per_s": E / (ms * 1e-3),
           "algorithmic_bytes": bytes_tot, "hbm_gbs_algorithmic": bytes_tot / (ms * 1e-3) / 1e9,
           "hbm_frac": bytes_tot / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "gflops": flops_tot / (ms * 1e-3) / 1e9,
           "ms_one_launch_per_class_sum": float(sum(per_class)), "ms_one_launch_per_class": per_class_ms,
           "tuned": {"grid_per_cu": tuned["hetero_grid_per_cu"], "tile_lds_budget": tuned["hetero_lds_budget"],
                     "elements_per_tile": {f"N{c['order']}m{c['nquant']}": c["elements_per_tile"]
                                           for c in tuned["classes"] if c["tiled"]}}}
    log(f"[bench] heterogeneous: eager {ms:.3f} ms, graph {res['ms_graph']:.3f} ms, "
        f"{res['hbm_gbs_algorithmic']:.0f} GB/s algorithmic; per-class launches sum {sum(per_class):.3f} ms")
    del d, qavg, favg, qface
    torch.cuda.empty_cache()
    return res


def bench_serving(args, torch, stp, W):
    """Serving loop: batches of log-uniform size 1..4096 (contiguous runs of element ids) from two resident
    p-adaptive meshes (acoustic m=4 and elastic m=9, N ~ U{2..9}), FP32 with FP64 accumulation at N >= 8,
    admission budget 2 GiB. Measures the saturated throughput (batches submitted back to back), then
    Poisson arrivals at 50 % and 80 % of it; latency = completion - submission (library timestamps)."""
    import ctypes as C
    E = args.serve_mesh
    log(f"[bench] serving: generating two resident meshes of {E} elements")
    meshes = [W.serving_mesh(W.ACOUSTIC, E, W.SEED0 + 50, 0), W.serving_mesh(W.ELASTIC, E, W.SEED0 + 51, 8)]
    classes = [(N, 4, stp.ACOUSTIC, 0) for N in range(2, 10)] + [(N, 9, stp.ELASTIC, 0) for N in range(2, 10)]
    plan = stp.Plan(classes, prec=stp.FP32, acc64_min_order=8, serve_mem_budget=2 << 30)
    for mh in meshes:
        mh["qavg"] = torch.empty(mh["size_q"], device="cuda")
        mh["favg"] = torch.empty(3 * mh["size_q"], device="cuda")
        mh["qface"] = torch.empty(mh["size_face"], device="cuda")
    L = stp.lib()
    rng = np.random.default_rng(W.SEED0 + 52)

    def make_batches(n, seed):
        sizes = W.serving_batch_sizes(n, seed)
        which = rng.integers(0, 2, n)
        out = []
        for k, w in zip(sizes, which):
            mh = meshes[w]
            a = int(rng.integers(0, E - k + 1))
            b = stp.Batch()
            b.nelem = int(k)
            b.cls = mh["cls"].data_ptr() + 4 * a
            for f in ("off_q", "off_coef", "off_face", "dt", "h"):
                setattr(b, f, mh[f].data_ptr() + 8 * a)
            b.dt_h_scalar = 0
            b.Q, b.params = mh["Q"].data_ptr(), mh["params"].data_ptr()
            b.qavg, b.favg, b.qface = mh["qavg"].data_ptr(), mh["favg"].data_ptr(), mh["qface"].data_ptr()
            out.append(b)
        return out, int(sizes.sum())

    def run(batches, gaps=None):
        """Submit (back to back, or at the scheduled arrival times), drain, return per-batch latencies."""
        tickets = np.zeros(len(batches), dtype=np.uint64)
        t = C.c_uint64()
        t0 = time.perf_counter()
        due = t0
        for i, b in enumerate(batches):
            if gaps is not None:
                due += gaps[i]
                while time.perf_counter() < due:
                    pass
            st = L.stp_submit(plan.handle, C.byref(b), C.byref(t))
            if st != stp.OK:
                raise stp.StpError(st, stp.last_error())
            tickets[i] = t.value
        plan.drain()
        info = stp.TicketInfo()
        lat, first, last = np.zeros(len(batches)), None, 0.0
        for i, tk in enumerate(tickets):
            st = L.stp_poll(plan.handle, C.c_uint64(int(tk)), C.byref(info))
            assert st == stp.OK, (st, stp.last_error())
            lat[i] = info.t_done - info.t_submit
            first = info.t_submit if first is None else min(first, info.t_submit)
            last = max(last, info.t_done)
        return lat, last - first

    warm, _ = make_batches(500, W.SEED0 + 53)
    run(warm)
    sat_b, sat_el = make_batches(max(2000, args.serve_batches // 3), W.SEED0 + 54)
    _, span = run(sat_b)
    sat_rate = len(sat_b) / span
    res = {"workload": f"two resident meshes of {E} elements (acoustic m=4, elastic m=9), N ~ U{{2..9}}, "
                       "batches of log-uniform size 1..4096, FP32 with FP64 accumulation at N >= 8, "
                       "2 GiB admission budget",
           "saturated": {"batches_per_s": sat_rate, "elements_per_s": sat_el / span,
                         "mean_batch_elements": sat_el / len(sat_b)}}
    log(f"[bench] serving saturated: {sat_rate:.0f} batches/s, {sat_el / span:.3g} el/s")
    for frac in (0.5, 0.8):
        bs, n_el = make_batches(args.serve_batches, W.SEED0 + 55 + int(frac * 10))
        gaps = rng.exponential(1.0 / (frac * sat_rate), len(bs))
        lat, span = run(bs, gaps)
        key = f"load_{int(frac * 100)}pct"
        res[key] = {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                    "mean_ms": float(lat.mean() * 1e3), "batches": len(bs),
                    "offered_batches_per_s": frac * sat_rate, "achieved_batches_per_s": len(bs) / span,
                    "elements_per_s": n_el / span}
        log(f"[bench] serving {key}: p50 {res[key]['p50_ms']:.3f} ms, p99 {res[key]['p99_ms']:.3f} ms")
    plan.close()
    del meshes
    torch.cuda.empty_cache()
    return res


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
    # inputs rounded to FP32 once: every variant (FP64 included) and the oracle see the same values
    b = runner.rounded(W.c3_elastic_n7(nelem=E), stp.FP32)
    err_ids = np.linspace(0, E - 1, min(E, 2048)).astype(np.int64)  # elements checked against the oracle
    sampled = {}
    cls = runner.class_of(b)
    results = {}
    variants = args.variants.split(",")
    specs = {
        "fp64_plain": (stp.FP64, stp.VARIANT_PLAIN),
        "fp32_plain": (stp.FP32, stp.VARIANT_PLAIN),
        "fp32_fused": (stp.FP32, stp.VARIANT_FUSED),
        "bf16x3_mfma": (stp.BF16X3, stp.VARIANT_MFMA),
        "fp32_mfma": (stp.FP32, stp.VARIANT_MFMA),
    }
    for name in variants:
        prec, var = specs[name]
        plan = stp.Plan([cls], prec=prec, variant=var)
        db = runner.DeviceBatch(plan, b)
        r = time_variant(name, plan, db, args.steps, args.warmup, torch)
        idx = torch.from_numpy(err_ids).cuda()
        sampled[name] = {k: v.index_select(0, idx).double().cpu().numpy() for k, v in
                         (("qavg", db.qavg), ("favg", db.favg), ("qface", db.qface))}
        bytes_el, flops_el = plan.cost(0)
        r["elements_per_s"] = E / (r["ms_median"] * 1e-3)
        r["gflops"] = flops_el * E / (r["ms_median"] * 1e-3) / 1e9
        r["hbm_gbs_algorithmic"] = bytes_el * E / (r["ms_median"] * 1e-3) / 1e9
        r["bytes_per_element"] = bytes_el
        r["flops_per_element"] = flops_el
        # arithmetic of the path: FP64, FP32, or split-BF16x3 contractions with FP32 accumulation and FP32 VALU
        r["dtype"] = {stp.FP64: "f64", stp.FP32: "f32", stp.BF16X3: "bf16x3"}[prec]
        results[name] = r
        del db
        plan.close()
        torch.cuda.empty_cache()

    fp32_names = [k for k in results if results[k]["dtype"] != "f64"]  # FP32 I/O variants
    head = max(fp32_names, key=lambda k: results[k]["elements_per_s"]) if fp32_names else variants[0]
    h = results[head]
    # Roofline of the dominant (only) kernel of a step: which ceiling binds at the algorithmic counts. The
    # derivative contractions are 2 n n^3 q_d flops per direction and application (q_d = 6 quantities read
    # by the elastic B_d), N+1 applications; on the split-BF16x3 variant they run on the matrix cores: one
    # 16x16x32 BF16 product per 16 lines of 8 nodes, 8 times the contraction's multiply-adds (the six split
    # products, two output rows per node, the other line group's zero blocks), at the dense BF16 peak; the
    # rest of its flops run on the VALU. The FP32 MFMA variant forms exactly the contraction's products on the
    # matrix cores (4x4 blocks of the lanes' own lines, nothing wasted) at the dense FP32 matrix peak.
    valu = "f64" if h["dtype"] == "f64" else "f32"  # the VALU type of the non-contraction work
    n = b.N + 1
    contr = (b.N + 1) * 3 * 2 * n * n ** 3 * 6
    t_hbm = h["bytes_per_element"] / (HBM_PEAK_GBS * 1e9)
    if head == "bf16x3_mfma":
        t_cmp = 8 * contr / (MFMA_BF16_PEAK_TFS * 1e12) + (h["flops_per_element"] - contr) / (ALU_PEAK_TFS["f32"] * 1e12)
    elif head == "fp32_mfma":
        t_cmp = contr / (MFMA_F32_PEAK_TFS * 1e12) + (h["flops_per_element"] - contr) / (ALU_PEAK_TFS["f32"] * 1e12)
    else:
        t_cmp = h["flops_per_element"] / (ALU_PEAK_TFS[valu] * 1e12)
    if t_hbm >= t_cmp:
        roof = {"bound": "hbm", "achieved": h["hbm_gbs_algorithmic"], "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": h["gflops"] / 1e3, "peak": ALU_PEAK_TFS[valu], "unit": "TFLOP/s"}
    roof["t_hbm_ns_per_element"] = t_hbm * 1e9
    roof["t_compute_ns_per_element"] = t_cmp * 1e9
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"], roof["traffic_over_algorithmic"] = measured_traffic(head, h["bytes_per_element"] * E)
    roof["kernel"] = head
    roof["hbm_frac"] = h["hbm_gbs_algorithmic"] / HBM_PEAK_GBS
    roof["alu_frac"] = h["gflops"] / 1e3 / ALU_PEAK_TFS[valu]

    copy = None
    if args.copy_gib > 0:
        copy = copy_bandwidth(args.copy_gib, torch)

    c1, c1_batch, c1_out = bench_c1(args, torch, stp, W, runner)
    lob_ids = np.linspace(0, E - 1, min(E, 256)).astype(np.int64)
    lobatto = None if args.no_hetero else bench_lobatto(args, torch, stp, runner, b, lob_ids)
    acoustic = None if args.no_hetero else bench_acoustic(args, torch, stp, W, runner)
    full_step = None if args.no_hetero else bench_full_step(args, torch, stp, W)
    curv = None if args.no_hetero else bench_curvilinear(args, torch, stp, W)
    hetero = None if args.no_hetero else bench_hetero(args, torch, stp, W)
    serving = None if args.no_serve else bench_serving(args, torch, stp, W)

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
        k = int(min(E, max(threads, rate * args.cpu_seconds / 3)))
        ids = np.unique(np.concatenate([np.linspace(0, E - 1, k).astype(np.int64), err_ids]))
        k = len(ids)
        log(f"[bench] CPU oracle on {k} elements, {threads} threads, 3 runs")
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            ref = oracle.stp(b.N, b.physics, b.Q[ids], b.dt[ids], b.h[ids], params=b.params[ids], nthreads=threads)
            times.append(time.perf_counter() - t0)
        t = float(np.median(times))
        # per-output max-relative error of every variant on the checked elements (a subset of the sample)
        pos = np.searchsorted(ids, err_ids)
        for name, got in sampled.items():
            errs = {}
            for key in ("qavg", "favg", "qface"):
                y = ref[key][pos].reshape(len(pos), -1)
                x = got[key].reshape(len(pos), -1)
                errs[key] = float((np.abs(x - y).max(axis=1) / np.abs(y).max(axis=1)).max())
            results[name]["max_rel_err_vs_oracle"] = errs
            results[name]["checked_elements"] = int(len(pos))
            log(f"[bench] {name}: max rel err vs oracle {errs}")
        del ref
        if lobatto is not None:  # sampled parity on Gauss-Lobatto nodes
            ref = oracle.stp(b.N, b.physics, b.Q[lob_ids], b.dt[lob_ids], b.h[lob_ids], params=b.params[lob_ids],
                             nthreads=threads, nodes=1)
            for name in ("bf16x3_mfma", "fp32_mfma", "fp32_fused"):
                got = lobatto[name]["sampled"]
                errs = {}
                for key in ("qavg", "favg", "qface"):
                    y = ref[key].reshape(len(lob_ids), -1)
                    x = got[key].reshape(len(lob_ids), -1)
                    errs[key] = float((np.abs(x - y).max(axis=1) / np.abs(y).max(axis=1)).max())
                lobatto[name]["max_rel_err_vs_oracle"] = errs
                lobatto[name]["checked_elements"] = int(len(lob_ids))
                log(f"[bench] Gauss-Lobatto {name}: max rel err vs oracle {errs}")
            del ref
        if curv is not None:  # sampled parity of the curvilinear workload
            ck = curv["check"]
            ref = oracle.stp(7, W.ELASTIC_CURV, ck["Q"], ck["dt"], 1.0, params=ck["params"], nthreads=threads)
            for name in ("bf16x3_mfma", "fp32_plain", "fp64_plain"):
                got = curv[name]["sampled"]
                errs = {}
                for key in ("qavg", "favg", "qface"):
                    y = ref[key].reshape(len(ck["ids"]), -1)
                    x = got[key].reshape(len(ck["ids"]), -1)
                    errs[key] = float((np.abs(x - y).max(axis=1) / np.abs(y).max(axis=1)).max())
                curv[name]["max_rel_err_vs_oracle"] = errs
                curv[name]["checked_elements"] = int(len(ck["ids"]))
                log(f"[bench] curvilinear {name}: max rel err vs oracle {errs}")
            del ref
        # C1: every element of the small FP64 batch against the oracle
        ref = oracle.stp(c1_batch.N, c1_batch.physics, c1_batch.Q, c1_batch.dt, c1_batch.h, params=c1_batch.params,
                         nthreads=threads)
        errs = {}
        for key in ("qavg", "favg", "qface"):
            y = ref[key].reshape(c1_batch.nelem, -1)
            x = c1_out[key].reshape(c1_batch.nelem, -1)
            errs[key] = float((np.abs(x - y).max(axis=1) / np.abs(y).max(axis=1)).max())
        c1["max_rel_err_vs_oracle"] = errs
        log(f"[bench] C1: max rel err vs oracle {errs}")
        del ref
        # one host thread on a small sample, for the per-core rate
        one = np.linspace(0, E - 1, min(E, 256)).astype(np.int64)
        t0 = time.perf_counter()
        oracle.stp(b.N, b.physics, b.Q[one], b.dt[one], b.h[one], params=b.params[one], nthreads=1)
        t1 = time.perf_counter() - t0
        desc = cpu_description(threads)
        cpu = {"value": k / t, "unit": "element-updates/s", "cores": threads, "kind": "oracle",
               "sample": f"{k} of the {E} elements (evenly spaced), FP64; median of 3 runs "
                         f"({', '.join(f'{x:.1f}' for x in times)} s)",
               "value_1thread": len(one) / t1, "sample_1thread": f"{len(one)} elements, {t1:.2f} s",
               "cpu_model": desc.get("model name", ""), "cpu": desc}
        log(f"[bench] CPU oracle: {k / t:.1f} el/s ({threads} threads, median of 3), {len(one) / t1:.1f} el/s "
            f"(1 thread), {desc}")

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
        "acoustic_n5": acoustic,
        "ader_dg_step": full_step,
        "gauss_lobatto": None if lobatto is None else {k: ({kk: vv for kk, vv in v.items() if kk != "sampled"}
                                                           if isinstance(v, dict) else v)
                                                       for k, v in lobatto.items()},
        "curvilinear": None if curv is None else {k: ({kk: vv for kk, vv in v.items() if kk != "sampled"}
                                                      if isinstance(v, dict) else v)
                                                  for k, v in curv.items() if k != "check"},
        "c1_latency": c1,
        "heterogeneous": hetero,
        "serving": serving,
        "latency_p50_ms": serving["load_80pct"]["p50_ms"] if serving else None,
        "latency_p99_ms": serving["load_80pct"]["p99_ms"] if serving else None,
        "speedup_vs_fp64_plain": (h["elements_per_s"] / results["fp64_plain"]["elements_per_s"]
                                  if "fp64_plain" in results else None),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
