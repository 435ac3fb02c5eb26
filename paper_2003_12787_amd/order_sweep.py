"""Per-order timing of the predictor's FP32 kernels: where the matrix cores could pay.

For the acoustic and elastic presets at N = 1..9 (per-node material, Q ~ N(0, 1), inputs drawn on the device),
every kernel variant that exists for the class in FP32 I/O (plain, fused; the FP32 MFMA kernel at N = 7 and
the split-BF16x3 MFMA kernels at N = 7..9) is timed with HIP events over a batch of about 2 GB of algorithmic traffic. The algorithmic bytes
(inputs read once, outputs written once) and flops come from stp_class_cost. A variant that moves its bytes
near the measured device-copy rate is bound by HBM, and faster contractions cannot shorten it; a variant well
below it is bound by its instruction issue, and that is where the matrix cores can pay.

usage: python -m paper_2003_12787_amd.order_sweep [--orders 1-9] [--steps 10]
Prints one JSON object (and a table on stderr).
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--orders", default="1-9")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--target-gb", type=float, default=2.0)
    args = ap.parse_args()
    lo, hi = (int(x) for x in args.orders.split("-"))
    import torch

    from . import stp

    assert torch.cuda.is_available(), "order_sweep needs a GPU"
    torch.cuda.set_device(0)
    # measured HBM reference: a 1 GiB device-to-device copy
    x = torch.empty(1 << 28, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(10):
        y.copy_(x)
    e.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * x.numel() * 4 / (s.elapsed_time(e) / 10 * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    out = {"copy_gbs": copy_gbs, "rows": []}
    print(f"copy {copy_gbs:.0f} GB/s", file=sys.stderr)
    names = {(stp.FP32, stp.VARIANT_PLAIN): "plain", (stp.FP32, stp.VARIANT_FUSED): "fused",
             (stp.FP32, stp.VARIANT_MFMA): "mfma32", (stp.BF16X3, stp.VARIANT_MFMA): "mfma"}
    g = torch.Generator(device="cuda")
    for phys, m, npar, pname in ((stp.ACOUSTIC, 4, 2, "acoustic"), (stp.ELASTIC, 9, 3, "elastic")):
        for N in range(lo, hi + 1):
            n3 = (N + 1) ** 3
            cls = [(N, m, phys, 0)]
            probe = stp.Plan(cls, prec=stp.FP32)
            bytes_el, flops_el = probe.cost(0)
            probe.close()
            E = int(min(262144, max(1024, args.target_gb * 1e9 / bytes_el)))
            g.manual_seed(2003127870 + 100 * N + m)
            Q = torch.randn(E * n3 * m, generator=g, device="cuda")
            par = 1.0 + torch.rand(E * n3 * npar, generator=g, device="cuda")  # positive material in [1, 2)
            qavg = torch.empty(E * n3 * m, device="cuda")
            favg = torch.empty(3 * E * n3 * m, device="cuda")
            qface = torch.empty(E * 6 * (N + 1) ** 2 * m, device="cuda")
            dt = 0.4 / ((2 * N + 1) * 2.0)
            variants = [stp.VARIANT_PLAIN] + ([stp.VARIANT_FUSED] if N <= 7 else [])
            precs = [(stp.FP32, v) for v in variants]
            if N == 7:
                precs.append((stp.FP32, stp.VARIANT_MFMA))
            if N >= 7:
                precs.append((stp.BF16X3, stp.VARIANT_MFMA))
            for prec, var in precs:
                plan = stp.Plan(cls, prec=prec, variant=var)
                b = plan.batch(E, Q, qavg, favg, qface, dt, 1.0, params=par)
                stream = torch.cuda.Stream()
                for _ in range(2):
                    plan.run(b, stream)
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(args.steps)]
                for a0, a1 in ev:
                    a0.record(stream)
                    plan.run(b, stream)
                    a1.record(stream)
                torch.cuda.synchronize()
                ms = float(np.median([a0.elapsed_time(a1) for a0, a1 in ev]))
                gbs = bytes_el * E / (ms * 1e-3) / 1e9
                row = {"physics": pname, "N": N, "variant": names[(prec, var)], "nelem": E, "ms": ms,
                       "elements_per_s": E / (ms * 1e-3), "hbm_gbs": gbs, "frac_of_copy": gbs / copy_gbs,
                       "frac_of_8tbs": gbs / 8000.0, "tflops": flops_el * E / (ms * 1e-3) / 1e12,
                       "bytes_per_element": bytes_el, "flops_per_element": flops_el}
                out["rows"].append(row)
                print(f"{pname:9s} N={N} {names[(prec, var)]:6s} E={E:7d} {ms:8.3f} ms  {gbs:6.0f} GB/s "
                      f"({gbs / copy_gbs:5.1%} of copy)  {row['tflops']:5.1f} TFLOP/s", file=sys.stderr)
                plan.close()
            del Q, par, qavg, favg, qface
            torch.cuda.empty_cache()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
