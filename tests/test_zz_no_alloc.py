"""stp_run_noalloc (the entry point for callers that cannot allocate): heterogeneous batches through the
library's static scratch give, bit for bit, what stp_run gives through the plan's allocated scratch, on two
calls in a row (the second with a smaller batch, so stale lists and counts of the first call would show), and
match the FP64 oracle on a sample. Sizes beyond the static array are refused on the host."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2003_12787_amd import stp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    oracle.build()
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def device_batch(plan, mb):
    import torch
    to = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
    f = torch.float32
    keep = dict(Q=to(mb.Q, f), params=to(mb.params, f), B=to(mb.B, f), A=to(mb.A, f), src=to(mb.src, f),
                qavg=torch.full((mb.size_q,), float("nan"), device="cuda"),
                favg=torch.full((3 * mb.size_q,), float("nan"), device="cuda"),
                qface=torch.full((mb.size_face,), float("nan"), device="cuda"),
                fface=torch.zeros(mb.size_face, device="cuda"),
                cls=to(mb.cls, torch.int32), off_q=to(mb.off_q, torch.int64), off_coef=to(mb.off_coef, torch.int64),
                off_face=to(mb.off_face, torch.int64), off_src=to(mb.off_src, torch.int64),
                dt=to(mb.dt, torch.float64), h=to(mb.h, torch.float64))
    k = keep
    b = plan.batch(len(mb.cls), k["Q"], k["qavg"], k["favg"], k["qface"], k["dt"], k["h"], params=k["params"],
                   A=k["A"], B=k["B"], src=k["src"], fface=k["fface"], cls=k["cls"], off_q=k["off_q"],
                   off_coef=k["off_coef"], off_face=k["off_face"], off_src=k["off_src"])
    return b, keep


def outputs(keep):
    return {k: keep[k].double().cpu().numpy() for k in ("qavg", "favg", "qface", "fface")}


def test_noalloc_matches_run_on_two_calls_then_smaller():
    import torch
    from test_gpu_parity import check_mixed, mixed_batch
    big = mixed_batch(E_scale=12, seed=931)
    small = mixed_batch(E_scale=1, seed=932)
    assert big.classes == small.classes and len(small.cls) < len(big.cls)
    plan = stp.Plan(big.classes, prec=stp.FP32)
    for label, mb in (("first, larger", big), ("second, smaller", small)):
        say(f"[noalloc] {label}: classes={len(mb.classes)} E={len(mb.cls)}")
        b_ref, k_ref = device_batch(plan, mb)
        plan.run(b_ref)
        b_na, k_na = device_batch(plan, mb)
        plan.run_noalloc(b_na)
        torch.cuda.synchronize()
        ref, got = outputs(k_ref), outputs(k_na)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (label, k)
        say(f"[noalloc]   bitwise equal to stp_run; worst vs oracle {check_mixed(mb, stp.FP32, got, 4):.2e}")
    plan.close()


def test_noalloc_uniform_plan_and_limits():
    import torch
    from paper_2003_12787_amd import runner
    from paper_2003_12787_amd import workloads as W
    b = W.elastic_batch(5, 50, 933)
    plan = stp.Plan([runner.class_of(b)], prec=stp.FP32)
    say("[noalloc] uniform elastic N=5 E=50")
    ref = runner.run(plan, b)
    db = runner.DeviceBatch(plan, b)
    plan.run_noalloc(db.cbatch)
    torch.cuda.synchronize()
    got = db.outputs()
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    plan.close()
    # nclass * nelem beyond the static lists: refused on the host before any launch (buffers never read)
    from test_gpu_parity import mixed_batch
    mb = mixed_batch(seed=934)
    plan = stp.Plan(mb.classes, prec=stp.FP32)
    bb, keep = device_batch(plan, mb)
    bb.nelem = (4 << 20) // len(mb.classes) + 1
    assert plan.run_noalloc_status(bb) == stp.E_INVAL and "static scratch" in stp.last_error()
    assert stp.lib().stp_run_noalloc(None, C.byref(bb), None) == stp.E_INVAL
    bb.nelem = 0
    assert plan.run_noalloc_status(bb) == stp.OK
    torch.cuda.synchronize()
    plan.close()
