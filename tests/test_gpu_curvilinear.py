"""GPU parity of curvilinear elastic elements (STP_ELASTIC_CURV: material and metric terms per node) against
the oracle, through the C ABI: every precision of the plain kernel, per-node (curved) and per-element
(affine) parameters, a heterogeneous batch mixing curvilinear and Cartesian classes, and the
unsupported combinations."""
import sys

import numpy as np
import pytest

import oracle
from paper_2003_12787_amd import runner, stp
from paper_2003_12787_amd import workloads as W
from parity import TOL, max_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check(b, prec, acc64_min_order=0, variant=stp.VARIANT_AUTO):
    plan = stp.Plan([runner.class_of(b)], prec=prec, acc64_min_order=acc64_min_order, variant=variant)
    say(f"[curvilinear] N={b.N} E={b.nelem} per_element={b.coef_per_element} prec={prec} "
        f"acc64_min_order={acc64_min_order} -> {plan.describe()['classes'][0]['variant']}")
    got = runner.run(plan, b)
    rb = runner.rounded(b, prec)
    ref = oracle.stp(rb.N, rb.physics, rb.Q, rb.dt, rb.h, params=rb.params, coef_per_element=rb.coef_per_element)
    err = max_rel_err(got, ref, rb.Q, rb.h)
    say(f"[curvilinear]   max rel err {err}")
    for k, v in err.items():
        assert v < TOL[prec], (k, v)
    plan.close()


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9])
def test_curvilinear_fp64(N):
    check(W.curvilinear_batch(N, 40, 800 + N), stp.FP64)


@pytest.mark.parametrize("N", [3, 7, 8])
def test_curvilinear_fp32(N):
    check(W.curvilinear_batch(N, 40, 810 + N), stp.FP32)


def test_curvilinear_fp32_acc64_and_bf16x3_plan():
    check(W.curvilinear_batch(9, 24, 821), stp.FP32, acc64_min_order=8)
    check(W.curvilinear_batch(7, 24, 822), stp.BF16X3)  # no MFMA kernel: the plan takes the FP32 plain one


@pytest.mark.parametrize("N", [2, 6])
def test_curvilinear_per_element(N):
    check(W.curvilinear_batch(N, 36, 830 + N, per_node=False), stp.FP32)
    check(W.curvilinear_batch(N, 36, 840 + N, per_node=False), stp.FP64)


def test_identity_metric_matches_cartesian_kernel(gpu):
    """Curvilinear elements with G = I on the GPU against the Cartesian elastic kernel on the same data."""
    b = W.elastic_batch(5, 48, 850)
    par = np.concatenate([b.params, np.broadcast_to(np.eye(3).ravel(), b.params.shape[:-1] + (9,))], axis=-1)
    bc = W.Batch(b.N, 9, W.ELASTIC_CURV, b.Q, b.dt, b.h, params=par)
    outs = []
    for batch in (b, bc):
        plan = stp.Plan([runner.class_of(batch)], prec=stp.FP64, variant=stp.VARIANT_PLAIN)
        outs.append(runner.run(plan, batch))
        plan.close()
    for k in ("qavg", "favg", "qface"):
        err = np.abs(outs[0][k] - outs[1][k]).max() / np.abs(outs[0][k]).max()
        say(f"[curvilinear] G = I vs Cartesian {k}: {err:.2e}")
        assert err < 1e-13, (k, err)


def test_mixed_batch_with_curvilinear_classes():
    """Curvilinear classes run on launches of their own beside the persistent launch of the Cartesian
    buckets; the whole batch is one stp_run."""
    from test_gpu_parity import check_mixed, run_mixed
    parts = [W.curvilinear_batch(3, 30, 861), W.elastic_batch(3, 40, 862), W.curvilinear_batch(7, 10, 863),
             W.acoustic_batch(4, 25, 864), W.curvilinear_batch(2, 20, 865, per_node=False)]
    classes = [runner.class_of(p) for p in parts]
    mb = W.interleave(parts, classes, 866)
    plan = stp.Plan(classes, prec=stp.FP32)
    say(f"[curvilinear] mixed batch: {len(mb.cls)} elements, classes {classes}")
    got = run_mixed(plan, mb, stp.FP32)
    worst = check_mixed(mb, stp.FP32, got)
    say(f"[curvilinear]   worst rel err {worst:.2e}")
    plan.close()


def test_unsupported_combinations(gpu):
    torch = gpu
    cls = [(7, 9, stp.ELASTIC_CURV, 0)]
    for prec, variant in ((stp.FP32, stp.VARIANT_FUSED), (stp.BF16X3, stp.VARIANT_MFMA)):
        with pytest.raises(stp.StpError) as ei:
            stp.Plan(cls, prec=prec, variant=variant)
        assert ei.value.status == stp.E_UNSUPPORTED
    plan = stp.Plan([(3, 9, stp.ELASTIC_CURV, stp.PARAM_PER_ELEMENT)], prec=stp.FP32)
    z = torch.zeros(8 * 64 * 9 * 3, device="cuda")
    out = torch.zeros(8 * 64 * 9, device="cuda")
    st = stp.Step(2, 2, 2, 0.01, 0.5, z.data_ptr(), z.data_ptr(), None, None, z.data_ptr(), z.data_ptr(), None,
                  out.data_ptr())
    assert plan.correct_status(st) == stp.E_UNSUPPORTED and "curvilinear" in stp.last_error()
    plan.close()
    torch.cuda.synchronize()
