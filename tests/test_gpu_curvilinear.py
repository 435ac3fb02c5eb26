"""GPU parity of curvilinear elastic elements (STP_ELASTIC_CURV: material and metric terms per node) against
the oracle, through the C ABI: every precision of the plain kernel, the split-BF16x3 MFMA kernel at N = 7,
per-node (curved) and per-element (affine) parameters, a heterogeneous batch mixing curvilinear and
Cartesian classes, and the unsupported combinations."""
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
    chosen = plan.describe()["classes"][0]["variant"]
    say(f"[curvilinear] N={b.N} E={b.nelem} per_element={b.coef_per_element} prec={prec} "
        f"acc64_min_order={acc64_min_order} -> {chosen}")
    if prec == stp.BF16X3 and b.N == 7 and variant == stp.VARIANT_AUTO:
        assert chosen == "mfma", chosen
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


def test_curvilinear_fp32_acc64():
    check(W.curvilinear_batch(9, 24, 821), stp.FP32, acc64_min_order=8)


@pytest.mark.parametrize("per_node", [True, False])
def test_curvilinear_mfma(per_node):
    """Split-BF16x3 MFMA kernel (all 9 quantities differentiated per direction, metric rows re-read per
    direction) against the oracle on the FP32-rounded inputs."""
    b = W.curvilinear_batch(7, 40, 823 + per_node, per_node=per_node)
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA)
    check(b, stp.BF16X3)  # the automatic choice at N = 7 is the MFMA kernel


def test_curvilinear_bf16x3_other_orders_take_plain():
    check(W.curvilinear_batch(5, 24, 825), stp.BF16X3)


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
    for prec, variant in ((stp.FP32, stp.VARIANT_FUSED), (stp.FP32, stp.VARIANT_MFMA)):
        with pytest.raises(stp.StpError) as ei:
            stp.Plan(cls, prec=prec, variant=variant)
        assert ei.value.status == stp.E_UNSUPPORTED
    # the corrector rejects point sources for curvilinear classes as for the others
    plan = stp.Plan([(3, 9, stp.ELASTIC_CURV, stp.SRC_POINT)], prec=stp.FP32)
    z = torch.zeros(8 * 64 * 12 * 3, device="cuda")
    out = torch.zeros(8 * 64 * 9, device="cuda")
    st = stp.Step(2, 2, 2, 0.01, 0.5, z.data_ptr(), z.data_ptr(), None, None, z.data_ptr(), z.data_ptr(), None,
                  out.data_ptr())
    assert plan.correct_status(st) == stp.E_UNSUPPORTED and "point source" in stp.last_error()
    plan.close()
    torch.cuda.synchronize()


def test_curvilinear_mfma_full_size_sampled(gpu):
    """65536 curvilinear N = 7 elements generated on the device (the bench's workload and launch), 24 of them
    checked against the oracle on the same FP32 inputs."""
    torch = gpu
    N, E, n3, n2 = 7, 65536, 512, 64
    Q, par, dt = W.curvilinear_device(N, E, W.SEED0 + 7)
    plan = stp.Plan([(N, 9, stp.ELASTIC_CURV, 0)], prec=stp.BF16X3, variant=stp.VARIANT_MFMA)
    qavg = torch.empty((E, n3, 9), device="cuda")
    favg = torch.empty((E, 3, n3, 9), device="cuda")
    qface = torch.empty((E, 6, n2, 9), device="cuda")
    say(f"[curvilinear] full size E={E} MFMA")
    plan.run(plan.batch(E, Q, qavg, favg, qface, dt, 1.0, params=par))
    torch.cuda.synchronize()
    ids = torch.from_numpy(np.linspace(0, E - 1, 24).astype(np.int64)).cuda()
    pick = lambda t: t.index_select(0, ids).double().cpu().numpy()
    ref = oracle.stp(N, W.ELASTIC_CURV, pick(Q), dt, 1.0, params=pick(par))
    got = {"qavg": pick(qavg), "favg": pick(favg), "qface": pick(qface)}
    err = max_rel_err(got, ref, pick(Q), np.ones(24))
    say(f"[curvilinear]   max rel err {err}")
    for k, v in err.items():
        assert v < TOL[stp.BF16X3], (k, v)
    plan.close()
    del Q, par, qavg, favg, qface
    torch.cuda.empty_cache()
