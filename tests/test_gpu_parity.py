"""GPU parity: the HIP predictor through the C ABI against the FP64 oracle on the same seeded inputs.

Reduced-precision runs feed the oracle the inputs rounded to FP32, so input quantisation is not counted as
kernel error. The metric is the per-element max-relative error of each output (see parity.py) with the
tolerances FP64 1e-12, FP32 1e-5 and split-BF16x3 1e-4. Full-size workloads are checked on a sample of
elements spread over the batch, in the same launch configuration the benchmark times.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2003_12787_amd import stp
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


def oracle_run(b, **kw):
    return oracle.stp(b.N, b.physics, b.Q, b.dt, b.h, params=b.params, A=b.A, B=b.B, src=b.src,
                      coef_per_element=b.coef_per_element, **kw)


def subset(b, ids):
    import copy
    s = copy.copy(b)
    for k in ("Q", "dt", "h", "params", "A", "B", "src"):
        v = getattr(b, k)
        if v is not None:
            setattr(s, k, v[ids])
    return s


def check(b, prec, variant=stp.VARIANT_AUTO, acc64=0, sample=None, favg_sum=False, label="", tol=None):
    from paper_2003_12787_amd import runner
    cls = runner.class_of(b, stp.FAVG_SUM if favg_sum else 0)
    plan = stp.Plan([cls], prec=prec, variant=variant, acc64_min_order=acc64)
    say(f"[parity] {label} N={b.N} m={b.m} phys={b.physics} E={b.nelem} prec={prec} variant={variant}")
    got = runner.run(plan, b, favg_sum=favg_sum)
    rb = runner.rounded(b, prec)
    ids = np.arange(b.nelem) if sample is None else sample
    rb = subset(rb, ids)
    got = {k: v[ids] for k, v in got.items()}
    ref = oracle_run(rb)
    if favg_sum:
        ref["favg"] = ref["favg"].sum(axis=1)
    err = max_rel_err(got, ref, rb.Q, rb.h)
    say(f"[parity]   max rel err {err}")
    for k, v in err.items():
        assert v < (tol or TOL[prec]), (k, v)
    plan.close()
    return err


def spread(E, k, seed=0):
    rng = np.random.default_rng(seed)
    ids = np.unique(np.concatenate([[0, E - 1], rng.choice(E, size=min(k, E), replace=False)]))
    return np.sort(ids)


# ------------------------------------------------------------------------------------------------ presets
def test_c1_elastic_n3_fp64():
    check(W.c1_elastic_n3(), stp.FP64, label="C1")


@pytest.mark.parametrize("acc64", [0, 1])
def test_c1_elastic_n3_fp32(acc64):
    check(W.c1_elastic_n3(), stp.FP32, acc64=acc64, label="C1")


@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_c2_acoustic_plane_wave_small(prec):
    check(W.c2_acoustic_n5(nelem=1000), prec, label="C2-small")


@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_c3_elastic_n7_small(prec):
    check(W.c3_elastic_n7(nelem=300), prec, label="C3-small")


@pytest.mark.parametrize("N", [1, 2, 4, 6, 8, 9])
@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_elastic_all_orders(N, prec):
    check(W.elastic_batch(N, 70, 500 + N), prec, acc64=8, label="elastic-orders")


@pytest.mark.parametrize("N", [1, 3, 9])
def test_acoustic_orders_per_node(N):
    check(W.acoustic_batch(N, 65, 600 + N), stp.FP32, label="acoustic-per-node")
    check(W.acoustic_batch(N, 65, 600 + N), stp.FP64, label="acoustic-per-node")


@pytest.mark.parametrize("phys,N,acc64", [("elastic", 8, 0), ("acoustic", 9, 0), ("elastic", 6, 6)])
def test_plain_register_bounded_instances(phys, N, acc64):
    """The plain instances compiled under a waves-per-SIMD bound (FP32 elastic N = 8, FP32 acoustic N = 9, FP32
    I/O with FP64 accumulation at elastic N = 6), with per-node and per-element material and favg summed."""
    gen = W.elastic_batch if phys == "elastic" else W.acoustic_batch
    check(gen(N, 45, 640 + N), stp.FP32, variant=stp.VARIANT_PLAIN, acc64=acc64, label=f"plain-bounded-{phys}")
    check(gen(N, 30, 650 + N, per_node=False), stp.FP32, variant=stp.VARIANT_PLAIN, acc64=acc64, favg_sum=True,
          label=f"plain-bounded-{phys}-fsum")


def test_elastic_per_element_material_and_favg_sum():
    b = W.elastic_batch(5, 130, 21, per_node=False)
    check(b, stp.FP32, label="elastic-per-element")
    check(b, stp.FP64, favg_sum=True, label="elastic-favg-sum")


def test_fp64_order7_register_bound_favg_sum():
    """The FP64 elastic order-7 kernel runs under a 128-register bound with favg stored one direction at a time:
    per-node material, separate and summed fluxes, an element count that is not a multiple of the grid."""
    b = W.elastic_batch(7, 45, 23)
    check(b, stp.FP64, label="fp64-n7")
    check(b, stp.FP64, favg_sum=True, label="fp64-n7-favg-sum")


def test_c3_full_size_sampled():
    b = W.c3_elastic_n7()
    check(b, stp.FP32, sample=spread(b.nelem, 40), label="C3-full")


def test_c2_full_size_sampled():
    b = W.c2_acoustic_n5()
    check(b, stp.FP32, sample=spread(b.nelem, 40, 1), label="C2-full")
    check(b, stp.FP64, sample=spread(b.nelem, 40, 2), label="C2-full")


# ------------------------------------------------------------------------------------------------ variants
@pytest.mark.parametrize("variant", [stp.VARIANT_PLAIN, stp.VARIANT_FUSED])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_fp32_variants_elastic(variant, N):
    check(W.elastic_batch(N, 37 + 13 * N, 900 + N), stp.FP32, variant=variant, label="elastic-variant")


@pytest.mark.parametrize("variant", [stp.VARIANT_PLAIN, stp.VARIANT_FUSED])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_fp32_variants_acoustic(variant, N):
    check(W.acoustic_batch(N, 41 + 11 * N, 950 + N), stp.FP32, variant=variant, label="acoustic-variant")


@pytest.mark.parametrize("variant", [stp.VARIANT_PLAIN, stp.VARIANT_FUSED])
def test_c3_full_size_variants(variant):
    b = W.c3_elastic_n7()
    check(b, stp.FP32, variant=variant, sample=spread(b.nelem, 24, 7), label="C3-full")


def test_fused_per_element_material_favg_sum_and_hetero_offsets():
    b = W.acoustic_plane_wave_batch(5, 300, 17)
    check(b, stp.FP32, variant=stp.VARIANT_FUSED, favg_sum=True, label="fused-favg-sum")


@pytest.mark.parametrize("variant", [stp.VARIANT_AUTO, stp.VARIANT_MFMA])
def test_bf16x3_mfma_elastic_n7(variant):
    check(W.c3_elastic_n7(nelem=300), stp.BF16X3, variant=variant, label="bf16x3-C3-small")


def test_bf16x3_mfma_acoustic_n7_and_favg_sum():
    check(W.acoustic_batch(7, 150, 971), stp.BF16X3, variant=stp.VARIANT_MFMA, label="bf16x3-acoustic")
    check(W.acoustic_batch(7, 150, 971), stp.BF16X3, variant=stp.VARIANT_MFMA, favg_sum=True,
          label="bf16x3-acoustic-favg-sum")


def test_bf16x3_mfma_smooth_plane_wave_error_bound():
    """Smooth fields: the derivative of a nearly constant line cancels entries of D whose absolute row sum
    reaches 129 at n = 8 while |D u| ~ k h |u|, so favg (a derivative of the smooth q-bar) is where a short
    split of the operands shows. The three-piece split keeps the contraction at about FP32 accuracy, and the
    split-BF16 tolerance holds here as on random data. The FP32 kernel is checked on the same data."""
    b = W.acoustic_plane_wave_batch(7, 125, 972)
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA, favg_sum=True, label="bf16x3-plane-wave")
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA, label="bf16x3-plane-wave-per-direction")
    check(b, stp.FP32, variant=stp.VARIANT_FUSED, favg_sum=True, label="fp32-plane-wave")


def test_bf16x3_mfma_smooth_elastic_plane_wave():
    """The benchmark's physics on smooth data: elastic N = 7 with per-node material, a P- plus S-wave and
    1e-2 noise; per-direction favg."""
    b = W.elastic_plane_wave_batch(7, 216, 974)
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA, label="bf16x3-elastic-plane-wave")
    check(b, stp.FP32, variant=stp.VARIANT_FUSED, label="fp32-elastic-plane-wave")


def test_bf16x3_mfma_per_element_material_and_dt_h():
    b = W.elastic_batch(7, 77, 973, per_node=False)
    rng = np.random.default_rng(9)
    b.h = rng.uniform(0.5, 2.0, b.nelem)
    b.dt = b.dt * b.h * rng.uniform(0.2, 1.0, b.nelem)
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA, label="bf16x3-per-element")


def test_bf16x3_full_size_sampled():
    b = W.c3_elastic_n7()
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA, sample=spread(b.nelem, 24, 11), label="bf16x3-C3-full")


# FP32 matrix-core kernel (order 7, Cartesian presets): FP32 products and accumulation, FP32 tolerance
def test_fp32_mfma_elastic_n7():
    check(W.c3_elastic_n7(nelem=300), stp.FP32, variant=stp.VARIANT_MFMA, label="fp32-mfma-C3-small")


def test_fp32_mfma_acoustic_n7_and_favg_sum():
    check(W.acoustic_batch(7, 150, 975), stp.FP32, variant=stp.VARIANT_MFMA, label="fp32-mfma-acoustic")
    check(W.acoustic_batch(7, 150, 975), stp.FP32, variant=stp.VARIANT_MFMA, favg_sum=True,
          label="fp32-mfma-acoustic-favg-sum")
    check(W.elastic_batch(7, 60, 976), stp.FP32, variant=stp.VARIANT_MFMA, favg_sum=True,
          label="fp32-mfma-elastic-favg-sum")


def test_fp32_mfma_smooth_plane_waves():
    """Smooth fields, where favg is a derivative of a nearly constant q-bar: per-direction and summed favg."""
    check(W.acoustic_plane_wave_batch(7, 125, 977), stp.FP32, variant=stp.VARIANT_MFMA, favg_sum=True,
          label="fp32-mfma-acoustic-plane-wave")
    check(W.elastic_plane_wave_batch(7, 216, 978), stp.FP32, variant=stp.VARIANT_MFMA,
          label="fp32-mfma-elastic-plane-wave")


def test_fp32_mfma_per_element_material_and_dt_h():
    b = W.elastic_batch(7, 77, 979, per_node=False)
    rng = np.random.default_rng(12)
    b.h = rng.uniform(0.5, 2.0, b.nelem)
    b.dt = b.dt * b.h * rng.uniform(0.2, 1.0, b.nelem)
    check(b, stp.FP32, variant=stp.VARIANT_MFMA, label="fp32-mfma-per-element")


def test_fp32_mfma_full_size_sampled():
    b = W.c3_elastic_n7()
    check(b, stp.FP32, variant=stp.VARIANT_MFMA, sample=spread(b.nelem, 24, 13), label="fp32-mfma-C3-full")


@pytest.mark.parametrize("N", [2, 5])
def test_bf16x3_plan_other_orders_use_fp32_kernels(N):
    check(W.elastic_batch(N, 40, 980 + N), stp.BF16X3, label="bf16x3-fallback")


# Orders 8 and 9: two chained 32x32x16 products per derivative, five nodes per lane, n = 9 with a stand-in pad
# node, and more lanes than lines (repeated lines in the last wave).
@pytest.mark.parametrize("variant", [stp.VARIANT_AUTO, stp.VARIANT_MFMA])
@pytest.mark.parametrize("N", [8, 9])
def test_bf16x3_mfma_elastic_orders_8_9(N, variant):
    check(W.elastic_batch(N, 45, 990 + N), stp.BF16X3, variant=variant, label="bf16x3-elastic-hi")


@pytest.mark.parametrize("N", [8, 9])
def test_bf16x3_mfma_acoustic_orders_8_9_and_favg_sum(N):
    b = W.acoustic_batch(N, 60, 992 + N)
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA, label="bf16x3-acoustic-hi")
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA, favg_sum=True, label="bf16x3-acoustic-hi-favg-sum")


@pytest.mark.parametrize("N", [8, 9])
def test_bf16x3_mfma_smooth_plane_waves_orders_8_9(N):
    """Smooth fields at the orders where D's rows are largest (absolute row sums grow with n)."""
    check(W.elastic_plane_wave_batch(N, 64, 994 + N), stp.BF16X3, variant=stp.VARIANT_MFMA,
          label="bf16x3-elastic-plane-wave-hi")
    check(W.acoustic_plane_wave_batch(N, 64, 996 + N), stp.BF16X3, variant=stp.VARIANT_MFMA, favg_sum=True,
          label="bf16x3-acoustic-plane-wave-hi")


@pytest.mark.parametrize("N", [8, 9])
def test_bf16x3_mfma_orders_8_9_per_element_material_and_dt_h(N):
    b = W.elastic_batch(N, 33, 998 + N, per_node=False)
    rng = np.random.default_rng(N)
    b.h = rng.uniform(0.5, 2.0, b.nelem)
    b.dt = b.dt * b.h * rng.uniform(0.2, 1.0, b.nelem)
    check(b, stp.BF16X3, variant=stp.VARIANT_MFMA, label="bf16x3-per-element-hi")


def test_bf16x3_heterogeneous_with_orders_8_9():
    """A split-BF16x3 heterogeneous plan: orders 8 and 9 take their own MFMA launches over element lists (on
    the side streams), beside the persistent launch of the low orders."""
    parts = [W.elastic_batch(9, 14, 1001), W.acoustic_batch(8, 20, 1002), W.elastic_batch(3, 40, 1003),
             W.elastic_batch(8, 11, 1004, per_node=False), W.acoustic_batch(9, 17, 1005),
             W.acoustic_batch(4, 30, 1006)]
    from paper_2003_12787_amd import runner
    mb = W.interleave(parts, [runner.class_of(p) for p in parts], 1007)
    plan = stp.Plan(mb.classes, prec=stp.BF16X3)
    got = run_mixed(plan, mb, stp.BF16X3)
    say(f"[parity]   worst {check_mixed(mb, stp.BF16X3, got)}")
    plan.close()


def test_unsupported_variant_is_reported():
    with pytest.raises(stp.StpError) as ei:
        stp.Plan([(8, 9, stp.ELASTIC, 0)], prec=stp.FP32, variant=stp.VARIANT_FUSED)
    assert ei.value.status == stp.E_UNSUPPORTED
    with pytest.raises(stp.StpError) as ei:
        stp.Plan([(6, 9, stp.ELASTIC, 0)], prec=stp.BF16X3, variant=stp.VARIANT_MFMA)
    assert ei.value.status == stp.E_UNSUPPORTED


# ------------------------------------------------------------------------------------------------ generic
@pytest.mark.parametrize("N,m", [(1, 1), (2, 5), (3, 9), (4, 16), (8, 9), (9, 4), (9, 16)])
@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_generic_dense_B_per_node(N, m, prec):
    check(W.generic_batch(N, m, 67, 700 + N * 20 + m), prec, label="generic")


@pytest.mark.parametrize("N,m", [(7, 9), (8, 9), (9, 9), (4, 4), (5, 4), (6, 4), (7, 4), (8, 4), (9, 4)])
def test_generic_on_chip_B(N, m):
    """Generic classes with dense per-node B_d and no other terms take the kernel that holds B_d on chip
    (registers and LDS, the rest streamed): FP32 parity at every order and m it covers, odd element counts."""
    from paper_2003_12787_amd import runner
    b = W.generic_batch(N, m, 37, 760 + N * 20 + m)
    plan = stp.Plan([runner.class_of(b)], prec=stp.FP32)
    assert plan.describe()["classes"][0]["on_chip_B"]
    plan.close()
    check(b, stp.FP32, label="generic-on-chip-B")


def test_generic_on_chip_B_favg_sum_and_routing():
    """The summed-flux output of the on-chip B_d kernel; classes with A, a point source, per-element coefficients,
    FP64 accumulation or FP64 I/O, m = 9 below order 7, m = 4 below order 4 and other m keep the plain kernel."""
    from paper_2003_12787_amd import runner
    check(W.generic_batch(7, 9, 23, 777), stp.FP32, favg_sum=True, label="generic-on-chip-B-favg-sum")
    for cls, prec, acc64 in [((7, 9, W.GENERIC, stp.A_PRESENT), stp.FP32, 0),
                             ((7, 9, W.GENERIC, stp.SRC_POINT), stp.FP32, 0),
                             ((7, 9, W.GENERIC, stp.COEF_PER_ELEMENT), stp.FP32, 0),
                             ((8, 9, W.GENERIC, 0), stp.FP32, 8),
                             ((7, 9, W.GENERIC, 0), stp.FP64, 0),
                             ((6, 9, W.GENERIC, 0), stp.FP32, 0),
                             ((3, 4, W.GENERIC, 0), stp.FP32, 0),
                             ((8, 5, W.GENERIC, 0), stp.FP32, 0)]:
        plan = stp.Plan([cls], prec=prec, acc64_min_order=acc64)
        assert not plan.describe()["classes"][0]["on_chip_B"], cls
        plan.close()
    plan = stp.Plan([(7, 9, W.GENERIC, 0)], prec=stp.BF16X3)
    assert plan.describe()["classes"][0]["on_chip_B"]
    plan.close()


@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_generic_high_orders_with_A_source_and_per_element(prec):
    """Orders 8 and 9 form B_d (D x_d u) column by column: with A_d and a point source (per node), and with
    per-element coefficients (B_d from LDS)."""
    b = W.generic_batch(9, 7, 40, 805, with_A=True)
    b.src = W.point_source(b, 806)
    check(b, prec, label="generic-N9-A-src")
    check(W.generic_batch(8, 9, 40, 807, with_A=True, per_node=False), prec, label="generic-N8-per-element")


def test_generic_high_orders_fp64_accumulation():
    """FP32 I/O with FP64 accumulation (the serving configuration at N >= 8) through the column form."""
    check(W.generic_batch(9, 9, 40, 808), stp.FP32, acc64=8, label="generic-N9-acc64")
    check(W.generic_batch(8, 12, 30, 809, with_A=True), stp.FP32, acc64=8, label="generic-N8-m12-A-acc64")


@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_generic_with_A_and_point_source(prec):
    b = W.generic_batch(3, 6, 66, 801, with_A=True)
    b.src = W.point_source(b, 802)
    check(b, prec, label="generic-A-src")


@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_generic_per_element_coefficients(prec):
    b = W.generic_batch(5, 9, 65, 803, with_A=True, per_node=False)
    check(b, prec, label="generic-per-element")


def test_per_element_dt_and_h():
    b = W.elastic_batch(4, 90, 804)
    rng = np.random.default_rng(5)
    b.h = rng.uniform(0.5, 2.0, b.nelem)
    b.dt = b.dt * b.h * rng.uniform(0.2, 1.0, b.nelem)
    check(b, stp.FP64, label="per-element-dt-h")
    check(b, stp.FP32, label="per-element-dt-h")


def test_dt_zero_returns_Q():
    from paper_2003_12787_amd import runner
    b = W.elastic_batch(3, 10, 805)
    b.dt = np.zeros(b.nelem)
    plan = stp.Plan([runner.class_of(b)], prec=stp.FP64)
    got = runner.run(plan, b)
    assert np.array_equal(got["qavg"], b.Q)


# ------------------------------------------------------------------------------------------------ hetero
def _hetero(hb, prec, sample_per_class=None, label="hetero"):
    import torch
    dt = torch.float64 if prec == stp.FP64 else torch.float32
    dev = "cuda"
    plan = stp.Plan(hb.classes, prec=prec)
    say(f"[parity] {label} classes={len(hb.classes)} E={len(hb.cls)} prec={prec}")
    Q = torch.from_numpy(hb.Q).to(dev, dt)
    B = torch.from_numpy(hb.coef).to(dev, dt)
    qavg = torch.zeros(hb.size_q, device=dev, dtype=dt)
    favg = torch.zeros(3 * hb.size_q, device=dev, dtype=dt)
    qface = torch.zeros(hb.size_face, device=dev, dtype=dt)
    to = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to(dev, t)
    cls, oq, oc, of = to(hb.cls, torch.int32), to(hb.off_q, torch.int64), to(hb.off_coef, torch.int64), to(hb.off_face, torch.int64)
    dts, hs = to(hb.dt, torch.float64), to(hb.h, torch.float64)
    batch = plan.batch(len(hb.cls), Q, qavg, favg, qface, dts, hs, B=B, cls=cls, off_q=oq, off_coef=oc, off_face=of)
    plan.run(batch)
    torch.cuda.synchronize()
    qa, fa, qf = qavg.double().cpu().numpy(), favg.double().cpu().numpy(), qface.double().cpu().numpy()
    worst = 0.0
    for c, (N, m, _, _) in enumerate(hb.classes):
        ids = hb.members[c]
        pick = np.arange(len(ids)) if sample_per_class is None else spread(len(ids), sample_per_class, c)[:sample_per_class]
        part = subset(hb.parts[c], pick)
        if prec != stp.FP64:
            part.Q = part.Q.astype(np.float32).astype(np.float64)
            part.B = part.B.astype(np.float32).astype(np.float64)
        ref = oracle_run(part)
        n3, n2 = (N + 1) ** 3, (N + 1) ** 2
        got = {"qavg": [], "favg": [], "qface": []}
        for j in pick:
            e = ids[j]
            got["qavg"].append(qa[hb.off_q[e]:hb.off_q[e] + n3 * m].reshape(n3, m))
            got["favg"].append(fa[3 * hb.off_q[e]:3 * hb.off_q[e] + 3 * n3 * m].reshape(3, n3, m))
            got["qface"].append(qf[hb.off_face[e]:hb.off_face[e] + 6 * n2 * m].reshape(6, n2, m))
        got = {k: np.stack(v) for k, v in got.items()}
        err = max_rel_err(got, ref, part.Q, part.h)
        worst = max(worst, max(err.values()))
        for k, v in err.items():
            assert v < TOL[prec], (N, m, k, v)
    say(f"[parity]   worst max rel err {worst}")
    plan.close()


@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_heterogeneous_small(prec):
    _hetero(W.hetero_generic_batch(600, 901, orders=[1, 2, 3, 5], nquants=[1, 4, 9]), prec)


def test_c4_heterogeneous_full_size_sampled():
    _hetero(W.hetero_generic_batch(16384, W.SEED0 + 3), stp.FP32, sample_per_class=6, label="C4-full")


def mixed_batch(E_scale=1, seed=905):
    """Every physics bucket of the persistent launch, classes with their own launch (high orders, run-time m, and
    generic m = 4 with B_d on chip) in one batch."""
    G = W.GENERIC
    parts = [
        W.elastic_batch(3, 40 * E_scale, seed + 1),
        W.elastic_batch(7, 12 * E_scale, seed + 2, per_node=False),
        W.acoustic_batch(5, 30 * E_scale, seed + 3),
        W.acoustic_batch(1, 70 * E_scale, seed + 4, per_node=False),
        W.generic_batch(2, 9, 25 * E_scale, seed + 5, with_A=True),
        W.generic_batch(4, 3, 20 * E_scale, seed + 6, per_node=False),
        W.generic_batch(3, 12, 15 * E_scale, seed + 7),
        W.generic_batch(8, 4, 6 * E_scale, seed + 8),
        W.generic_batch(6, 4, 10 * E_scale, seed + 9),
        W.generic_batch(3, 4, 12 * E_scale, seed + 11),
    ]
    parts[5].src = W.point_source(parts[5], seed + 10)
    from paper_2003_12787_amd import runner
    classes = [runner.class_of(p) for p in parts]
    return W.interleave(parts, classes, seed)


def run_mixed(plan, mb, prec, graph_replays=0):
    """Run a MixedBatch through one heterogeneous plan; returns host outputs (and, with graph_replays,
    checks that replays of a captured graph reproduce the eager result bit for bit)."""
    import torch
    dt = torch.float64 if prec == stp.FP64 else torch.float32
    to = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
    ins = dict(Q=to(mb.Q, dt), params=to(mb.params, dt), B=to(mb.B, dt), A=to(mb.A, dt), src=to(mb.src, dt))
    outs = dict(qavg=torch.zeros(mb.size_q, device="cuda", dtype=dt),
                favg=torch.zeros(3 * mb.size_q, device="cuda", dtype=dt),
                qface=torch.zeros(mb.size_face, device="cuda", dtype=dt),
                fface=torch.zeros(mb.size_face, device="cuda", dtype=dt))
    idx = dict(cls=to(mb.cls, torch.int32), off_q=to(mb.off_q, torch.int64), off_coef=to(mb.off_coef, torch.int64),
               off_face=to(mb.off_face, torch.int64), off_src=to(mb.off_src, torch.int64))
    dts, hs = to(mb.dt, torch.float64), to(mb.h, torch.float64)
    batch = plan.batch(len(mb.cls), ins["Q"], outs["qavg"], outs["favg"], outs["qface"], dts, hs,
                       params=ins["params"], A=ins["A"], B=ins["B"], src=ins["src"], fface=outs["fface"], **idx)
    plan.run(batch)
    torch.cuda.synchronize()
    host = {k: v.double().cpu().numpy() for k, v in outs.items()}
    if graph_replays:
        plan.reserve(len(mb.cls))
        g = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        with torch.cuda.graph(g, stream=cap):
            plan.run(batch)
        other = torch.randn(1 << 20, device="cuda")
        for r in range(graph_replays):
            for k, v in outs.items():
                v.fill_(0.0 if k == "fface" else float("nan"))  # fface is written only for classes with A
            _ = (other * 2).sum().item()  # eager work and a synchronisation between replays
            g.replay()
            torch.cuda.synchronize()
            for k, v in outs.items():
                assert np.array_equal(v.double().cpu().numpy(), host[k]), (r, k)
            say(f"[parity]   graph replay {r} bitwise equal")
        del g
    return host


def check_mixed(mb, prec, got, sample_per_class=None):
    worst = 0.0
    for c, (N, m, phys, flags) in enumerate(mb.classes):
        ids = mb.members[c]
        if len(ids) == 0:
            continue
        pick = np.arange(len(ids)) if sample_per_class is None else spread(len(ids), sample_per_class, c)[:sample_per_class]
        from paper_2003_12787_amd import runner
        part = subset(runner.rounded(mb.parts[c], prec), pick)
        ref = oracle_run(part)
        n3, n2 = (N + 1) ** 3, (N + 1) ** 2
        res = {"qavg": [], "favg": [], "qface": []}
        hasA = bool(flags & stp.A_PRESENT)
        if hasA:
            res["fface"] = []
        for j in pick:
            e = ids[j]
            oq, of = mb.off_q[e], mb.off_face[e]
            res["qavg"].append(got["qavg"][oq:oq + n3 * m].reshape(n3, m))
            res["favg"].append(got["favg"][3 * oq:3 * oq + 3 * n3 * m].reshape(3, n3, m))
            res["qface"].append(got["qface"][of:of + 6 * n2 * m].reshape(6, n2, m))
            if hasA:
                res["fface"].append(got["fface"][of:of + 6 * n2 * m].reshape(6, n2, m))
        res = {k: np.stack(v) for k, v in res.items()}
        if not hasA:
            ref.pop("fface", None)
        err = max_rel_err(res, ref, part.Q, part.h)
        say(f"[parity]   class {c} N={N} m={m} phys={phys} flags={flags} E={len(ids)} err={max(err.values()):.2e}")
        worst = max(worst, max(err.values()))
        for k, v in err.items():
            assert v < TOL[prec], (c, N, m, k, v)
    return worst


@pytest.mark.parametrize("prec,acc64", [(stp.FP64, 0), (stp.FP32, 0), (stp.FP32, 6)])
def test_heterogeneous_mixed_physics(prec, acc64):
    mb = mixed_batch()
    say(f"[parity] mixed physics classes={len(mb.classes)} E={len(mb.cls)} prec={prec} acc64={acc64}")
    plan = stp.Plan(mb.classes, prec=prec, acc64_min_order=acc64)
    got = run_mixed(plan, mb, prec)
    say(f"[parity]   worst {check_mixed(mb, prec, got)}")
    plan.close()


def test_heterogeneous_graph_capture_replays():
    mb = mixed_batch(E_scale=4, seed=906)
    say(f"[graph] mixed physics E={len(mb.cls)} captured after stp_reserve")
    plan = stp.Plan(mb.classes, prec=stp.FP32)
    got = run_mixed(plan, mb, stp.FP32, graph_replays=3)
    check_mixed(mb, stp.FP32, got, sample_per_class=8)
    plan.close()


def test_heterogeneous_graph_capture_replays_with_side_streams():
    """A batch large enough (>= 8192 elements) that the own-launch classes fork onto side streams: the
    captured fork/join replays bit for bit and matches the oracle on a sample."""
    mb = mixed_batch(E_scale=40, seed=908)
    assert len(mb.cls) >= 8192
    say(f"[graph] mixed physics E={len(mb.cls)} (side streams) captured after stp_reserve")
    plan = stp.Plan(mb.classes, prec=stp.FP32)
    got = run_mixed(plan, mb, stp.FP32, graph_replays=3)
    check_mixed(mb, stp.FP32, got, sample_per_class=6)
    plan.close()


def test_uniform_graph_capture_replays():
    import torch
    from paper_2003_12787_amd import runner
    for b, prec, variant in ((W.c3_elastic_n7(2048), stp.FP32, stp.VARIANT_FUSED),
                             (W.c3_elastic_n7(2048), stp.FP32, stp.VARIANT_MFMA),
                             (W.c3_elastic_n7(2048), stp.BF16X3, stp.VARIANT_MFMA),
                             (W.elastic_batch(9, 300, 1010), stp.BF16X3, stp.VARIANT_MFMA)):
        say(f"[graph] N={b.N} E={b.nelem} prec={prec} variant={variant}")
        plan = stp.Plan([runner.class_of(b)], prec=prec, variant=variant)
        db = runner.DeviceBatch(plan, b)
        plan.run(db.cbatch)
        torch.cuda.synchronize()
        ref = db.outputs()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=torch.cuda.Stream()):
            plan.run(db.cbatch)
        for r in range(3):
            db.clear_outputs(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            out = db.outputs()
            for k in ref:
                assert np.array_equal(out[k], ref[k]), (prec, r, k)
        del g
        plan.close()


def test_serving_heterogeneous_batches_match_run():
    """Mixed-physics batches through the serving lanes (each with its own scratch) equal stp_run's output, and
    the served outputs match the oracle."""
    import torch
    mb = mixed_batch(seed=907)
    plan = stp.Plan(mb.classes, prec=stp.FP32, serve_mem_budget=256 << 20)
    ref = run_mixed(plan, mb, stp.FP32)
    to = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
    ins = dict(Q=to(mb.Q, torch.float32), params=to(mb.params, torch.float32), B=to(mb.B, torch.float32),
               A=to(mb.A, torch.float32), src=to(mb.src, torch.float32))
    idx = dict(cls=to(mb.cls, torch.int32), off_q=to(mb.off_q, torch.int64), off_coef=to(mb.off_coef, torch.int64),
               off_face=to(mb.off_face, torch.int64), off_src=to(mb.off_src, torch.int64))
    dts, hs = to(mb.dt, torch.float64), to(mb.h, torch.float64)
    outs, tickets = [], []
    say(f"[serve] mixed physics E={len(mb.cls)} x 8 submissions")
    for _ in range(8):
        o = dict(qavg=torch.zeros(mb.size_q, device="cuda"), favg=torch.zeros(3 * mb.size_q, device="cuda"),
                 qface=torch.zeros(mb.size_face, device="cuda"), fface=torch.zeros(mb.size_face, device="cuda"))
        b = plan.batch(len(mb.cls), ins["Q"], o["qavg"], o["favg"], o["qface"], dts, hs, params=ins["params"],
                       A=ins["A"], B=ins["B"], src=ins["src"], fface=o["fface"], **idx)
        outs.append((o, b))
    torch.cuda.synchronize()  # the serving streams do not wait for the caller's streams (the zero fills)
    for _, b in outs:
        tickets.append(plan.submit(b))
    plan.drain()
    for t in tickets:
        st, _ = plan.poll(t)
        assert st == stp.OK
    for o, _ in outs:
        for k, v in o.items():
            assert np.array_equal(v.double().cpu().numpy(), ref[k]), k
    say(f"[serve]   served outputs vs oracle: worst {check_mixed(mb, stp.FP32, {k: v.double().cpu().numpy() for k, v in outs[0][0].items()}):.2e}")
    plan.close()


# ------------------------------------------------------------------------------------------------ autotuner
def test_autotune_single_class_variant_is_cached_and_correct(tmp_path, monkeypatch):
    import json
    from paper_2003_12787_amd import runner
    monkeypatch.setenv("STP_TUNE_CACHE", str(tmp_path / "tune.json"))
    b = W.c3_elastic_n7(512)
    cls = runner.class_of(b)
    say("[tune] elastic N=7 BF16X3, autotune=1")
    plan = stp.Plan([cls], prec=stp.BF16X3, autotune=1)
    d = plan.describe()
    say(f"[tune]   chose {d['classes'][0]['variant']}")
    assert d["classes"][0]["variant"] in ("plain", "fused", "mfma")
    cache = json.load(open(tmp_path / "tune.json"))
    entry = [v for k, v in cache.items() if "|class|N7,m9,p1" in k]
    assert len(entry) == 1 and entry[0]["us_per_elem"] > 0
    got = runner.run(plan, b)
    ref = oracle_run(runner.rounded(b, stp.BF16X3))
    err = max_rel_err(got, ref, runner.rounded(b, stp.BF16X3).Q, b.h)
    assert max(err.values()) < TOL[stp.BF16X3], err
    plan.close()
    again = stp.Plan([cls], prec=stp.BF16X3, autotune=0)  # from the cache
    assert again.describe()["classes"][0]["variant"] == d["classes"][0]["variant"]
    again.close()


def test_autotune_heterogeneous_grid_and_tiles(tmp_path, monkeypatch):
    import json
    monkeypatch.setenv("STP_TUNE_CACHE", str(tmp_path / "tune.json"))
    mb = mixed_batch()
    say(f"[tune] mixed physics classes={len(mb.classes)} autotune=1")
    plan = stp.Plan(mb.classes, prec=stp.FP32, autotune=1)
    d = plan.describe()
    say(f"[tune]   grid/CU {d['hetero_grid_per_cu']} LDS budget {d['hetero_lds_budget']}")
    assert d["hetero_grid_per_cu"] in (2, 4, 8)
    assert d["hetero_lds_budget"] in (48 * 1024, 80 * 1024, 128 * 1024)
    for c, (N, m, phys, flags) in zip(d["classes"], mb.classes):
        # tiled: order <= 7, preset physics or a generic class with m = 4 or 9, unless B_d is kept on chip
        assert c["tiled"] == (N <= 7 and (phys != stp.GENERIC or m in (4, 9)) and not c["on_chip_B"]), c
        assert c["on_chip_B"] == (phys == stp.GENERIC and not flags and ((m == 4 and N >= 4) or (m == 9 and N >= 7)))
        if c["tiled"]:
            assert 1 <= c["elements_per_tile"] <= 512 // (N + 1) ** 3
    cache = json.load(open(tmp_path / "tune.json"))
    assert any("|hetero|" in k for k in cache)
    got = run_mixed(plan, mb, stp.FP32)
    check_mixed(mb, stp.FP32, got)
    plan.close()
    again = stp.Plan(mb.classes, prec=stp.FP32, autotune=0)
    d2 = again.describe()
    assert (d2["hetero_grid_per_cu"], d2["hetero_lds_budget"]) == (d["hetero_grid_per_cu"], d["hetero_lds_budget"])
    again.close()


# ------------------------------------------------------------------------------------------------ edges
def test_empty_batch_is_noop():
    from paper_2003_12787_amd import runner
    b = W.elastic_batch(3, 0, 1)
    plan = stp.Plan([runner.class_of(b)], prec=stp.FP32)
    db = runner.DeviceBatch(plan, b)
    assert plan.run_status(db.cbatch) == stp.OK


def test_deterministic_bitwise():
    from paper_2003_12787_amd import runner
    b = W.elastic_batch(7, 200, 31)
    for prec in (stp.FP32, stp.FP64):
        plan = stp.Plan([runner.class_of(b)], prec=prec)
        o1 = runner.run(plan, b)
        o2 = runner.run(plan, b)
        for k in o1:
            assert np.array_equal(o1[k], o2[k]), k


def test_host_validation_errors():
    import torch
    from paper_2003_12787_amd import runner
    b = W.elastic_batch(3, 8, 32)
    plan = stp.Plan([runner.class_of(b)], prec=stp.FP32)
    db = runner.DeviceBatch(plan, b)
    bad = plan.batch(8, db.Q, db.Q, db.favg, db.qface, db.dt, db.h, params=db.params)  # qavg aliases Q
    assert plan.run_status(bad) == stp.E_INVAL and "alias" in stp.last_error()
    bad = plan.batch(8, None, db.qavg, db.favg, db.qface, db.dt, db.h, params=db.params)
    assert plan.run_status(bad) == stp.E_INVAL
    bad = plan.batch(8, db.Q, db.qavg, db.favg, db.qface, db.dt, -1.0, params=db.params)
    assert plan.run_status(bad) == stp.E_INVAL
    bad = plan.batch(8, db.Q, db.qavg, db.favg, db.qface, -0.1, 1.0, params=db.params)
    assert plan.run_status(bad) == stp.E_INVAL
    bad = plan.batch(8, db.Q, db.qavg, db.favg, db.qface, db.dt, db.h, params=None)
    assert plan.run_status(bad) == stp.E_INVAL
    torch.cuda.synchronize()


# ------------------------------------------------------------------------------------------------ serving
def test_serving_submit_poll_matches_run():
    import time
    import torch
    from paper_2003_12787_amd import runner
    b = W.elastic_batch(4, 40, 33)
    cls = runner.class_of(b)
    plan = stp.Plan([cls], prec=stp.FP32, serve_mem_budget=64 << 20)
    ref = runner.run(plan, b)
    dbs = [runner.DeviceBatch(plan, b) for _ in range(5)]
    tickets = [plan.submit(db.cbatch) for db in dbs]
    plan.drain()
    for t in tickets:
        st, info = plan.poll(t)
        assert st == stp.OK and info.t_done >= info.t_start >= info.t_submit
        st, _ = plan.poll(t)
        assert st == stp.E_INVAL  # retired
    for db in dbs:
        out = db.outputs()
        for k in ref:
            assert np.array_equal(out[k], ref[k])
    # a batch larger than the whole budget is refused
    small = stp.Plan([cls], prec=stp.FP32, serve_mem_budget=1024)
    with pytest.raises(stp.StpError) as ei:
        small.submit(runner.DeviceBatch(small, b).cbatch)
    assert ei.value.status == stp.E_NOMEM
    st, _ = plan.poll(123456789)
    assert st == stp.E_INVAL
    torch.cuda.synchronize()
    del time
