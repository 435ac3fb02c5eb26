"""GPU: elements placed beyond 2^31 values in every input and output buffer (64-bit per-element offsets in
stp_batch), for the MFMA, fused, plain and on-chip B_d kernels and the heterogeneous persistent launch. The outputs at
those offsets must equal, bit for bit, those of the same elements run from small contiguous buffers on the
same plan, and match the oracle. About 60 GB of device memory per case (FP32), most of it never touched."""
import sys

import numpy as np
import pytest

import oracle
from paper_2003_12787_amd import runner, stp
from paper_2003_12787_amd import workloads as W
from parity import TOL, max_rel_err

pytestmark = pytest.mark.gpu

BASE = 2 ** 31 + 4096  # values: the first element sits past the int32 range of every array


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def offsets(sizes, misalign):
    """Offsets from BASE with a gap of 4 values (plus 1 on every other element when misalign)."""
    off, cur = [], BASE
    for k, s in enumerate(sizes):
        off.append(cur + (1 if misalign and k % 2 else 0))
        cur = off[-1] + s + 4
    return np.array(off, dtype=np.int64), cur


def coef_block(p, j):
    """Element j's coefficient block in the library layout: preset parameters, or a generic class's B_d."""
    if p.params is not None:
        return p.params[j].ravel()
    return W.coef_abi(p.B[j:j + 1], p.coef_per_element)[0].ravel()


def run_far(plan, parts, torch, misalign, classes_of=None):
    """Run the elements of `parts` (uniform host batches, FP32-rounded; all presets, or all generic without A)
    placed at 64-bit offsets; returns the outputs per element as host arrays."""
    elems = [(c, p, j) for c, p in enumerate(parts) for j in range(p.nelem)]
    generic = parts[0].params is None
    assert all((p.params is None) == generic and p.A is None for p in parts)
    sq = [p.Q[0].size for c, p, j in elems]
    sf = [6 * (p.N + 1) ** 2 * p.m for c, p, j in elems]
    sp = [coef_block(p, j).size for c, p, j in elems]
    oq, endq = offsets(sq, misalign)
    of, endf = offsets(sf, misalign)
    oc, endc = offsets(sp, misalign)
    say(f"[large] {len(elems)} elements, Q/qavg {endq} values, favg {3 * endq}, qface {endf}, params {endc}")
    f32 = dict(device="cuda", dtype=torch.float32)
    Q, qavg, favg = torch.empty(endq, **f32), torch.empty(endq, **f32), torch.empty(3 * endq, **f32)
    qface, par = torch.empty(endf, **f32), torch.empty(endc, **f32)
    for k, (c, p, j) in enumerate(elems):
        Q[oq[k]:oq[k] + sq[k]] = torch.from_numpy(p.Q[j].ravel()).to(**f32)
        par[oc[k]:oc[k] + sp[k]] = torch.from_numpy(coef_block(p, j)).to(**f32)
    i64 = lambda a: torch.from_numpy(a).to("cuda", torch.int64)
    kw = dict(off_q=i64(oq), off_coef=i64(oc), off_face=i64(of))
    if len(parts) > 1:
        kw["cls"] = torch.from_numpy(np.array([c for c, p, j in elems], dtype=np.int32)).cuda()
    dt = torch.from_numpy(np.array([p.dt[j] for c, p, j in elems])).to("cuda", torch.float64)
    h = torch.from_numpy(np.array([p.h[j] for c, p, j in elems])).to("cuda", torch.float64)
    coef = {"B": par} if generic else {"params": par}
    plan.run(plan.batch(len(elems), Q, qavg, favg, qface, dt, h, **coef, **kw))
    torch.cuda.synchronize()
    out = []
    for k, (c, p, j) in enumerate(elems):
        out.append({"qavg": qavg[oq[k]:oq[k] + sq[k]].cpu().numpy(),
                    "favg": favg[3 * oq[k]:3 * oq[k] + 3 * sq[k]].cpu().numpy(),
                    "qface": qface[of[k]:of[k] + sf[k]].cpu().numpy()})
    del Q, qavg, favg, qface, par
    torch.cuda.empty_cache()
    return elems, out


def check(plan_args, parts, torch, misalign):
    parts = [runner.rounded(p, stp.FP32) for p in parts]
    plan = stp.Plan([runner.class_of(p) for p in parts], **plan_args)
    elems, far = run_far(plan, parts, torch, misalign)
    near = {}
    if len(parts) == 1:  # the same elements from contiguous buffers
        got = runner.run(plan, parts[0])
        for j in range(parts[0].nelem):
            near[(0, j)] = {k: v[j].ravel() for k, v in got.items()}
    for c, p in enumerate(parts):
        ref = oracle.stp(p.N, p.physics, p.Q, p.dt, p.h, params=p.params, B=p.B, coef_per_element=p.coef_per_element)
        ks = [k for k, (cc, pp, j) in enumerate(elems) if cc == c]
        g = {key: np.stack([far[k][key].astype(np.float64).reshape(ref[key][0].shape) for k in ks])
             for key in ("qavg", "favg", "qface")}
        err = max_rel_err(g, {key: ref[key] for key in g}, p.Q, p.h)
        say(f"[large]   class {c} N={p.N} phys={p.physics}: max rel err {err}")
        for key, v in err.items():
            assert v < TOL[plan_args["prec"]], (c, key, v)
        for k in ks:
            if (c, elems[k][2]) in near:
                for key in ("qavg", "favg", "qface"):
                    assert np.array_equal(far[k][key], near[(c, elems[k][2])][key]), (key, k)
    plan.close()


@pytest.mark.parametrize("misalign", [False, True])
def test_mfma_beyond_int32_offsets(gpu, misalign):
    check(dict(prec=stp.BF16X3, variant=stp.VARIANT_MFMA), [W.elastic_batch(7, 6, 870)], gpu, misalign)


@pytest.mark.parametrize("misalign", [False, True])
@pytest.mark.parametrize("physics", ["elastic", "acoustic"])
def test_fp32_mfma_beyond_int32_offsets(gpu, physics, misalign):
    part = W.elastic_batch(7, 6, 869) if physics == "elastic" else W.acoustic_batch(7, 6, 868)
    check(dict(prec=stp.FP32, variant=stp.VARIANT_MFMA), [part], gpu, misalign)


def test_fused_beyond_int32_offsets(gpu):
    check(dict(prec=stp.FP32, variant=stp.VARIANT_FUSED), [W.elastic_batch(3, 6, 871)], gpu, True)


def test_plain_beyond_int32_offsets(gpu):
    check(dict(prec=stp.FP32, variant=stp.VARIANT_PLAIN), [W.curvilinear_batch(4, 6, 872)], gpu, True)


def test_heterogeneous_beyond_int32_offsets(gpu):
    """Persistent bucket launches (acoustic, elastic) and an own launch (order 8) in one stp_run."""
    parts = [W.elastic_batch(3, 5, 873), W.acoustic_batch(5, 5, 874), W.elastic_batch(8, 3, 875)]
    check(dict(prec=stp.FP32), parts, gpu, True)


@pytest.mark.parametrize("N", [8, 9])
def test_mfma_orders_8_9_beyond_int32_offsets(gpu, N):
    """Order 8 blocks hold an odd number of values, so misaligned placements reach every copy-out alignment."""
    check(dict(prec=stp.BF16X3, variant=stp.VARIANT_MFMA), [W.elastic_batch(N, 5, 876 + N)], gpu, True)


@pytest.mark.parametrize("N,m", [(7, 9), (9, 4)])
def test_on_chip_B_beyond_int32_offsets(gpu, N, m):
    """The generic kernel that holds B_d on chip: B_d blocks, like every other array, past 2^31 values."""
    part = W.generic_batch(N, m, 5, 880 + N + m)
    plan = stp.Plan([runner.class_of(part)], prec=stp.FP32)
    assert plan.describe()["classes"][0]["on_chip_B"]
    plan.close()
    check(dict(prec=stp.FP32), [part], gpu, True)
