"""Batch-level behaviour of the HIP predictor through the C ABI, against the FP64 oracle:

* heterogeneous batches above 65536 elements, which bucket their elements with a counting kernel and global
  atomics instead of the single-workgroup pass (sampled per class against the oracle, and bit for bit equal
  to the same elements run as two smaller batches);
* class ids outside the plan: skipped on the device, reported by stp_sync (stp_run, stp_run_noalloc) and by
  the ticket's status (serving), with the other elements unchanged;
* the serving path in the serving configuration (preset classes N = 2..9, m = 4 and 9, FP32 with FP64
  accumulation at N >= 8, per-element dt and h): every element of every ticket against the oracle.
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


def large_mixed(seed=941):
    """About 71 000 low-order elements in four classes: three tiled in the persistent launches (elastic N = 2,
    acoustic N = 3, generic m = 4 N = 1) and one with its own launch (generic m = 3, N = 2)."""
    from paper_2003_12787_amd import runner
    parts = [
        W.elastic_batch(2, 30000, seed + 1),
        W.acoustic_batch(3, 25000, seed + 2),
        W.generic_batch(1, 4, 6000, seed + 3),
        W.generic_batch(2, 3, 10000, seed + 4),
    ]
    return W.interleave(parts, [runner.class_of(p) for p in parts], seed)


class Dev:
    """Device copies of a MixedBatch (FP32 I/O) and NaN-filled outputs."""

    def __init__(self, mb):
        import torch
        to = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
        f = torch.float32
        self.mb = mb
        self.ins = dict(Q=to(mb.Q, f), params=to(mb.params, f), B=to(mb.B, f), A=to(mb.A, f), src=to(mb.src, f))
        self.idx = dict(cls=to(mb.cls, torch.int32), off_q=to(mb.off_q, torch.int64),
                        off_coef=to(mb.off_coef, torch.int64), off_face=to(mb.off_face, torch.int64),
                        off_src=to(mb.off_src, torch.int64))
        self.dt, self.h = to(mb.dt, torch.float64), to(mb.h, torch.float64)
        self.new_outputs()

    def new_outputs(self):
        import torch
        mb = self.mb
        self.outs = dict(qavg=torch.full((mb.size_q,), float("nan"), device="cuda"),
                         favg=torch.full((3 * mb.size_q,), float("nan"), device="cuda"),
                         qface=torch.full((mb.size_face,), float("nan"), device="cuda"),
                         fface=torch.full((mb.size_face,), float("nan"), device="cuda"))
        return self.outs

    def batch(self, plan, ids=None):
        """A stp_batch over the elements `ids` (all when None), reading and writing the full buffers."""
        i, o = self.ins, self.outs
        idx = self.idx if ids is None else {k: v[ids] for k, v in self.idx.items()}
        dt, h = (self.dt, self.h) if ids is None else (self.dt[ids], self.h[ids])
        b = plan.batch(int(idx["cls"].numel()), i["Q"], o["qavg"], o["favg"], o["qface"], dt, h,
                       params=i["params"], A=i["A"], B=i["B"], src=i["src"], fface=o["fface"], **idx)
        b._hold = (idx, dt, h)
        return b

    def host(self):
        return {k: v.double().cpu().numpy() for k, v in self.outs.items()}


def test_heterogeneous_over_65536_elements():
    import torch
    from test_gpu_parity import check_mixed
    mb = large_mixed()
    E = len(mb.cls)
    assert E > 65536
    say(f"[large] classes={len(mb.classes)} E={E} (counting-kernel bucketing)")
    plan = stp.Plan(mb.classes, prec=stp.FP32)
    d = Dev(mb)
    plan.run(d.batch(plan))
    assert plan.sync_status() == stp.OK
    full = d.host()
    say(f"[large]   worst vs oracle {check_mixed(mb, stp.FP32, full, sample_per_class=6):.2e}")
    # the same elements as two batches of at most 65536 (single-workgroup bucketing), into fresh outputs
    d.new_outputs()
    half = E // 2
    subs = [d.batch(plan, torch.arange(a, b, device="cuda")) for a, b in ((0, half), (half, E))]
    for sb in subs:
        plan.run(sb)
    torch.cuda.synchronize()
    split = d.host()
    for k in ("qavg", "favg", "qface"):
        assert np.array_equal(split[k], full[k]), k
    say("[large]   bitwise equal to two smaller batches")
    plan.close()


def _corrupt(mb, ids, values):
    import copy
    bad = copy.copy(mb)
    bad.cls = mb.cls.copy()
    bad.cls[ids] = values
    return bad


def _check_skipped(got, ref, mb, bad_ids):
    """Elements with invalid ids keep the NaN fill; every other element equals the clean run bit for bit."""
    keep_q = np.ones(mb.size_q, bool)
    keep_f = np.ones(mb.size_face, bool)
    for e in bad_ids:
        N, m = mb.classes[mb.cls[e]][:2]
        n3, n2 = (N + 1) ** 3, (N + 1) ** 2
        assert np.isnan(got["qavg"][mb.off_q[e]:mb.off_q[e] + n3 * m]).all()
        assert np.isnan(got["qface"][mb.off_face[e]:mb.off_face[e] + 6 * n2 * m]).all()
        keep_q[mb.off_q[e]:mb.off_q[e] + n3 * m] = False
        keep_f[mb.off_face[e]:mb.off_face[e] + 6 * n2 * m] = False
    assert np.array_equal(got["qavg"][keep_q], ref["qavg"][keep_q])
    assert np.array_equal(got["qface"][keep_f], ref["qface"][keep_f])


def test_invalid_class_ids_are_reported():
    import torch
    from test_gpu_parity import mixed_batch
    mb = mixed_batch(seed=942)
    nc = len(mb.classes)
    bad_ids = np.array([3, 17, len(mb.cls) - 1])
    bad = _corrupt(mb, bad_ids, [-1, nc, 1 << 20])
    plan = stp.Plan(mb.classes, prec=stp.FP32)
    clean = Dev(mb)
    plan.run(clean.batch(plan))
    assert plan.sync_status() == stp.OK
    ref = clean.host()
    for label, runner in (("stp_run", "run"), ("stp_run_noalloc", "run_noalloc")):
        say(f"[invalid] {label}: {len(bad_ids)} of {len(mb.cls)} class ids out of range")
        d = Dev(bad)
        getattr(plan, runner)(d.batch(plan))
        assert plan.sync_status() == stp.E_INVAL and "class ids outside" in stp.last_error()
        assert plan.sync_status() == stp.OK  # cleared
        _check_skipped(d.host(), ref, mb, bad_ids)
    plan.close()
    # the counting-kernel path (more than 65536 elements)
    big = large_mixed(seed=943)
    bad_big = _corrupt(big, np.array([0, 40000, len(big.cls) - 1]), [-7, len(big.classes), -1])
    plan = stp.Plan(big.classes, prec=stp.FP32)
    say(f"[invalid] stp_run, E={len(big.cls)} (counting kernel)")
    plan.run(Dev(bad_big).batch(plan))
    assert plan.sync_status() == stp.E_INVAL
    plan.run(Dev(big).batch(plan))
    assert plan.sync_status() == stp.OK
    plan.close()
    # serving: the ticket of the bad batch fails, the clean one completes
    plan = stp.Plan(mb.classes, prec=stp.FP32, serve_mem_budget=256 << 20)
    say("[invalid] serving")
    db, dc = Dev(bad), Dev(mb)
    torch.cuda.synchronize()
    tb, tc = plan.submit(db.batch(plan)), plan.submit(dc.batch(plan))
    plan.drain()
    st, _ = plan.poll(tb)
    assert st == stp.E_INVAL and "class ids outside" in stp.last_error()
    st, _ = plan.poll(tc)
    assert st == stp.OK
    _check_skipped(db.host(), ref, mb, bad_ids)
    for k in ("qavg", "favg", "qface"):
        assert np.array_equal(dc.host()[k], ref[k]), k
    plan.close()


def test_serving_preset_batches_match_oracle():
    """The serving configuration: acoustic and elastic classes N = 2..9 in one plan, FP32 with FP64
    accumulation at N >= 8, per-element dt and h (dt_h_scalar = 0), batches of contiguous element runs of a
    resident mesh submitted through stp_submit; every element of every ticket against the oracle."""
    import torch
    classes = [(N, 4, stp.ACOUSTIC, 0) for N in range(2, 10)] + [(N, 9, stp.ELASTIC, 0) for N in range(2, 10)]
    plan = stp.Plan(classes, prec=stp.FP32, acc64_min_order=8, serve_mem_budget=256 << 20)
    meshes = [W.serving_mesh(W.ACOUSTIC, 240, W.SEED0 + 60, 0), W.serving_mesh(W.ELASTIC, 160, W.SEED0 + 61, 8)]
    rng = np.random.default_rng(944)
    tickets = []
    for mh in meshes:
        mh["qavg"] = torch.full((mh["size_q"],), float("nan"), device="cuda")
        mh["favg"] = torch.full((3 * mh["size_q"],), float("nan"), device="cuda")
        mh["qface"] = torch.full((mh["size_face"],), float("nan"), device="cuda")
        mh["h"] = torch.from_numpy(rng.uniform(0.5, 2.0, mh["nelem"])).to("cuda", torch.float64)
        mh["dt"] = mh["dt"] * mh["h"] * torch.from_numpy(rng.uniform(0.3, 1.0, mh["nelem"])).to("cuda", torch.float64)
        # disjoint contiguous runs of log-uniform length
        a = 0
        while a < mh["nelem"]:
            k = min(int(np.exp(rng.uniform(0, np.log(65)))), mh["nelem"] - a)
            b = stp.Batch()
            b.nelem = k
            b.cls = mh["cls"].data_ptr() + 4 * a
            for f in ("off_q", "off_coef", "off_face", "dt", "h"):
                setattr(b, f, mh[f].data_ptr() + 8 * a)
            b.dt_h_scalar = 0
            b.Q, b.params = mh["Q"].data_ptr(), mh["params"].data_ptr()
            b.qavg, b.favg, b.qface = mh["qavg"].data_ptr(), mh["favg"].data_ptr(), mh["qface"].data_ptr()
            tickets.append((b, a, k, mh))
            a += k
    torch.cuda.synchronize()
    say(f"[serve-oracle] {len(tickets)} batches of 1..64 elements from two meshes (400 elements)")
    ids = [plan.submit(t[0]) for t in tickets]
    plan.drain()
    for t in ids:
        st, _ = plan.poll(t)
        assert st == stp.OK, stp.last_error()
    worst = 0.0
    for mh in meshes:
        phys, m = mh["physics"], W.NQUANT[mh["physics"]]
        npar = W.NPARAM[phys]
        host = {k: mh[k].cpu().numpy() for k in ("Q", "params", "qavg", "favg", "qface", "off_q", "off_coef",
                                                  "off_face", "dt", "h")}
        for N in range(2, 10):
            el = np.nonzero(mh["N"] == N)[0]
            if len(el) == 0:
                continue
            n3, n2 = (N + 1) ** 3, (N + 1) ** 2
            gq = lambda arr, off, size, mul=1: np.stack([arr[mul * host[off][e]:mul * host[off][e] + size] for e in el])
            Q = gq(host["Q"], "off_q", n3 * m).reshape(-1, n3, m).astype(np.float64)
            par = gq(host["params"], "off_coef", n3 * npar).reshape(-1, n3, npar).astype(np.float64)
            ref = oracle.stp(N, phys, Q, host["dt"][el], host["h"][el], params=par)
            got = {"qavg": gq(host["qavg"], "off_q", n3 * m).reshape(-1, n3, m),
                   "favg": gq(host["favg"], "off_q", 3 * n3 * m, 3).reshape(-1, 3, n3, m),
                   "qface": gq(host["qface"], "off_face", 6 * n2 * m).reshape(-1, 6, n2, m)}
            err = max_rel_err({k: v.astype(np.float64) for k, v in got.items()}, ref, Q, host["h"][el])
            worst = max(worst, max(err.values()))
            for k, v in err.items():
                assert v < TOL[stp.FP32], (phys, N, k, v)
    say(f"[serve-oracle]   every element of every ticket, worst max rel err {worst:.2e}")
    plan.close()


def test_serving_splits_large_batches_across_lanes(monkeypatch):
    """With STP_SERVE_SPLIT = 1024, batches above 1024 elements are queued as parts on different lanes; the
    outputs equal stp_run's bit for bit: a uniform batch with contiguous storage and host scalars dt, h; the
    same with per-element dt, h; and a heterogeneous batch with per-element offsets."""
    import torch
    monkeypatch.setenv("STP_SERVE_SPLIT", "1024")
    from paper_2003_12787_amd import runner
    from test_gpu_parity import mixed_batch
    b = W.elastic_batch(2, 3000, 945)
    rng = np.random.default_rng(946)
    bv = W.elastic_batch(3, 2500, 947)
    bv.h = rng.uniform(0.5, 2.0, bv.nelem)
    bv.dt = bv.dt * bv.h * rng.uniform(0.2, 1.0, bv.nelem)
    for label, ub in (("uniform, scalar dt/h", b), ("uniform, per-element dt/h", bv)):
        plan = stp.Plan([runner.class_of(ub)], prec=stp.FP32, serve_mem_budget=512 << 20)
        ref = runner.run(plan, ub)
        db = runner.DeviceBatch(plan, ub)
        db.clear_outputs(float("nan"))
        torch.cuda.synchronize()
        say(f"[split] {label}: E={ub.nelem}")
        t = plan.submit(db.cbatch)
        plan.drain()
        st, info = plan.poll(t)
        assert st == stp.OK and info.t_done >= info.t_start >= info.t_submit
        out = db.outputs()
        for k in ref:
            assert np.array_equal(out[k], ref[k]), (label, k)
        plan.close()
    mb = mixed_batch(E_scale=12, seed=948)
    assert len(mb.cls) > 1024
    plan = stp.Plan(mb.classes, prec=stp.FP32, serve_mem_budget=512 << 20)
    ref_d = Dev(mb)
    plan.run(ref_d.batch(plan))
    torch.cuda.synchronize()
    ref = ref_d.host()
    d = Dev(mb)
    torch.cuda.synchronize()
    say(f"[split] heterogeneous: E={len(mb.cls)}")
    t = plan.submit(d.batch(plan))
    plan.drain()
    st, _ = plan.poll(t)
    assert st == stp.OK
    got = d.host()
    for k in ref:  # fface is written only for the classes with A; both runs leave the rest at NaN
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    plan.close()


def test_serving_deadline(monkeypatch):
    """A ticket whose deadline has passed before its batch is launched fails with STP_E_TIMEOUT and writes
    nothing; tickets without a deadline (or with a generous one) complete. Split into parts (STP_SERVE_SPLIT)."""
    import torch
    monkeypatch.setenv("STP_SERVE_SPLIT", "1024")
    from paper_2003_12787_amd import runner
    b = W.elastic_batch(3, 2100, 949)  # three parts
    plan = stp.Plan([runner.class_of(b)], prec=stp.FP32, serve_mem_budget=512 << 20)
    ref = runner.run(plan, b)
    late, ok1, ok2 = (runner.DeviceBatch(plan, b) for _ in range(3))
    for db in (late, ok1, ok2):
        db.clear_outputs(float("nan"))
    torch.cuda.synchronize()
    t_late = plan.submit_deadline(late.cbatch, 0.0)  # the deadline is the submission time itself
    t_ok1 = plan.submit_deadline(ok1.cbatch, 60.0)
    t_ok2 = plan.submit(ok2.cbatch)
    plan.drain()
    st, _ = plan.poll(t_late)
    assert st == stp.E_TIMEOUT and "deadline" in stp.last_error()
    assert np.isnan(late.outputs()["qavg"]).all()
    for t, db in ((t_ok1, ok1), (t_ok2, ok2)):
        st, _ = plan.poll(t)
        assert st == stp.OK
        out = db.outputs()
        for k in ref:
            assert np.array_equal(out[k], ref[k]), k
    with pytest.raises(stp.StpError) as ei:
        plan.submit_deadline(ok1.cbatch, -1.0)
    assert ei.value.status == stp.E_INVAL
    plan.close()
