"""GPU parity with Gauss-Lobatto nodes (stp_plan_desc.nodes = 1): the predictor variants against the oracle's
Lobatto predictor, and the full ADER-DG step (predictor + corrector) converging on a plane wave."""
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


def check(b, prec, variant=stp.VARIANT_AUTO):
    plan = stp.Plan([runner.class_of(b)], prec=prec, variant=variant, nodes=stp.GAUSS_LOBATTO)
    assert plan.describe()["nodes"] == "lobatto"
    say(f"[lobatto] N={b.N} m={b.m} phys={b.physics} E={b.nelem} prec={prec} variant={variant}")
    got = runner.run(plan, b)
    rb = runner.rounded(b, prec)
    ref = oracle.stp(rb.N, rb.physics, rb.Q, rb.dt, rb.h, params=rb.params, A=rb.A, B=rb.B, src=rb.src,
                     coef_per_element=rb.coef_per_element, nodes=1)
    err = max_rel_err(got, ref, rb.Q, rb.h)
    say(f"[lobatto]   max rel err {err}")
    for k, v in err.items():
        assert v < TOL[prec], (k, v)
    plan.close()


@pytest.mark.parametrize("N,prec,variant", [(3, stp.FP64, stp.VARIANT_PLAIN), (3, stp.FP32, stp.VARIANT_FUSED),
                                            (7, stp.FP32, stp.VARIANT_FUSED), (7, stp.FP32, stp.VARIANT_MFMA),
                                            (7, stp.BF16X3, stp.VARIANT_MFMA),
                                            (9, stp.FP32, stp.VARIANT_PLAIN)])
def test_elastic_lobatto_variants(N, prec, variant):
    check(W.elastic_batch(N, 40, 700 + N), prec, variant)


def test_acoustic_and_generic_lobatto():
    check(W.acoustic_batch(5, 30, 711), stp.FP32)
    check(W.generic_batch(4, 5, 20, 712, with_A=True), stp.FP64)


@pytest.mark.parametrize("N", [2, 3])
def test_lobatto_full_step_plane_wave_converges(N, gpu):
    torch = gpu
    rho, K = 1.0, 2.25
    c = np.sqrt(K / rho)
    n = N + 1
    xi, _ = oracle.gll_nodes(n)
    plan = stp.Plan([(N, 4, stp.ACOUSTIC, stp.PARAM_PER_ELEMENT)], prec=stp.FP64, nodes=stp.GAUSS_LOBATTO)
    errs = []
    for nx in (8, 16):
        h = 1.0 / nx
        x = np.zeros((nx, n, n, n))
        for e in range(nx):
            x[e] = (e + xi)[None, None, :] * h
        x = x.reshape(nx, n ** 3)
        f = lambda t: np.sin(2 * np.pi * (x - c * t))
        Q0 = np.zeros((nx, n ** 3, 4))
        Q0[..., 0] = f(0.0)
        Q0[..., 1] = f(0.0) / (rho * c)
        T = 0.2
        steps = int(np.ceil(T / (0.2 * h / ((2 * N + 1) * c))))
        dt = T / steps
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64)
        Q, Qn, par = dev(Q0), torch.empty((nx, n ** 3, 4), device="cuda", dtype=torch.float64), dev(np.tile([rho, K], (nx, 1)))
        qavg = torch.empty_like(Q)
        favg = torch.empty((nx, 3, n ** 3, 4), device="cuda", dtype=torch.float64)
        qface = torch.empty((nx, 6, n * n, 4), device="cuda", dtype=torch.float64)
        for _ in range(steps):
            plan.run(plan.batch(nx, Q, qavg, favg, qface, dt, h, params=par))
            plan.correct((nx, 1, 1), dt, h, Q, favg, qface, Qn, params=par)
            Q, Qn = Qn, Q
        torch.cuda.synchronize()
        got = Q.cpu().numpy()
        errs.append(max(np.abs(got[..., 0] - f(T)).max(), np.abs(got[..., 1] - f(T) / (rho * c)).max()))
    rate = np.log2(errs[0] / errs[1])
    say(f"[lobatto] full step N={N} errors {errs} rate {rate:.2f}")
    assert rate > N + 1 - 0.5, (errs, rate)
    plan.close()
