"""GPU parity of the corrector (stp_correct) and of full ADER-DG steps (stp_run + stp_correct) against the
oracle on periodic Cartesian meshes, plus end-to-end plane-wave convergence on the GPU."""
import sys

import numpy as np
import pytest

import oracle
from oracle import corrector as OC
from paper_2003_12787_amd import stp
from paper_2003_12787_amd import workloads as W
from parity import TOL

pytestmark = pytest.mark.gpu

ACOUSTIC, ELASTIC, GENERIC, ELASTIC_CURV = 0, 1, 2, 3


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(x, y):
    return float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300))


def mesh_inputs(physics, N, grid, seed, m=None, with_A=False):
    rng = np.random.default_rng(seed)
    E = grid[0] * grid[1] * grid[2]
    n3 = (N + 1) ** 3
    if physics == ELASTIC:
        params, A, B, m = W.elastic_material(rng, (E,)), None, None, 9
    elif physics == ELASTIC_CURV:  # affine elements: material and a non-symmetric metric near I per element
        G = np.eye(3) + 0.2 * rng.standard_normal((E, 3, 3))
        params, A, B, m = np.concatenate([W.elastic_material(rng, (E,)), G.reshape(E, 9)], axis=1), None, None, 9
    elif physics == ACOUSTIC:
        params, A, B, m = np.stack([rng.uniform(2, 3, E), rng.uniform(1, 2, E)], axis=1), None, None, 4
    else:
        params = None
        B = rng.standard_normal((E, 3, m, m)) / np.sqrt(m)
        A = rng.standard_normal((E, 3, m, m)) / np.sqrt(m) if with_A else None
    Q = rng.standard_normal((E, n3, m))
    return Q, params, A, B, m


def flags_of(physics, with_A):
    if physics == GENERIC:
        return stp.COEF_PER_ELEMENT | (stp.A_PRESENT if with_A else 0)
    return stp.PARAM_PER_ELEMENT


def gpu_step(plan, prec, physics, N, grid, Q, params, A, B, dt, h, with_A, torch):
    """stp_run then stp_correct on the device; returns (q_new, predictor outputs) as host arrays."""
    tdt = torch.float64 if prec == stp.FP64 else torch.float32
    up = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda", tdt)
    E, n3, m = Q.shape
    n2 = (N + 1) ** 2
    dQ, dpar, dA, dB = up(Q), up(params), up(A), up(B)
    qavg = torch.empty((E, n3, m), device="cuda", dtype=tdt)
    favg = torch.empty((E, 3, n3, m), device="cuda", dtype=tdt)
    qface = torch.empty((E, 6, n2, m), device="cuda", dtype=tdt)
    fface = torch.empty((E, 6, n2, m), device="cuda", dtype=tdt) if with_A else None
    Qn = torch.empty_like(dQ)
    plan.run(plan.batch(E, dQ, qavg, favg, qface, dt, h, params=dpar, A=dA, B=dB, fface=fface))
    plan.correct(grid, dt, h, dQ, favg, qface, Qn, params=dpar, A=dA, B=dB, fface=fface)
    torch.cuda.synchronize()
    return Qn.double().cpu().numpy()


@pytest.mark.parametrize("physics,N,prec,with_A", [(ELASTIC, 3, stp.FP64, False), (ELASTIC, 3, stp.FP32, False),
                                                   (ACOUSTIC, 5, stp.FP64, False), (GENERIC, 2, stp.FP64, True),
                                                   (GENERIC, 4, stp.FP32, True), (ELASTIC_CURV, 3, stp.FP64, False),
                                                   (ELASTIC_CURV, 7, stp.FP32, False)])
def test_corrector_matches_oracle_on_oracle_predictor_outputs(physics, N, prec, with_A, gpu):
    """stp_correct alone, fed with the oracle predictor's outputs (rounded to the I/O precision)."""
    torch = gpu
    grid = (4, 3, 2)
    Q, params, A, B, m = mesh_inputs(physics, N, grid, 11 + N, m=3, with_A=with_A)
    h, dt = 0.5, 0.01
    rnd = (lambda a: a) if prec == stp.FP64 else (lambda a: None if a is None else a.astype(np.float32).astype(np.float64))
    Q, params, A, B = rnd(Q), rnd(params), rnd(A), rnd(B)
    pred = oracle.stp(N, physics, Q, dt, h, params=params, A=A, B=B, coef_per_element=True)
    favg, qface, fface = rnd(pred["favg"]), rnd(pred["qface"]), rnd(pred.get("fface"))
    ref = OC.correct(N, physics, grid, Q, favg, qface, dt, h, params=params, A=A, B=B, fface=fface)
    say(f"[corrector] physics={physics} N={N} m={m} prec={prec} A={with_A} mesh={grid}")
    plan = stp.Plan([(N, m, physics, flags_of(physics, with_A))], prec=prec)
    tdt = torch.float64 if prec == stp.FP64 else torch.float32
    up = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda", tdt)
    Qn = torch.empty(Q.shape, device="cuda", dtype=tdt)
    plan.correct(grid, dt, h, up(Q), up(favg), up(qface), Qn, params=up(params), A=up(A), B=up(B), fface=up(fface))
    torch.cuda.synchronize()
    got = Qn.double().cpu().numpy()
    err = rel(got, ref)
    say(f"[corrector]   max rel err {err:.2e}")
    assert err < TOL[prec], err
    plan.close()


@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_full_steps_match_oracle(prec, gpu):
    """Three ADER-DG steps (predictor + corrector on the GPU) against the oracle's steps."""
    torch = gpu
    N, grid = 3, (3, 2, 2)
    Q, params, _, _, m = mesh_inputs(ELASTIC, N, grid, 21)
    if prec != stp.FP64:
        Q, params = Q.astype(np.float32).astype(np.float64), params.astype(np.float32).astype(np.float64)
    h = 0.5
    dt = 0.2 * h / ((2 * N + 1) * np.sqrt((params[:, 1] + 2 * params[:, 2]) / params[:, 0]).max())
    plan = stp.Plan([(N, m, ELASTIC, stp.PARAM_PER_ELEMENT)], prec=prec)
    qg, qo = Q.copy(), Q.copy()
    for k in range(3):
        qg = gpu_step(plan, prec, ELASTIC, N, grid, qg, params, None, None, dt, h, False, torch)
        qo = OC.ader_step(N, ELASTIC, grid, qo, dt, h, params=params)
        err = rel(qg, qo)
        say(f"[full step] prec={prec} step {k}: max rel err {err:.2e}")
        assert err < 3 * TOL[prec], err
    plan.close()


@pytest.mark.parametrize("N", [2, 3])
def test_gpu_plane_wave_converges(N, gpu):
    """End to end on the GPU (FP64): an acoustic plane wave along x converges at order N + 1."""
    torch = gpu
    rho, K = 1.0, 2.25
    c = np.sqrt(K / rho)
    errs = []
    plan = stp.Plan([(N, 4, ACOUSTIC, stp.PARAM_PER_ELEMENT)], prec=stp.FP64)
    for nx in (8, 16):
        h = 1.0 / nx
        xi, _ = oracle.gl_nodes(N + 1)
        n = N + 1
        x = np.zeros((nx, n, n, n))
        for e in range(nx):
            x[e] = (e + xi)[None, None, :] * h
        x = x.reshape(nx, n ** 3)
        f = lambda t: np.sin(2 * np.pi * (x - c * t))
        Q = np.zeros((nx, n ** 3, 4))
        Q[..., 0] = f(0.0)
        Q[..., 1] = f(0.0) / (rho * c)
        params = np.tile([rho, K], (nx, 1))
        T = 0.2
        steps = int(np.ceil(T / (0.2 * h / ((2 * N + 1) * c))))
        dt = T / steps
        for _ in range(steps):
            Q = gpu_step(plan, stp.FP64, ACOUSTIC, N, (nx, 1, 1), Q, params, None, None, dt, h, False, torch)
        errs.append(max(np.abs(Q[..., 0] - f(T)).max(), np.abs(Q[..., 1] - f(T) / (rho * c)).max()))
    rate = np.log2(errs[0] / errs[1])
    say(f"[convergence] N={N} errors {errs} rate {rate:.2f}")
    assert rate > N + 1 - 0.25, (errs, rate)
    plan.close()


def test_corrector_validation(gpu):
    torch = gpu
    plan = stp.Plan([(3, 9, ELASTIC, 0)], prec=stp.FP32)  # per-node material: not supported by the corrector
    z = torch.zeros(64 * 9 * 8, device="cuda")
    st = stp.Step(2, 2, 2, 0.01, 0.5, z.data_ptr(), z.data_ptr(), None, None, z.data_ptr(), z.data_ptr(), None,
                  z.data_ptr())
    assert plan.correct_status(st) == stp.E_UNSUPPORTED
    plan.close()
    plan = stp.Plan([(3, 9, ELASTIC, stp.PARAM_PER_ELEMENT)], prec=stp.FP32)
    assert plan.correct_status(st) == stp.E_INVAL and "alias" in stp.last_error()
    out = torch.zeros(8 * 64 * 9, device="cuda")
    st.Qnew = out.data_ptr()
    st.h = 0.0
    assert plan.correct_status(st) == stp.E_INVAL
    st.h, st.nx = 0.5, 0
    assert plan.correct_status(st) == stp.E_INVAL
    plan.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_curvilinear_full_steps_match_oracle(prec, gpu):
    """Three ADER-DG steps on affine curvilinear elements (a different metric per element)."""
    torch = gpu
    N, grid = 3, (3, 2, 2)
    Q, params, _, _, m = mesh_inputs(ELASTIC_CURV, N, grid, 31)
    if prec != stp.FP64:
        Q, params = Q.astype(np.float32).astype(np.float64), params.astype(np.float32).astype(np.float64)
    h = 0.5
    dt = 0.2 * h / ((2 * N + 1) * OC.wave_speed(ELASTIC_CURV, params).max())
    plan = stp.Plan([(N, m, ELASTIC_CURV, stp.PARAM_PER_ELEMENT)], prec=prec)
    qg, qo = Q.copy(), Q.copy()
    for k in range(3):
        qg = gpu_step(plan, prec, ELASTIC_CURV, N, grid, qg, params, None, None, dt, h, False, torch)
        qo = OC.ader_step(N, ELASTIC_CURV, grid, qo, dt, h, params=params)
        err = rel(qg, qo)
        say(f"[curvilinear full step] prec={prec} step {k}: max rel err {err:.2e}")
        assert err < 3 * TOL[prec], err
    plan.close()


@pytest.mark.parametrize("N", [2, 3])
def test_gpu_affine_curvilinear_plane_wave_converges(N, gpu):
    """End to end on the GPU (FP64): a P-wave on a mesh mapped by a non-symmetric affine map (the oracle's
    convergence pin) converges at order N + 1."""
    torch = gpu
    rng = np.random.default_rng(12)
    J = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    G = np.linalg.inv(J)
    rho, lam, mu = 2.0, 3.0, 1.5
    cp = np.sqrt((lam + 2 * mu) / rho)
    k = 2 * np.pi * G.T[:, 0]
    kh = k / np.linalg.norm(k)
    S = -(lam * np.eye(3) + 2 * mu * np.outer(kh, kh)) / cp
    r = np.concatenate([kh, [S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]]])
    omega = cp * np.linalg.norm(k)
    alpha = cp * np.linalg.norm(G, axis=1).max()
    plan = stp.Plan([(N, 9, ELASTIC_CURV, stp.PARAM_PER_ELEMENT)], prec=stp.FP64)
    errs = []
    for nx in (8, 16):
        h = 1.0 / nx
        n = N + 1
        xi, _ = oracle.gl_nodes(n)
        xg = np.zeros((nx, n, n, n))
        for e in range(nx):
            xg[e] = (e + xi)[None, None, :] * h
        xg = xg.reshape(nx, n ** 3)
        f = lambda t: np.sin(2 * np.pi * xg - omega * t)
        Q = f(0.0)[..., None] * r
        params = np.tile(np.concatenate([[rho, lam, mu], G.ravel()]), (nx, 1))
        T = 0.1
        steps = int(np.ceil(T / (0.2 * h / ((2 * N + 1) * alpha))))
        dt = T / steps
        for _ in range(steps):
            Q = gpu_step(plan, stp.FP64, ELASTIC_CURV, N, (nx, 1, 1), Q, params, None, None, dt, h, False, torch)
        errs.append(np.abs(Q - f(T)[..., None] * r).max())
    rate = np.log2(errs[0] / errs[1])
    say(f"[curvilinear convergence] N={N} errors {errs} rate {rate:.2f}")
    assert rate > N + 1 - 0.5, (errs, rate)
    plan.close()


def curved_inputs(N, grid, seed):
    """Per-node curvilinear parameters of a small deformed box and random Q. The material is constant in each
    element (it jumps between elements); the face values extrapolate it, so it has to be smooth inside an
    element, as the metric is."""
    rng = np.random.default_rng(seed)
    _, G = W.curvilinear_geometry(N, grid, 0.5, 0.15)
    E, n3 = G.shape[:2]
    mat = np.broadcast_to(W.elastic_material(rng, (E,))[:, None, :], (E, n3, 3))
    params = np.concatenate([mat, G.reshape(E, n3, 9)], axis=2)
    return rng.standard_normal((E, n3, 9)), params


@pytest.mark.parametrize("N,prec,nodes", [(2, stp.FP64, stp.GAUSS_LEGENDRE), (3, stp.FP64, stp.GAUSS_LEGENDRE),
                                           (7, stp.FP32, stp.GAUSS_LEGENDRE), (3, stp.FP64, stp.GAUSS_LOBATTO),
                                           (5, stp.FP32, stp.GAUSS_LOBATTO)])
def test_curved_corrector_matches_oracle(N, prec, nodes, gpu):
    """stp_correct on curved elements (12 parameters per node), fed with the oracle predictor's outputs; then
    stp_face_params against the oracle's face extrapolation of the parameters, and the corrector given those
    face parameters reproduces its own extrapolation bit for bit."""
    torch = gpu
    grid = (3, 2, 2)
    Q, params = curved_inputs(N, grid, 40 + N)
    h, dt = 0.5, 0.005
    rnd = (lambda a: a) if prec == stp.FP64 else (lambda a: None if a is None else a.astype(np.float32).astype(np.float64))
    Q, params = rnd(Q), rnd(params)
    pred = oracle.stp(N, ELASTIC_CURV, Q, dt, h, params=params, nodes=nodes)
    favg, qface = rnd(pred["favg"]), rnd(pred["qface"])
    ref = OC.correct(N, ELASTIC_CURV, grid, Q, favg, qface, dt, h, params=params, nodes=nodes)
    say(f"[curved corrector] N={N} prec={prec} nodes={nodes} mesh={grid}")
    plan = stp.Plan([(N, 9, ELASTIC_CURV, 0)], prec=prec, nodes=nodes)
    tdt = torch.float64 if prec == stp.FP64 else torch.float32
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", tdt)
    Qn = torch.empty(Q.shape, device="cuda", dtype=tdt)
    dQ, dfavg, dqface, dpar = up(Q), up(favg), up(qface), up(params)
    plan.correct(grid, dt, h, dQ, dfavg, dqface, Qn, params=dpar)
    torch.cuda.synchronize()
    err = rel(Qn.double().cpu().numpy(), ref)
    say(f"[curved corrector]   max rel err {err:.2e}")
    assert err < TOL[prec], err
    n = N + 1
    E = Q.shape[0]
    fp = plan.face_params(E, dpar)
    torch.cuda.synchronize()
    fref = OC.face_values(params, n, nodes).reshape(E, 6, n * n, 12)
    ferr = np.abs(fp.double().cpu().numpy() - fref).max() / np.abs(fref).max()
    say(f"[curved corrector]   face parameters max rel err {ferr:.2e}")
    assert ferr < (1e-13 if prec == stp.FP64 else 1e-5), ferr
    Qf = torch.empty_like(Qn)
    plan.correct(grid, dt, h, dQ, dfavg, dqface, Qf, params=dpar, fparams=fp)
    torch.cuda.synchronize()
    assert torch.equal(Qf, Qn)
    plan.close()


def test_face_params_argument_errors(gpu):
    torch = gpu
    N, grid = 2, (2, 2, 2)
    E, n3, n2 = 8, 27, 9
    z = torch.zeros(E * n3 * 12 * 8, device="cuda")
    out = torch.zeros(E * n3 * 9, device="cuda")
    fp = torch.zeros(E * 6 * n2 * 12, device="cuda")
    cart = stp.Plan([(N, 9, ELASTIC, stp.PARAM_PER_ELEMENT)], prec=stp.FP32)
    affine = stp.Plan([(N, 9, ELASTIC_CURV, stp.PARAM_PER_ELEMENT)], prec=stp.FP32)
    curved = stp.Plan([(N, 9, ELASTIC_CURV, 0)], prec=stp.FP32)
    for plan in (cart, affine):  # face parameters are for curved elements only
        with pytest.raises(stp.StpError) as ei:
            plan.face_params(E, z, fp)
        assert ei.value.status == stp.E_UNSUPPORTED
        with pytest.raises(stp.StpError) as ei:
            plan.correct(grid, 0.01, 0.5, z, z, z, out, params=z, fparams=fp)
        assert ei.value.status == stp.E_INVAL and "fparams" in stp.last_error()
    for args in ((-1, z, fp), (E, None, fp), (E, z, z[1:])):  # nelem < 0, NULL params, fparams overlapping
        with pytest.raises(stp.StpError) as ei:
            curved.face_params(*args)
        assert ei.value.status == stp.E_INVAL
    with pytest.raises(stp.StpError) as ei:  # Qnew aliasing fparams
        curved.correct(grid, 0.01, 0.5, z, z, z, fp, params=z, fparams=fp)
    assert ei.value.status == stp.E_INVAL and "fparams" in stp.last_error()
    curved.face_params(0, z, fp)  # an empty batch queues nothing
    torch.cuda.synchronize()
    for plan in (cart, affine, curved):
        plan.close()


@pytest.mark.parametrize("N", [2, 3])
def test_gpu_curved_mesh_plane_wave_converges(N, gpu):
    """End to end on the GPU (FP64): the oracle's curved-box P-wave (metric per node). The errors at 4^3
    elements equal the oracle's, and the rate over 4^3 -> 8^3 -> 16^3 stays >= N + 1 - 0.5."""
    from test_corrector_oracle import curved_wave_setup
    torch = gpu
    plan = stp.Plan([(N, 9, ELASTIC_CURV, 0)], prec=stp.FP64)
    errs = []
    for M in (4, 8, 16):
        x, params, r, cp, alpha = curved_wave_setup(N, M)
        h = 1.0 / M
        f = lambda t: np.sin(2 * np.pi * (x[..., 0] - cp * t))
        Q = f(0.0)[..., None] * r
        T = 0.05
        steps = int(np.ceil(T / (0.2 * h / ((2 * N + 1) * alpha))))
        dt = T / steps
        qo = Q.copy()
        for k in range(steps):
            Q = gpu_step(plan, stp.FP64, ELASTIC_CURV, N, (M, M, M), Q, params, None, None, dt, h, False, torch)
            if M == 4:
                qo = OC.ader_step(N, ELASTIC_CURV, (M, M, M), qo, dt, h, params=params)
        if M == 4:
            say(f"[curved convergence] N={N} M=4 GPU vs oracle after {steps} steps: {rel(Q, qo):.2e}")
            assert rel(Q, qo) < 1e-11
        errs.append(np.abs(Q - f(T)[..., None] * r).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    say(f"[curved convergence] N={N} errors {errs} rates {rates}")
    assert rates[-1] > N + 1 - 0.5, (errs, rates)
    plan.close()


def test_time_loop_captured_in_a_graph(gpu):
    """stp_face_params and four full ADER-DG steps (stp_run then stp_correct with those face parameters, Q
    ping-ponging between two buffers) captured in one HIP graph: every replay, with other work and
    synchronisations in between, reproduces the eager steps (which extrapolate the parameters in the
    corrector) bit for bit (curved curvilinear elements, FP32)."""
    torch = gpu
    N, grid = 3, (4, 3, 2)
    Q0, params = curved_inputs(N, grid, 50)
    E, n3, m = Q0.shape
    n2 = (N + 1) ** 2
    h = 0.5
    dt = 0.2 * h / ((2 * N + 1) * 2.5)
    plan = stp.Plan([(N, m, ELASTIC_CURV, 0)], prec=stp.FP32)
    f32 = dict(device="cuda", dtype=torch.float32)
    Qa, Qb = torch.from_numpy(Q0).to(**f32), torch.empty((E, n3, m), **f32)
    par = torch.from_numpy(np.ascontiguousarray(params)).to(**f32)
    qavg, favg = torch.empty((E, n3, m), **f32), torch.empty((E, 3, n3, m), **f32)
    qface = torch.empty((E, 6, n2, m), **f32)
    ba = plan.batch(E, Qa, qavg, favg, qface, dt, h, params=par)
    bb = plan.batch(E, Qb, qavg, favg, qface, dt, h, params=par)

    fpar = torch.empty((E, 6, n2, 12), **f32)

    def four_steps(st, fp=None):
        for _ in range(2):
            plan.run(ba, st)
            plan.correct(grid, dt, h, Qa, favg, qface, Qb, params=par, fparams=fp, stream=st)
            plan.run(bb, st)
            plan.correct(grid, dt, h, Qb, favg, qface, Qa, params=par, fparams=fp, stream=st)

    # eager reference: three times four steps from Q0
    ref = []
    four_steps(torch.cuda.current_stream())
    for _ in range(3):
        ref.append(Qa.clone())
        four_steps(torch.cuda.current_stream())
    torch.cuda.synchronize()
    Qa.copy_(torch.from_numpy(Q0).to(**f32))
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=cap):
        plan.face_params(E, par, fpar, stream=cap)
        four_steps(cap, fpar)
    other = torch.randn(1 << 20, device="cuda")
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        say(f"[graph] replay {k}: max |diff| {float((Qa - ref[k]).abs().max()):.3e}")
        assert torch.equal(Qa, ref[k]), k
        other.mul_(1.0001)  # unrelated work between replays
        torch.cuda.synchronize()
    plan.close()


def test_curved_full_step_full_size(gpu):
    """The bench's curved full step at full size (65536 elements of the deformed 64 x 32 x 32 box, N = 7, MFMA
    predictor, FP32; material constant in each element): stp_face_params against the oracle's face
    extrapolation on 24 sampled elements, and the corrector with those face parameters equal, bit for bit, to
    the corrector that extrapolates them, with finite results."""
    torch = gpu
    N, E, n3, n2 = 7, 65536, 512, 64
    Q, par, dt = W.curvilinear_device(N, E, W.SEED0 + 7)
    par[..., 0:3] = par[:, :1, 0:3].clone()  # smooth inside an element (R25 reading of curved elements)
    grid = W.grid_of(E)
    assert grid[0] * grid[1] * grid[2] == E
    plan = stp.Plan([(N, 9, ELASTIC_CURV, 0)], prec=stp.BF16X3, variant=stp.VARIANT_MFMA)
    f32 = dict(device="cuda", dtype=torch.float32)
    qavg, favg, qface = torch.empty((E, n3, 9), **f32), torch.empty((E, 3, n3, 9), **f32), torch.empty((E, 6, n2, 9), **f32)
    say(f"[curved full size] E={E} grid={grid}")
    plan.run(plan.batch(E, Q, qavg, favg, qface, dt / 2, 1.0, params=par))
    fp = plan.face_params(E, par)
    Qa, Qb = torch.empty_like(Q), torch.empty_like(Q)
    plan.correct(grid, dt / 2, 1.0, Q, favg, qface, Qa, params=par, fparams=fp)
    plan.correct(grid, dt / 2, 1.0, Q, favg, qface, Qb, params=par)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Qa).all())
    assert torch.equal(Qa, Qb)
    ids = torch.from_numpy(np.linspace(0, E - 1, 24).astype(np.int64)).cuda()
    p = par.index_select(0, ids).double().cpu().numpy()
    fref = OC.face_values(p, N + 1).reshape(24, 6, n2, 12)
    ferr = np.abs(fp.index_select(0, ids).double().cpu().numpy() - fref).max() / np.abs(fref).max()
    say(f"[curved full size]   face parameters max rel err {ferr:.2e}; corrector paths equal")
    assert ferr < 1e-5, ferr
    plan.close()
    del Q, par, qavg, favg, qface, fp, Qa, Qb
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N", [1, 4, 9])
@pytest.mark.parametrize("prec", [stp.FP64, stp.FP32])
def test_face_params_orders(N, prec, gpu):
    """stp_face_params against the oracle's face extrapolation at the lowest and highest orders."""
    torch = gpu
    _, params = curved_inputs(N, (3, 2, 2), 60 + N)
    if prec != stp.FP64:
        params = params.astype(np.float32).astype(np.float64)
    tdt = torch.float64 if prec == stp.FP64 else torch.float32
    plan = stp.Plan([(N, 9, ELASTIC_CURV, 0)], prec=prec)
    E, n = params.shape[0], N + 1
    fp = plan.face_params(E, torch.from_numpy(np.ascontiguousarray(params)).to("cuda", tdt))
    torch.cuda.synchronize()
    fref = OC.face_values(params, n).reshape(E, 6, n * n, 12)
    err = np.abs(fp.double().cpu().numpy() - fref).max() / np.abs(fref).max()
    say(f"[face params] N={N} prec={prec}: max rel err {err:.2e}")
    assert err < (1e-13 if prec == stp.FP64 else 1e-5), err
    plan.close()
