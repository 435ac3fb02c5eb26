"""Pins of the corrector oracle (the ADER-DG step on a periodic Cartesian mesh), against what the scheme and
the mathematics fix: steady constant states, the upwind flux for a scalar wave, and the convergence order of
a full space-time step on smooth plane waves."""
import numpy as np
import pytest

import oracle
from oracle import corrector as OC

ACOUSTIC, ELASTIC, GENERIC = 0, 1, 2


def node_x(N, nx, h):
    """x coordinate of every node [E, n^3] of a nx x 1 x 1 mesh (elements along x)."""
    n = N + 1
    xi, _ = oracle.gl_nodes(n)
    x = np.zeros((nx, n, n, n))
    for e in range(nx):
        x[e] = (e + xi)[None, None, :] * h
    return x.reshape(nx, n ** 3)


def full_step_dt(N, h, c):
    """Stable time step of the full 3D step: half the predictor workloads' rule 0.4 h / ((2N+1) c). At the
    full rule, transverse modes seeded by rounding grow on a 1-element-wide periodic mesh at N = 3."""
    return 0.2 * h / ((2 * N + 1) * c)


def test_constant_state_is_steady_with_jumps_in_material():
    rng = np.random.default_rng(1)
    N, grid = 2, (3, 2, 2)
    E, n3 = 12, 27
    params = np.stack([rng.uniform(2, 3, E), rng.uniform(1, 4, E), rng.uniform(1, 3, E)], axis=1)
    q0 = rng.standard_normal(9)
    Q = np.broadcast_to(q0, (E, n3, 9)).copy()
    out = OC.ader_step(N, ELASTIC, grid, Q, 0.01, 0.5, params=params)
    assert np.abs(out - Q).max() < 1e-13


def test_scalar_wave_gets_the_upwind_flux():
    """q_t + a q_x = 0 (generic m = 1, a > 0): the upper face sees no correction, the lower face a (q+ - q-)."""
    N, nx = 2, 3
    n = N + 1
    a, h, dt = 1.5, 0.5, 0.01
    B = np.zeros((nx, 3, 1, 1))
    B[:, 0, 0, 0] = a
    rng = np.random.default_rng(2)
    # varying along x only, so that the (self-periodic) y and z faces see no jump
    Q = np.broadcast_to(rng.standard_normal((nx, 1, 1, n)), (nx, n, n, n)).reshape(nx, n ** 3, 1).copy()
    pred = oracle.stp(N, GENERIC, Q, dt, h, B=B, coef_per_element=True)
    out = OC.correct(N, GENERIC, (nx, 1, 1), Q, pred["favg"], pred["qface"], dt, h, B=B)
    qf = pred["qface"].reshape(nx, 6, n, n)
    w = OC.gl_weights01(n)
    l0 = oracle.lagrange_at(n, 0.0)
    ref = Q.reshape(nx, n, n, n) + dt * pred["favg"].sum(axis=1).reshape(nx, n, n, n)
    for e in range(nx):
        up = (e - 1) % nx  # upstream neighbour
        jump = qf[up, 1] - qf[e, 0]  # its x+ face minus our x- face
        ref[e] += dt * (l0 / (h * w))[None, None, :] * (a * jump)[:, :, None]
    assert np.abs(out.reshape(nx, n, n, n) - ref).max() < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3])
def test_acoustic_plane_wave_converges_at_order_N_plus_1(N):
    """p = sin(2 pi (x - c t)), v_x = p / (rho c) on [0,1] periodic; error at the nodes after t = 0.2."""
    rho, K = 1.0, 2.25
    c = np.sqrt(K / rho)
    errs = []
    for nx in (8, 16):
        h = 1.0 / nx
        x = node_x(N, nx, h)
        f = lambda t: np.sin(2 * np.pi * (x - c * t))
        Q = np.zeros((nx, (N + 1) ** 3, 4))
        Q[..., 0] = f(0.0)
        Q[..., 1] = f(0.0) / (rho * c)
        params = np.tile([rho, K], (nx, 1))
        T = 0.2
        steps = int(np.ceil(T / full_step_dt(N, h, c)))
        dt = T / steps
        for _ in range(steps):
            Q = OC.ader_step(N, ACOUSTIC, (nx, 1, 1), Q, dt, h, params=params)
        err = max(np.abs(Q[..., 0] - f(T)).max(), np.abs(Q[..., 1] - f(T) / (rho * c)).max())
        assert np.abs(Q[..., 2:]).max() < 1e-12  # no transverse velocity appears
        errs.append(err)
    rate = np.log2(errs[0] / errs[1])
    assert rate > N + 1 - 0.25, (errs, rate)


def test_elastic_shear_wave_converges():
    """An S-wave along x: v_y = sin(2 pi (x - cs t)), s_xy = -rho cs v_y; N = 2, rate >= 2.75 (16 -> 32
    elements; the Rusanov speed is the P-wave speed, so the S-wave needs the finer pair to be asymptotic)."""
    N = 2
    rho, lam, mu = 2.0, 3.0, 1.5
    cs = np.sqrt(mu / rho)
    errs = []
    for nx in (16, 32):
        h = 1.0 / nx
        x = node_x(N, nx, h)
        f = lambda t: np.sin(2 * np.pi * (x - cs * t))
        Q = np.zeros((nx, (N + 1) ** 3, 9))
        Q[..., 1] = f(0.0)
        Q[..., 6] = -rho * cs * f(0.0)
        params = np.tile([rho, lam, mu], (nx, 1))
        T = 0.3
        cp = np.sqrt((lam + 2 * mu) / rho)
        steps = int(np.ceil(T / full_step_dt(N, h, cp)))
        dt = T / steps
        for _ in range(steps):
            Q = OC.ader_step(N, ELASTIC, (nx, 1, 1), Q, dt, h, params=params)
        errs.append(max(np.abs(Q[..., 1] - f(T)).max(), np.abs(Q[..., 6] + rho * cs * f(T)).max()))
    rate = np.log2(errs[0] / errs[1])
    assert rate > 2.75, (errs, rate)


@pytest.mark.parametrize("N", [2, 3])
def test_gauss_lobatto_plane_wave_converges(N):
    """The same acoustic plane wave with Gauss-Lobatto nodes (collocated boundary nodes, lumped mass)."""
    rho, K = 1.0, 2.25
    c = np.sqrt(K / rho)
    errs = []
    n = N + 1
    xi, _ = oracle.gll_nodes(n)
    for nx in (8, 16):
        h = 1.0 / nx
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
        steps = int(np.ceil(T / full_step_dt(N, h, c)))
        dt = T / steps
        for _ in range(steps):
            Q = OC.ader_step(N, ACOUSTIC, (nx, 1, 1), Q, dt, h, params=params, nodes=1)
        errs.append(max(np.abs(Q[..., 0] - f(T)).max(), np.abs(Q[..., 1] - f(T) / (rho * c)).max()))
    rate = np.log2(errs[0] / errs[1])
    assert rate > N + 1 - 0.5, (errs, rate)


@pytest.mark.parametrize("N", [2, 3])
def test_affine_curvilinear_plane_wave_converges(N):
    """Curvilinear elastic elements with affine geometry: the mesh is the image of the periodic box under
    x = J xi (J non-symmetric), each element carrying G = J^-1 and the material (12 parameters). A P-wave
    q = r sin(k.x - c_p |k| t) with k = 2 pi G^T e_x is periodic in xi; after full ADER-DG steps the error at
    the nodes falls at order N + 1."""
    ELASTIC_CURV = 3
    rng = np.random.default_rng(12)
    J = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    assert np.linalg.det(J) > 0.2 and np.abs(J - J.T).max() > 0.05
    G = np.linalg.inv(J)
    rho, lam, mu = 2.0, 3.0, 1.5
    cp = np.sqrt((lam + 2 * mu) / rho)
    k = 2 * np.pi * G.T[:, 0]
    kh = k / np.linalg.norm(k)
    S = -(lam * np.eye(3) + 2 * mu * np.outer(kh, kh)) / cp
    r = np.concatenate([kh, [S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]]])
    omega = cp * np.linalg.norm(k)
    alpha = cp * np.linalg.norm(G, axis=1).max()
    errs = []
    for nx in (8, 16):
        h = 1.0 / nx
        xg = node_x(N, nx, h)  # global reference coordinate xi_x of the nodes
        f = lambda t: np.sin(2 * np.pi * xg - omega * t)
        Q = f(0.0)[..., None] * r
        params = np.tile(np.concatenate([[rho, lam, mu], G.ravel()]), (nx, 1))
        T = 0.1
        steps = int(np.ceil(T / full_step_dt(N, h, alpha)))
        dt = T / steps
        for _ in range(steps):
            Q = OC.ader_step(N, ELASTIC_CURV, (nx, 1, 1), Q, dt, h, params=params)
        errs.append(np.abs(Q - f(T)[..., None] * r).max())
    rate = np.log2(errs[0] / errs[1])
    print(f"affine curvilinear N={N}: errors {errs}, rate {rate:.2f}")
    assert rate > N + 1 - 0.5, (errs, rate)


def test_curvilinear_with_identity_metric_is_the_cartesian_step():
    rng = np.random.default_rng(13)
    N, grid, E, n3 = 2, (3, 2, 2), 12, 27
    par = np.stack([rng.uniform(2, 3, E), rng.uniform(1, 4, E), rng.uniform(1, 3, E)], axis=1)
    pc = np.concatenate([par, np.tile(np.eye(3).ravel(), (E, 1))], axis=1)
    Q = rng.standard_normal((E, n3, 9))
    a = OC.ader_step(N, ELASTIC, grid, Q, 0.01, 0.5, params=par)
    b = OC.ader_step(N, 3, grid, Q, 0.01, 0.5, params=pc)
    assert np.abs(a - b).max() < 1e-14


def curved_wave_setup(N, M, eps=0.1):
    """M^3 elements of the unit box under the smooth periodic deformation of the curvilinear workloads; a
    P-wave along x_0, q = r sin(2 pi (x_0 - c_p t)), periodic on the deformed box. Returns the node positions,
    the per-node parameters [E, n^3, 12], r, c_p and the largest Rusanov speed."""
    from paper_2003_12787_amd import workloads as W
    rho, lam, mu = 2.0, 3.0, 1.5
    cp = np.sqrt((lam + 2 * mu) / rho)
    x, G = W.curvilinear_geometry(N, (M, M, M), 1.0 / M, eps)
    E, n3 = x.shape[:2]
    params = np.concatenate([np.broadcast_to([rho, lam, mu], (E, n3, 3)), G.reshape(E, n3, 9)], axis=2)
    S = -(lam * np.eye(3) + 2 * mu * np.outer([1, 0, 0], [1, 0, 0])) / cp
    r = np.concatenate([[1.0, 0, 0], [S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]]])
    alpha = cp * np.linalg.norm(G, axis=3).max()
    return x, params, r, cp, alpha


def test_curved_elements_constant_parameters_are_the_affine_step():
    """Parameters given per node but constant in every element reproduce the per-element (affine) step."""
    rng = np.random.default_rng(14)
    N, grid, E, n3 = 2, (3, 2, 2), 12, 27
    par = np.concatenate([np.stack([rng.uniform(2, 3, E), rng.uniform(1, 4, E), rng.uniform(1, 3, E)], axis=1),
                          (np.eye(3) + 0.2 * rng.standard_normal((E, 3, 3))).reshape(E, 9)], axis=1)
    Q = rng.standard_normal((E, n3, 9))
    a = OC.ader_step(N, 3, grid, Q, 0.01, 0.5, params=par)
    b = OC.ader_step(N, 3, grid, Q, 0.01, 0.5, params=np.repeat(par[:, None, :], n3, axis=1))
    assert np.abs(a - b).max() < 1e-14 * np.abs(a).max()


@pytest.mark.parametrize("N", [2, 3])
def test_curved_mesh_plane_wave_converges(N):
    """Curved elements (metric per node) of the deformed periodic box: a P-wave converges at order >= N + 1 -
    0.5 over full ADER-DG steps (4^3 -> 8^3 elements)."""
    errs = []
    for M in (4, 8):
        x, params, r, cp, alpha = curved_wave_setup(N, M)
        h = 1.0 / M
        f = lambda t: np.sin(2 * np.pi * (x[..., 0] - cp * t))
        Q = f(0.0)[..., None] * r
        T = 0.05
        steps = int(np.ceil(T / full_step_dt(N, h, alpha)))
        dt = T / steps
        for _ in range(steps):
            Q = OC.ader_step(N, 3, (M, M, M), Q, dt, h, params=params)
        errs.append(np.abs(Q - f(T)[..., None] * r).max())
    rate = np.log2(errs[0] / errs[1])
    print(f"curved mesh N={N}: errors {errs}, rate {rate:.2f}")
    assert rate > N + 1 - 0.5, (errs, rate)
