"""Pins of the FP64 oracle against what the paper and the mathematics fix (no GPU).

The paper prints no worked example, so every pin is a closed form, a textbook/library special case, a
brute-force construction or an invariant:
  - quadrature nodes: closed forms (n = 2, 3), numpy's leggauss, exactness of the rule;
  - derivative matrix: exact differentiation of polynomials up to degree N (Sec. II-A), nilpotency;
  - face vectors: exact interpolation of polynomials at 0 and 1;
  - sum factorisation (Sec. III-B): equals the densely assembled Kronecker operator;
  - CK Taylor loop (Eq. (4)): equals the dense truncated series and lies within the truncation bound
    of phi_1(dt V) = (exp(dt V) - I)/(dt V) from scipy's expm;
  - presets: the spectrum of sum_d k_d B_d is the textbook wave speeds; polynomial plane waves are
    reproduced exactly (q-bar, favg, faces);
  - invariants: linearity, constant state, Fig. 1 == Fig. 5, axis permutation, dt -> 0, favg ~ 1/h,
    point source with V = 0.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import dense
from paper_2003_12787_amd import workloads as W

ACOUSTIC, ELASTIC, GENERIC = 0, 1, 2


# ------------------------------------------------------------------------------------------------ nodes
def test_gl_nodes_closed_forms(oracle_mod):
    xi, w = oracle_mod.gl_nodes(2)
    assert np.allclose(xi, [0.5 - math.sqrt(3) / 6, 0.5 + math.sqrt(3) / 6], rtol=0, atol=1e-15)
    assert np.allclose(w, [0.5, 0.5], rtol=0, atol=1e-15)
    xi, w = oracle_mod.gl_nodes(3)
    assert np.allclose(xi, [0.5 - math.sqrt(15) / 10, 0.5, 0.5 + math.sqrt(15) / 10], rtol=0, atol=1e-15)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], rtol=0, atol=1e-15)
    xi, w = oracle_mod.gl_nodes(1)
    assert np.allclose(xi, [0.5]) and np.allclose(w, [1.0])


@pytest.mark.parametrize("n", range(1, 13))
def test_gl_nodes_vs_library_and_exactness(oracle_mod, n):
    xi, w = oracle_mod.gl_nodes(n)
    xr, wr = dense.np_nodes(n)
    assert np.max(np.abs(xi - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14
    assert np.all(np.diff(xi) > 0)
    for p in range(2 * n):  # Gauss rule with n points is exact up to degree 2n-1
        assert abs(np.dot(w, xi ** p) - 1.0 / (p + 1)) < 1e-14
    # degree 2n is not integrated exactly: the Gauss error for xi^(2n) on [0,1] is the closed form
    # (n!)^4 / ((2n+1) ((2n)!)^2), which catches a wrong node count or a shifted node set
    if n <= 6:
        err = 1.0 / (2 * n + 1) - np.dot(w, xi ** (2 * n))
        exact = math.factorial(n) ** 4 / ((2 * n + 1) * math.factorial(2 * n) ** 2)
        assert abs(err - exact) < 1e-6 * exact


# ------------------------------------------------------------------------------------------------ D
@pytest.mark.parametrize("N", range(0, 10))
def test_dmatrix_differentiates_polynomials_exactly(oracle_mod, N):
    n = N + 1
    D = oracle_mod.dmatrix(n)
    xi, _ = oracle_mod.gl_nodes(n)
    scale = np.abs(D).sum(axis=1).max() + 1.0
    for p in range(0, N + 1):
        exact = p * xi ** (p - 1) if p > 0 else np.zeros(n)
        assert np.max(np.abs(D @ xi ** p - exact)) < 2e-15 * scale * max(1, p)
    # orientation: rows are output nodes. The transposed matrix fails the p = 1 pin for n >= 2.
    if n >= 2:
        assert np.max(np.abs(D.T @ xi - 1.0)) > 1e-3
    # nilpotent: D^n annihilates every polynomial of degree <= N
    Dn = np.linalg.matrix_power(D, n)
    assert np.abs(Dn).max() <= 1e-13 * np.abs(D).max() ** n + 1e-12
    # agrees with the Lagrange derivative assembled from monomial coefficients by numpy
    assert np.max(np.abs(D - dense.np_dmatrix(n))) < 1e-9 * scale


@pytest.mark.parametrize("N", range(0, 10))
def test_face_vectors(oracle_mod, N):
    n = N + 1
    e0 = oracle_mod.lagrange_at(n, 0.0)
    e1 = oracle_mod.lagrange_at(n, 1.0)
    xi, _ = oracle_mod.gl_nodes(n)
    for p in range(0, N + 1):
        assert abs(np.dot(e0, xi ** p) - (1.0 if p == 0 else 0.0)) < 1e-12
        assert abs(np.dot(e1, xi ** p) - 1.0) < 1e-12
    assert np.allclose(e0[::-1], e1, atol=1e-13)  # symmetric node set


# ------------------------------------------------------------------------------------------------ contraction
def test_fig7_fused_y_contraction_layout(oracle_mod):
    """Fig. 7: the y-derivative with the x and quantity indices fused, 6 nodes per axis and 12 quantities
    (z stride 432 = 6*72, y stride 72 = 6*12, derivative matrix padded to leading dimension 8).
    Restated from the figure's index arithmetic, and compared to the oracle's axis-1 contraction."""
    n, m = 6, 12
    rng = np.random.default_rng(7)
    Q = rng.standard_normal(n * n * n * m)
    D = oracle_mod.dmatrix(n)
    dudx = np.zeros(n * 8)
    for j in range(n):
        for l in range(n):
            dudx[j * 8 + l] = D[j, l]
    grad = np.zeros_like(Q)
    for k in range(n):
        for j in range(n):
            for l in range(n):
                grad[k * 432 + j * 72:k * 432 + j * 72 + 72] += Q[k * 432 + l * 72:k * 432 + l * 72 + 72] * dudx[j * 8 + l]
    ref = oracle_mod.contract(D, 1, Q.reshape(n, n, n, m)).ravel()
    assert np.max(np.abs(grad - ref)) < 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_contract_matches_kronecker(oracle_mod, axis):
    n, m = 4, 3
    rng = np.random.default_rng(axis)
    M = rng.standard_normal((n, n))
    u = rng.standard_normal((n, n, n, m))
    K = np.kron(dense.axis_operator(M, axis, n), np.eye(m))
    assert np.max(np.abs(oracle_mod.contract(M, axis, u).ravel() - K @ u.ravel())) < 1e-13


# ------------------------------------------------------------------------------------------------ presets
def test_preset_spectra(oracle_mod):
    """sum_d k_d B_d has the textbook characteristic speeds: acoustic +-c, 0, 0; elastic +-c_p, +-c_s
    (twice), 0 (three times)."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        k = rng.standard_normal(3)
        k /= np.linalg.norm(k)
        rho, K = rng.uniform(2, 3), rng.uniform(1, 2)
        B = oracle_mod.preset_B(ACOUSTIC, [rho, K])
        ev = np.sort(np.linalg.eigvals(np.einsum("d,dij->ij", k, B)).real)
        c = math.sqrt(K / rho)
        assert np.allclose(ev, [-c, 0, 0, c], atol=1e-12)
        rho, lam, mu = rng.uniform(2, 3), rng.uniform(1, 4), rng.uniform(1, 3)
        B = oracle_mod.preset_B(ELASTIC, [rho, lam, mu])
        ev = np.sort(np.linalg.eigvals(np.einsum("d,dij->ij", k, B)).real)
        cp, cs = math.sqrt((lam + 2 * mu) / rho), math.sqrt(mu / rho)
        assert np.allclose(ev, [-cp, -cs, -cs, 0, 0, 0, cs, cs, cp], atol=1e-10)


def _node_B(oracle_mod, physics, params_nodes):
    return np.stack([oracle_mod.preset_B(physics, p) for p in params_nodes], axis=1)


# ------------------------------------------------------------------------------------------------ V
@pytest.mark.parametrize("N", [0, 1, 2, 3])
@pytest.mark.parametrize("kind", ["acoustic", "elastic", "generic", "generic_A"])
def test_apply_Vd_matches_dense_kronecker(oracle_mod, N, kind):
    n3 = (N + 1) ** 3
    rng = np.random.default_rng(N * 10 + len(kind))
    h = 0.7
    A3 = None
    if kind == "acoustic":
        m = 4
        par = np.stack([rng.uniform(2, 3, n3), rng.uniform(1, 2, n3)], axis=1)
        B3 = _node_B(oracle_mod, ACOUSTIC, par)
    elif kind == "elastic":
        m = 9
        par = W.elastic_material(rng, (n3,))
        B3 = _node_B(oracle_mod, ELASTIC, par)
    else:
        m = 5
        B3 = rng.standard_normal((3, n3, m, m))
        if kind == "generic_A":
            A3 = rng.standard_normal((3, n3, m, m))
    u = rng.standard_normal((n3, m))
    for d in range(3):
        ref = dense.dense_Vd(N, m, h, d, B3, A3) @ u.ravel()
        got = oracle_mod.apply_Vd(N, h, d, B3, u, A3).ravel()
        assert np.max(np.abs(got - ref)) < 1e-11 * max(1.0, np.abs(ref).max())


# ------------------------------------------------------------------------------------------------ Taylor loop
def _small_case(kind, N, seed, with_A=False):
    if kind == "elastic":
        return W.elastic_batch(N, 3, seed, h=0.9)
    if kind == "acoustic":
        return W.acoustic_batch(N, 3, seed, h=1.3)
    return W.generic_batch(N, 3, 3, seed, h=1.1, with_A=with_A)


def _batch_B3(oracle_mod, b, e):
    n3 = (b.N + 1) ** 3
    if b.physics == GENERIC:
        B3 = b.B[e] if not b.coef_per_element else np.repeat(b.B[e][:, None], n3, axis=1)
        A3 = None if b.A is None else (b.A[e] if not b.coef_per_element else np.repeat(b.A[e][:, None], n3, axis=1))
        return B3, A3
    par = b.params[e] if not b.coef_per_element else np.repeat(b.params[e][None], n3, axis=0)
    return _node_B(oracle_mod, b.physics, par), None


def run_oracle(oracle_mod, b, fig5=False, **kw):
    return oracle_mod.stp(b.N, b.physics, b.Q, b.dt, b.h, params=b.params, A=b.A, B=b.B, src=b.src,
                          coef_per_element=b.coef_per_element, fig5=fig5, **kw)


@pytest.mark.parametrize("N", [1, 2])
@pytest.mark.parametrize("kind", ["acoustic", "elastic", "generic", "generic_A"])
def test_taylor_sum_vs_dense_series_and_expm(oracle_mod, N, kind):
    b = _small_case(kind.replace("_A", ""), N, 100 + N, with_A=kind.endswith("_A"))
    out = run_oracle(oracle_mod, b)
    n3, m = (N + 1) ** 3, b.m
    for e in range(b.nelem):
        B3, A3 = _batch_B3(oracle_mod, b, e)
        Vds = [dense.dense_Vd(N, m, b.h[e], d, B3, A3) for d in range(3)]
        V = sum(Vds)
        q0 = b.Q[e].ravel()
        dt = b.dt[e]
        # truncated series with N+1 terms: sum_o dt^o/(o+1)! V^o Q, and favg_d = V_d of that
        terms = [q0]
        for o in range(1, N + 1):
            terms.append(V @ terms[-1])
        qbar = sum(dt ** o / math.factorial(o + 1) * t for o, t in enumerate(terms))
        scale = np.abs(qbar).max()
        assert np.max(np.abs(out["qavg"][e].ravel() - qbar)) < 1e-12 * scale
        for d in range(3):
            fd = Vds[d] @ qbar
            assert np.max(np.abs(out["favg"][e, d].ravel() - fd)) < 1e-11 * max(1.0, np.abs(fd).max())
        # phi_1(dt V) Q from the exponential of the augmented matrix [[dt V, I], [0, 0]]
        K = V.shape[0]
        aug = np.zeros((2 * K, 2 * K))
        aug[:K, :K] = dt * V
        aug[:K, K:] = np.eye(K)
        phi1 = scipy.linalg.expm(aug)[:K, K:]
        exact = phi1 @ q0
        lead = dt ** (N + 1) / math.factorial(N + 2) * np.abs(V @ terms[-1]).max()
        err = np.abs(out["qavg"][e].ravel() - exact).max()
        assert err <= 1.5 * lead + 1e-13 * scale
        # the truncation is visible above rounding, and one term fewer is clearly worse (N+1 terms, not N)
        assert err > 1e-6 * scale
        fewer = qbar - dt ** N / math.factorial(N + 1) * terms[-1]
        assert np.abs(fewer - exact).max() > 3.0 * err


# ------------------------------------------------------------------------------------------------ plane waves
def _plane_wave_setup(physics, N, wave, seed):
    """Constant-material plane wave q = r f(k.x - c t) with f a random polynomial of degree N."""
    rng = np.random.default_rng(seed)
    k = rng.standard_normal(3)
    k /= np.linalg.norm(k)
    if physics == ACOUSTIC:
        rho, K = 2.3, 1.7
        par = np.array([rho, K])
        c = math.sqrt(K / rho)
        r = np.concatenate([[1.0], k / (rho * c)])
    else:
        rho, lam, mu = 2.5, 2.0, 1.5
        par = np.array([rho, lam, mu])
        if wave == "P":
            c = math.sqrt((lam + 2 * mu) / rho)
            S = -(lam * np.eye(3) + 2 * mu * np.outer(k, k)) / c
            vel = k
        else:
            c = math.sqrt(mu / rho)
            a = np.cross(k, rng.standard_normal(3))
            a /= np.linalg.norm(a)
            S = -mu * (np.outer(a, k) + np.outer(k, a)) / c
            vel = a
        r = np.concatenate([vel, [S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]]])
    coef = rng.standard_normal(N + 1)
    return par, k, c, r, np.polynomial.Polynomial(coef)


@pytest.mark.parametrize("N", [1, 2, 3, 5])
@pytest.mark.parametrize("physics,wave", [(ACOUSTIC, "P"), (ELASTIC, "P"), (ELASTIC, "S")])
def test_polynomial_plane_wave_exact(oracle_mod, N, physics, wave):
    n = N + 1
    par, k, c, r, f = _plane_wave_setup(physics, N, wave, 40 + N)
    h, dt = 0.8, 0.05
    origin = np.array([0.3, -0.2, 0.5])
    xi, _ = dense.np_nodes(n)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")
    pos = origin[None, :] + h * np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    s = pos @ k
    F = f.integ()
    Q = np.outer(f(s), r)[None]
    out = oracle_mod.stp(N, physics, Q, dt, h, params=par[None], coef_per_element=True)
    # exact time average (1/dt) int_0^dt r f(s - c t) dt = r [F(s) - F(s - c dt)] / (c dt)
    qbar = np.outer((F(s) - F(s - c * dt)) / (c * dt), r)
    scale = np.abs(qbar).max()
    assert np.max(np.abs(out["qavg"][0] - qbar)) < 1e-12 * max(1, scale) * 10
    # favg_d = -k_d B_d r [f(s) - f(s - c dt)] / (c dt)
    B = oracle_mod.preset_B(physics, par)
    g = (f(s) - f(s - c * dt)) / (c * dt)
    for d in range(3):
        fd = -k[d] * np.outer(g, B[d] @ r)
        assert np.max(np.abs(out["favg"][0, d] - fd)) < 1e-11 * max(1, np.abs(fd).max()) * 10
    # faces: q-bar of the exact solution at the face points
    for fidx in range(6):
        axis, side = fidx // 2, fidx % 2
        A_, B_ = np.meshgrid(xi, xi, indexing="ij")
        coords = np.zeros((n * n, 3))
        other = [a for a in (2, 1, 0) if a != axis]  # slower axis first: z, y, x
        coords[:, axis] = float(side)
        coords[:, other[0]] = A_.ravel()
        coords[:, other[1]] = B_.ravel()
        sf = (origin[None, :] + h * coords) @ k
        qf = np.outer((F(sf) - F(sf - c * dt)) / (c * dt), r)
        assert np.max(np.abs(out["qface"][0, fidx] - qf)) < 1e-11 * max(1, scale) * 10


def test_sinusoidal_plane_wave_converges_at_order_N_plus_1(oracle_mod):
    """With f = sin and dt proportional to h, the error of q-bar against the exact average falls like
    h^(N+1) (space and time truncation are both of that order)."""
    physics, N = ELASTIC, 3
    n = N + 1
    par, k, c, r, _ = _plane_wave_setup(physics, N, "P", 9)
    xi, _ = dense.np_nodes(n)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")
    errs = []
    hs = [0.2, 0.1, 0.05]
    for h in hs:
        dt = 0.3 * h / c
        pos = h * np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        s = pos @ k + 0.37
        Q = np.outer(np.sin(s), r)[None]
        out = oracle_mod.stp(N, physics, Q, dt, h, params=par[None], coef_per_element=True)
        exact = np.outer((np.cos(s - c * dt) - np.cos(s)) / (c * dt), r)
        errs.append(np.abs(out["qavg"][0] - exact).max())
    rates = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
    assert min(rates) > N + 1 - 0.4, (errs, rates)


# ------------------------------------------------------------------------------------------------ invariants
@pytest.mark.parametrize("kind", ["acoustic", "elastic", "generic_A"])
def test_linearity(oracle_mod, kind):
    N = 3
    b1 = _small_case(kind.replace("_A", ""), N, 5, with_A=kind.endswith("_A"))
    b2 = _small_case(kind.replace("_A", ""), N, 5, with_A=kind.endswith("_A"))
    b2.Q = np.random.default_rng(77).standard_normal(b1.Q.shape)
    a, c = 0.7, -1.9
    b3 = _small_case(kind.replace("_A", ""), N, 5, with_A=kind.endswith("_A"))
    b3.Q = a * b1.Q + c * b2.Q
    o1, o2, o3 = (run_oracle(oracle_mod, b) for b in (b1, b2, b3))
    for key in o1:
        comb = a * o1[key] + c * o2[key]
        assert np.max(np.abs(o3[key] - comb)) < 1e-12 * max(1, np.abs(comb).max())


@pytest.mark.parametrize("kind", ["acoustic", "elastic", "generic"])
def test_constant_state_zero_update(oracle_mod, kind):
    N = 4
    b = _small_case(kind, N, 6)
    b.Q = np.broadcast_to(np.random.default_rng(1).standard_normal((b.nelem, 1, b.m)), b.Q.shape).copy()
    out = run_oracle(oracle_mod, b)
    assert np.max(np.abs(out["qavg"] - b.Q)) < 1e-13
    assert np.max(np.abs(out["favg"])) < 1e-11
    n2 = (N + 1) ** 2
    for f in range(6):
        assert np.max(np.abs(out["qface"][:, f] - b.Q[:, :n2])) < 1e-13


@pytest.mark.parametrize("kind", ["acoustic", "elastic", "generic_A"])
def test_fig1_equals_fig5(oracle_mod, kind):
    """Fig. 1 accumulates favg over the Taylor terms; Fig. 5 recomputes it from q-bar by linearity."""
    for N in (2, 5):
        b = _small_case(kind.replace("_A", ""), N, 8, with_A=kind.endswith("_A"))
        out = run_oracle(oracle_mod, b, fig5=True)
        scale = np.abs(out["favg"]).max()
        assert np.max(np.abs(out["favg"] - out["favg_fig5"])) < 1e-13 * scale


def test_axis_permutation(oracle_mod):
    """Cyclic relabelling x->y->z->x of space, velocity and stress components permutes the outputs."""
    N = 3
    n = N + 1
    b = W.elastic_batch(N, 2, 11)
    out = run_oracle(oracle_mod, b)
    # new coordinates: x' = z, y' = x, z' = y (so node (z,y,x) of the new element is (y', x', z') ...)
    perm_q = np.array([2, 0, 1, 5, 3, 4, 8, 6, 7])  # new quantity j takes old quantity perm_q[j]

    def permute_nodes(a):  # a [E, n^3, ...]: new[z', y', x'] = old[z=y', y=x', x=z']
        sh = a.shape
        a = a.reshape(sh[0], n, n, n, *sh[2:])
        # old axes (z, y, x); new (z', y', x') = (old y, old x, old z)
        a = np.moveaxis(a, (1, 2, 3), (3, 1, 2))
        return a.reshape(sh)

    b2 = W.elastic_batch(N, 2, 11)
    b2.Q = permute_nodes(b.Q)[..., perm_q]
    b2.params = permute_nodes(b.params)
    out2 = run_oracle(oracle_mod, b2)
    assert np.max(np.abs(out2["qavg"] - permute_nodes(out["qavg"])[..., perm_q])) < 1e-12
    # direction d' of the new frame is old direction: x' = z (2), y' = x (0), z' = y (1)
    for dn, do in ((0, 2), (1, 0), (2, 1)):
        ref = permute_nodes(out["favg"][:, do])[..., perm_q]
        assert np.max(np.abs(out2["favg"][:, dn] - ref)) < 1e-11 * np.abs(ref).max()


def test_preset_equals_generic(oracle_mod):
    N = 2
    b = W.elastic_batch(N, 2, 12)
    out = run_oracle(oracle_mod, b)
    B = np.stack([_node_B(oracle_mod, ELASTIC, b.params[e]) for e in range(b.nelem)])
    out2 = oracle_mod.stp(N, GENERIC, b.Q, b.dt, b.h, B=B)
    for key in out:
        assert np.max(np.abs(out[key] - out2[key])) < 1e-13 * max(1, np.abs(out[key]).max())


def test_dt_zero_and_small(oracle_mod):
    N = 3
    b = W.elastic_batch(N, 2, 13)
    b.dt = np.zeros(b.nelem)
    out = run_oracle(oracle_mod, b)
    assert np.array_equal(out["qavg"], b.Q)
    # favg -> V_d(Q) as dt -> 0
    for e in range(b.nelem):
        B3, _ = _batch_B3(oracle_mod, b, e)
        for d in range(3):
            ref = oracle_mod.apply_Vd(N, b.h[e], d, B3, b.Q[e])
            assert np.max(np.abs(out["favg"][e, d] - ref)) < 1e-12 * np.abs(ref).max()
    b.dt = np.full(b.nelem, 1e-9)
    out2 = run_oracle(oracle_mod, b)
    assert np.max(np.abs(out2["qavg"] - b.Q)) < 1e-6


def test_favg_scales_with_inverse_h(oracle_mod):
    """Outputs depend on dt/h only, except favg which carries one more factor 1/h."""
    N = 3
    b = W.elastic_batch(N, 2, 14)
    out = run_oracle(oracle_mod, b)
    b.h = b.h * 2.0
    b.dt = b.dt * 2.0
    out2 = run_oracle(oracle_mod, b)
    assert np.max(np.abs(out2["qavg"] - out["qavg"])) < 1e-12
    assert np.max(np.abs(out2["qface"] - out["qface"])) < 1e-12
    assert np.max(np.abs(2.0 * out2["favg"] - out["favg"])) < 1e-12 * np.abs(out["favg"]).max()


@pytest.mark.parametrize("N", [1, 3, 5])
def test_point_source_with_zero_operator(oracle_mod, N):
    """With A = B = 0 the predictor integrates the source: q(t) = Q + int_0^t S, S(t) a polynomial of
    degree N-1 with Taylor coefficients sigma^(o); the time average is computed here by exact polynomial
    integration."""
    m, n3 = 3, (N + 1) ** 3
    b = W.generic_batch(N, m, 2, 15)
    b.B = np.zeros_like(b.B)
    b.src = W.point_source(b, 16)
    out = run_oracle(oracle_mod, b)
    for e in range(b.nelem):
        P, a, sig = b.src[e, :n3], b.src[e, n3:n3 + m], b.src[e, n3 + m:]
        S = np.polynomial.Polynomial([sig[o] / math.factorial(o) for o in range(N)])
        dt = b.dt[e]
        Sint = S.integ()           # int_0^t S
        avg = (Sint.integ()(dt) - Sint.integ()(0.0)) / dt
        ref = b.Q[e] + np.outer(P, a) * avg
        assert np.max(np.abs(out["qavg"][e] - ref)) < 1e-13 * np.abs(ref).max()
        assert np.max(np.abs(out["favg"][e])) == 0.0


def test_point_source_enters_recursion(oracle_mod):
    """With a non-zero operator the source enters p_{o+1} = V p_o + S_o: compare with the dense
    recursion."""
    N, m = 2, 3
    b = W.generic_batch(N, m, 2, 17)
    b.src = W.point_source(b, 18)
    out = run_oracle(oracle_mod, b)
    n3 = (N + 1) ** 3
    for e in range(b.nelem):
        B3, _ = _batch_B3(oracle_mod, b, e)
        V = dense.dense_V(N, m, b.h[e], B3)
        P, a, sig = b.src[e, :n3], b.src[e, n3:n3 + m], b.src[e, n3 + m:]
        p = [b.Q[e].ravel()]
        for o in range(N):
            p.append(V @ p[-1] + np.outer(P, a).ravel() * sig[o])
        dt = b.dt[e]
        ref = sum(dt ** o / math.factorial(o + 1) * po for o, po in enumerate(p))
        assert np.max(np.abs(out["qavg"][e].ravel() - ref)) < 1e-12 * np.abs(ref).max()


def test_fface_is_extrapolated_conservative_flux(oracle_mod):
    N, m = 2, 3
    b = W.generic_batch(N, m, 2, 19, with_A=True)
    out = run_oracle(oracle_mod, b)
    n = N + 1
    e0, e1 = oracle_mod.lagrange_at(n, 0.0), oracle_mod.lagrange_at(n, 1.0)
    for e in range(b.nelem):
        q = out["qavg"][e]
        for f in range(6):
            d = f // 2
            flux = np.einsum("ksr,kr->ks", b.A[e, d], q).reshape(n, n, n, m)
            ev = e1 if f % 2 else e0
            face = np.tensordot(flux, ev, axes=([2 - d], [0]))  # remaining axes in (slow, fast) order
            assert np.max(np.abs(out["fface"][e, f] - face.reshape(n * n, m))) < 1e-12 * np.abs(face).max()


def test_empty_batch(oracle_mod):
    b = W.elastic_batch(3, 0, 1)
    out = run_oracle(oracle_mod, b)
    assert out["qavg"].shape == (0, 64, 9)


# ------------------------------------------------------------------------------------------------ Gauss-Lobatto
def test_gll_nodes_closed_forms(oracle_mod):
    """Lobatto rules on [0, 1]: n = 3 is Simpson's rule; n = 4 has the nodes 1/2 -+ sqrt(5)/10 with weights
    1/12, 5/12; n = 5 has 1/2 -+ sqrt(21)/14 and the weights 1/20, 49/180, 16/45."""
    x, w = oracle_mod.gll_nodes(3)
    assert np.allclose(x, [0, 0.5, 1], atol=1e-15) and np.allclose(w, [1 / 6, 2 / 3, 1 / 6], atol=1e-15)
    x, w = oracle_mod.gll_nodes(4)
    s5 = math.sqrt(5) / 10
    assert np.allclose(x, [0, 0.5 - s5, 0.5 + s5, 1], atol=1e-15)
    assert np.allclose(w, [1 / 12, 5 / 12, 5 / 12, 1 / 12], atol=1e-15)
    x, w = oracle_mod.gll_nodes(5)
    s21 = math.sqrt(21) / 14
    assert np.allclose(x, [0, 0.5 - s21, 0.5, 0.5 + s21, 1], atol=1e-15)
    assert np.allclose(w, [1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20], atol=1e-15)


@pytest.mark.parametrize("n", [2, 3, 4, 6, 8, 10])
def test_gll_quadrature_degree_is_2n_minus_3(oracle_mod, n):
    x, w = oracle_mod.gll_nodes(n)
    for p in range(2 * n - 2):
        assert abs(np.dot(w, x ** p) - 1.0 / (p + 1)) < 1e-14, p
    # one degree higher the rule errs by exactly the Lobatto remainder term (f^(2n-2) is constant here):
    # n (n-1)^3 2^(2n-1) ((n-2)!)^4 / ((2n-1) ((2n-2)!)^3) times f^(2n-2) of x^(2n-2) mapped to [-1, 1]
    f = math.factorial
    rem = n * (n - 1) ** 3 * 2 ** (2 * n - 1) * f(n - 2) ** 4 / ((2 * n - 1) * f(2 * n - 2) ** 3)
    rem *= 0.5 * f(2 * n - 2) / 2 ** (2 * n - 2)
    err = np.dot(w, x ** (2 * n - 2)) - 1.0 / (2 * n - 1)
    assert abs(err / rem - 1.0) < 1e-5, (err, rem)


@pytest.mark.parametrize("N", [1, 3, 7])
def test_gll_predictor_matches_dense_series(oracle_mod, N):
    """With Gauss-Lobatto nodes the predictor is the truncated series of the dense operator built from the
    Lobatto derivative matrix (numpy's polynomial routines on the oracle's Lobatto nodes)."""
    n, m = N + 1, 9
    xi, _ = oracle_mod.gll_nodes(n)
    D = np.zeros((n, n))
    for j in range(n):
        others = np.delete(xi, j)
        coef = np.poly(others) / np.prod(xi[j] - others)
        D[:, j] = np.polyval(np.polyder(coef), xi)
    rng = np.random.default_rng(40 + N)
    par = np.array([2.4, 2.1, 1.3])
    Q = rng.standard_normal((1, n ** 3, m))
    h, dt = 0.7, 0.01
    out = oracle_mod.stp(N, ELASTIC, Q, dt, h, params=par[None], coef_per_element=True, nodes=1)
    B3 = np.broadcast_to(oracle_mod.preset_B(ELASTIC, par)[:, None], (3, n ** 3, m, m))
    Vds = [dense.dense_Vd(N, m, h, d, B3, None, D) for d in range(3)]
    V = sum(Vds)
    terms = [Q[0].ravel()]
    for o in range(1, N + 1):
        terms.append(V @ terms[-1])
    qbar = sum(dt ** o / math.factorial(o + 1) * t for o, t in enumerate(terms))
    assert np.abs(out["qavg"][0].ravel() - qbar).max() < 1e-12 * np.abs(qbar).max()
    # Lobatto faces are the boundary nodes themselves
    q = out["qavg"][0].reshape(n, n, n, m)
    assert np.array_equal(out["qface"][0, 0].reshape(n, n, m), q[:, :, 0])
    assert np.array_equal(out["qface"][0, 5].reshape(n, n, m), q[n - 1])
