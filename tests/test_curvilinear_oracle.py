"""Pins of the oracle's curvilinear elastic physics (no GPU).

Curvilinear elements carry the metric terms G[d][j] = h dxi_d/dx_j per node, and the oracle forms
B_d = sum_j G[d][j] M_j from the Cartesian elastic matrices M_j (the chain rule). The pins:
  - spectrum: sum_d kappa_d B_d has the elastic wave speeds scaled by |G^T kappa|;
  - G = I reproduces the Cartesian elastic predictor;
  - an affine element (constant, non-symmetric G) reproduces a polynomial plane wave of the physical
    coordinates exactly: q-bar, every favg[d] (whose split over d involves J and G) and the faces;
  - a curved element converges to the exact time average of a smooth plane wave at order N + 1.
"""
import math

import numpy as np
import pytest

import dense
from paper_2003_12787_amd import workloads as W

ELASTIC, ELASTIC_CURV = 1, 3


def _J(seed):
    """A non-symmetric Jacobian with positive determinant."""
    rng = np.random.default_rng(seed)
    J = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    assert np.linalg.det(J) > 0.2 and np.abs(J - J.T).max() > 0.05
    return J


def test_curvilinear_spectrum(oracle_mod):
    rng = np.random.default_rng(5)
    for t in range(5):
        rho, lam, mu = rng.uniform(2, 3), rng.uniform(1, 4), rng.uniform(1, 3)
        G = np.linalg.inv(_J(100 + t))
        B = oracle_mod.preset_B(ELASTIC_CURV, np.concatenate([[rho, lam, mu], G.ravel()]))
        kappa = rng.standard_normal(3)
        ev = np.sort(np.linalg.eigvals(np.einsum("d,dij->ij", kappa, B)).real)
        k = np.linalg.norm(G.T @ kappa)
        cp, cs = math.sqrt((lam + 2 * mu) / rho), math.sqrt(mu / rho)
        assert np.allclose(ev, k * np.array([-cp, -cs, -cs, 0, 0, 0, cs, cs, cp]), atol=1e-10)


def test_identity_metric_is_cartesian(oracle_mod):
    N = 3
    b = W.elastic_batch(N, 4, 17)
    par = np.concatenate([b.params, np.broadcast_to(np.eye(3).ravel(), b.params.shape[:-1] + (9,))], axis=-1)
    ref = oracle_mod.stp(N, ELASTIC, b.Q, b.dt, b.h, params=b.params)
    got = oracle_mod.stp(N, ELASTIC_CURV, b.Q, b.dt, b.h, params=par)
    for k in ("qavg", "favg", "qface"):
        assert np.abs(got[k] - ref[k]).max() <= 1e-13 * np.abs(ref[k]).max(), k


def _plane_wave(k, wave, rng):
    rho, lam, mu = 2.5, 2.0, 1.5
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
    return np.array([rho, lam, mu]), c, r


@pytest.mark.parametrize("N", [1, 2, 3, 5])
@pytest.mark.parametrize("wave", ["P", "S"])
def test_affine_element_polynomial_plane_wave_exact(oracle_mod, N, wave):
    """x = origin + h J xi: a plane wave r f(k.x - c t) with f of degree N is a polynomial of degree N in xi,
    so the predictor is exact. favg[d] = -(k . J e_d) (sum_j G[d][j] M_j r) [f(s) - f(s - c dt)] / (c dt)."""
    rng = np.random.default_rng(60 + N)
    n = N + 1
    k = rng.standard_normal(3)
    k /= np.linalg.norm(k)
    par, c, r = _plane_wave(k, wave, rng)
    J = _J(70 + N)
    G = np.linalg.inv(J)
    h, dt = 0.7, 0.04
    origin = np.array([0.2, -0.4, 0.1])
    xi, _ = dense.np_nodes(n)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")
    ref = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    s = (origin[None, :] + h * ref @ J.T) @ k
    f = np.polynomial.Polynomial(rng.standard_normal(N + 1))
    F = f.integ()
    Q = np.outer(f(s), r)[None]
    pc = np.concatenate([par, G.ravel()])
    out = oracle_mod.stp(N, ELASTIC_CURV, Q, dt, h, params=pc[None], coef_per_element=True)
    qbar = np.outer((F(s) - F(s - c * dt)) / (c * dt), r)
    scale = np.abs(qbar).max()
    assert np.abs(out["qavg"][0] - qbar).max() < 1e-11 * max(1, scale)
    M = oracle_mod.preset_B(ELASTIC, par)
    g = (f(s) - f(s - c * dt)) / (c * dt)
    for d in range(3):
        Bd = np.einsum("j,jab->ab", G[d], M)
        fd = -(k @ J[:, d]) * np.outer(g, Bd @ r)
        assert np.abs(out["favg"][0, d] - fd).max() < 1e-10 * max(1, np.abs(fd).max()), d
    for fidx in range(6):
        axis, side = fidx // 2, fidx % 2
        A_, B_ = np.meshgrid(xi, xi, indexing="ij")
        coords = np.zeros((n * n, 3))
        other = [a for a in (2, 1, 0) if a != axis]  # slower axis first: z, y, x
        coords[:, axis] = float(side)
        coords[:, other[0]] = A_.ravel()
        coords[:, other[1]] = B_.ravel()
        sf = (origin[None, :] + h * coords @ J.T) @ k
        qf = np.outer((F(sf) - F(sf - c * dt)) / (c * dt), r)
        assert np.abs(out["qface"][0, fidx] - qf).max() < 1e-10 * max(1, scale)


def test_transposed_metric_fails_the_affine_pin(oracle_mod):
    """The affine pin detects an orientation mistake: G transposed gives a different q-bar."""
    N, n = 2, 3
    rng = np.random.default_rng(9)
    k = np.array([0.6, 0.0, 0.8])
    par, c, r = _plane_wave(k, "P", rng)
    J = _J(71)
    G = np.linalg.inv(J)
    xi, _ = dense.np_nodes(n)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")
    s = (np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) @ J.T) @ k
    Q = np.outer(s ** 2, r)[None]
    good = oracle_mod.stp(N, ELASTIC_CURV, Q, 0.05, 1.0, params=np.concatenate([par, G.ravel()])[None],
                          coef_per_element=True)
    bad = oracle_mod.stp(N, ELASTIC_CURV, Q, 0.05, 1.0, params=np.concatenate([par, G.T.ravel()])[None],
                         coef_per_element=True)
    assert np.abs(good["qavg"] - bad["qavg"]).max() > 1e-3


@pytest.mark.parametrize("N", [2, 3])
def test_curved_element_converges(oracle_mod, N):
    """One element of side h at a fixed place of the deformed unit box (the map stays fixed while the element
    shrinks); a smooth P plane wave; the error of q-bar against the exact time average at the mapped nodes
    falls at order >= N + 1 as h halves."""
    rng = np.random.default_rng(80)
    k = np.array([1.0, 2.0, 2.0]) / 3.0
    par, c, r = _plane_wave(k, "P", rng)
    w = 2 * math.pi
    errs = []
    for h in (0.1, 0.05):
        t, _ = dense.np_nodes(N + 1)
        Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
        xi = np.array([0.3, 0.1, 0.6]) + h * np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        x, J = W.curved_map(xi, (1.0, 1.0, 1.0), 0.3)
        G = np.linalg.inv(J)  # xi = origin + h xi_loc, so h dxi_loc_d/dx_j = dxi_d/dx_j = (J^-1)[d][j]
        s = x @ k
        Q = np.outer(np.sin(w * s), r)[None]
        par_n = np.concatenate([np.broadcast_to(par, (len(s), 3)), G.reshape(-1, 9)], axis=1)[None]
        dt = 0.2 * h / ((2 * N + 1) * c)
        out = oracle_mod.stp(N, ELASTIC_CURV, Q, dt, h, params=par_n)
        exact = np.outer((np.cos(w * (s - c * dt)) - np.cos(w * s)) / (w * c * dt), r)
        errs.append(np.abs(out["qavg"][0] - exact).max())
    rate = math.log2(errs[0] / errs[1])
    print(f"curved element N={N}: errors {errs}, rate {rate:.2f}")
    assert rate > N + 1 - 0.5, (errs, rate)
