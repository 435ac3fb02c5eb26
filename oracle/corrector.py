"""Oracle of the ADER-DG corrector step on a periodic Cartesian mesh (test infrastructure only).

Only tests/, the package's smoke check and the benchmark's CPU leg use this module; the product never
imports it. Plain numpy in FP64, written from the paper's scheme (Sec. II-A): the time-integrated
semi-discrete update of Eq. (5) -- the corrector -- uses the predictor's outputs (the time-averaged DOFs
q-bar, their face projections and the face projections of the conservative flux) and a numerical flux that
is linear in the face states. The paper leaves that flux open; this oracle takes the reading (R22 in the
design notes):

  strong form, Gauss-Legendre collocation, diagonal mass matrix h^3 w_k1 w_k2 w_k3 (w: weights on [0,1]);
  for the face f of an element with outward normal n = s e_d (s = -1 for the lower face, +1 for the upper)
  and the states q- (own face projection of q-bar), q+ (the neighbour's projection on the same face),
  F-/F+ (the face projections of A_d q-bar), the face correction entering the element is

      C_f = 1/2 alpha (q+ - q-) - 1/2 s (F+ - F-) - 1/2 s Bbar_d (q+ - q-),

  Bbar_d = (B_d(e) + B_d(neighbour)) / 2, alpha = max(alpha(e), alpha(neighbour)) (Rusanov), with alpha the
  fastest wave speed of the element: sqrt(K/rho) acoustic, sqrt((lambda+2 mu)/rho) elastic, and for generic
  coefficients the bound max_d ||A_d + B_d||_inf (maximum absolute row sum). Curvilinear elastic elements with
  affine geometry (12 parameters per element: the material and the constant metric G[d][j] = h dxi_d/dx_j)
  take B_d = sum_j G[d][j] M_j and alpha = sqrt((lambda+2 mu)/rho) max_d |G[d][:]|_2 (the spectral radius of
  B_d in its worst direction): the scheme is the Cartesian one in the reference coordinates of the mesh.
  Curved elements (the 12 parameters per node) take, at every face point, the parameters extrapolated from
  each side's nodes with the face vectors l_j(0), l_j(1), B_d and alpha of those parameters on each side,
  Bbar_d the mean of the two sides' B_d and alpha the larger speed.

  q(t_{n+1})_k = q(t_n)_k + dt sum_d favg[d]_k + dt sum_f l_{k_d}(x_f) / (h w_{k_d}) C_f(k_a, k_b)

  where favg[d] = V_d(q-bar) is the predictor's time-averaged volume term, l_j(x_f) the Lagrange basis at the
  face (0 or 1 along d) and (k_a, k_b) the face node of k. For a single linear wave with speed a > 0 along
  x this reduces to the upwind flux (the lower face receives a (q+ - q-), the upper face nothing).

Elements are numbered e = (iz * ny + iy) * nx + ix; the mesh is periodic in all three directions. Material
or coefficients are per element: presets [E, np] (rho, K) or (rho, lambda, mu); generic A, B [E, 3, m, m].
"""
from __future__ import annotations

import hashlib

import numpy as np

import oracle

ACOUSTIC, ELASTIC, GENERIC, ELASTIC_CURV = 0, 1, 2, 3


def gl_weights01(n: int, nodes: int = 0) -> np.ndarray:
    """Quadrature weights on [0, 1] of the node family (0 Gauss-Legendre, 1 Gauss-Lobatto)."""
    return oracle.nodes_of(n, nodes)[1]


def element_B(physics: int, params=None, B=None):
    """B_d [E, 3, m, m] per element: presets from the material (same matrices as the predictor), generic as
    given."""
    if physics == GENERIC:
        return np.asarray(B, dtype=np.float64)
    params = np.asarray(params, dtype=np.float64)
    return np.stack([oracle.preset_B(physics, p) for p in params])


def wave_speed(physics: int, params=None, A=None, B=None) -> np.ndarray:
    """alpha per element (see the module docstring)."""
    if physics == ACOUSTIC:
        return np.sqrt(params[:, 1] / params[:, 0])
    if physics == ELASTIC:
        return np.sqrt((params[:, 1] + 2 * params[:, 2]) / params[:, 0])
    if physics == ELASTIC_CURV:
        G = np.asarray(params[:, 3:], dtype=np.float64).reshape(-1, 3, 3)
        return np.sqrt((params[:, 1] + 2 * params[:, 2]) / params[:, 0]) * np.linalg.norm(G, axis=2).max(axis=1)
    M = np.asarray(B, dtype=np.float64) + (0.0 if A is None else np.asarray(A, dtype=np.float64))
    return np.abs(M).sum(axis=-1).max(axis=(1, 2))


def lagrange(xi, x: float) -> np.ndarray:
    """l_j(x) for the nodes xi (product formula)."""
    n = len(xi)
    return np.array([np.prod([(x - xi[k]) / (xi[j] - xi[k]) for k in range(n) if k != j]) for j in range(n)])


def face_values(u, n: int, nodes: int = 0) -> np.ndarray:
    """Nodal data u [E, n^3, c] extrapolated to the six faces [E, 6, n, n, c] (face node (a, b) = the two other
    axes, slower first) with the face vectors l_j(0), l_j(1) along the normal."""
    E = u.shape[0]
    U = np.asarray(u, dtype=np.float64).reshape(E, n, n, n, -1)  # [e][z][y][x][c]
    xi, _ = oracle.nodes_of(n, nodes)
    l0, l1 = lagrange(xi, 0.0), lagrange(xi, 1.0)
    out = np.empty((E, 6, n, n, U.shape[-1]))
    for side, lv in ((0, l0), (1, l1)):
        out[:, 0 + side] = np.einsum("j,ezyjc->ezyc", lv, U)  # x faces: (a, b) = (z, y)
        out[:, 2 + side] = np.einsum("j,ezjxc->ezxc", lv, U)  # y faces: (a, b) = (z, x)
        out[:, 4 + side] = np.einsum("j,ejyxc->eyxc", lv, U)  # z faces: (a, b) = (y, x)
    return out


def curved_speed(P) -> float:
    """alpha of one face point's curvilinear parameters (rho, lambda, mu, G)."""
    G = np.asarray(P[3:]).reshape(3, 3)
    return float(np.sqrt((P[1] + 2 * P[2]) / P[0]) * np.linalg.norm(G, axis=1).max())


_face_cache: dict = {}


def curved_face_coefficients(params, n: int, nodes: int = 0):
    """B_{d_f} [E, 6, n, n, 9, 9] and alpha [E, 6, n, n] of the parameters extrapolated to every face point
    (memoised on the parameter values: they do not change between steps)."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    key = (hashlib.sha1(params.tobytes()).hexdigest(), params.shape, n, nodes)
    if key not in _face_cache:
        fp = face_values(params, n, nodes)
        E = fp.shape[0]
        Bf = np.empty((E, 6, n, n, 9, 9))
        af = np.empty((E, 6, n, n))
        for e in range(E):
            for f in range(6):
                for ia in range(n):
                    for ib in range(n):
                        P = fp[e, f, ia, ib]
                        Bf[e, f, ia, ib] = oracle.preset_B(ELASTIC_CURV, P)[f // 2]
                        af[e, f, ia, ib] = curved_speed(P)
        _face_cache.clear()
        _face_cache[key] = (Bf, af)
    return _face_cache[key]


def neighbour(e: int, d: int, s: int, nx: int, ny: int, nz: int) -> int:
    """The periodic neighbour of element e across its face along d on side s (-1 lower, +1 upper)."""
    ix, iy, iz = e % nx, (e // nx) % ny, e // (nx * ny)
    if d == 0:
        ix = (ix + s) % nx
    elif d == 1:
        iy = (iy + s) % ny
    else:
        iz = (iz + s) % nz
    return (iz * ny + iy) * nx + ix


def correct(N: int, physics: int, grid, Q, favg, qface, dt: float, h: float, params=None, A=None, B=None,
            fface=None, favg_sum: bool = False, nodes: int = 0):
    """q(t_{n+1}) [E, n^3, m] from q(t_n) and the predictor outputs of every element of the mesh.

    Q [E, n^3, m]; favg [E, 3, n^3, m] (or [E, n^3, m] with favg_sum); qface, fface [E, 6, n^2, m] with the
    faces ordered x-, x+, y-, y+, z-, z+ and the face nodes (a, b) = the two other axes, slower first.
    Presets take params [E, np] (np = 2, 3, or 12 for affine curvilinear elements); curved curvilinear elements
    take params [E, n^3, 12]."""
    nx, ny, nz = grid
    n = N + 1
    E = nx * ny * nz
    Q = np.asarray(Q, dtype=np.float64).reshape(E, n, n, n, -1)  # [e][z][y][x][s]
    m = Q.shape[-1]
    fa = np.asarray(favg, dtype=np.float64)
    vol = fa.reshape(E, n ** 3, m) if favg_sum else fa.reshape(E, 3, n ** 3, m).sum(axis=1)
    qf = np.asarray(qface, dtype=np.float64).reshape(E, 6, n, n, m)
    ff = None if fface is None else np.asarray(fface, dtype=np.float64).reshape(E, 6, n, n, m)
    curved = physics == ELASTIC_CURV and np.asarray(params).ndim == 3
    if curved:
        Bf, af = curved_face_coefficients(params, n, nodes)
    else:
        Bd = element_B(physics, params, B)
        alpha = wave_speed(physics, params, A, B)
    xi, w = oracle.nodes_of(n, nodes)
    l0 = lagrange(xi, 0.0)
    l1 = lagrange(xi, 1.0)
    out = Q + dt * vol.reshape(E, n, n, n, m)
    for e in range(E):
        for d in range(3):
            for side, s in ((0, -1), (1, 1)):
                f = 2 * d + side
                nb = neighbour(e, d, s, nx, ny, nz)
                fo = 2 * d + (1 - side)  # the neighbour's face on the shared plane
                jump = qf[nb, fo] - qf[e, f]  # [a][b][m]
                if curved:  # B_d and alpha of each side's extrapolated parameters at every face point
                    Bbar = 0.5 * (Bf[e, f] + Bf[nb, fo])  # [a][b][m][m]
                    a = np.maximum(af[e, f], af[nb, fo])[..., None]
                    C = 0.5 * a * jump - 0.5 * s * np.einsum("abrc,abc->abr", Bbar, jump)
                else:
                    Bbar = 0.5 * (Bd[e, d] + Bd[nb, d])
                    a = max(alpha[e], alpha[nb])
                    C = 0.5 * a * jump - 0.5 * s * jump @ Bbar.T
                if ff is not None:
                    C -= 0.5 * s * (ff[nb, fo] - ff[e, f])
                lift = (l1 if side else l0) / (h * w)  # [k_d]
                # face node (a, b) = the two other axes, slower first; scatter along the normal axis
                if d == 0:    # (a, b) = (z, y), normal x
                    out[e] += dt * lift[None, None, :, None] * C[:, :, None, :]
                elif d == 1:  # (a, b) = (z, x), normal y
                    out[e] += dt * lift[None, :, None, None] * C[:, None, :, :]
                else:         # (a, b) = (y, x), normal z
                    out[e] += dt * lift[:, None, None, None] * C[None, :, :, :]
    return out.reshape(E, n ** 3, m)


def ader_step(N: int, physics: int, grid, Q, dt: float, h: float, params=None, A=None, B=None, nodes: int = 0):
    """One full ADER-DG step: the oracle predictor on every element, then the corrector. Per-element
    coefficients (params [E, np] or A, B [E, 3, m, m]), or curvilinear parameters per node [E, n^3, 12];
    nodes 0 Gauss-Legendre, 1 Gauss-Lobatto."""
    per_elem = not (physics == ELASTIC_CURV and np.asarray(params).ndim == 3)
    pred = oracle.stp(N, physics, Q, dt, h, params=params, A=A, B=B, coef_per_element=per_elem, nodes=nodes)
    return correct(N, physics, grid, Q, pred["favg"], pred["qface"], dt, h, params=params, A=A, B=B,
                   fface=pred.get("fface"), nodes=nodes)
