"""Seeded synthetic inputs shaped like the paper's workloads (elastic / acoustic waves).

This module holds input recipes only: random materials, random or plane-wave DOFs, element sizes and the
CFL time-step rule. It contains none of the predictor's arithmetic, and both the oracle tests and the HIP
path draw their inputs from it. Everything is generated in FP64 with ``numpy.random.default_rng(seed)``;
reduced-precision runs round these values to the I/O dtype and the oracle is then run on the rounded
values.

The paper's benchmark (LOH1 on a curvilinear mesh, m = 21) is not available; these inputs stand in for
it with the same physics (first-order elastic velocity-stress, three material parameters per node) and, for
the curvilinear elements, nine geometry parameters per node from a smooth synthetic mesh deformation.

Quantity order: acoustic (p, v_x, v_y, v_z), params (rho, K); elastic (v_x, v_y, v_z, s_xx, s_yy, s_zz,
s_xy, s_yz, s_xz), params (rho, lambda, mu); curvilinear elastic params (rho, lambda, mu, G[0][0], ...,
G[2][2]) with G[d][j] = h dxi_d/dx_j. Nodal arrays are [element][z][y][x][quantity].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ACOUSTIC, ELASTIC, GENERIC, ELASTIC_CURV = 0, 1, 2, 3
NQUANT = {ACOUSTIC: 4, ELASTIC: 9, ELASTIC_CURV: 9}
NPARAM = {ACOUSTIC: 2, ELASTIC: 3, ELASTIC_CURV: 12}
SEED0 = 2003127870


@dataclasses.dataclass
class Batch:
    """One uniform-class batch of elements (FP64 host arrays)."""
    N: int
    m: int
    physics: int
    Q: np.ndarray                    # [E, n^3, m]
    dt: np.ndarray                   # [E]
    h: np.ndarray                    # [E]
    params: np.ndarray | None = None  # presets: [E, n^3, np] or [E, np]
    A: np.ndarray | None = None       # generic: [E, 3, n^3, m, m] or [E, 3, m, m]
    B: np.ndarray | None = None       # generic: same layout as A
    src: np.ndarray | None = None     # [E, n^3 + m + N]
    coef_per_element: bool = False

    @property
    def nelem(self) -> int:
        return self.Q.shape[0]


def coef_abi(M: np.ndarray | None, per_element: bool) -> np.ndarray | None:
    """Per-node coefficient matrices [E, 3, n^3, m, m] (the generators' and the oracle's layout) in the
    library's layout [E, 3, m, m, n^3] (node fastest); per-element matrices [E, 3, m, m] are unchanged."""
    if M is None or per_element:
        return M
    return np.ascontiguousarray(np.moveaxis(M, 2, -1))


def _node_positions(n: int) -> np.ndarray:
    """Gauss-Legendre points on [0, 1] from numpy's library routine (used only to sample waves)."""
    x, _ = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0)


def elastic_material(rng, shape):
    """rho ~ U[2,3], lambda ~ U[1,4], mu ~ U[1,3] (per node or per element)."""
    rho = rng.uniform(2.0, 3.0, shape)
    lam = rng.uniform(1.0, 4.0, shape)
    mu = rng.uniform(1.0, 3.0, shape)
    return np.stack([rho, lam, mu], axis=-1)


def cfl_dt(N: int, h: float, c: float, cfl: float = 0.4) -> float:
    """dt = cfl * h / ((2N+1) c), the time-step rule of the workloads."""
    return cfl * h / ((2 * N + 1) * c)


def elastic_batch(N: int, nelem: int, seed: int, h: float = 1.0, per_node: bool = True,
                  q_scale: float = 1.0) -> Batch:
    """Elastic waves, m = 9: per-node material, Q ~ N(0, 1), dt from the fastest P-wave in the batch."""
    rng = np.random.default_rng(seed)
    n3 = (N + 1) ** 3
    par = elastic_material(rng, (nelem, n3) if per_node else (nelem,))
    Q = q_scale * rng.standard_normal((nelem, n3, 9))
    cp = np.sqrt((par[..., 1] + 2 * par[..., 2]) / par[..., 0]).max() if nelem else 1.0
    dt = np.full(nelem, cfl_dt(N, h, cp))
    return Batch(N, 9, ELASTIC, Q, dt, np.full(nelem, h), params=par, coef_per_element=not per_node)


def grid_of(nelem: int):
    """(nx, ny, nz) of the box the curvilinear workloads tile: nx = 2 ny = 2 nz when nelem = 2 k^3 (65536 ->
    64 x 32 x 32), else the smallest cube holding nelem elements."""
    k = round((nelem / 2) ** (1.0 / 3.0))
    if 2 * k ** 3 == nelem:
        return 2 * k, k, k
    g = max(1, int(round(nelem ** (1.0 / 3.0))))
    while g ** 3 < nelem:
        g += 1
    return g, g, g


def _map_terms(xi, L, eps, sin, cos):
    """The deformation of curved_map on coordinate arrays xi = [xi_0, xi_1, xi_2] (broadcastable; numpy or
    torch, with their sin and cos): returns x as a list of 3 arrays and J as nested lists J[i][j]."""
    a = min(L) / (2 * math.pi)
    k = [2 * math.pi / Lj for Lj in L]
    s = [sin(k[j] * xi[j]) for j in range(3)]
    c = [cos(k[j] * xi[j]) for j in range(3)]
    x, J = [], [[None] * 3 for _ in range(3)]
    for i in range(3):
        j1, j2 = [j for j in range(3) if j != i]
        x.append(xi[i] + eps * a * s[j1] * s[j2])
        J[i][i] = 1.0
        J[i][j1] = eps * a * k[j1] * c[j1] * s[j2]
        J[i][j2] = eps * a * k[j2] * s[j1] * c[j2]
    return x, J


def curved_map(xi, L, eps):
    """A smooth, periodic deformation of the box [0, L_0] x [0, L_1] x [0, L_2] (xi [..., 3] -> x [..., 3]) and
    its Jacobian J[..., i, j] = dx_i/dxi_j:
        x_i = xi_i + eps a prod_{j != i} sin(2 pi xi_j / L_j),   a = min(L) / (2 pi).
    Each off-diagonal entry of J is at most eps in magnitude, so J is invertible for eps < 1/2."""
    x, J = _map_terms([xi[..., j] for j in range(3)], [float(v) for v in L], eps, np.sin, np.cos)
    Jm = np.zeros(xi.shape + (3,))
    for i in range(3):
        for j in range(3):
            Jm[..., i, j] = J[i][j]
    return np.stack(x, axis=-1), Jm


def _inverse3(J):
    """Inverse of 3 x 3 matrices given as nested lists J[i][j] of equally shaped arrays (adjugate / det)."""
    c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1]
    c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2]
    c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0]
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02
    return [[c00 / det, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det, (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det],
            [c01 / det, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det, (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det],
            [c02 / det, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det, (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det]]


def _element_coords(N, grid, h, e, t):
    """Global reference coordinates [xi_0, xi_1, xi_2], each [E, n^3], of the nodes of elements e of the grid;
    t are the 1D node positions."""
    nx, ny, _ = grid
    n = N + 1
    ix, iy, iz = e % nx, (e // nx) % ny, e // (nx * ny)
    tz, ty, tx = t.reshape(n, 1, 1), t.reshape(1, n, 1), t.reshape(1, 1, n)
    zero = 0 * tx * ty * tz
    node = [(tx + zero).reshape(1, -1), (ty + zero).reshape(1, -1), (tz + zero).reshape(1, -1)]
    return [(ix[:, None] + node[0]) * h, (iy[:, None] + node[1]) * h, (iz[:, None] + node[2]) * h]


def curvilinear_geometry(N: int, grid, h: float, eps: float, elements=None):
    """Node positions x [E, n^3, 3] and metric terms G [E, n^3, 3, 3] (G[d][j] = h dxi_d/dx_j = the inverse of
    dx/dxi_global) of the elements of a grid (nx, ny, nz) of cubes of side h under curved_map; element
    e = (iz ny + iy) nx + ix, nodes (z, y, x) at Gauss-Legendre points."""
    nx, ny, nz = grid
    e = np.arange(nx * ny * nz) if elements is None else np.asarray(elements)
    xi = _element_coords(N, grid, h, e, _node_positions(N + 1))
    x, J = _map_terms(xi, (nx * h, ny * h, nz * h), eps, np.sin, np.cos)
    Gl = _inverse3(J)
    X = np.stack(x, axis=-1)
    G = np.empty(X.shape + (3,))
    for i in range(3):
        for j in range(3):
            G[..., i, j] = Gl[i][j]
    return X, G


def curvilinear_device(N: int, nelem: int, seed: int, device="cuda", h: float = 1.0, eps: float = 0.2):
    """The curvilinear workload of curvilinear_batch generated on the device (torch, FP64 arithmetic, FP32
    results): the same grid, map and metric; material rho ~ U[2,3], lambda ~ U[1,4], mu ~ U[1,3] and
    Q ~ N(0, 1) from a torch generator seeded with `seed`. Returns (Q [E, n^3, 9], params [E, n^3, 12], dt)."""
    import torch
    grid = grid_of(nelem)
    n3 = (N + 1) ** 3
    t = torch.from_numpy(_node_positions(N + 1)).to(device)
    e = torch.arange(nelem, device=device, dtype=torch.float64)
    ef = torch.floor
    nx, ny, nz = grid
    ix = e - nx * ef(e / nx)
    iy = ef(e / nx) - ny * ef(e / (nx * ny))
    iz = ef(e / (nx * ny))
    tz, ty, tx = t.reshape(-1, 1, 1), t.reshape(1, -1, 1), t.reshape(1, 1, -1)
    zero = 0 * tx * ty * tz
    xi = [(ix[:, None] + (tx + zero).reshape(1, -1)) * h, (iy[:, None] + (ty + zero).reshape(1, -1)) * h,
          (iz[:, None] + (tz + zero).reshape(1, -1)) * h]
    _, J = _map_terms(xi, (nx * h, ny * h, nz * h), eps, torch.sin, torch.cos)
    del xi
    Gl = _inverse3(J)
    del J
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    u = torch.rand((nelem, n3, 3), generator=g, device=device, dtype=torch.float64)
    params = torch.empty((nelem, n3, 12), device=device, dtype=torch.float32)
    params[..., 0] = 2.0 + u[..., 0]
    params[..., 1] = 1.0 + 3.0 * u[..., 1]
    params[..., 2] = 1.0 + 2.0 * u[..., 2]
    gmax = 0.0
    for d in range(3):
        gmax = max(gmax, float((Gl[d][0].abs() + Gl[d][1].abs() + Gl[d][2].abs()).max()))
        for j in range(3):
            params[..., 3 + 3 * d + j] = Gl[d][j]
    del Gl, u
    Q = torch.randn((nelem, n3, 9), generator=g, device=device, dtype=torch.float32)
    p = params.double()
    cp = float(torch.sqrt((p[..., 1] + 2 * p[..., 2]) / p[..., 0]).max())
    del p
    return Q, params, cfl_dt(N, h, cp * gmax)


def curvilinear_batch(N: int, nelem: int, seed: int, h: float = 1.0, eps: float = 0.2, per_node: bool = True,
                      q_scale: float = 1.0) -> Batch:
    """Elastic waves on curvilinear elements (m = 9, 12 parameters per node): the material of elastic_batch,
    the metric terms of curvilinear_geometry on grid_of(nelem), Q ~ N(0, 1). dt from the fastest P-wave
    times the largest row sum of |G| in the batch (the fastest reference-space speed). per_node = False
    keeps the first node's parameters for the whole element (an affine element)."""
    rng = np.random.default_rng(seed)
    n3 = (N + 1) ** 3
    grid = grid_of(nelem)
    _, G = curvilinear_geometry(N, grid, h, eps, elements=np.arange(nelem))
    mat = elastic_material(rng, (nelem, n3) if per_node else (nelem,))
    if not per_node:
        G = G[:, 0]
    par = np.concatenate([mat, G.reshape(G.shape[:-2] + (9,))], axis=-1)
    Q = q_scale * rng.standard_normal((nelem, n3, 9))
    cp = np.sqrt((mat[..., 1] + 2 * mat[..., 2]) / mat[..., 0]).max() if nelem else 1.0
    gmax = (np.abs(G[..., 0]) + np.abs(G[..., 1]) + np.abs(G[..., 2])).max() if nelem else 1.0
    dt = np.full(nelem, cfl_dt(N, h, cp * gmax))
    return Batch(N, 9, ELASTIC_CURV, Q, dt, np.full(nelem, h), params=par, coef_per_element=not per_node)


def acoustic_plane_wave_batch(N: int, nelem: int, seed: int, h: float = 1.0, noise: float = 1e-2,
                              grid: int | None = None) -> Batch:
    """Acoustic waves, m = 4: rho = 1, K_e ~ U[1,2] per element; Q is a smooth plane wave
    p = sin(k.x), v = k_hat p / (rho c_e), k = (2 pi / 8h) (1,2,2)/3, plus N(0, noise^2) per DOF.
    Elements sit on a cubic grid (grid^3 >= nelem, x fastest)."""
    rng = np.random.default_rng(seed)
    n = N + 1
    if grid is None:
        grid = max(1, int(round(nelem ** (1.0 / 3.0))))
        while grid ** 3 < nelem:
            grid += 1
    K = rng.uniform(1.0, 2.0, nelem)
    rho = np.ones(nelem)
    par = np.stack([rho, K], axis=-1)
    c = np.sqrt(K / rho)
    kvec = (2 * math.pi / (8 * h)) * np.array([1.0, 2.0, 2.0]) / 3.0
    khat = kvec / np.linalg.norm(kvec)
    xi = _node_positions(n)
    e = np.arange(nelem)
    ex, ey, ez = e % grid, (e // grid) % grid, e // (grid * grid)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")  # node (z, y, x)
    px = (ex[:, None] + X.reshape(1, -1)) * h
    py = (ey[:, None] + Y.reshape(1, -1)) * h
    pz = (ez[:, None] + Z.reshape(1, -1)) * h
    phase = kvec[0] * px + kvec[1] * py + kvec[2] * pz
    p = np.sin(phase)
    v = khat[None, None, :] * (p / (rho * c)[:, None])[:, :, None]
    Q = np.concatenate([p[..., None], v], axis=-1)
    Q = Q + noise * rng.standard_normal(Q.shape)
    dt = np.full(nelem, cfl_dt(N, h, c.max() if nelem else 1.0))
    return Batch(N, 4, ACOUSTIC, Q, dt, np.full(nelem, h), params=par, coef_per_element=True)


def elastic_plane_wave_batch(N: int, nelem: int, seed: int, h: float = 1.0, noise: float = 1e-2,
                             per_node: bool = True) -> Batch:
    """Elastic waves, m = 9, smooth fields: the per-node material of the elastic workloads, and Q a P-wave plus
    an S-wave of the reference material (rho, lambda, mu) = (2.5, 2.5, 2), both sin(k.x) with
    k = (2 pi / 8h) (1,2,2)/3, plus N(0, noise^2) per DOF. Elements sit on a cubic grid (x fastest). Q is
    smooth but not a solution for the sampled material; it is an input recipe for accuracy tests on smooth
    data."""
    rng = np.random.default_rng(seed)
    n = N + 1
    grid = max(1, int(round(nelem ** (1.0 / 3.0))))
    while grid ** 3 < nelem:
        grid += 1
    par = elastic_material(rng, (nelem, n ** 3) if per_node else (nelem,))
    rho0, lam0, mu0 = 2.5, 2.5, 2.0
    cp0, cs0 = math.sqrt((lam0 + 2 * mu0) / rho0), math.sqrt(mu0 / rho0)
    kvec = (2 * math.pi / (8 * h)) * np.array([1.0, 2.0, 2.0]) / 3.0
    khat = kvec / np.linalg.norm(kvec)
    a = np.cross(khat, [1.0, 0.0, 0.0])
    a /= np.linalg.norm(a)
    def voigt(S):  # (xx, yy, zz, xy, yz, xz)
        return np.array([S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]])
    rP = np.concatenate([khat, -voigt(lam0 * np.eye(3) + 2 * mu0 * np.outer(khat, khat)) / cp0])
    rS = np.concatenate([a, -voigt(mu0 * (np.outer(a, khat) + np.outer(khat, a))) / cs0])
    xi = _node_positions(n)
    e = np.arange(nelem)
    ex, ey, ez = e % grid, (e // grid) % grid, e // (grid * grid)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")
    phase = (kvec[0] * (ex[:, None] + X.reshape(1, -1)) + kvec[1] * (ey[:, None] + Y.reshape(1, -1))
             + kvec[2] * (ez[:, None] + Z.reshape(1, -1))) * h
    Q = np.sin(phase)[..., None] * rP + 0.5 * np.sin(phase + 1.0)[..., None] * rS
    Q = Q + noise * rng.standard_normal(Q.shape)
    cp = np.sqrt((par[..., 1] + 2 * par[..., 2]) / par[..., 0]).max() if nelem else 1.0
    dt = np.full(nelem, cfl_dt(N, h, cp))
    return Batch(N, 9, ELASTIC, Q, dt, np.full(nelem, h), params=par, coef_per_element=not per_node)


def acoustic_batch(N: int, nelem: int, seed: int, h: float = 1.0, per_node: bool = True) -> Batch:
    """Acoustic waves with random per-node material rho ~ U[2,3], K ~ U[1,2] and Q ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    n3 = (N + 1) ** 3
    shape = (nelem, n3) if per_node else (nelem,)
    par = np.stack([rng.uniform(2.0, 3.0, shape), rng.uniform(1.0, 2.0, shape)], axis=-1)
    Q = rng.standard_normal((nelem, n3, 4))
    c = np.sqrt(par[..., 1] / par[..., 0]).max() if nelem else 1.0
    dt = np.full(nelem, cfl_dt(N, h, c))
    return Batch(N, 4, ACOUSTIC, Q, dt, np.full(nelem, h), params=par, coef_per_element=not per_node)


def generic_batch(N: int, m: int, nelem: int, seed: int, h: float = 1.0, with_A: bool = False,
                  per_node: bool = True) -> Batch:
    """Generic linear system: dense B_d (and optionally A_d) with entries ~ N(0, 1/m) per node,
    Q ~ N(0, 1); dt_e from c_e = max over nodes and directions of the Frobenius norm of B_d."""
    rng = np.random.default_rng(seed)
    n3 = (N + 1) ** 3
    shape = (nelem, 3, n3, m, m) if per_node else (nelem, 3, m, m)
    B = rng.standard_normal(shape) / math.sqrt(m)
    A = rng.standard_normal(shape) / math.sqrt(m) if with_A else None
    Q = rng.standard_normal((nelem, n3, m))
    axes = tuple(range(1, B.ndim))
    cB = np.sqrt((B ** 2).sum(axis=(-1, -2)))
    c = cB.reshape(nelem, -1).max(axis=1) if nelem else np.ones(0)
    if with_A:
        cA = np.sqrt((A ** 2).sum(axis=(-1, -2))).reshape(nelem, -1).max(axis=1)
        c = c + cA
    del axes
    dt = np.array([cfl_dt(N, h, ci) for ci in c])
    return Batch(N, m, GENERIC, Q, dt, np.full(nelem, h), A=A, B=B, coef_per_element=not per_node)


def point_source(batch: Batch, seed: int) -> np.ndarray:
    """A point source per element: nodal projection P ~ U[0,1], amplitude a ~ N(0,1), and the time
    derivatives sigma^(o)(t_n) ~ N(0,1) for o = 0..N-1. Layout [E, n^3 + m + N]."""
    rng = np.random.default_rng(seed)
    n3 = (batch.N + 1) ** 3
    E = batch.nelem
    return np.concatenate([rng.uniform(0, 1, (E, n3)), rng.standard_normal((E, batch.m)),
                           rng.standard_normal((E, batch.N))], axis=1)


# ------------------------------------------------------------------------------------------------
# The named workloads (element counts as in the paper-shaped configurations).

def c1_elastic_n3(seed: int = SEED0 + 0) -> Batch:
    """Elastic, N=3, 64 elements, h=1, per-node material, FP64."""
    return elastic_batch(3, 64, seed)


def c2_acoustic_n5(nelem: int = 32768, seed: int = SEED0 + 1) -> Batch:
    """Acoustic, N=5, 32768 = 32^3 elements, plane wave + noise."""
    return acoustic_plane_wave_batch(5, nelem, seed, grid=32 if nelem == 32768 else None)


def c3_elastic_n7(nelem: int = 65536, seed: int = SEED0 + 2) -> Batch:
    """Elastic, N=7, 65536 elements, per-node material, Q ~ N(0,1)."""
    return elastic_batch(7, nelem, seed)


def c4_classes(nelem: int = 16384, seed: int = SEED0 + 3):
    """Heterogeneous mix: N_e ~ U{2..9}, m_e ~ U{4, 9} independently. Returns (N[e], m[e])."""
    rng = np.random.default_rng(seed)
    return rng.integers(2, 10, nelem), rng.choice(np.array([4, 9]), nelem)


def serving_batch_sizes(nbatch: int, seed: int) -> np.ndarray:
    """Log-uniform batch sizes floor(exp(U[0, ln 4097))) in 1..4096."""
    rng = np.random.default_rng(seed)
    return np.minimum(4096, np.floor(np.exp(rng.uniform(0, math.log(4097), nbatch))).astype(np.int64))


@dataclasses.dataclass
class HeteroBatch:
    """A batch of elements of several classes in one flat buffer per array (FP64 host arrays).

    classes: list of (N, m, physics, flags); cls[e] is the class of element e; off_q / off_coef /
    off_face are per-element offsets (in values) into Q / B (or params) / qface; `parts` holds the
    uniform sub-batch of each class with `members[c]` the element ids of class c. `coef` holds the
    per-node B in the library's node-fastest layout (coef_abi)."""
    classes: list
    cls: np.ndarray
    off_q: np.ndarray
    off_coef: np.ndarray
    off_face: np.ndarray
    Q: np.ndarray
    coef: np.ndarray
    dt: np.ndarray
    h: np.ndarray
    parts: list
    members: list
    size_q: int
    size_face: int


def hetero_generic_batch(nelem: int, seed: int, orders=None, nquants=None, h: float = 1.0) -> HeteroBatch:
    """Heterogeneous elements with dense per-node B_d ~ N(0, 1/m) (no A), Q ~ N(0,1), dt_e from
    c_e = max over nodes and directions of ||B_d||_F. Orders N_e ~ U{2..9} and m_e ~ U{4, 9} by default."""
    rng = np.random.default_rng(seed)
    if orders is None:
        Ns, ms = c4_classes(nelem, seed)
    else:
        Ns = rng.choice(np.asarray(orders), nelem)
        ms = rng.choice(np.asarray(nquants), nelem)
    keys = sorted(set(zip(Ns.tolist(), ms.tolist())))
    classes = [(N, m, GENERIC, 0) for N, m in keys]
    index = {k: i for i, k in enumerate(keys)}
    cls = np.array([index[(int(a), int(b))] for a, b in zip(Ns, ms)], dtype=np.int32)
    parts, members = [], []
    for c, (N, m) in enumerate(keys):
        ids = np.nonzero(cls == c)[0]
        members.append(ids)
        parts.append(generic_batch(N, m, len(ids), seed + 1000 + c, h=h))
    size_q = np.array([(N + 1) ** 3 * m for N, m in keys])
    size_face = np.array([6 * (N + 1) ** 2 * m for N, m in keys])
    size_coef = np.array([3 * (N + 1) ** 3 * m * m for N, m in keys])
    sq, sf, sc = size_q[cls], size_face[cls], size_coef[cls]
    off_q = np.concatenate([[0], np.cumsum(sq)[:-1]]).astype(np.int64)
    off_face = np.concatenate([[0], np.cumsum(sf)[:-1]]).astype(np.int64)
    off_coef = np.concatenate([[0], np.cumsum(sc)[:-1]]).astype(np.int64)
    Q = np.zeros(int(sq.sum()))
    coef = np.zeros(int(sc.sum()))
    dt = np.zeros(nelem)
    hh = np.full(nelem, h)
    for c, ids in enumerate(members):
        p = parts[c]
        for j, e in enumerate(ids):
            Q[off_q[e]:off_q[e] + sq[e]] = p.Q[j].ravel()
            coef[off_coef[e]:off_coef[e] + sc[e]] = np.moveaxis(p.B[j], 1, -1).ravel()
            dt[e] = p.dt[j]
    return HeteroBatch(classes, cls, off_q, off_coef, off_face, Q, coef, dt, hh, parts, members,
                       int(sq.sum()), int(sf.sum()))


@dataclasses.dataclass
class MixedBatch:
    """Uniform batches of any physics interleaved into one flat buffer per array (FP64 host arrays).

    Element e of class cls[e] reads Q at off_q[e], its coefficients at off_coef[e] (into `params` for a
    preset class, into `B` and `A` for a generic one; A shares B's offsets), its source at off_src[e];
    its faces go to off_face[e] and its time-averaged fluxes to 3 * off_q[e]. `members[c]` are the
    element ids of class c in the order of `parts[c]`. Per-node A and B are in the library's node-fastest
    layout (coef_abi)."""
    classes: list
    cls: np.ndarray
    off_q: np.ndarray
    off_coef: np.ndarray
    off_face: np.ndarray
    off_src: np.ndarray
    Q: np.ndarray
    params: np.ndarray
    B: np.ndarray
    A: np.ndarray
    src: np.ndarray
    dt: np.ndarray
    h: np.ndarray
    parts: list
    members: list
    size_q: int
    size_face: int


def interleave(parts, classes, seed: int) -> MixedBatch:
    """Shuffle the elements of several uniform batches (class c = parts[c], classes[c] its stp class
    tuple) into one heterogeneous batch with per-element offsets."""
    rng = np.random.default_rng(seed)
    cls = np.concatenate([np.full(p.nelem, c, dtype=np.int32) for c, p in enumerate(parts)])
    rng.shuffle(cls)
    members = [np.nonzero(cls == c)[0] for c in range(len(parts))]
    E = len(cls)
    rank = np.zeros(E, dtype=np.int64)
    for ids in members:
        rank[ids] = np.arange(len(ids))
    sq = np.array([parts[c].Q[0].size if parts[c].nelem else 0 for c in cls], dtype=np.int64)
    sf = np.array([6 * (parts[c].N + 1) ** 2 * parts[c].m for c in cls], dtype=np.int64)

    def coef_of(p):
        return p.params if p.physics != GENERIC else p.B

    sp = np.array([coef_of(parts[c])[0].size if parts[c].physics != GENERIC else 0 for c in cls], dtype=np.int64)
    sb = np.array([coef_of(parts[c])[0].size if parts[c].physics == GENERIC else 0 for c in cls], dtype=np.int64)
    ss = np.array([parts[c].src[0].size if parts[c].src is not None else 0 for c in cls], dtype=np.int64)
    ex = lambda s: np.concatenate([[0], np.cumsum(s)[:-1]]).astype(np.int64)
    off_q, off_face, off_src = ex(sq), ex(sf), ex(ss)
    off_p, off_b = ex(sp), ex(sb)
    off_coef = np.where(sb > 0, off_b, off_p)
    Q, params, B, A = np.zeros(sq.sum()), np.zeros(max(sp.sum(), 1)), np.zeros(max(sb.sum(), 1)), np.zeros(max(sb.sum(), 1))
    src = np.zeros(max(ss.sum(), 1))
    dt, hh = np.zeros(E), np.zeros(E)
    for e in range(E):
        p, j = parts[cls[e]], rank[e]
        Q[off_q[e]:off_q[e] + sq[e]] = p.Q[j].ravel()
        if p.physics != GENERIC:
            params[off_coef[e]:off_coef[e] + sp[e]] = p.params[j].ravel()
        else:
            lay = (lambda M: M.ravel()) if p.coef_per_element else (lambda M: np.moveaxis(M, 1, -1).ravel())
            B[off_coef[e]:off_coef[e] + sb[e]] = lay(p.B[j])
            if p.A is not None:
                A[off_coef[e]:off_coef[e] + sb[e]] = lay(p.A[j])
        if p.src is not None:
            src[off_src[e]:off_src[e] + ss[e]] = p.src[j].ravel()
        dt[e], hh[e] = p.dt[j], p.h[j]
    return MixedBatch(list(classes), cls, off_q, off_coef, off_face, off_src, Q, params, B, A, src, dt, hh,
                      list(parts), members, int(sq.sum()), int(sf.sum()))


# ------------------------------------------------------------------------------------------------------------
# Device-side generators for the full-size heterogeneous and serving workloads (the host generators above
# build these sizes too slowly). Same distributions as the host recipes; values are drawn with a seeded
# torch generator on the device, so they differ from the host generators' values.

def _exclusive(sizes: np.ndarray) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)


def c4_device(nelem: int = 16384, seed: int = SEED0 + 3, device="cuda", h: float = 1.0):
    """The heterogeneous generic workload on the device, FP32: N_e ~ U{2..9}, m_e ~ U{4, 9}, per-node dense
    B_d ~ N(0, 1/m), Q ~ N(0, 1), dt_e from c_e = max over nodes and directions of ||B_d||_F (FP64).

    Element ids are in random class order; storage is class-contiguous (offsets map ids to storage), so each
    class's elements also form a uniform batch (`class_ranges`). Returns a dict of device tensors and
    host metadata (classes, counts, class_ranges)."""
    import torch
    Ns, ms = c4_classes(nelem, seed)
    keys = sorted(set(zip(Ns.tolist(), ms.tolist())))
    classes = [(N, m, GENERIC, 0) for N, m in keys]
    index = {k: i for i, k in enumerate(keys)}
    cls = np.array([index[(int(a), int(b))] for a, b in zip(Ns, ms)], dtype=np.int32)
    order = np.argsort(cls, kind="stable")            # storage slot -> element id
    counts = np.bincount(cls, minlength=len(keys))
    n3 = np.array([(N + 1) ** 3 for N, _ in keys])
    mm = np.array([m for _, m in keys])
    sq_c, sf_c, sc_c = n3 * mm, 6 * np.array([(N + 1) ** 2 for N, _ in keys]) * mm, 3 * n3 * mm * mm
    sq, sf, sc = sq_c[cls[order]], sf_c[cls[order]], sc_c[cls[order]]
    oq_s, of_s, oc_s = _exclusive(sq), _exclusive(sf), _exclusive(sc)
    off_q, off_face, off_coef = (np.empty(nelem, np.int64) for _ in range(3))
    off_q[order], off_face[order], off_coef[order] = oq_s, of_s, oc_s
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Q = torch.randn(int(sq.sum()), generator=g, device=device, dtype=torch.float32)
    B = torch.randn(int(sc.sum()), generator=g, device=device, dtype=torch.float32)
    dt = np.empty(nelem)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]])
    ranges = []
    for c, (N, m) in enumerate(keys):
        k = int(counts[c])
        ranges.append((int(first[c]), k))
        if k == 0:
            continue
        s0 = int(oc_s[first[c]])
        blk = B[s0:s0 + k * int(sc_c[c])].view(k, 3, m, m, int(n3[c]))  # node-fastest library layout
        blk.mul_(1.0 / math.sqrt(m))
        cmax = torch.linalg.matrix_norm(blk.double(), dim=(2, 3)).amax(dim=(1, 2)).cpu().numpy()
        dt[order[first[c]:first[c] + k]] = [cfl_dt(N, h, ci) for ci in cmax]
    to = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to(device, t)
    return dict(classes=classes, counts=counts, class_ranges=ranges, order=order, nelem=nelem,
                cls=to(cls, torch.int32), off_q=to(off_q, torch.int64), off_coef=to(off_coef, torch.int64),
                off_face=to(off_face, torch.int64), Q=Q, B=B, dt=to(dt, torch.float64),
                h=torch.full((nelem,), h, device=device, dtype=torch.float64),
                size_q=int(sq.sum()), size_face=int(sf.sum()), size_coef=int(sc.sum()),
                storage_q=oq_s, storage_face=of_s, storage_coef=oc_s, sizes_q=sq_c, sizes_face=sf_c, sizes_coef=sc_c)


# Sup of the material ranges: the fastest wave speed any element can have (serving dt rule).
C_MAX = {ACOUSTIC: math.sqrt(2.0 / 2.0), ELASTIC: math.sqrt((4.0 + 2 * 3.0) / 2.0)}


def serving_mesh(physics: int, nelem: int, seed: int, class_base: int, device="cuda", h: float = 1.0):
    """A resident p-adaptive mesh for the serving workload: N_e ~ U{2..9} per element, per-node material
    (acoustic rho ~ U[2,3], K ~ U[1,2]; elastic as elastic_material), Q ~ N(0, 1), FP32 on the device,
    element-contiguous storage. Class id of element e = class_base + N_e - 2. dt_e = 0.4 h / ((2N_e+1) c_max)
    with c_max the fastest wave speed the material ranges allow."""
    import torch
    rng = np.random.default_rng(seed)
    m, npar = NQUANT[physics], NPARAM[physics]
    Ns = rng.integers(2, 10, nelem)
    n3 = (Ns + 1) ** 3
    sq, sf, sp = n3 * m, 6 * (Ns + 1) ** 2 * m, n3 * npar
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Q = torch.randn(int(sq.sum()), generator=g, device=device, dtype=torch.float32)
    u = torch.rand(int(sp.sum()) // npar, npar, generator=g, device=device, dtype=torch.float32)
    if physics == ACOUSTIC:
        lo, hi = torch.tensor([2.0, 1.0], device=device), torch.tensor([3.0, 2.0], device=device)
    else:
        lo, hi = torch.tensor([2.0, 1.0, 1.0], device=device), torch.tensor([3.0, 4.0, 3.0], device=device)
    params = (lo + (hi - lo) * u).reshape(-1)
    dt = np.array([cfl_dt(int(N), h, C_MAX[physics]) for N in Ns])
    to = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to(device, t)
    return dict(physics=physics, nelem=nelem, N=Ns, cls=to(class_base + Ns - 2, torch.int32),
                off_q=to(_exclusive(sq), torch.int64), off_coef=to(_exclusive(sp), torch.int64),
                off_face=to(_exclusive(sf), torch.int64), Q=Q, params=params, dt=to(dt, torch.float64),
                h=torch.full((nelem,), h, device=device, dtype=torch.float64),
                size_q=int(sq.sum()), size_face=int(sf.sum()))
