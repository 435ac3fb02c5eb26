"""The seeded input generators: shapes, seeding and the recipe's value ranges (no GPU)."""
import numpy as np

from paper_2003_12787_amd import workloads as W


def test_named_workload_shapes_and_dt():
    b = W.c1_elastic_n3()
    assert b.Q.shape == (64, 64, 9) and b.params.shape == (64, 64, 3)
    assert abs(b.dt[0] - 0.4 / (7 * np.sqrt((b.params[..., 1] + 2 * b.params[..., 2]) / b.params[..., 0]).max())) < 1e-15
    assert 0.0255 < b.dt[0] < 0.027  # the bound 0.4/(7 sqrt(5)) for the sup of the material ranges
    b = W.c2_acoustic_n5(nelem=1000)
    assert b.Q.shape == (1000, 216, 4) and b.params.shape == (1000, 2) and b.coef_per_element
    assert np.all(b.params[:, 0] == 1.0) and 1 <= b.params[:, 1].min() and b.params[:, 1].max() <= 2
    assert 0.0257 < b.dt[0] < 0.0258
    b = W.c3_elastic_n7(nelem=10)
    assert b.Q.shape == (10, 512, 9)


def test_seeding_is_reproducible():
    a, b = W.elastic_batch(3, 5, 7), W.elastic_batch(3, 5, 7)
    assert np.array_equal(a.Q, b.Q) and np.array_equal(a.params, b.params)
    c = W.elastic_batch(3, 5, 8)
    assert not np.array_equal(a.Q, c.Q)


def test_plane_wave_recipe():
    b = W.acoustic_plane_wave_batch(3, 27, 1, noise=0.0)
    p, v = b.Q[..., 0], b.Q[..., 1:]
    c = np.sqrt(b.params[:, 1] / b.params[:, 0])
    khat = np.array([1.0, 2.0, 2.0]) / 3.0
    assert np.allclose(v, khat[None, None, :] * (p / c[:, None])[..., None])


def test_generic_and_hetero():
    g = W.generic_batch(2, 5, 4, 3, with_A=True)
    assert g.B.shape == (4, 3, 27, 5, 5) and g.A.shape == g.B.shape
    s = W.point_source(g, 4)
    assert s.shape == (4, 27 + 5 + 2)
    hb = W.hetero_generic_batch(200, 5, orders=[1, 2], nquants=[1, 4])
    assert len(hb.cls) == 200 and hb.Q.size == hb.size_q
    for c, ids in enumerate(hb.members):
        N, m = hb.classes[c][:2]
        e = ids[0]
        assert np.array_equal(hb.Q[hb.off_q[e]:hb.off_q[e] + (N + 1) ** 3 * m], hb.parts[c].Q[0].ravel())
    Ns, ms = W.c4_classes(1000)
    assert set(np.unique(Ns)) == set(range(2, 10)) and set(np.unique(ms)) == {4, 9}
    sz = W.serving_batch_sizes(10000, 1)
    assert sz.min() >= 1 and sz.max() <= 4096


def test_coef_abi_is_node_fastest():
    g = W.generic_batch(2, 3, 2, 5, with_A=True)
    L = W.coef_abi(g.B, False)
    assert L.shape == (2, 3, 3, 3, 27)
    e, d, node, s, r = 1, 2, 13, 0, 2
    assert L.ravel()[(((e * 3 + d) * 3 + s) * 3 + r) * 27 + node] == g.B[e, d, node, s, r]
    pe = W.generic_batch(2, 3, 2, 5, per_node=False)
    assert W.coef_abi(pe.B, True) is pe.B


def test_interleave_offsets_round_trip():
    parts = [W.elastic_batch(2, 5, 1), W.acoustic_batch(3, 4, 2, per_node=False),
             W.generic_batch(2, 3, 6, 3, with_A=True)]
    parts[2].src = W.point_source(parts[2], 4)
    classes = [(p.N, p.m, p.physics, 0) for p in parts]
    mb = W.interleave(parts, classes, 7)
    assert sorted(np.concatenate(mb.members).tolist()) == list(range(15))
    for c, p in enumerate(parts):
        for j, e in enumerate(mb.members[c]):
            assert mb.cls[e] == c
            n = p.Q[j].size
            assert np.array_equal(mb.Q[mb.off_q[e]:mb.off_q[e] + n], p.Q[j].ravel())
            coef = p.params if p.physics != W.GENERIC else W.coef_abi(p.B, p.coef_per_element)
            arr = mb.params if p.physics != W.GENERIC else mb.B
            k = coef[j].size
            assert np.array_equal(arr[mb.off_coef[e]:mb.off_coef[e] + k], coef[j].ravel())
            if p.A is not None:
                A = W.coef_abi(p.A, p.coef_per_element)
                assert np.array_equal(mb.A[mb.off_coef[e]:mb.off_coef[e] + k], A[j].ravel())
            if p.src is not None:
                s = p.src[j].size
                assert np.array_equal(mb.src[mb.off_src[e]:mb.off_src[e] + s], p.src[j].ravel())
            assert mb.dt[e] == p.dt[j] and mb.h[e] == p.h[j]
    # offsets tile the flat arrays without overlap
    sq = [parts[mb.cls[e]].Q[0].size for e in range(15)]
    order = np.argsort(mb.off_q)
    assert np.all(np.diff(mb.off_q[order]) == np.array(sq)[order][:-1])
    assert mb.size_q == sum(sq)


def test_curvilinear_geometry_matches_the_map_and_its_inverse_jacobian():
    """The per-element metric terms are the inverse of the map's Jacobian at the nodes (numpy's inverse),
    the node positions are the map of the grid points, and the device generator reproduces the metric."""
    N, grid, h, eps = 3, (4, 3, 2), 0.5, 0.3
    x, G = W.curvilinear_geometry(N, grid, h, eps)
    t = W._node_positions(N + 1)
    e = np.arange(24)
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    xi = np.stack([((e % 4)[:, None] + X.reshape(1, -1)) * h, (((e // 4) % 3)[:, None] + Y.reshape(1, -1)) * h,
                   ((e // 12)[:, None] + Z.reshape(1, -1)) * h], axis=-1)
    xr, J = W.curved_map(xi, (2.0, 1.5, 1.0), eps)
    assert np.abs(x - xr).max() < 1e-14
    assert np.abs(G - np.linalg.inv(J)).max() < 1e-13
    _, Gs = W.curvilinear_geometry(N, grid, h, eps, elements=[5, 17])
    assert np.array_equal(Gs, G[[5, 17]])
    # the map is a periodic deformation: x - xi is periodic, and every J is invertible
    assert np.linalg.det(J).min() > 0.5
    import torch
    Q, par, dt = W.curvilinear_device(N, 16, 7, device="cpu")
    _, Gg = W.curvilinear_geometry(N, W.grid_of(16), 1.0, 0.2)
    assert par.shape == (16, 64, 12) and Q.shape == (16, 64, 9) and dt > 0
    assert np.abs(par[..., 3:].double().numpy() - Gg.reshape(16, 64, 9)).max() < 1e-6
    p = par.double().numpy()
    assert p[..., 0].min() >= 2 and p[..., 0].max() <= 3 and p[..., 1].min() >= 1 and p[..., 2].max() <= 3
