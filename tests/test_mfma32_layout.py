"""Host emulation of the FP32 MFMA kernel's derivative layouts (csrc/stp_mfma_f32.hpp), in float64.

v_mfma_f32_4x4x1f32 (16 blocks of four lanes): lane l's accumulator register r gains A of lane 4 (l // 4) + r
times B of lane l; with cbsz = 1 the A values of the pair of blocks (2k, 2k + 1) come from block 2k + abid.
(These are the lane layouts the kernel relies on, read off the hardware with a probe; the GPU parity tests check
the kernel end to end.) DPP row_half_mirror hands lane i of each group of eight the value of lane 7 - i.

The emulation builds each lane's A and B constants with the kernel's formulas, runs the x-derivative (two chains
of four products and one mirror add) and the role derivative (one broadcast chain of eight products) on random
lines, and compares with D u. It also checks the lane-to-line maps: every line once per half, partners where the
kernel expects them.
"""
import numpy as np
import pytest

from dense import np_dmatrix, np_nodes

n = 8


def lagrange_at(x):
    """l_j(x) for the n Gauss-Legendre nodes on [0, 1]."""
    xi, _ = np_nodes(n)
    return np.array([np.prod([(x - xi[k]) / (xi[j] - xi[k]) for k in range(n) if k != j]) for j in range(n)])


def mfma_4x4x1(a, b, c, cbsz=0, abid=0):
    """One v_mfma_f32_4x4x1f32 over 64 lanes: a, b [64], c [64][4]."""
    out = c.copy()
    for l in range(64):
        blk = l // 4
        src = ((blk >> cbsz) << cbsz) + abid if cbsz else blk
        for r in range(4):
            out[l, r] += a[4 * src + r] * b[l]
    return out


def mirror(v):
    """DPP row_half_mirror: lane i of each group of eight takes lane 7 - i."""
    return np.array([v[(l & ~7) | (7 - (l & 7))] for l in range(64)])


def half(l):
    return (l >> 2) & 1


def lslot(l):
    i = l & 7
    return 4 * ((l >> 3) & 3) + (i if i < 4 else 7 - i)


def la(w, l):
    return (lslot(l) >> 2) + 4 * w


def lb(l):
    return (lslot(l) & 3) + 4 * (l >> 5)


def rslot(l):
    return 4 * ((l >> 3) & 3) + (l & 3)


def ra(w, l):
    return (rslot(l) >> 2) + 4 * w


def rb(l):
    return (rslot(l) & 3) + 4 * (l >> 5)


@pytest.fixture(scope="module")
def D():
    return np_dmatrix(n)


def test_lane_maps_cover_every_line_once_per_half():
    for line_of in ((lambda w, l: 8 * la(w, l) + lb(l)), (lambda w, l: 8 * ra(w, l) + rb(l))):
        seen = np.zeros((2, 64), int)
        for w in range(2):
            for l in range(64):
                seen[half(l), line_of(w, l)] += 1
        assert (seen == 1).all()
    for w in range(2):
        for l in range(64):
            # owner partners (the mirror add) and role partners (the broadcast pair) share a line
            assert (la(w, l), lb(l)) == (la(w, l ^ 7), lb(l ^ 7)) and half(l) != half(l ^ 7)
            assert (ra(w, l), rb(l)) == (ra(w, l ^ 4), rb(l ^ 4)) and half(l) != half(l ^ 4)
            # the lanes of a 4x4 block share their half (and so the node indices they feed)
            assert half(l) == half(4 * (l // 4))


def test_x_derivative_chains_and_mirror_add(D):
    rng = np.random.default_rng(5)
    for w in range(2):
        lines = rng.standard_normal((64, n))  # u along every owner line L = 8a + b
        u = np.array([[lines[8 * la(w, l) + lb(l), 4 * half(l) + t] for t in range(4)] for l in range(64)])
        # A[g][m] = D[4 (g ^ h) + l % 4][4h + m]
        A = np.array([[[D[4 * (g ^ half(l)) + (l & 3), 4 * half(l) + m] for m in range(4)] for g in range(2)]
                      for l in range(64)])
        c0 = np.zeros((64, 4))
        c1 = np.zeros((64, 4))
        for m in range(4):
            c0 = mfma_4x4x1(A[:, 0, m], u[:, m], c0)
            c1 = mfma_4x4x1(A[:, 1, m], u[:, m], c1)
        out = np.stack([c0[:, i] + mirror(c1[:, i]) for i in range(4)], axis=1)
        for l in range(64):
            ref = D @ lines[8 * la(w, l) + lb(l)]
            np.testing.assert_allclose(out[l], ref[4 * half(l):4 * half(l) + 4], rtol=0, atol=1e-12)


def test_role_derivative_broadcast_chain(D):
    rng = np.random.default_rng(6)
    for w in range(2):
        lines = rng.standard_normal((64, n))  # u along every role line L = 8a + b
        u = np.array([[lines[8 * ra(w, l) + rb(l), 4 * half(l) + t] for t in range(4)] for l in range(64)])
        # B[abid][m] = D[4h + l % 4][4 abid + m]
        B = np.array([[[D[4 * half(l) + (l & 3), 4 * ab + m] for m in range(4)] for ab in range(2)]
                      for l in range(64)])
        c = np.zeros((64, 4))
        for ab in range(2):
            for m in range(4):
                c = mfma_4x4x1(u[:, m], B[:, ab, m], c, cbsz=1, abid=ab)
        for l in range(64):
            for r in range(4):
                row_lane = (l & ~3) | r  # the lane of row r in the block: its line is the line of register r
                ref = D @ lines[8 * ra(w, row_lane) + rb(row_lane)]
                assert abs(c[l, r] - ref[4 * half(l) + (l & 3)]) < 1e-12, (w, l, r)


def test_face_mirror_sums():
    """Faces: the lane's sum with l_j(h) plus its mirror partner's sum with l_j(1 - h) is the line's side-h face."""
    e0, e1 = lagrange_at(0.0), lagrange_at(1.0)
    rng = np.random.default_rng(7)
    lines = rng.standard_normal((64, n))
    u = np.array([[lines[8 * la(0, l) + lb(l), 4 * half(l) + t] for t in range(4)] for l in range(64)])
    e = (e0, e1)
    so = np.array([sum(e[half(l)][4 * half(l) + t] * u[l, t] for t in range(4)) for l in range(64)])
    sp = np.array([sum(e[1 - half(l)][4 * half(l) + t] * u[l, t] for t in range(4)) for l in range(64)])
    face = so + mirror(sp)
    for l in range(64):
        assert abs(face[l] - e[half(l)] @ lines[8 * la(0, l) + lb(l)]) < 1e-12
