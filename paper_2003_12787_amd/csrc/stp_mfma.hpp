// stp_mfma.hpp -- predictor kernel with the derivative contractions on the matrix cores (MFMA), for the
// physics presets (acoustic, elastic, curvilinear elastic) at order N = 7 (8 nodes per axis), FP32 I/O.
//
// Mathematics as in the other kernels (Sec. II-A, Eq. (4), Fig. 5 recompute of favg, Sec. II-B faces). Only
// the 1D derivative u -> D u (the sum-factorised contraction of Sec. III-B) runs on MFMA, as split-BF16
// products with FP32 accumulation: u = u_hi + u_lo and D = D_hi + D_lo with hi = bf16(x) (nearest) and
// lo = bf16(x - hi); the products D_hi u_hi + D_hi u_lo + D_lo u_hi + D_lo u_lo are formed by two
// v_mfma_f32_16x16x32_bf16 per 32 lines (the K dimension carries [hi | lo] of the lines of both 16-line
// groups, so the fourth product costs nothing).
//
// Lane layout: an element is 128 lanes (two waves). Lane (wave w, lane l): line c = l % 16 of group
// g = l / 32, half h = (l / 16) % 2, line index 32 w + 16 g + c, nodes 4h..4h+3 along the line. For the
// x-direction the owner's registers already hold its half-line: each lane forms hi/lo of its 4 values, and two
// permlane16 swaps of (hi, lo) give every lane the 8 K values of its row block of the B operand
//   B = [hi of group 0 | lo of group 0 | hi of group 1 | lo of group 1]   (8 nodes each, column = line c)
// With A_x = [[D_x, D_x, 0, 0]; [0, 0, D_x, D_x]] (rows 0..7: group 0, rows 8..15: group 1; x = hi, lo),
//   C = A_hi B + A_lo B
// leaves D u exactly at each owner's 4 nodes. The y- and
// z-directions use the same lane roles on lines read from an LDS tile of p, and return the derivatives to the
// owners through an LDS exchange buffer (as in the fused kernel). Pointwise terms, the time accumulation and
// the faces stay on the VALU in FP32.
#pragma once
#include "stp_device.hpp"
#include "stp_fused.hpp"
#include "stp_kernels.hpp"

namespace stp {
namespace mfma {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// hi = bf16(x) (round to nearest even), lo = bf16(x - hi); two values packed per 32-bit word (one packed
// conversion per pair; the hi parts are widened back to FP32 by shifting the bit patterns)
__device__ inline void split_pair(float a, float b, unsigned& hi, unsigned& lo)
{
    const f32x2 v = {a, b};
    const unsigned hu = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
    const f32x2 r = {a - __builtin_bit_cast(float, hu << 16), b - __builtin_bit_cast(float, hu & 0xffff0000u)};
    hi = hu;
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2));
}

__device__ inline bf16x8 as_bf16x8(unsigned w0, unsigned w1, unsigned w2, unsigned w3)
{
    const u32x4 t = {w0, w1, w2, w3};
    return __builtin_bit_cast(bf16x8, t);
}

// opaque_zero() (stp_device.hpp) launders the LDS base addresses: they are recomputed where they are used
// instead of being hoisted out of the Taylor loop (each quantity slot needs its own base register for the
// paired LDS accesses, and keeping them all live would halve the occupancy).

// A operands of the split contraction: D_hi and D_lo in the block layout [[D, D, 0, 0]; [0, 0, D, D]]
struct AOps {
    bf16x8 hi, lo;
};

// The split of the lane's 4 values: hi and lo of nodes (0, 1) and (2, 3), two bf16 per word.
struct Split4 {
    unsigned h0, l0, h1, l1;
};

__device__ inline Split4 split4(const float (&u)[4])
{
    Split4 s;
    split_pair(u[0], u[1], s.h0, s.l0);
    split_pair(u[2], u[3], s.h1, s.l1);
    return s;
}

// Node words of the LDS tile: hi of the node in the low half, lo in the high half (one word per node, the size of
// the FP32 value), so that the y- and z-roles reassemble the hi and lo pairs with two byte permutes per pair
// instead of splitting again.
__device__ inline unsigned node_word(unsigned h, unsigned l, bool second)
{
    return __builtin_amdgcn_perm(l, h, second ? 0x07060302u : 0x05040100u);
}

__device__ inline Split4 from_words(unsigned w0, unsigned w1, unsigned w2, unsigned w3)
{
    return {__builtin_amdgcn_perm(w1, w0, 0x05040100u), __builtin_amdgcn_perm(w1, w0, 0x07060302u),
            __builtin_amdgcn_perm(w3, w2, 0x05040100u), __builtin_amdgcn_perm(w3, w2, 0x07060302u)};
}

// D u for the lane's half-line, from the split of u[0..3]; the B operand of both 16-line groups of the wave is
// formed by two permlane16 swaps.
__device__ inline void deriv_mfma(const AOps& A, const Split4& sp, float (&out)[4])
{
    const unsigned h0 = sp.h0, l0 = sp.l0, h1 = sp.h1, l1 = sp.l1;
    // The swap exchanges the odd 16-lane rows of the first operand with the even rows of the second: rows 0 and
    // 2 (h = 0) end with the hi parts of nodes 0..7 of their line, rows 1 and 3 (h = 1) with the lo parts, in
    // node order (0, 1), (2, 3), (4, 5), (6, 7): the lane's 8 K values of B.
    auto s0 = __builtin_amdgcn_permlane16_swap(h0, l0, false, false);
    auto s1 = __builtin_amdgcn_permlane16_swap(h1, l1, false, false);
    const bf16x8 b = as_bf16x8(s0[0], s1[0], s0[1], s1[1]);
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.hi, b, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.lo, b, c, 0, 0, 0);
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

template <int PHYS>
struct Mfma8 {
    static constexpr int N = 7, n = 8, n2 = 64, n3 = 512;
    static constexpr int M = PhysTraits<PHYS>::m;
    static constexpr int NP = PhysTraits<PHYS>::np;
    static constexpr int WG = 128;  // one element per workgroup (two waves)
    using S = fused::Sets<PHYS>;
    static constexpr int NPS = S::NPS, NG = S::NG;
    // Exchange-buffer slots: the derivatives of one direction come back in chunks of NGX quantities (all of
    // them at once for the Cartesian presets; 5 + 4 for curvilinear elements, which differentiate all 9
    // quantities in every direction) so that four elements per CU still fit in LDS.
    static constexpr int NGX = NG <= 6 ? NG : 5;
    static constexpr int C1 = NGX;  // end of the first chunk
    static constexpr int SLOT = n3;  // one quantity's tile, swizzled (at()): 4 elements per CU fit in LDS
    static constexpr int ELDS = (NPS + NGX) * SLOT;
    static constexpr int STAGE = 16 * n * M;  // per-wave staging of 16 lines of an output block (floats)
    static constexpr int LDS_FLOATS = ELDS + 2 * STAGE;
    static constexpr int FACE_OFF = M * SLOT;  // face staging after the q-bar tile of the face pass
    static_assert(FACE_OFF + 6 * n2 * M <= LDS_FLOATS, "face staging fits the LDS region");
    static_assert(NPS + NGX >= M, "face pass reuses the tile for all quantities");

    // Row D of the metric terms at the lane's 4 nodes (curvilinear elements): re-read from the parameter array
    // for each direction (the laundered offset keeps the loads inside the Taylor loop; L2 holds the element's
    // parameters) instead of holding 36 registers for the whole kernel.
    using GRow = float[4][3];
    template <int D>
    __device__ static inline void load_grow(const float* gp, int stride, GRow& Gd)
    {
        if constexpr (PHYS == kElasticCurv) {
            const float* q = gp + opaque_zero() + 3 + 3 * D;
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < 3; ++j) Gd[t][j] = q[t * stride + j];
        }
    }

    // Accumulator rows of a Taylor step on curvilinear elements: the reference derivatives of all directions are
    // first mapped to the 9 velocity gradients h dv_i/dx_j (rows 3i + j) and the 3 stress divergences
    // h sum_j ds_ij/dx_j (rows 9 + i), 18 FMAs per node and direction; the elastic operator is applied once to
    // those (grad_finish) instead of 36 operations per node and direction. The time-averaged fluxes need each
    // direction's term on its own and keep the per-direction form (rows = M).
    static constexpr int kGradRows = 12;
    static constexpr int TR = PHYS == kElasticCurv ? kGradRows : M;  // accumulator rows of a Taylor step

    // r[.][t] += contribution of the derivative g (quantity dq(D, K)) at the lane's 4 nodes; with R ==
    // kGradRows (curvilinear Taylor steps) to the gradient accumulators instead
    template <int D, int K, int R>
    __device__ static inline void ncp(const Material<float, PHYS> (&mt)[4], const GRow& Gd, const float (&g)[4],
                                      float (&r)[R][4])
    {
        if constexpr (PHYS == kElasticCurv && R == kGradRows) {
            if constexpr (K < 3) {  // v_K: h dv_K/dx_j += G[D][j] g
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int j = 0; j < 3; ++j) r[3 * K + j][t] = fma(Gd[t][j], g[t], r[3 * K + j][t]);
            } else if constexpr (K < 6) {  // s_aa: row a of the divergence gets G[D][a] g
                constexpr int a = K - 3;
#pragma unroll
                for (int t = 0; t < 4; ++t) r[9 + a][t] = fma(Gd[t][a], g[t], r[9 + a][t]);
            } else {  // s_ab: rows a and b get G[D][b] g and G[D][a] g
                constexpr int a = K == 6 ? 0 : (K == 7 ? 1 : 0), b = K == 6 ? 1 : 2;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    r[9 + a][t] = fma(Gd[t][b], g[t], r[9 + a][t]);
                    r[9 + b][t] = fma(Gd[t][a], g[t], r[9 + b][t]);
                }
            }
        } else if constexpr (PHYS == kElasticCurv) {
            // g = d/dxi_D of quantity K contributes G[D][j] g / h to its derivative along x_j (1/h is in c);
            // the elastic operator's column K of sum_j G[D][j] M_j:
            using P = PhysTraits<kElastic>;
            if constexpr (K < 3) {  // v_K: s_KK <- (lam+2mu) dv_K/dx_K, s_ii <- lam dv_K/dx_K, s_jK <- mu dv_K/dx_j
                constexpr int j1 = (K + 1) % 3, j2 = (K + 2) % 3;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float gk = Gd[t][K] * g[t];
                    const float gm = mt[t].c[2] * g[t];
                    r[3 + K][t] = fma(mt[t].c[3], gk, r[3 + K][t]);
                    r[3 + j1][t] = fma(mt[t].c[1], gk, r[3 + j1][t]);
                    r[3 + j2][t] = fma(mt[t].c[1], gk, r[3 + j2][t]);
                    r[P::sig(j1, K)][t] = fma(Gd[t][j1], gm, r[P::sig(j1, K)][t]);
                    r[P::sig(j2, K)][t] = fma(Gd[t][j2], gm, r[P::sig(j2, K)][t]);
                }
            } else if constexpr (K < 6) {  // s_aa: v_a <- (1/rho) ds_aa/dx_a
                constexpr int a = K - 3;
#pragma unroll
                for (int t = 0; t < 4; ++t) r[a][t] = fma(mt[t].c[0] * Gd[t][a], g[t], r[a][t]);
            } else {  // s_ab (a != b): v_a <- (1/rho) ds_ab/dx_b, v_b <- (1/rho) ds_ab/dx_a
                constexpr int a = K == 6 ? 0 : (K == 7 ? 1 : 0), b = K == 6 ? 1 : 2;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float gr = mt[t].c[0] * g[t];
                    r[a][t] = fma(Gd[t][b], gr, r[a][t]);
                    r[b][t] = fma(Gd[t][a], gr, r[b][t]);
                }
            }
        } else if constexpr (PHYS == kElastic) {
            using P = PhysTraits<kElastic>;
            if constexpr (K < 3) {
                if constexpr (K == D) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        r[3 + D][t] = fma(mt[t].c[3], g[t], r[3 + D][t]);
                        r[3 + (D + 1) % 3][t] = fma(mt[t].c[1], g[t], r[3 + (D + 1) % 3][t]);
                        r[3 + (D + 2) % 3][t] = fma(mt[t].c[1], g[t], r[3 + (D + 2) % 3][t]);
                    }
                } else {
                    constexpr int q = P::sig(D, K);
#pragma unroll
                    for (int t = 0; t < 4; ++t) r[q][t] = fma(mt[t].c[2], g[t], r[q][t]);
                }
            } else {
                constexpr int i = K - 3;
#pragma unroll
                for (int t = 0; t < 4; ++t) r[i][t] = fma(mt[t].c[0], g[t], r[i][t]);
            }
        } else {
            if constexpr (K == 0) {
#pragma unroll
                for (int t = 0; t < 4; ++t) r[1 + D][t] = fma(mt[t].c[1], g[t], r[1 + D][t]);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) r[0][t] = fma(mt[t].c[0], g[t], r[0][t]);
            }
        }
    }

    // The elastic operator on the gradient accumulators: r = (1/rho) div s, s_ii = lambda tr(grad v) +
    // 2 mu dv_i/dx_i, s_ab = mu (dv_a/dx_b + dv_b/dx_a), with 1/h in the material coefficients.
    __device__ static inline void grad_finish(const Material<float, PHYS> (&mt)[4], const float (&a)[TR][4],
                                              float (&r)[M][4])
    {
        if constexpr (TR == kGradRows) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float tr = a[0][t] + a[4][t] + a[8][t];
                const float mu2 = mt[t].c[3] - mt[t].c[1];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    r[i][t] = mt[t].c[0] * a[9 + i][t];
                    r[3 + i][t] = fma(mt[t].c[1], tr, mu2 * a[4 * i][t]);
                }
                r[6][t] = mt[t].c[2] * (a[1][t] + a[3][t]);
                r[7][t] = mt[t].c[2] * (a[5][t] + a[7][t]);
                r[8][t] = mt[t].c[2] * (a[2][t] + a[6][t]);
            }
        }
    }

    template <int K = 0, int R = M>
    __device__ static inline void xpass(const AOps& A, const Material<float, PHYS> (&mt)[4], const GRow& Gd,
                                        const Split4 (&p)[M],
                                        float (&r)[R][4])
    {
        if constexpr (K < NG) {
            float g[4];
            deriv_mfma(A, p[S::dq(0, K)], g);
            ncp<0, K>(mt, Gd, g, r);
            __builtin_amdgcn_sched_barrier(0);  // one quantity at a time: bounds the live registers
            xpass<K + 1>(A, mt, Gd, p, r);
        }
    }

    // Tile address of node (z, y, x), an XOR swizzle. The LDS serves 32 lanes at a time from 32 banks, and in
    // each of the three access patterns (owner lines along x: z in {2j, 2j+1}, all y, x = 4h + t; y-role lines:
    // y = 4h + t, all x; z-role lines: z = 4h + t, y in {2j, 2j+1}, all x) the 32 lanes of a half-wave vary in
    // five node bits. The bank bits
    //   b0 = x0 ^ y0, b1 = x1 ^ y1, b2 = x2, b3 = y0 ^ y2, b4 = z0 ^ z2
    // are independent over each of those five-bit sets, so every pattern hits 32 distinct banks; the
    // remaining bits (z1, x0, x1, z0) select one of 16 groups of 32 words. A padded linear layout leaves 2- to
    // 4-way conflicts.
    __host__ __device__ static constexpr int at(int z, int y, int x)
    {
        const int bank = ((x ^ y) & 3) | (x & 4) | (((y ^ (y >> 2)) & 1) << 3) | (((z ^ (z >> 2)) & 1) << 4);
        const int group = ((z >> 1) & 1) | ((x & 3) << 1) | ((z & 1) << 3);
        return 32 * group + bank;
    }

    static constexpr bool at_is_permutation()
    {
        bool seen[n3] = {};
        for (int z = 0; z < n; ++z)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) {
                    const int v = at(z, y, x);
                    if (v < 0 || v >= n3 || seen[v]) return false;
                    seen[v] = true;
                }
        return true;
    }
    static_assert(at_is_permutation(), "the swizzled tile covers [0, n^3) once");

    // A lane's tile offsets for its four nodes t = 0..3 in the owner, y-role and z-role patterns (fixed for
    // the kernel's lifetime: the lane's line never changes).
    struct Offs {
        int o[4], y[4], z[4];
    };
    __device__ static inline Offs offsets(int la, int lb, int h)
    {
        Offs f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f.o[t] = at(la, lb, 4 * h + t);
            f.y[t] = at(la, 4 * h + t, lb);
            f.z[t] = at(4 * h + t, la, lb);
        }
        return f;
    }

    // y- or z-role: lines (a, b) = (z, x) resp. (y, x), nodes 4h..4h+3 along the line; derivatives of the
    // quantities dq(D, k), k in [K0, K1), into exchange slots k - K0
    template <int D, int K0, int K1>
    __device__ static inline void transposed(const AOps& A, const float* P0, float* G0, const Offs& f)
    {
        const int z0 = opaque_zero();
        const unsigned* P = reinterpret_cast<const unsigned*>(P0) + z0;  // node words (node_word)
        float* G = G0 + z0;
        const int(&off)[4] = D == 1 ? f.y : f.z;
#pragma unroll
        for (int k = K0; k < K1; ++k) {
            const int s = S::slot(S::dq(D, k));
            float g[4];
            const unsigned* Ps = P + s * SLOT;
            deriv_mfma(A, from_words(Ps[off[0]], Ps[off[1]], Ps[off[2]], Ps[off[3]]), g);
#pragma unroll
            for (int t = 0; t < 4; ++t) G[(k - K0) * SLOT + off[t]] = g[t];
            // The Cartesian presets leave the scheduler free to overlap the quantities' chains (LDS read,
            // MFMA pair, LDS write): 231 registers, still two waves per SIMD. Curvilinear elements (244
            // registers) overlap them in pairs.
            if constexpr (PHYS == kElasticCurv)
                if (((k - K0) & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
    }

    template <int D, int K0, int K1, int K = K0, int R = M>
    __device__ static inline void gather(const float* G0, const Offs& f, const Material<float, PHYS> (&mt)[4],
                                         const GRow& Gd, float (&r)[R][4])
    {
        const float* G = G0 + (K == K0 ? opaque_zero() : 0);
        if constexpr (K < K1) {
            float g[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) g[t] = G[(K - K0) * SLOT + f.o[t]];
            ncp<D, K>(mt, Gd, g, r);
            gather<D, K0, K1, K + 1>(G, f, mt, Gd, r);
        }
    }

    // r += the y- or z-contributions, once every lane has written the first chunk of direction D (transposed
    // <D, 0, C1>) and passed a barrier; the other chunk, if any, goes through the exchange buffer here. gp, gs:
    // the lane's first node's parameters and the per-node stride (0 for per-element parameters).
    template <int D, int R>
    __device__ static inline void finish_dir(const AOps& A, const float* P, float* G, const Offs& f,
                                             const Material<float, PHYS> (&mt)[4], const float* gp, int gs,
                                             float (&r)[R][4])
    {
        GRow Gd;
        load_grow<D>(gp, gs, Gd);
        gather<D, 0, C1>(G, f, mt, Gd, r);
        if constexpr (NG > NGX) {
            __syncthreads();
            transposed<D, C1, NG>(A, P, G, f);
            __syncthreads();
            gather<D, C1, NG>(G, f, mt, Gd, r);
        }
    }

    // the split of every quantity at the lane's 4 nodes (the x-pass and the tile use it; each value is split once)
    __device__ static inline void split_all(const float (&v)[M][4], Split4 (&sp)[M])
    {
#pragma unroll
        for (int q = 0; q < M; ++q) sp[q] = split4(v[q]);
    }

    __device__ static inline void write_tile(float* P0, const Offs& f, const Split4 (&sp)[M])
    {
        unsigned* P = reinterpret_cast<unsigned*>(P0) + opaque_zero();
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const int s = S::slot(q);
            if (s < 0) continue;
            P[s * SLOT + f.o[0]] = node_word(sp[q].h0, sp[q].l0, false);
            P[s * SLOT + f.o[1]] = node_word(sp[q].h0, sp[q].l0, true);
            P[s * SLOT + f.o[2]] = node_word(sp[q].h1, sp[q].l1, false);
            P[s * SLOT + f.o[3]] = node_word(sp[q].h1, sp[q].l1, true);
        }
    }

    // 4 nodes x M quantities = 4M contiguous floats
    __device__ static inline void load4(const float* src, float (&v)[M][4])
    {
        if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const float4 t = s4[i];
                const int w = 4 * i;
                v[(w + 0) % M][(w + 0) / M] = t.x;
                v[(w + 1) % M][(w + 1) / M] = t.y;
                v[(w + 2) % M][(w + 2) / M] = t.z;
                v[(w + 3) % M][(w + 3) / M] = t.w;
            }
        } else {
#pragma unroll
            for (int w = 0; w < 4 * M; ++w) v[w % M][w / M] = src[w];
        }
    }

    __device__ static inline void store4(float* dst, const float (&v)[M][4])
    {
        if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
            float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int w = 4 * i;
                d4[i] = make_float4(v[(w + 0) % M][(w + 0) / M], v[(w + 1) % M][(w + 1) / M],
                                    v[(w + 2) % M][(w + 2) / M], v[(w + 3) % M][(w + 3) / M]);
            }
        } else {
#pragma unroll
            for (int w = 0; w < 4 * M; ++w) dst[w] = v[w % M][w / M];
        }
    }

    // Store the wave's 32 half-line pairs of one output block (32 lines x 8 nodes x M contiguous floats at
    // `dst`) through the wave's LDS staging area, 16 lines per round, so that each 16-byte store instruction
    // of the wave covers 1 KB of consecutive addresses. Falls back to per-lane stores when misaligned.
    __device__ static inline void store_block(float* S, float* dst, const float (&v)[M][4], int l, int g, int c, int h,
                                              bool aligned)
    {
        if (!aligned) {
            store4(dst + ((16 * g + c) * n + 4 * h) * M, v);
            return;
        }
#pragma unroll
        for (int rnd = 0; rnd < 2; ++rnd) {
            if (g == rnd) {
                float4* s4 = reinterpret_cast<float4*>(S + (c * 2 + h) * 4 * M);
#pragma unroll
                for (int i = 0; i < M; ++i) {
                    const int w = 4 * i;
                    s4[i] = make_float4(v[(w + 0) % M][(w + 0) / M], v[(w + 1) % M][(w + 1) / M],
                                        v[(w + 2) % M][(w + 2) / M], v[(w + 3) % M][(w + 3) / M]);
                }
            }
            __syncthreads();
            const float4* r4 = reinterpret_cast<const float4*>(S);
            float4* d4 = reinterpret_cast<float4*>(dst + rnd * STAGE);
#pragma unroll 2
            for (int i = l; i < STAGE / 4; i += 64) d4[i] = r4[i];
            __syncthreads();
        }
    }

    __device__ static void run(const StpArgs& a)
    {
        extern __shared__ __align__(16) unsigned char smem[];
        const int tid = threadIdx.x;
        const int wv = tid >> 6, l = tid & 63;
        const int c = l & 15, h = (l >> 4) & 1, g = l >> 5;
        const int line = 32 * wv + 16 * g + c;
        const int la = line >> 3, lb = line & 7;  // owner (z, y); y-role (z, x); z-role (y, x)
        const Offs off = offsets(la, lb, h);
        float* P = reinterpret_cast<float*>(smem);
        float* G = P + NPS * SLOT;
        float* Sw = P + ELDS + wv * STAGE;  // this wave's staging area
        const bool per_elem = (a.flags & kParamPerElement) != 0;

        AOps A;
        {
            // table: [2 matrices (A_hi, A_lo)][64 lanes][8 bf16]
            const unsigned* t = static_cast<const unsigned*>(a.Dsplit);
            A.hi = as_bf16x8(t[l * 4], t[l * 4 + 1], t[l * 4 + 2], t[l * 4 + 3]);
            A.lo = as_bf16x8(t[(64 + l) * 4], t[(64 + l) * 4 + 1], t[(64 + l) * 4 + 2], t[(64 + l) * 4 + 3]);
        }
        const int64_t cnt = a.count ? (int64_t)*a.count : a.nelem;

        for (int64_t it = blockIdx.x; it < cnt; it += gridDim.x) {
            ElemRef er;
            elem_ref(a, it, er);
            const int64_t node0 = (int64_t)line * n + 4 * h;  // first of the lane's 4 nodes
            float p[M][4], qb[M][4];
            Material<float, PHYS> mt[4];
            load4(static_cast<const float*>(a.Q) + er.q + node0 * M, p);
            {
                const double inv_h = 1.0 / er.h;
                const float* par = static_cast<const float*>(a.params) + er.coef;
#pragma unroll
                for (int t = 0; t < 4; ++t) mt[t].load(per_elem ? par : par + (node0 + t) * NP, inv_h);
            }
            const float* gp = static_cast<const float*>(a.params) + er.coef + (per_elem ? 0 : node0 * NP);
            const int gs = per_elem ? 0 : NP;
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int t = 0; t < 4; ++t) qb[q][t] = p[q][t];
            float w = 1.f;
            const float dt = (float)er.dt;
#pragma unroll 1
            for (int o = 1; o <= N; ++o) {
                Split4 sp[M];
                split_all(p, sp);
                write_tile(P, off, sp);
                __syncthreads();
                float r[TR][4];
#pragma unroll
                for (int q = 0; q < TR; ++q)
#pragma unroll
                    for (int t = 0; t < 4; ++t) r[q][t] = 0.f;
                transposed<1, 0, C1>(A, P, G, off);
                {
                    GRow G0;
                    load_grow<0>(gp, gs, G0);
                    xpass(A, mt, G0, sp, r);
                }
                __syncthreads();
                finish_dir<1>(A, P, G, off, mt, gp, gs, r);
                __syncthreads();
                transposed<2, 0, C1>(A, P, G, off);
                __syncthreads();
                finish_dir<2>(A, P, G, off, mt, gp, gs, r);
                w = w * dt * __builtin_amdgcn_rcpf((float)(o + 1));
                if constexpr (TR == kGradRows) {
                    grad_finish(mt, r, p);
                } else {
#pragma unroll
                    for (int q = 0; q < M; ++q)
#pragma unroll
                        for (int t = 0; t < 4; ++t) p[q][t] = r[q][t];
                }
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int t = 0; t < 4; ++t) qb[q][t] = fma(w, p[q][t], qb[q][t]);
                __syncthreads();
            }

            // outputs
            const bool fsum = (a.flags & kFavgSum) != 0;
            const bool al = (er.q & 3) == 0;  // 16-byte aligned element blocks (float offsets)
            const int64_t wbase = (int64_t)32 * wv * n * M;  // first float of this wave's lines in a block
            store_block(Sw, static_cast<float*>(a.qavg) + er.q + wbase, qb, l, g, c, h, al);
            Split4 sq[M];
            split_all(qb, sq);
            write_tile(P, off, sq);
            __syncthreads();
            {
                float fx[M][4];
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int t = 0; t < 4; ++t) fx[q][t] = 0.f;
                transposed<1, 0, C1>(A, P, G, off);
                {
                    GRow G0;
                    load_grow<0>(gp, gs, G0);
                    xpass(A, mt, G0, sq, fx);
                }
                float* fav = static_cast<float*>(a.favg) + (fsum ? er.q : 3 * er.q) + wbase;
                if (!fsum) {
                    store_block(Sw, fav, fx, l, g, c, h, al);
#pragma unroll
                    for (int q = 0; q < M; ++q)
#pragma unroll
                        for (int t = 0; t < 4; ++t) fx[q][t] = 0.f;
                }
                __syncthreads();
                finish_dir<1>(A, P, G, off, mt, gp, gs, fx);
                if (!fsum) {
                    store_block(Sw, fav + (int64_t)n3 * M, fx, l, g, c, h, al);
#pragma unroll
                    for (int q = 0; q < M; ++q)
#pragma unroll
                        for (int t = 0; t < 4; ++t) fx[q][t] = 0.f;
                }
                __syncthreads();
                transposed<2, 0, C1>(A, P, G, off);
                __syncthreads();
                finish_dir<2>(A, P, G, off, mt, gp, gs, fx);
                store_block(Sw, fsum ? fav : fav + 2 * (int64_t)n3 * M, fx, l, g, c, h, al);
            }
            // faces: partial sums over the lane's 4 nodes, completed with the other half-line (lane ^ 16); the
            // face values are staged in LDS in the output layout [f][a][b][s] and written with coalesced stores
            float* F = P + FACE_OFF;
            float e0[4], e1[4];  // face vectors at the lane's 4 nodes along a line
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                e0[t] = ld<float>(a.e0, 4 * h + t);
                e1[t] = ld<float>(a.e1, 4 * h + t);
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int t = 0; t < 4; ++t) P[q * SLOT + off.o[t]] = qb[q][t];
#pragma unroll
            for (int q = 0; q < M; ++q) {
                float s0 = 0.f, s1 = 0.f;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    s0 = fma(e0[t], qb[q][t], s0);
                    s1 = fma(e1[t], qb[q][t], s1);
                }
                s0 += __shfl_xor(s0, 16);
                s1 += __shfl_xor(s1, 16);
                F[(h * n2 + line) * M + q] = h ? s1 : s0;  // x- (h = 0) and x+ (h = 1)
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < M; ++q) {
                float y0 = 0.f, y1 = 0.f, z0 = 0.f, z1 = 0.f;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float vy = P[q * SLOT + off.y[t]];  // y-role (z, x)
                    const float vz = P[q * SLOT + off.z[t]];  // z-role (y, x)
                    y0 = fma(e0[t], vy, y0);
                    y1 = fma(e1[t], vy, y1);
                    z0 = fma(e0[t], vz, z0);
                    z1 = fma(e1[t], vz, z1);
                }
                y0 += __shfl_xor(y0, 16);
                y1 += __shfl_xor(y1, 16);
                z0 += __shfl_xor(z0, 16);
                z1 += __shfl_xor(z1, 16);
                F[((2 + h) * n2 + line) * M + q] = h ? y1 : y0;
                F[((4 + h) * n2 + line) * M + q] = h ? z1 : z0;
            }
            __syncthreads();
            float* qf = static_cast<float*>(a.qface) + er.face;
            if ((er.face & 3) == 0) {
                const float4* f4 = reinterpret_cast<const float4*>(F);
                float4* d4 = reinterpret_cast<float4*>(qf);
#pragma unroll 2
                for (int i = tid; i < 6 * n2 * M / 4; i += WG) d4[i] = f4[i];
            } else {
                for (int i = tid; i < 6 * n2 * M; i += WG) qf[i] = F[i];
            }
            __syncthreads();
        }
    }
};

template <int PHYS>
__global__ void __launch_bounds__(128) stp_mfma_kernel(StpArgs a)
{
    Mfma8<PHYS>::run(a);
}

template <int PHYS>
KernelInfo mfma_info()
{
    using K = Mfma8<PHYS>;
    KernelInfo ki;
    ki.fn = reinterpret_cast<const void*>(&stp_mfma_kernel<PHYS>);
    ki.block = K::WG;
    ki.mb = K::M;
    ki.elems_per_block = 1;
    ki.lds = [](int, bool) -> size_t { return sizeof(float) * (size_t)K::LDS_FLOATS; };
    ki.aux = KernelInfo::kAuxMfmaSplit;
    return ki;
}

}  // namespace mfma
}  // namespace stp
