// stp_mfma.hpp -- predictor kernel with the derivative contractions on the matrix cores (MFMA), for the
// physics presets (acoustic, elastic, curvilinear elastic) at order N = 7 (8 nodes per axis), FP32 I/O.
//
// Mathematics as in the other kernels (Sec. II-A, Eq. (4), Fig. 5 recompute of favg, Sec. II-B faces). Only
// the 1D derivative u -> D u (the sum-factorised contraction of Sec. III-B) runs on MFMA, as BF16 products
// with FP32 accumulation. Both operands are split into three BF16 pieces:
//   u = hi + mid + lo     (truncation: hi keeps the 8 leading significant bits of u, mid the next 8 of the
//                          exact remainder, lo the rest, so the sum is exact)
//   D = D0 + D1 + D2      (the same split of the FP32 derivative matrix, done once on the host)
// and the six products of relative order up to 2^-16 are formed:
//   D u ~ D0 (hi + mid + lo) + D1 (hi + mid) + D2 hi,
// dropping terms of order 2^-24 and below, so the contraction is about as accurate as FP32 arithmetic. Smooth
// fields need this: the derivative of a nearly constant line cancels entries of D whose absolute row sum
// reaches 129 at n = 8, and a two-piece split (16 bits) leaves errors of a few 1e-4 in favg.
//
// Lane layout: an element is 256 lanes (four waves). Lane (wave w, lane l) has q = l / 16 and c = l % 16; it
// owns line L = 16 w + c (lines are (z, y) = (L / 8, L % 8) along x) at the nodes 2q and 2q + 1. The y- and
// z-roles of the same lane take the line (z, x) resp. (y, x) = (L / 8, L % 8) at the same two node
// positions along y resp. z. A derivative of a wave's 16 lines is one v_mfma_f32_16x16x32_bf16 whose B operand
// is every lane's own two nodes (2q and 2q+1): lane group q supplies K entries 8q..8q+7 as the BF16 pairs
//   [(hi | mid) of node 2q, (hi | mid) of node 2q+1, (lo of 2q | lo of 2q+1), (hi of 2q | hi of 2q+1)].
// The A operand (a host table, one row per lane) has two rows per output node: in part a the entries are D0
// on hi, mid and lo and D1 on the second copy of hi; in part b D2 on hi and D1 on mid. Rows 4q', 4q'+1 are
// part a and rows 4q'+2, 4q'+3 part b of the nodes 2q', 2q'+1, so the lane that owns those nodes receives both
// parts in its accumulator and adds them: D u at its own nodes with no data movement between lanes. The
// x-direction uses the owner's registers; the y- and z-directions read their lines from an LDS tile of the
// split (per node the (hi | mid) word of every quantity, and words holding the lo pieces of two quantities)
// and return the derivatives to the owners through an LDS exchange buffer. Pointwise terms, the time
// accumulation and the faces stay on the VALU in FP32.
#pragma once
#include "stp_device.hpp"
#include "stp_fused.hpp"
#include "stp_kernels.hpp"

namespace stp {
namespace mfma {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ inline bf16x8 as_bf16x8(unsigned w0, unsigned w1, unsigned w2, unsigned w3)
{
    const u32x4 t = {w0, w1, w2, w3};
    return __builtin_bit_cast(bf16x8, t);
}

// The split of the lane's 2 values, as the four words of the B operand: (hi | mid) of each node, the two lo
// pieces, the two hi pieces (low half first).
struct Split2 {
    unsigned hm[2], lo2, hi2;
};

// u = hi + mid + lo exactly: hi = u with the low 16 bits cleared, r = u - hi (exact), mid = r with the low 16
// bits cleared, lo = r - mid (exact, at most 8 significant bits, so its upper 16 bits are lo in BF16). The
// tile's 16-bit lo of node t is the upper half of lo_bits[t].
__device__ inline Split2 split2(const float (&u)[2], unsigned (&lo_bits)[2])
{
    Split2 s;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const unsigned ub = __builtin_bit_cast(unsigned, u[t]);
        const float r = u[t] - __builtin_bit_cast(float, ub & 0xffff0000u);
        const unsigned rb = __builtin_bit_cast(unsigned, r);
        lo_bits[t] = __builtin_bit_cast(unsigned, r - __builtin_bit_cast(float, rb & 0xffff0000u));
        s.hm[t] = __builtin_amdgcn_perm(rb, ub, 0x07060302u);  // (hi | mid)
    }
    const unsigned u0 = __builtin_bit_cast(unsigned, u[0]), u1 = __builtin_bit_cast(unsigned, u[1]);
    s.lo2 = __builtin_amdgcn_perm(lo_bits[1], lo_bits[0], 0x07060302u);
    s.hi2 = __builtin_amdgcn_perm(u1, u0, 0x07060302u);
    return s;
}

// D u at the lane's own 2 nodes: one MFMA, then part a + part b.
__device__ inline void deriv_mfma(const bf16x8& A, const Split2& s, float (&out)[2])
{
    const bf16x8 b = as_bf16x8(s.hm[0], s.hm[1], s.lo2, s.hi2);
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, b, c, 0, 0, 0);
    out[0] = c[0] + c[2];
    out[1] = c[1] + c[3];
}

// r[.][t] += the pointwise term of a Cartesian preset (acoustic or elastic) for g, the derivative along
// direction D of the quantity dq(D, K) of the direction's derivative set, at L nodes (1/h is folded into the
// material coefficients).
template <int PHYS, int D, int K, int L, int R>
__device__ inline void ncp_cart(const Material<float, PHYS> (&mt)[L], const float (&g)[L], float (&r)[R][L])
{
    if constexpr (PHYS == kElastic) {
        using P = PhysTraits<kElastic>;
        if constexpr (K < 3) {
            if constexpr (K == D) {
#pragma unroll
                for (int t = 0; t < L; ++t) {
                    r[3 + D][t] = fma(mt[t].c[3], g[t], r[3 + D][t]);
                    r[3 + (D + 1) % 3][t] = fma(mt[t].c[1], g[t], r[3 + (D + 1) % 3][t]);
                    r[3 + (D + 2) % 3][t] = fma(mt[t].c[1], g[t], r[3 + (D + 2) % 3][t]);
                }
            } else {
                constexpr int q = P::sig(D, K);
#pragma unroll
                for (int t = 0; t < L; ++t) r[q][t] = fma(mt[t].c[2], g[t], r[q][t]);
            }
        } else {
            constexpr int i = K - 3;
#pragma unroll
            for (int t = 0; t < L; ++t) r[i][t] = fma(mt[t].c[0], g[t], r[i][t]);
        }
    } else {
        static_assert(PHYS == kAcoustic, "Cartesian presets only");
        if constexpr (K == 0) {
#pragma unroll
            for (int t = 0; t < L; ++t) r[1 + D][t] = fma(mt[t].c[1], g[t], r[1 + D][t]);
        } else {
#pragma unroll
            for (int t = 0; t < L; ++t) r[0][t] = fma(mt[t].c[0], g[t], r[0][t]);
        }
    }
}

template <int PHYS>
struct Mfma8 {
    static constexpr int N = 7, n = 8, n2 = 64, n3 = 512;
    static constexpr int NL = 2;     // nodes per lane
    static constexpr int WG = 256;   // one element per workgroup (four waves)
    static constexpr int M = PhysTraits<PHYS>::m;
    static constexpr int NP = PhysTraits<PHYS>::np;
    using S = fused::Sets<PHYS>;
    static constexpr int NPS = S::NPS, NG = S::NG;
    // Exchange-buffer slots: the derivatives of one direction come back in chunks of NGX quantities. All of
    // them come back at once: curvilinear elements differentiate all 9 quantities in every direction, and their
    // 143 registers hold three elements per CU, whose 47 KB of LDS each fit (two chunks would save LDS that
    // cannot host a fourth element, at two more barriers per direction). The chunked path stays for NGX < NG.
    static constexpr int NGX = NG;
    static constexpr int C1 = NGX;  // end of the first chunk
    static constexpr int SLOT = n3;  // one quantity's tile, swizzled (at())
    // Quantity pairs of the tile's lo words: each 32-bit word holds the lo pieces of two quantities at one node,
    // paired so that the y- and z-passes read few words. Elastic: (v_x, v_y) and (v_z, s_yz), which both
    // directions differentiate, (s_xy, s_yy) for y and (s_xz, s_zz) for z: three words per node and direction.
    // lo_pair(q) = word index * 2 + half, or -1 outside the tile.
    static constexpr int lo_pair(int q)
    {
        if constexpr (PHYS == kElastic) {
            constexpr int t[9] = {0, 1, 2, -1, 5, 7, 4, 3, 6};  // v_x v_y v_z s_xx s_yy s_zz s_xy s_yz s_xz
            return t[q];
        } else if constexpr (PHYS == kAcoustic) {
            constexpr int t[4] = {0, -1, 1, 2};  // p, v_x, v_y, v_z: (p, v_y), (v_z, -)
            return t[q];
        } else {
            return q;  // curvilinear: (0, 1), (2, 3), (4, 5), (6, 7), (8, -)
        }
    }
    static constexpr int NLP = PHYS == kElastic ? 4 : (PHYS == kAcoustic ? 2 : 5);  // lo words per node
    // Orders in which a pass takes its quantities, pair partners adjacent (so a lo word is read or assembled
    // once for both): the owner's split over all M quantities, and the k of direction D (dq(D, k)).
    static constexpr int qord(int i)
    {
        if constexpr (PHYS == kElastic) {
            constexpr int t[9] = {0, 1, 2, 7, 6, 4, 8, 5, 3};
            return t[i];
        } else if constexpr (PHYS == kAcoustic) {
            constexpr int t[4] = {0, 2, 3, 1};
            return t[i];
        } else {
            return i;
        }
    }
    static constexpr int kord(int D, int i)
    {
        if constexpr (PHYS == kElastic) {
            // y: v_x v_y | v_z s_yz | s_xy s_yy;  z: v_x v_y | v_z s_yz | s_xz s_zz  (k: 3 + i is s_{D,i})
            constexpr int ty[6] = {0, 1, 2, 5, 3, 4}, tz[6] = {0, 1, 2, 4, 3, 5};
            return D == 1 ? ty[i] : (D == 2 ? tz[i] : i);
        } else {
            return i;
        }
    }
    // LDS (32-bit words): the (hi | mid) words of the tile, the lo words, then the exchange buffer, which
    // also stages the output blocks (two waves of 16 lines at a time, lines padded by 4 floats so that the
    // lanes' 8-byte writes spread over the banks)
    static constexpr int HM_OFF = 0, LO_OFF = NPS * SLOT, G_OFF = LO_OFF + NLP * SLOT;
    static constexpr int ELDS = G_OFF + NGX * SLOT;
    static constexpr int LINE = n * M;            // floats of one line of an output block
    static constexpr int SLINE = LINE + 4;        // staged line (16-byte aligned)
    static constexpr int STAGE_END = G_OFF + 32 * SLINE;
    static constexpr int FACE_OFF = M * SLOT;  // face staging after the q-bar tile of the face pass
    static constexpr int max3(int x, int y, int z) { return x > y ? (x > z ? x : z) : (y > z ? y : z); }
    static constexpr int LDS_FLOATS = max3(ELDS, FACE_OFF + 6 * n2 * M, STAGE_END);

    // x-derivative index of quantity q (k with dq(0, k) == q), or -1
    static constexpr int kx(int q)
    {
        for (int k = 0; k < NG; ++k)
            if (S::dq(0, k) == q) return k;
        return -1;
    }

    // Row D of the metric terms at the lane's 2 nodes (curvilinear elements): re-read from the parameter array
    // for each direction (the laundered offset keeps the loads inside the Taylor loop; L2 holds the element's
    // parameters) instead of being held in registers for the whole kernel. Each row is loaded one phase before
    // the phase that uses it, so at most two rows are live at a time.
    using GRow = float[NL][3];
    template <int D>
    __device__ static inline void load_grow(const float* gp, int stride, GRow& Gd)
    {
        if constexpr (PHYS == kElasticCurv) {
            const float* q = gp + opaque_zero() + 3 + 3 * D;
#pragma unroll
            for (int t = 0; t < NL; ++t)
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

    // r[.][t] += contribution of the derivative g (quantity dq(D, K)) at the lane's nodes; with R ==
    // kGradRows (curvilinear Taylor steps) to the gradient accumulators instead
    template <int D, int K, int R>
    __device__ static inline void ncp(const Material<float, PHYS> (&mt)[NL], const GRow& Gd, const float (&g)[NL],
                                      float (&r)[R][NL])
    {
        if constexpr (PHYS == kElasticCurv && R == kGradRows) {
            if constexpr (K < 3) {  // v_K: h dv_K/dx_j += G[D][j] g
#pragma unroll
                for (int t = 0; t < NL; ++t)
#pragma unroll
                    for (int j = 0; j < 3; ++j) r[3 * K + j][t] = fma(Gd[t][j], g[t], r[3 * K + j][t]);
            } else if constexpr (K < 6) {  // s_aa: row a of the divergence gets G[D][a] g
                constexpr int a = K - 3;
#pragma unroll
                for (int t = 0; t < NL; ++t) r[9 + a][t] = fma(Gd[t][a], g[t], r[9 + a][t]);
            } else {  // s_ab: rows a and b get G[D][b] g and G[D][a] g
                constexpr int a = K == 6 ? 0 : (K == 7 ? 1 : 0), b = K == 6 ? 1 : 2;
#pragma unroll
                for (int t = 0; t < NL; ++t) {
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
                for (int t = 0; t < NL; ++t) {
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
                for (int t = 0; t < NL; ++t) r[a][t] = fma(mt[t].c[0] * Gd[t][a], g[t], r[a][t]);
            } else {  // s_ab (a != b): v_a <- (1/rho) ds_ab/dx_b, v_b <- (1/rho) ds_ab/dx_a
                constexpr int a = K == 6 ? 0 : (K == 7 ? 1 : 0), b = K == 6 ? 1 : 2;
#pragma unroll
                for (int t = 0; t < NL; ++t) {
                    const float gr = mt[t].c[0] * g[t];
                    r[a][t] = fma(Gd[t][b], gr, r[a][t]);
                    r[b][t] = fma(Gd[t][a], gr, r[b][t]);
                }
            }
        } else {
            ncp_cart<PHYS, D, K>(mt, g, r);
        }
    }

    // The elastic operator on the gradient accumulators: r = (1/rho) div s, s_ii = lambda tr(grad v) +
    // 2 mu dv_i/dx_i, s_ab = mu (dv_a/dx_b + dv_b/dx_a), with 1/h in the material coefficients.
    __device__ static inline void grad_finish(const Material<float, PHYS> (&mt)[NL], const float (&a)[TR][NL],
                                              float (&r)[M][NL])
    {
        if constexpr (TR == kGradRows) {
#pragma unroll
            for (int t = 0; t < NL; ++t) {
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

    // Tile address of node (z, y, x), an XOR swizzle. The LDS serves 32 lanes at a time from 32 banks. In each
    // of the three access patterns of a half-wave (owner: y, z0 and x1 vary; y-role: x, z0 and y1 vary;
    // z-role: x, y0 and z1 vary) the bank bits
    //   b0 = x0 ^ y0, b1 = x1, b2 = x2 ^ y2, b3 = y1 ^ z1, b4 = z0 ^ y0
    // are independent over the five varying node bits, so every pattern hits 32 distinct banks; the group
    // bits (x0, x2, y1, z2) complete a permutation of the 512 nodes.
    __host__ __device__ static constexpr int at(int z, int y, int x)
    {
        const int x0 = x & 1, x1 = (x >> 1) & 1, x2 = (x >> 2) & 1;
        const int y0 = y & 1, y1 = (y >> 1) & 1, y2 = (y >> 2) & 1;
        const int z0 = z & 1, z1 = (z >> 1) & 1, z2 = (z >> 2) & 1;
        const int bank = (x0 ^ y0) | (x1 << 1) | ((x2 ^ y2) << 2) | ((y1 ^ z1) << 3) | ((z0 ^ y0) << 4);
        const int group = x0 | (x2 << 1) | (y1 << 2) | (z2 << 3);
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

    // A lane's tile offsets for its two nodes t in the owner, y-role and z-role patterns (fixed for the
    // kernel's lifetime: the lane's line never changes).
    struct Offs {
        int o[NL], y[NL], z[NL];
    };
    __device__ static inline Offs offsets(int la, int lb, int q)
    {
        Offs f;
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            f.o[t] = at(la, lb, 2 * q + t);
            f.y[t] = at(la, 2 * q + t, lb);
            f.z[t] = at(2 * q + t, la, lb);
        }
        return f;
    }

    // LDS byte addresses of the lane's two nodes at offsets off[t] in the (hi | mid) words (also the exchange
    // buffer and the FP32 face tile, at constant distances) and in the 16-bit lo array. Slots and regions are
    // constant distances, folded into the instructions' offset fields, so each access pattern needs its two
    // word addresses and two halfword addresses only.
    struct Addr {
        unsigned w[NL], h[NL];
    };
    __device__ static inline Addr addr(const int (&off)[NL])
    {
        Addr a;
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            a.w[t] = (unsigned)(off[t] << 2);
            a.h[t] = (unsigned)(off[t] << 1);
        }
        return a;
    }
    template <typename T>
    __device__ static inline T& lds(unsigned char* smem, unsigned byte)
    {
        return *reinterpret_cast<T*>(smem + byte);
    }

    // For every quantity (in the order qord): split the lane's 2 values, store the split in the tile (if the
    // quantity is differentiated along y or z), and if it is differentiated along x form its x-derivative from
    // the split and apply its pointwise terms. `pend` carries the lo pieces of a pair's first quantity to its
    // second, which writes the pair's lo word.
    template <int I, int R>
    __device__ static inline void split_xpass_q(const bf16x8& A, unsigned char* smem, const Addr& ad,
                                                const Material<float, PHYS> (&mt)[NL], const GRow& Gd,
                                                const float (&v)[M][NL], float (&r)[R][NL], unsigned (&pend)[NL])
    {
        if constexpr (I < M) {
            constexpr int Q = qord(I);
            unsigned lo_bits[NL];
            const Split2 sp = split2(v[Q], lo_bits);
            constexpr int s = S::slot(Q), lp = lo_pair(Q);
            if constexpr (s >= 0) {
#pragma unroll
                for (int t = 0; t < NL; ++t) lds<unsigned>(smem, ad.w[t] + 4 * (HM_OFF + s * SLOT)) = sp.hm[t];
                constexpr bool last = (lp & 1) == 1 || I + 1 >= M || lo_pair(qord(I + 1)) != lp + 1;
                if constexpr (!last) {
#pragma unroll
                    for (int t = 0; t < NL; ++t) pend[t] = lo_bits[t];
                } else {
#pragma unroll
                    for (int t = 0; t < NL; ++t) {
                        // (lo of the pair's first quantity | lo of the second), or the lone lo in the low half
                        const unsigned w = (lp & 1) ? __builtin_amdgcn_perm(lo_bits[t], pend[t], 0x07060302u)
                                                    : (lo_bits[t] >> 16);
                        lds<unsigned>(smem, ad.w[t] + 4 * (LO_OFF + (lp >> 1) * SLOT)) = w;
                    }
                }
            }
            constexpr int k = kx(Q);
            if constexpr (k >= 0) {
                float g[NL];
                deriv_mfma(A, sp, g);
                ncp<0, k>(mt, Gd, g, r);
            }
            split_xpass_q<I + 1>(A, smem, ad, mt, Gd, v, r, pend);
        }
    }

    template <int R>
    __device__ static inline void split_xpass(const bf16x8& A, unsigned char* smem, const Offs& f,
                                              const Material<float, PHYS> (&mt)[NL], const GRow& Gd,
                                              const float (&v)[M][NL], float (&r)[R][NL])
    {
        unsigned pend[NL] = {0u, 0u};
        split_xpass_q<0>(A, smem, addr(f.o), mt, Gd, v, r, pend);
    }

    // y- or z-role: lines (a, b) = (z, x) resp. (y, x), nodes 2q, 2q+1 along the line; derivatives of the
    // quantities dq(D, kord(D, i)), i in [K0, K1), into exchange slots i - K0. A lo word is read once for the
    // two quantities of its pair when they follow each other.
    template <int D, int K0, int K1>
    __device__ static inline void transposed(const bf16x8& A, unsigned char* smem, const Offs& f)
    {
        const Addr ad = addr(D == 1 ? f.y : f.z);
        unsigned lw[NL] = {0u, 0u};
#pragma unroll
        for (int i = K0; i < K1; ++i) {
            const int q = S::dq(D, kord(D, i));
            const int s = S::slot(q), lp = lo_pair(q);
            const bool reuse = i > K0 && (lp & 1) == 1 && lo_pair(S::dq(D, kord(D, i - 1))) == lp - 1;
            Split2 sp;
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                sp.hm[t] = lds<unsigned>(smem, ad.w[t] + 4 * (HM_OFF + s * SLOT));
                if (!reuse) lw[t] = lds<unsigned>(smem, ad.w[t] + 4 * (LO_OFF + (lp >> 1) * SLOT));
            }
            // (lo of node 2q | lo of node 2q+1) from the quantity's half of the two lo words
            sp.lo2 = __builtin_amdgcn_perm(lw[1], lw[0], (lp & 1) ? 0x07060302u : 0x05040100u);
            sp.hi2 = __builtin_amdgcn_perm(sp.hm[1], sp.hm[0], 0x05040100u);  // (hi of 2q | hi of 2q+1)
            float g[NL];
            deriv_mfma(A, sp, g);
#pragma unroll
            for (int t = 0; t < NL; ++t) lds<float>(smem, ad.w[t] + 4 * (G_OFF + (i - K0) * SLOT)) = g[t];
        }
    }

    template <int D, int K0, int K1, int I = K0, int R = M>
    __device__ static inline void gather(const unsigned char* smem, const Addr& ad,
                                         const Material<float, PHYS> (&mt)[NL], const GRow& Gd, float (&r)[R][NL])
    {
        if constexpr (I < K1) {
            float g[NL];
#pragma unroll
            for (int t = 0; t < NL; ++t)
                g[t] = *reinterpret_cast<const float*>(smem + ad.w[t] + 4 * (G_OFF + (I - K0) * SLOT));
            ncp<D, kord(D, I)>(mt, Gd, g, r);
            gather<D, K0, K1, I + 1>(smem, ad, mt, Gd, r);
        }
    }

    // r += the y- or z-contributions, once every lane has written the first chunk of direction D (transposed
    // <D, 0, C1>) and passed a barrier; the other chunk, if any, goes through the exchange buffer here. Gd: the
    // direction's metric row at the lane's nodes (curvilinear elements; loaded by the caller a phase ahead).
    template <int D, int R>
    __device__ static inline void finish_dir(const bf16x8& A, unsigned char* smem, const Offs& f,
                                             const Material<float, PHYS> (&mt)[NL], const GRow& Gd,
                                             float (&r)[R][NL])
    {
        gather<D, 0, C1>(smem, addr(f.o), mt, Gd, r);
        if constexpr (NG > NGX) {
            __syncthreads();
            transposed<D, C1, NG>(A, smem, f);
            __syncthreads();
            gather<D, C1, NG>(smem, addr(f.o), mt, Gd, r);
        }
    }

    // 2 nodes x M quantities = 2M contiguous floats (8-byte aligned when the element block is)
    __device__ static inline void load2(const float* src, bool aligned, float (&v)[M][NL])
    {
        if (aligned) {
            const float2* s2 = reinterpret_cast<const float2*>(src);
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const float2 t = s2[i];
                v[(2 * i) % M][(2 * i) / M] = t.x;
                v[(2 * i + 1) % M][(2 * i + 1) / M] = t.y;
            }
        } else {
#pragma unroll
            for (int w = 0; w < NL * M; ++w) v[w % M][w / M] = src[w];
        }
    }

    // Store the wave's 16 lines of one output block (16 lines x 8 nodes x M contiguous floats per wave, the
    // four waves' parts consecutive at `dst`) through the staging area S (the exchange buffer), two waves per
    // round, lines padded to SLINE floats; each 16-byte store instruction of a wave covers 1 KB of consecutive
    // addresses. Falls back to per-lane stores when misaligned. Ends with a workgroup barrier either way
    // (`aligned` is uniform over the workgroup); the caller has passed a barrier after the last read of S.
    __device__ static inline void store_block(float* S, float* dst, const float (&v)[M][NL], int tid, int wv, int c,
                                              int q, bool aligned)
    {
        if (!aligned) {
            float* d = dst + ((16 * wv + c) * n + 2 * q) * M;
#pragma unroll
            for (int w = 0; w < NL * M; ++w) d[w] = v[w % M][w / M];
            __syncthreads();
            return;
        }
        constexpr int L4 = LINE / 4;  // float4 per line
#pragma unroll
        for (int rnd = 0; rnd < 2; ++rnd) {
            if ((wv >> 1) == rnd) {
                float2* s2 = reinterpret_cast<float2*>(S + ((wv & 1) * 16 + c) * SLINE + 2 * q * M);
#pragma unroll
                for (int i = 0; i < M; ++i)
                    s2[i] = make_float2(v[(2 * i) % M][(2 * i) / M], v[(2 * i + 1) % M][(2 * i + 1) / M]);
            }
            __syncthreads();
            float4* d4 = reinterpret_cast<float4*>(dst + rnd * 32 * LINE);
#pragma unroll
            for (int j = tid; j < 32 * L4; j += WG) {
                const int line = j / L4, k = j - line * L4;
                d4[j] = *reinterpret_cast<const float4*>(S + line * SLINE + 4 * k);
            }
            __syncthreads();
        }
    }

    // Sums over the four lanes of a line (rows 0..3 of the lane's column) of the face partials of two
    // quantities a and b: s0 = sum over the lane's nodes of l_j(0) u_j, s1 likewise with l_j(1). Returns, in
    // row 0, 1, 2, 3, the total of s0a, s1a, s0b, s1b. A swap of the odd with the even 16-lane rows pairs
    // rows (0, 1) and (2, 3); a swap of the 32-lane halves then pairs (0, 2) and (1, 3).
    //
    // Each swap's second result passes through an empty asm before it is added: this compiler otherwise
    // rewrites the sum of a swap's two results as the sum of its two operands, as if the swap exchanged values
    // within a lane.
    __device__ static inline unsigned opaque_u(unsigned x)
    {
        asm volatile("" : "+v"(x));
        return x;
    }
    __device__ static inline float face_reduce(float s0a, float s1a, float s0b, float s1b)
    {
        const auto xa = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, s0a),
                                                         __builtin_bit_cast(unsigned, s1a), false, false);
        const auto xb = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, s0b),
                                                         __builtin_bit_cast(unsigned, s1b), false, false);
        const float ta = __builtin_bit_cast(float, xa[0]) + __builtin_bit_cast(float, opaque_u(xa[1]));
        const float tb = __builtin_bit_cast(float, xb[0]) + __builtin_bit_cast(float, opaque_u(xb[1]));
        const auto y = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, ta),
                                                        __builtin_bit_cast(unsigned, tb), false, false);
        return __builtin_bit_cast(float, y[0]) + __builtin_bit_cast(float, opaque_u(y[1]));
    }

    // The faces of direction D (0 x, 1 y, 2 z) from the q-bar values u[s][t] at the lane's nodes along its line
    // in that direction: F[(2D + side) n^2 + line][s]. Quantities go in pairs (a, a + 1); an odd one out is
    // paired with zeros.
    template <int D>
    __device__ static inline void faces_dir(float* F, const float (&u)[M][NL], const float (&e0)[NL],
                                            const float (&e1)[NL], int line, int q)
    {
#pragma unroll
        for (int a = 0; a < M; a += 2) {
            const int b = a + 1 < M ? a + 1 : a;
            const float s0a = fma(e0[1], u[a][1], e0[0] * u[a][0]), s1a = fma(e1[1], u[a][1], e1[0] * u[a][0]);
            const float s0b = a + 1 < M ? fma(e0[1], u[b][1], e0[0] * u[b][0]) : 0.f;
            const float s1b = a + 1 < M ? fma(e1[1], u[b][1], e1[0] * u[b][0]) : 0.f;
            const float v = face_reduce(s0a, s1a, s0b, s1b);
            const int sq = q < 2 ? a : b;  // rows 0, 1: quantity a (sides 0, 1); rows 2, 3: quantity b
            if (q < 2 || a + 1 < M) F[((2 * D + (q & 1)) * n2 + line) * M + sq] = v;
        }
    }

    __device__ static void run(const StpArgs& a)
    {
        extern __shared__ __align__(16) unsigned char smem[];
        const int tid = threadIdx.x;
        const int wv = tid >> 6, l = tid & 63;
        const int q = l >> 4, c = l & 15;
        const int line = 16 * wv + c;
        const int la = line >> 3, lb = line & 7;  // owner (z, y); y-role (z, x); z-role (y, x)
        const Offs off = offsets(la, lb, q);
        float* G = reinterpret_cast<float*>(smem) + G_OFF;
        const bool per_elem = (a.flags & kParamPerElement) != 0;

        bf16x8 A;
        {
            // table: [64 lanes][8 bf16], one A row per lane
            const unsigned* t = static_cast<const unsigned*>(a.Dsplit);
            A = as_bf16x8(t[l * 4], t[l * 4 + 1], t[l * 4 + 2], t[l * 4 + 3]);
        }
        const int64_t cnt = a.count ? (int64_t)*a.count : a.nelem;

        for (int64_t it = blockIdx.x; it < cnt; it += gridDim.x) {
            ElemRef er;
            elem_ref(a, it, er);
            const int64_t node0 = (int64_t)line * n + 2 * q;  // first of the lane's 2 nodes
            const bool al = (er.q & 3) == 0;  // 16-byte aligned element blocks (float offsets)
            float p[M][NL], qb[M][NL];
            Material<float, PHYS> mt[NL];
            load2(static_cast<const float*>(a.Q) + er.q + node0 * M, (er.q & 1) == 0, p);
            {
                const float ih = (float)(1.0 / er.h);
                const float* par = static_cast<const float*>(a.params) + er.coef;
#pragma unroll
                for (int t = 0; t < NL; ++t) mt[t].load_f32(per_elem ? par : par + (node0 + t) * NP, ih);
            }
            const float* gp = static_cast<const float*>(a.params) + er.coef + (per_elem ? 0 : node0 * NP);
            const int gs = per_elem ? 0 : NP;
#pragma unroll
            for (int s = 0; s < M; ++s)
#pragma unroll
                for (int t = 0; t < NL; ++t) qb[s][t] = p[s][t];
            float w = 1.f;
            const float dt = (float)er.dt;
            // curvilinear elements: each direction's metric row is loaded one phase ahead of its use (row 0 of the
            // next application during this step's z-gather), so the L2 latency overlaps the previous phase's work
            GRow G0;
            load_grow<0>(gp, gs, G0);
#pragma unroll 1
            for (int o = 1; o <= N; ++o) {
                float r[TR][NL];
#pragma unroll
                for (int s = 0; s < TR; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) r[s][t] = 0.f;
                GRow G1;
                load_grow<1>(gp, gs, G1);
                split_xpass(A, smem, off, mt, G0, p, r);
                __syncthreads();
                transposed<1, 0, C1>(A, smem, off);
                __syncthreads();
                GRow G2;
                load_grow<2>(gp, gs, G2);
                finish_dir<1>(A, smem, off, mt, G1, r);
                __syncthreads();
                transposed<2, 0, C1>(A, smem, off);
                __syncthreads();
                load_grow<0>(gp, gs, G0);
                finish_dir<2>(A, smem, off, mt, G2, r);
                w = w * dt * __builtin_amdgcn_rcpf((float)(o + 1));
                if constexpr (TR == kGradRows) {
                    grad_finish(mt, r, p);
                } else {
#pragma unroll
                    for (int s = 0; s < M; ++s)
#pragma unroll
                        for (int t = 0; t < NL; ++t) p[s][t] = r[s][t];
                }
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) qb[s][t] = fma(w, p[s][t], qb[s][t]);
                // No barrier here: the next step writes the tile after every lane has passed the barrier that
                // precedes this step's last gather (the tile's last reads come before it), and the exchange
                // buffer after the barrier that follows its own tile writes.
            }
            __syncthreads();  // the last gather's reads of the exchange buffer, which stages the outputs

            // outputs. The output blocks are staged in the exchange buffer, so each staging round starts
            // after every lane's last read of the buffer (a barrier) and ends with one (inside store_block).
            const bool fsum = (a.flags & kFavgSum) != 0;
            store_block(G, static_cast<float*>(a.qavg) + er.q, qb, tid, wv, c, q, al);
            {
                float fx[M][NL];
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) fx[s][t] = 0.f;
                GRow G1;
                load_grow<1>(gp, gs, G1);
                split_xpass(A, smem, off, mt, G0, qb, fx);  // G0: loaded during the last step's z-gather
                float* fav = static_cast<float*>(a.favg) + (fsum ? er.q : 3 * er.q);
                if (!fsum) {
                    store_block(G, fav, fx, tid, wv, c, q, al);  // ends with a barrier: the tile is complete
#pragma unroll
                    for (int s = 0; s < M; ++s)
#pragma unroll
                        for (int t = 0; t < NL; ++t) fx[s][t] = 0.f;
                } else {
                    __syncthreads();
                }
                transposed<1, 0, C1>(A, smem, off);
                __syncthreads();
                GRow G2;
                load_grow<2>(gp, gs, G2);
                finish_dir<1>(A, smem, off, mt, G1, fx);
                __syncthreads();
                if (!fsum) {
                    store_block(G, fav + (int64_t)n3 * M, fx, tid, wv, c, q, al);
#pragma unroll
                    for (int s = 0; s < M; ++s)
#pragma unroll
                        for (int t = 0; t < NL; ++t) fx[s][t] = 0.f;
                }
                transposed<2, 0, C1>(A, smem, off);
                __syncthreads();
                finish_dir<2>(A, smem, off, mt, G2, fx);
                __syncthreads();
                store_block(G, fsum ? fav : fav + 2 * (int64_t)n3 * M, fx, tid, wv, c, q, al);
            }
            // faces: partial sums over the lane's 2 nodes along each direction, completed over the line's four
            // lanes (face_reduce); the x-faces from the registers, the y- and z-faces from an FP32 q-bar tile.
            // The face values are staged in LDS in the output layout [f][a][b][s] and written with coalesced
            // stores.
            float* PF = reinterpret_cast<float*>(smem);
            float* F = PF + FACE_OFF;
            float e0[NL], e1[NL];  // face vectors at the lane's 2 nodes along a line
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                e0[t] = ld<float>(a.e0, 2 * q + t);
                e1[t] = ld<float>(a.e1, 2 * q + t);
            }
#pragma unroll
            for (int s = 0; s < M; ++s)
#pragma unroll
                for (int t = 0; t < NL; ++t) PF[s * SLOT + off.o[t]] = qb[s][t];
            faces_dir<0>(F, qb, e0, e1, line, q);
            __syncthreads();
            {
                float u[M][NL];
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) u[s][t] = PF[s * SLOT + off.y[t]];  // y-role (z, x)
                faces_dir<1>(F, u, e0, e1, line, q);
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) u[s][t] = PF[s * SLOT + off.z[t]];  // z-role (y, x)
                faces_dir<2>(F, u, e0, e1, line, q);
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
__global__ void __launch_bounds__(256) stp_mfma_kernel(StpArgs a)
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
