// stp_mfma_hi.hpp -- predictor kernel with the derivative contractions on the matrix cores for the Cartesian
// presets (acoustic, elastic) at orders N = 8 and 9 (9 and 10 nodes per axis), FP32 I/O.
//
// Mathematics, split and accuracy as in the order-7 kernel (Sec. II-A, Eq. (4), Fig. 5 recompute of favg,
// Sec. II-B faces; the 1D derivative of the sum factorisation, Sec. III-B): u = hi + mid + lo (exact truncation
// split), D = D0 + D1 + D2 (host tables), BF16 products with FP32 accumulation. The contraction shape changes
// with n: ten (or nine) nodes per line with three pieces each are 30 (27) K entries, which fill the K = 32 of two
// chained v_mfma_f32_32x32x16_bf16.
//
// Lane layout: a wave covers 32 lines. Lane l has c = l % 32 (its line's column in the products) and
// h = l / 32; it holds the nodes 5h .. 5h + 4 of its line (for n = 9 the fifth node of the upper half is a zero
// pad). In the first product, lane half h supplies the K entries 8h .. 8h + 7 as the (hi | mid) words of its
// nodes 5h .. 5h + 3; in the second, the (hi | mid) word of node 5h + 4 and the lo pieces in pairs
// (5h | 5h + 1), (5h + 2 | 5h + 3), (5h + 4 | 0). The A operand has three rows per output node, one per piece
// D_P, each holding D_P on every piece of every input node. Lane half h' receives the accumulator rows
// 8i + 4h' + k (i, k < 4); its r-th row is output node 5h' + r / 3, piece r % 3. So the three rows of node j land
// in the lane that owns j, which adds them: D u at its own nodes with all nine products D_P u_Q, and no data
// moves between lanes.
//
// Each lane has a line in each of three roles: the owner role (an x-line (z, y): the lane loads, accumulates and
// stores its values), the y-role (line (z, x)) and the z-role (line (y, x)). The lines of each role come from a
// host-built table chosen so that the 32 lines of a wave fall in distinct LDS banks (as far as the residues
// allow). There are n^2 = 100 (81) lines and 128 (96) lanes. The remaining lanes of the last wave repeat lines
// of other waves: they compute the same values as the lane that holds the line (same inputs, same operations)
// and skip the stores.
//
// Per Taylor step: the owner splits its values, writes the split to the LDS tile and forms the x-derivatives
// from its registers; the y- and z-roles read their lines' split words from the tile and return the
// derivatives to the owners through an exchange buffer. The pointwise terms, the time accumulation and the faces
// stay on the VALU in FP32.
#pragma once
#include "stp_mfma.hpp"
#include "stp_mfma_hi_layout.hpp"

namespace stp {
namespace mfma {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// The split of a lane's 5 values as the B words of the two products: the (hi | mid) word of each node and the
// lo pieces in pairs (low half first).
struct Split5 {
    unsigned hm[5], lo[3];
};

// u = hi + mid + lo exactly (as split2 of the order-7 kernel). The tile's 16-bit lo of node t is the upper half
// of lo_bits[t].
__device__ inline Split5 split5(const float (&u)[5], unsigned (&lo_bits)[5])
{
    Split5 s;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const unsigned ub = __builtin_bit_cast(unsigned, u[t]);
        const float r = u[t] - __builtin_bit_cast(float, ub & 0xffff0000u);
        const unsigned rb = __builtin_bit_cast(unsigned, r);
        lo_bits[t] = __builtin_bit_cast(unsigned, r - __builtin_bit_cast(float, rb & 0xffff0000u));
        s.hm[t] = __builtin_amdgcn_perm(rb, ub, 0x07060302u);  // (hi | mid)
    }
    s.lo[0] = __builtin_amdgcn_perm(lo_bits[1], lo_bits[0], 0x07060302u);
    s.lo[1] = __builtin_amdgcn_perm(lo_bits[3], lo_bits[2], 0x07060302u);
    s.lo[2] = lo_bits[4] >> 16;
    return s;
}

// D u at the lane's own 5 nodes: two chained products, then the three pieces' rows of each node added.
__device__ inline void deriv_mfma32(const bf16x8 (&A)[2], const Split5& s, float (&out)[5])
{
    f32x16 c = {};
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0], as_bf16x8(s.hm[0], s.hm[1], s.hm[2], s.hm[3]), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1], as_bf16x8(s.hm[4], s.lo[0], s.lo[1], s.lo[2]), c, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 5; ++t) out[t] = (c[3 * t] + c[3 * t + 1]) + c[3 * t + 2];
}

template <int PHYS, int NORD>
struct MfmaHi {
    static constexpr int N = NORD, n = N + 1, n2 = n * n, n3 = n2 * n;
    static_assert(n == 9 || n == 10, "orders 8 and 9");
    static_assert(PHYS == kAcoustic || PHYS == kElastic, "Cartesian presets");
    static constexpr int NL = mfma_hi::kNodesPerLane;
    static constexpr bool kPad = n < 2 * NL;  // the upper half's fifth node is a pad
    static constexpr int W = mfma_hi::waves(n), WG = 64 * W;
    static constexpr int M = PhysTraits<PHYS>::m, NP = PhysTraits<PHYS>::np;
    using S = fused::Sets<PHYS>;
    using K8 = Mfma8<PHYS>;  // quantity pairs of the lo words and the pass orders (independent of n)
    static constexpr int NPS = S::NPS, NG = S::NG, NLP = K8::NLP;
    static constexpr int PY = n, PZ = mfma_hi::zstride(n), SLOT = mfma_hi::slot_words(n);
    static constexpr int align4(int x) { return (x + 3) & ~3; }
    // LDS (32-bit words): the (hi | mid) words of the tile, the lo words, the exchange buffer (which also stages
    // the output blocks, ROUND lines at a time, shifted by up to 3 floats to match the destination's alignment)
    static constexpr int HM_OFF = 0, LO_OFF = NPS * SLOT, G_OFF = align4(LO_OFF + NLP * SLOT);
    static constexpr int ELDS = G_OFF + NG * SLOT;
    static constexpr int LINE = n * M;  // floats of one line of an output block
    static constexpr int ROUND = ((ELDS - G_OFF - 3) / LINE) & ~3;
    static_assert(ROUND >= 4, "the staging holds four lines");
    // face pass: an FP32 q-bar tile (M slots), then the face values in the output layout
    static constexpr int FACE_OFF = align4(M * SLOT);
    static constexpr int FACE_END = FACE_OFF + 3 + 6 * n2 * M;
    static constexpr int LDS_FLOATS = ELDS > FACE_END ? ELDS : FACE_END;

    struct Lane {
        int h;
        bool v4;                       // node 5h + 4 exists
        int lo, ly, lz;                // lines of the owner, y- and z-roles
        bool dup_o, dup_y, dup_z;      // the lane repeats that role's line of another lane
        unsigned bo, by, bz;           // byte address of node 0 of the lane's nodes in each role's pattern
    };
    // node t of the lane in the owner, y- and z-patterns: bo + 4 t, by + 4 t PY, bz + 4 t PZ
    static constexpr unsigned SO = 4, SY = 4 * PY, SZ = 4 * PZ;

    // The pad node (n = 9, upper half, t = 4) stands in for the lane's fourth node: it loads, splits, writes and
    // reads that node's values at that node's addresses (the same values to the same words), and the A table
    // gives it zero columns and that node's rows, so it adds nothing to the products and stays a copy of the
    // fourth node through every step. Only the stores and the face sums (zero face weights) leave it out. This
    // keeps the loop free of per-lane predication.
    __device__ static inline bool valid(const Lane& L, int t) { return !kPad || t < NL - 1 || L.v4; }

    // A pass takes the byte addresses of the lane's five nodes in one pattern, from `region` on. Every access is
    // one of these plus a slot offset that fits the instruction's 16-bit offset field (each region plus its
    // slots stays under 64 KB). For the elastic tile of n = 10 (74 KB, 18 slots) the five addresses are separate
    // registers made opaque to the compiler, so no two accesses share a register and none is merged into a
    // two-address instruction that would need a new base (a VALU add) for each slot. The smaller tiles keep one
    // opaque base per pass, whose few merged pairs cost fewer adds than five registers cost occupancy.
    struct Pat {
        unsigned b[NL];
    };
    static constexpr bool kNodeRegs = PHYS == kElastic && n == 10;
    __device__ static inline Pat pat(unsigned base, unsigned st, bool v4, unsigned region)
    {
        Pat P;
        if constexpr (!kNodeRegs) base += (unsigned)opaque_zero();
#pragma unroll
        for (int t = 0; t < NL - 1; ++t) P.b[t] = base + region + st * t;
        P.b[NL - 1] = base + region + (!kPad || v4 ? 4u * st : 3u * st);
        if constexpr (kNodeRegs) asm volatile("" : "+v"(P.b[0]), "+v"(P.b[1]), "+v"(P.b[2]), "+v"(P.b[3]), "+v"(P.b[4]));
        return P;
    }
    static constexpr unsigned kTile = 4 * HM_OFF, kExch = 4 * G_OFF;  // region byte offsets
    static_assert(4 * (LO_OFF + NLP * SLOT) <= 65536 && 4 * NG * SLOT <= 65536 && 4 * M * SLOT <= 65536,
                  "slot offsets fit the 16-bit LDS offset field");

    __device__ static inline Lane lane_setup(const uint16_t* tab, int wv, int l)
    {
        Lane L;
        const int c = l & 31;
        L.h = l >> 5;
        L.v4 = NL * L.h + NL - 1 < n;
        const uint16_t* roles = tab + mfma_hi::kTableA + 32 * wv + c;
        const unsigned eo = roles[0], ey = roles[32 * W], ez = roles[64 * W];
        L.lo = (int)(eo & 0x7fffu);
        L.ly = (int)(ey & 0x7fffu);
        L.lz = (int)(ez & 0x7fffu);
        L.dup_o = (eo & mfma_hi::kDupBit) != 0;
        L.dup_y = (ey & mfma_hi::kDupBit) != 0;
        L.dup_z = (ez & mfma_hi::kDupBit) != 0;
        const int k0 = NL * L.h;
        L.bo = 4u * (unsigned)((L.lo / n) * PZ + (L.lo % n) * PY + k0);  // (z, y, k0 + t)
        L.by = 4u * (unsigned)((L.ly / n) * PZ + k0 * PY + L.ly % n);    // (z, k0 + t, x)
        L.bz = 4u * (unsigned)(k0 * PZ + (L.lz / n) * PY + L.lz % n);    // (k0 + t, y, x)
        return L;
    }

    template <typename T>
    __device__ static inline T& lds(unsigned char* smem, unsigned byte)
    {
        return *reinterpret_cast<T*>(smem + byte);
    }

    // For every quantity (in the order qord) that the tile holds: split the lane's 5 values and store the split
    // in the tile. `pend` carries the lo pieces of a pair's first quantity to its second, which writes the
    // pair's lo word. The values die here, before the derivatives' accumulators fill, which keeps the register
    // count within two waves per SIMD.
    template <int I>
    __device__ static inline void split_q(unsigned char* smem, const Pat& P, const float (&v)[M][NL],
                                          unsigned (&pend)[NL])
    {
        if constexpr (I < M) {
            constexpr int Q = K8::qord(I);
            constexpr int s = S::slot(Q), lp = K8::lo_pair(Q);
            if constexpr (s >= 0) {
                unsigned lo_bits[NL];
                const Split5 sp = split5(v[Q], lo_bits);
#pragma unroll
                for (int t = 0; t < NL; ++t)
                    lds<unsigned>(smem, P.b[t] + 4 * (s * SLOT)) = sp.hm[t];
                constexpr bool last = (lp & 1) == 1 || I + 1 >= M || K8::lo_pair(K8::qord(I + 1)) != lp + 1;
                if constexpr (!last) {
#pragma unroll
                    for (int t = 0; t < NL; ++t) pend[t] = lo_bits[t];
                } else {
#pragma unroll
                    for (int t = 0; t < NL; ++t) {
                        // (lo of the pair's first quantity | lo of the second), or the lone lo in the low half
                        const unsigned w = (lp & 1) ? __builtin_amdgcn_perm(lo_bits[t], pend[t], 0x07060302u)
                                                    : (lo_bits[t] >> 16);
                        lds<unsigned>(smem, P.b[t] + 4 * (LO_OFF + (lp >> 1) * SLOT)) = w;
                    }
                }
            }
            split_q<I + 1>(smem, P, v, pend);
        }
    }

    // x-derivatives of the quantities only differentiated along x (outside the tile), from the registers
    template <int I, int R>
    __device__ static inline void xpass_reg(const bf16x8 (&A)[2], const Material<float, PHYS> (&mt)[NL],
                                            const float (&v)[M][NL], float (&r)[R][NL])
    {
        if constexpr (I < M) {
            if constexpr (S::slot(I) < 0 && K8::kx(I) >= 0) {
                unsigned lo_bits[NL];
                const Split5 sp = split5(v[I], lo_bits);
                float g[NL];
                deriv_mfma32(A, sp, g);
                ncp_cart<PHYS, 0, K8::kx(I)>(mt, g, r);
            }
            xpass_reg<I + 1>(A, mt, v, r);
        }
    }

    // The split of the lane's values of quantity q at its nodes along its line in the pattern (P, ST), read
    // from the tile. `lw` holds the lo words of q's pair, read unless `reuse` (the pair's other quantity was read
    // just before).
    __device__ static inline Split5 read_split(unsigned char* smem, const Pat& P, int q, bool reuse,
                                               unsigned (&lw)[NL])
    {
        const int s = S::slot(q), lp = K8::lo_pair(q);
        Split5 sp;
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            sp.hm[t] = lds<unsigned>(smem, P.b[t] + 4 * (s * SLOT));
            if (!reuse) lw[t] = lds<unsigned>(smem, P.b[t] + 4 * (LO_OFF + (lp >> 1) * SLOT));
        }
        // the quantity's half of the lo words, packed by node pairs
        const unsigned sel = (lp & 1) ? 0x07060302u : 0x05040100u;
        sp.lo[0] = __builtin_amdgcn_perm(lw[1], lw[0], sel);
        sp.lo[1] = __builtin_amdgcn_perm(lw[3], lw[2], sel);
        sp.lo[2] = (lp & 1) ? (lw[4] >> 16) : (lw[4] & 0xffffu);
        return sp;
    }

    // x-derivatives of the tile's quantities, from the owner's own tile entries (no barrier needed: the lane
    // wrote them), with their pointwise terms
    template <int R>
    __device__ static inline void xpass_tile(const bf16x8 (&A)[2], unsigned char* smem, const Lane& L,
                                             const Material<float, PHYS> (&mt)[NL], float (&r)[R][NL])
    {
        unsigned lw[NL] = {0u, 0u, 0u, 0u, 0u};
        xpass_tile_q<0>(A, smem, pat(L.bo, SO, L.v4, kTile), mt, r, lw);
    }
    template <int I, int R>
    __device__ static inline void xpass_tile_q(const bf16x8 (&A)[2], unsigned char* smem, const Pat& P,
                                               const Material<float, PHYS> (&mt)[NL], float (&r)[R][NL],
                                               unsigned (&lw)[NL])
    {
        if constexpr (I < NG) {
            constexpr int q = S::dq(0, K8::kord(0, I));
            if constexpr (S::slot(q) >= 0) {
                constexpr int lp = K8::lo_pair(q);
                constexpr bool reuse = I > 0 && (lp & 1) == 1 && S::slot(S::dq(0, K8::kord(0, I - 1))) >= 0 &&
                                       K8::lo_pair(S::dq(0, K8::kord(0, I - 1))) == lp - 1;
                const Split5 sp = read_split(smem, P, q, reuse, lw);
                float g[NL];
                deriv_mfma32(A, sp, g);
                ncp_cart<PHYS, 0, K8::kord(0, I)>(mt, g, r);
            }
            xpass_tile_q<I + 1>(A, smem, P, mt, r, lw);
        }
    }

    // One direction-x pass of a Taylor step (or of the favg pass): split v into the tile, then r += the
    // x-contributions.
    template <int R>
    __device__ static inline void split_xpass(const bf16x8 (&A)[2], unsigned char* smem, const Lane& L,
                                              const Material<float, PHYS> (&mt)[NL], const float (&v)[M][NL],
                                              float (&r)[R][NL])
    {
        unsigned pend[NL] = {0u, 0u, 0u, 0u, 0u};
        split_q<0>(smem, pat(L.bo, SO, L.v4, kTile), v, pend);
        xpass_reg<0>(A, mt, v, r);
        xpass_tile(A, smem, L, mt, r);
    }

    // y- or z-role: the derivatives along D of the quantities dq(D, kord(D, i)), i < NG, into exchange slot i.
    // A lo word is read once for the two quantities of its pair when they follow each other. The pad node reads
    // nothing and contributes zeros.
    template <int D>
    __device__ static inline void transposed(const bf16x8 (&A)[2], unsigned char* smem, const Lane& L)
    {
        constexpr unsigned ST = D == 1 ? SY : SZ;
        const unsigned base = D == 1 ? L.by : L.bz;
        const Pat P = pat(base, ST, L.v4, kTile), PG = pat(base, ST, L.v4, kExch);
        unsigned lw[NL] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            const int q = S::dq(D, K8::kord(D, i));
            const int lp = K8::lo_pair(q);
            const bool reuse = i > 0 && (lp & 1) == 1 && K8::lo_pair(S::dq(D, K8::kord(D, i - 1))) == lp - 1;
            const Split5 sp = read_split(smem, P, q, reuse, lw);
            float g[NL];
            deriv_mfma32(A, sp, g);
#pragma unroll
            for (int t = 0; t < NL; ++t)
                lds<float>(smem, PG.b[t] + 4 * (i * SLOT)) = g[t];
        }
    }

    // r += the y- or z-contributions from the exchange buffer (after a barrier that follows transposed<D>)
    template <int D, int R>
    __device__ static inline void gather(unsigned char* smem, const Lane& L, const Material<float, PHYS> (&mt)[NL],
                                         float (&r)[R][NL])
    {
        gather_q<D, 0>(smem, pat(L.bo, SO, L.v4, kExch), mt, r);
    }
    template <int D, int I, int R>
    __device__ static inline void gather_q(unsigned char* smem, const Pat& P, const Material<float, PHYS> (&mt)[NL],
                                           float (&r)[R][NL])
    {
        if constexpr (I < NG) {
            float g[NL];
#pragma unroll
            for (int t = 0; t < NL; ++t) g[t] = lds<float>(smem, P.b[t] + 4 * (I * SLOT));
            ncp_cart<PHYS, D, K8::kord(D, I)>(mt, g, r);
            gather_q<D, I + 1>(smem, P, mt, r);
        }
    }

    // Copy nf floats from LDS S to dst, which agree modulo 16 bytes: 16-byte stores between a scalar head and
    // tail.
    __device__ static inline void copy_out(const float* S, float* dst, int nf, int tid)
    {
        int head = (int)((4u - ((unsigned)((uintptr_t)dst >> 2) & 3u)) & 3u);
        if (head > nf) head = nf;
        if (tid < head) dst[tid] = S[tid];
        const int nb = (nf - head) >> 2;
        const float4* s4 = reinterpret_cast<const float4*>(S + head);
        float4* d4 = reinterpret_cast<float4*>(dst + head);
        for (int j = tid; j < nb; j += WG) d4[j] = s4[j];
        const int t0 = head + 4 * nb;
        if (t0 + tid < nf) dst[t0 + tid] = S[t0 + tid];
    }

    // Store an output block (n^2 lines of LINE contiguous floats at dst) through the exchange buffer G, ROUND
    // lines per round: each owner lane writes its nodes' values, then the workgroup copies the round out. The
    // staging is shifted by dst's misalignment so that both sides of the copy are 16-byte aligned together. Ends
    // with a workgroup barrier; the caller has passed a barrier after the last read of G.
    __device__ static inline void store_block(float* G, float* dst, const float (&v)[M][NL], const Lane& L, int tid)
    {
        float* S = G + (int)(((uintptr_t)dst >> 2) & 3u);
#pragma unroll 1
        for (int l0 = 0; l0 < n2; l0 += ROUND) {
            const int cnt = n2 - l0 < ROUND ? n2 - l0 : ROUND;
            if (!L.dup_o && L.lo >= l0 && L.lo < l0 + cnt) {
                float* d = S + (L.lo - l0) * LINE + NL * L.h * M;
#pragma unroll
                for (int t = 0; t < NL; ++t)
                    if (valid(L, t))
#pragma unroll
                        for (int s = 0; s < M; ++s) d[t * M + s] = v[s][t];
            }
            __syncthreads();
            copy_out(S, dst + (int64_t)l0 * LINE, cnt * LINE, tid);
            __syncthreads();
        }
    }

    // The faces of direction D from the q-bar values u[s][t] at the lane's nodes along its line of that
    // direction: the partial sums over the lane's nodes, completed over the line's two lanes by one
    // permlane32_swap per quantity, which leaves side 0 in the lower half (h = 0) and side 1 in the upper half.
    template <int D>
    __device__ static inline void faces_dir(float* F, const float (&u)[M][NL], const float (&e0)[NL],
                                            const float (&e1)[NL], int line, int h, bool dup)
    {
#pragma unroll
        for (int s = 0; s < M; ++s) {
            float s0 = e0[0] * u[s][0], s1 = e1[0] * u[s][0];
#pragma unroll
            for (int t = 1; t < NL; ++t) {
                s0 = fma(e0[t], u[s][t], s0);
                s1 = fma(e1[t], u[s][t], s1);
            }
            const auto y = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, s0),
                                                            __builtin_bit_cast(unsigned, s1), false, false);
            const float v = __builtin_bit_cast(float, y[0]) + __builtin_bit_cast(float, K8::opaque_u(y[1]));
            if (!dup) F[((2 * D + h) * n2 + line) * M + s] = v;
        }
    }

    __device__ static void run(const StpArgs& a)
    {
        extern __shared__ __align__(16) unsigned char smem[];
        float* smf = reinterpret_cast<float*>(smem);
        const int tid = threadIdx.x;
        const int wv = tid >> 6, l = tid & 63;
        const uint16_t* tab = static_cast<const uint16_t*>(a.Dsplit);
        const Lane L = lane_setup(tab, wv, l);
        bf16x8 A[2];
        {
            const unsigned* t = reinterpret_cast<const unsigned*>(tab) + 8 * l;  // [64 lanes][2][8 BF16]
            A[0] = as_bf16x8(t[0], t[1], t[2], t[3]);
            A[1] = as_bf16x8(t[4], t[5], t[6], t[7]);
        }
        float* G = smf + G_OFF;
        const bool per_elem = (a.flags & kParamPerElement) != 0;
        const int64_t cnt = a.count ? (int64_t)*a.count : a.nelem;

        for (int64_t it = blockIdx.x; it < cnt; it += gridDim.x) {
            ElemRef er;
            elem_ref(a, it, er);
            const int64_t node0 = (int64_t)L.lo * n + NL * L.h;  // first of the lane's owner nodes
            float p[M][NL], qb[M][NL];
            Material<float, PHYS> mt[NL];
            {
                const float* q = static_cast<const float*>(a.Q) + er.q + node0 * M;
                const float ih = (float)(1.0 / er.h);
                const float* par = static_cast<const float*>(a.params) + er.coef;
#pragma unroll
                for (int t = 0; t < NL; ++t) {
                    const int x = t < NL - 1 || valid(L, t) ? t : t - 1;  // the pad loads the fourth node
#pragma unroll
                    for (int s = 0; s < M; ++s) p[s][t] = q[x * M + s];
                    mt[t].load_f32(per_elem ? par : par + (node0 + x) * NP, ih);
                }
            }
#pragma unroll
            for (int s = 0; s < M; ++s)
#pragma unroll
                for (int t = 0; t < NL; ++t) qb[s][t] = p[s][t];
            float w = 1.f;
            const float dt = (float)er.dt;
            // Tile and exchange buffer are each read only between two barriers that follow their writes, so a
            // step needs four barriers: the next step's tile writes come after the barrier that precedes this
            // step's last gather, and its exchange writes after the barrier that follows its own tile writes.
#pragma unroll 1
            for (int o = 1; o <= N; ++o) {
                float r[M][NL];
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) r[s][t] = 0.f;
                split_xpass(A, smem, L, mt, p, r);
                __syncthreads();
                transposed<1>(A, smem, L);
                __syncthreads();
                gather<1>(smem, L, mt, r);
                __syncthreads();
                transposed<2>(A, smem, L);
                __syncthreads();
                gather<2>(smem, L, mt, r);
                w = w * dt * __builtin_amdgcn_rcpf((float)(o + 1));
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) {
                        p[s][t] = r[s][t];
                        qb[s][t] = fma(w, p[s][t], qb[s][t]);
                    }
            }
            __syncthreads();  // the last gather's reads of the exchange buffer, which stages the outputs

            const bool fsum = (a.flags & kFavgSum) != 0;
            store_block(G, static_cast<float*>(a.qavg) + er.q, qb, L, tid);
            {
                float fx[M][NL];
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) fx[s][t] = 0.f;
                split_xpass(A, smem, L, mt, qb, fx);
                float* fav = static_cast<float*>(a.favg) + (fsum ? er.q : 3 * er.q);
                if (!fsum) {
                    store_block(G, fav, fx, L, tid);  // ends with a barrier: the tile is complete
#pragma unroll
                    for (int s = 0; s < M; ++s)
#pragma unroll
                        for (int t = 0; t < NL; ++t) fx[s][t] = 0.f;
                } else {
                    __syncthreads();
                }
                transposed<1>(A, smem, L);
                __syncthreads();
                gather<1>(smem, L, mt, fx);
                __syncthreads();
                if (!fsum) {
                    store_block(G, fav + (int64_t)n3 * M, fx, L, tid);
#pragma unroll
                    for (int s = 0; s < M; ++s)
#pragma unroll
                        for (int t = 0; t < NL; ++t) fx[s][t] = 0.f;
                }
                transposed<2>(A, smem, L);
                __syncthreads();
                gather<2>(smem, L, mt, fx);
                __syncthreads();
                store_block(G, fsum ? fav : fav + 2 * (int64_t)n3 * M, fx, L, tid);
            }
            // faces: the x-faces from the registers, the y- and z-faces from an FP32 q-bar tile; staged in LDS
            // in the output layout [f][a][b][s] and copied out with 16-byte stores
            float* qf = static_cast<float*>(a.qface) + er.face;
            float* F = smf + FACE_OFF + (int)(((uintptr_t)qf >> 2) & 3u);
            float e0[NL], e1[NL];
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                e0[t] = valid(L, t) ? ld<float>(a.e0, NL * L.h + t) : 0.f;
                e1[t] = valid(L, t) ? ld<float>(a.e1, NL * L.h + t) : 0.f;
            }
            const Pat Po = pat(L.bo, SO, L.v4, 0), Py = pat(L.by, SY, L.v4, 0), Pz = pat(L.bz, SZ, L.v4, 0);
#pragma unroll
            for (int s = 0; s < M; ++s)
#pragma unroll
                for (int t = 0; t < NL; ++t) lds<float>(smem, Po.b[t] + 4 * s * SLOT) = qb[s][t];
            faces_dir<0>(F, qb, e0, e1, L.lo, L.h, L.dup_o);
            __syncthreads();
            {
                float u[M][NL];
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t)
                        u[s][t] = lds<float>(smem, Py.b[t] + 4 * s * SLOT);
                faces_dir<1>(F, u, e0, e1, L.ly, L.h, L.dup_y);
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t)
                        u[s][t] = lds<float>(smem, Pz.b[t] + 4 * s * SLOT);
                faces_dir<2>(F, u, e0, e1, L.lz, L.h, L.dup_z);
            }
            __syncthreads();
            copy_out(F, qf, 6 * n2 * M, tid);
            __syncthreads();
        }
    }
};

// At least two waves per SIMD: two elastic workgroups share a CU (the LDS bound).
template <int PHYS, int NORD>
__global__ void __launch_bounds__(64 * mfma_hi::waves(NORD + 1)) __attribute__((amdgpu_waves_per_eu(2)))
stp_mfma_hi_kernel(StpArgs a)
{
    MfmaHi<PHYS, NORD>::run(a);
}

template <int PHYS, int NORD>
KernelInfo mfma_hi_info()
{
    using K = MfmaHi<PHYS, NORD>;
    KernelInfo ki;
    ki.fn = reinterpret_cast<const void*>(&stp_mfma_hi_kernel<PHYS, NORD>);
    ki.block = K::WG;
    ki.mb = K::M;
    ki.elems_per_block = 1;
    ki.lds = [](int, bool) -> size_t { return sizeof(float) * (size_t)K::LDS_FLOATS; };
    ki.aux = KernelInfo::kAuxMfmaSplit;
    return ki;
}

}  // namespace mfma
}  // namespace stp
