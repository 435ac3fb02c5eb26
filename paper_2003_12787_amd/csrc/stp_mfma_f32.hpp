// stp_mfma_f32.hpp -- predictor kernel with the derivative contractions on the FP32 matrix cores, for the
// Cartesian presets (acoustic, elastic) at order N = 7 (8 nodes per axis), FP32 I/O and FP32 arithmetic.
//
// Mathematics as in the other kernels (Sec. II-A, Eq. (4), Fig. 5 recompute of favg, Sec. II-B faces). The 1D
// derivative u -> D u (the sum-factorised contraction of Sec. III-B) runs as FP32 matrix products; pointwise
// terms, the time accumulation and the faces stay on the VALU.
//
// Lane layout: an element is 128 lanes (two waves). In every group of eight lanes, lanes i = 0..3 hold the nodes
// 0..3 (h = 0) and lanes i = 4..7 the nodes 4..7 (h = 1) of four lines, lane i and lane 7 - i the same line. A
// lane's line (a, b) (la(), lb()) is the same pair in its three roles: the owner holds the x-line (z, y) = (a, b),
// the y-role the y-line (z, x) = (a, b), the z-role the z-line (y, x) = (a, b), each at the four node positions
// 4h .. 4h + 3 along its line; line index L = 8a + b.
//
// The derivative: v_mfma_f32_4x4x1f32 forms 16 independent 4x4 outer products, one per block of four lanes: lane
// l's accumulator register r gains A of lane 4 (l / 4) + r times B of lane l. The lanes of a block share h. With
// B = the lane's value at node 4h + m and A = D[4G + l % 4][4h + m] (eight constants per lane), four products
// (m = 0..3) accumulate in register r of every lane of the block the sum over the lane's own four nodes of
// D[4G + r][k] u_k: its half's share of the derivative at output node 4G + r of its own line. Chain 0 takes the
// lane's own output group (G = h), chain 1 its partner's (G = 1 - h); one DPP add (row_half_mirror, lane i <->
// 7 - i) then completes each of the lane's four derivatives with the partner's chain-1 share. Every product is
// useful (the 4x4 blocks are the lanes' own lines), and the 8 products per line and quantity run at the FP32
// matrix rate with no VALU work but the four adds. This is the x-derivative, which the owner needs at its own
// nodes.
//
// The y- and z-derivatives go to the owners through LDS, so their lanes (the roles) may hold any nodes: there
// lanes i and i + 4 of a group of eight hold the same line (row r = i % 4 of both blocks of the pair), and the
// tile values are the A operand, broadcast from one block of the pair to both (cbsz = 1; abid = 0 takes the
// nodes 0..3 of the h = 0 block, abid = 1 the nodes 4..7 of the h = 1 block). With B = D[4h + l % 4][4 abid + m],
// one chain of eight products leaves in register r of lane l the derivative at node 4h + l % 4 of the line of
// row r: complete, with no VALU work at all, and stored to the exchange buffer from there.
#pragma once
#include "stp_device.hpp"
#include "stp_fused.hpp"
#include "stp_kernels.hpp"
#include "stp_mfma.hpp"

namespace stp {
namespace mfma32 {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// v of the lane's partner: lane i <-> 7 - i in its group of eight lanes (DPP row_half_mirror)
__device__ inline float mirror(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xf, 0xf,
                                                                 false));
}

// Orders a wave's LDS accesses before and after this point against each other (the LDS executes a wave's
// accesses in order; this keeps the compiler from moving them across).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// D u at the lane's four nodes 4h .. 4h + 3 of its line, from u at the same nodes (A as above).
__device__ inline void deriv4(const float (&A)[2][4], const float (&u)[4], float (&out)[4])
{
    f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(A[0][m], u[m], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(A[1][m], u[m], c1, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = c0[i] + mirror(c1[i]);
}

template <int PHYS>
struct MfmaF {
    static_assert(PHYS == kElastic || PHYS == kAcoustic, "Cartesian presets");
    static constexpr int N = 7, n = 8, n2 = 64, n3 = 512;
    static constexpr int NL = 4;     // nodes per lane
    static constexpr int WG = 128;   // one element per workgroup (two waves)
    static constexpr int M = PhysTraits<PHYS>::m;
    static constexpr int NP = PhysTraits<PHYS>::np;
    using S = fused::Sets<PHYS>;
    static constexpr int NPS = S::NPS, NG = S::NG;
    static constexpr int SLOT = n3;  // one quantity's tile, swizzled (at())
    // The y- and z-derivatives are formed in one phase between two barriers. A quantity that only one of the two
    // directions differentiates gets its derivative written over its own tile values: the lanes of a wave read
    // those nodes before they write them, and no other wave reads them in that phase (the y-role lines of wave w
    // have z2 = w, its z-role lines y2 = w). The quantities both directions differentiate (shared) need exchange
    // slots, one set per direction.
    static constexpr bool shared(int q)
    {
        bool y = false, z = false;
        for (int k = 0; k < NG; ++k) {
            y = y || S::dq(1, k) == q;
            z = z || S::dq(2, k) == q;
        }
        return y && z;
    }
    static constexpr int NGS = [] {
        int c = 0;
        for (int q = 0; q < M; ++q) c += shared(q) ? 1 : 0;
        return c;
    }();
    // exchange slot of a shared quantity (its rank among the shared ones), -1 for the others
    static constexpr int gslot(int q)
    {
        if (!shared(q)) return -1;
        int c = 0;
        for (int i = 0; i < q; ++i) c += shared(i) ? 1 : 0;
        return c;
    }
    // LDS (floats): the tile of the quantities differentiated along y or z, then the exchange slots of the y- and
    // of the z-derivatives. Outputs are staged over them (each wave's half of an output block, its lines padded by
    // 4 floats), and the face pass holds an FP32 q-bar tile of all quantities followed by the face values. The
    // elastic kernel's 32 KB leave room for the four elements per CU that its registers allow.
    static constexpr int P_OFF = 0, GY_OFF = NPS * SLOT, GZ_OFF = GY_OFF + NGS * SLOT;
    static constexpr int ELDS = GZ_OFF + NGS * SLOT;
    // tile word offset of the direction-D derivative of quantity q (exchange slot or in place)
    static constexpr int dslot(int D, int q)
    {
        return gslot(q) >= 0 ? (D == 1 ? GY_OFF : GZ_OFF) + gslot(q) * SLOT : P_OFF + S::slot(q) * SLOT;
    }
    static constexpr int LINE = n * M;        // floats of one line of an output block
    static constexpr int SLINE = LINE + 4;    // staged line (16-byte aligned)
    static constexpr int WSTAGE = 32 * SLINE; // one wave's staging area (its 32 owner lines)
    static constexpr int FACE_OFF = M * SLOT;
    static constexpr int max3(int x, int y, int z) { return x > y ? (x > z ? x : z) : (y > z ? y : z); }
    static constexpr int LDS_FLOATS = max3(ELDS, FACE_OFF + 6 * n2 * M, 2 * WSTAGE);

    // x-derivative index of quantity q (k with dq(0, k) == q), or -1
    static constexpr int kx(int q)
    {
        for (int k = 0; k < NG; ++k)
            if (S::dq(0, k) == q) return k;
        return -1;
    }

    // The lane's line (a, b): slot q = 4 (l / 8 % 4) + (i < 4 ? i : 7 - i) of its half-wave p = l / 32, with
    // i = l % 8, gives b = q % 4 + 4p and a = q / 4 + 4w. The 32 lanes of a half-wave hold 16 lines, each at the
    // nodes of both halves h.
    __host__ __device__ static constexpr int lslot(int l)
    {
        return 4 * ((l >> 3) & 3) + ((l & 7) < 4 ? (l & 7) : 7 - (l & 7));
    }
    __host__ __device__ static constexpr int la(int w, int l) { return (lslot(l) >> 2) + 4 * w; }
    __host__ __device__ static constexpr int lb(int l) { return (lslot(l) & 3) + 4 * (l >> 5); }
    __host__ __device__ static constexpr int half(int l) { return (l >> 2) & 1; }

    // Tile address of node (z, y, x), an XOR swizzle. The LDS serves 32 lanes at a time from 32 banks; the 32
    // lanes of a half-wave hold 16 lines at one node position t of each half h. Per access (fixed w, p, t) the
    // owner lanes vary y0, y1, z0, z1 and x2 (= h), the y-role lanes x0, x1, z0, z1 and y2, the z-role lanes x0,
    // x1, y0, y1 and z2. The bank bits
    //   b0 = x0 ^ y0, b1 = x1 ^ y1, b2 = x2 ^ y2 ^ z2, b3 = z0 ^ x0, b4 = z1 ^ x1
    // are independent over each of these sets, so every pattern hits 32 distinct banks; the group bits (y0, y1,
    // y2, z2) complete a permutation of the 512 nodes.
    __host__ __device__ static constexpr int at(int z, int y, int x)
    {
        const int x0 = x & 1, x1 = (x >> 1) & 1, x2 = (x >> 2) & 1;
        const int y0 = y & 1, y1 = (y >> 1) & 1, y2 = (y >> 2) & 1;
        const int z0 = z & 1, z1 = (z >> 1) & 1, z2 = (z >> 2) & 1;
        const int bank = (x0 ^ y0) | ((x1 ^ y1) << 1) | ((x2 ^ y2 ^ z2) << 2) | ((z0 ^ x0) << 3) | ((z1 ^ x1) << 4);
        const int group = y0 | (y1 << 1) | (y2 << 2) | (z2 << 3);
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
    // The y- and z-role lines (a, b): slot q = 4 (l / 8 % 4) + l % 4, b = q % 4 + 4p, a = q / 4 + 4w; lanes i and
    // i + 4 of a group (the two blocks of a broadcast pair) hold the same line, at the nodes of either half.
    __host__ __device__ static constexpr int rslot(int l) { return 4 * ((l >> 3) & 3) + (l & 3); }
    __host__ __device__ static constexpr int ra(int w, int l) { return (rslot(l) >> 2) + 4 * w; }
    __host__ __device__ static constexpr int rb(int l) { return (rslot(l) & 3) + 4 * (l >> 5); }

    // every role covers the 64 lines once per half h; lanes i and 7 - i of a group hold the same owner line,
    // lanes i and i + 4 the same role line
    static constexpr bool lines_ok()
    {
        int seen[2][2][n2] = {};
        for (int w = 0; w < 2; ++w)
            for (int l = 0; l < 64; ++l) {
                if (la(w, l) != la(w, l ^ 7) || lb(l) != lb(l ^ 7) || half(l) == half(l ^ 7)) return false;
                if (ra(w, l) != ra(w, l ^ 4) || rb(l) != rb(l ^ 4)) return false;
                seen[0][half(l)][8 * la(w, l) + lb(l)]++;
                seen[1][half(l)][8 * ra(w, l) + rb(l)]++;
            }
        for (int r = 0; r < 2; ++r)
            for (int hh = 0; hh < 2; ++hh)
                for (int L = 0; L < n2; ++L)
                    if (seen[r][hh][L] != 1) return false;
        return true;
    }
    static_assert(lines_ok(), "lane-to-line maps");
    // the 32 lanes of a half-wave at one node position t hit 32 distinct banks in each role
    static constexpr bool conflict_free()
    {
        for (int w = 0; w < 2; ++w)
            for (int p = 0; p < 2; ++p)
                for (int t = 0; t < NL; ++t)
                    for (int role = 0; role < 3; ++role) {
                        bool bank[32] = {};
                        for (int l = 32 * p; l < 32 * p + 32; ++l) {
                            const int a = la(w, l), b = lb(l), pos = 4 * half(l) + t;
                            const int v = role == 0 ? at(a, b, pos) : (role == 1 ? at(a, pos, b) : at(pos, a, b));
                            if (bank[v % 32]) return false;
                            bank[v % 32] = true;
                        }
                    }
        return true;
    }
    static_assert(conflict_free(), "every access pattern of a half-wave is free of bank conflicts");
    // the roles' reads (lane's own line at node 4h + t) and writes (register r: the line of row r of the lane's
    // group at node 4h + l % 4) of a half-wave hit 32 distinct banks
    static constexpr bool roles_conflict_free()
    {
        for (int w = 0; w < 2; ++w)
            for (int p = 0; p < 2; ++p)
                for (int t = 0; t < NL; ++t)
                    for (int role = 1; role < 3; ++role)
                        for (int wr = 0; wr < 2; ++wr) {
                            bool bank[32] = {};
                            for (int l = 32 * p; l < 32 * p + 32; ++l) {
                                const int ll = wr ? (l & ~3) | t : l;  // lane of the written line's row
                                const int a = ra(w, ll), b = rb(ll), pos = 4 * half(l) + (wr ? (l & 3) : t);
                                const int v = role == 1 ? at(a, pos, b) : at(pos, a, b);
                                if (bank[v % 32]) return false;
                                bank[v % 32] = true;
                            }
                        }
        return true;
    }
    static_assert(roles_conflict_free(), "the roles' reads and writes are free of bank conflicts");

    // LDS byte addresses (fixed for the kernel's lifetime): the owner's four nodes (o), the roles' reads of their
    // own line's four nodes (yr, zr) and writes of the four lines of their group at one node (yw, zw). Slots and
    // regions are constant distances, folded into the instructions' offset fields.
    struct Offs {
        unsigned o[NL], yr[NL], yw[NL], zr[NL], zw[NL];
    };
    __device__ static inline Offs offsets(int wv, int l)
    {
        Offs f;
        const int h = half(l), ca = la(wv, l), cb = lb(l), a = ra(wv, l), b = rb(l);
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int ll = (l & ~3) | t, wa = ra(wv, ll), wb = rb(ll), node = 4 * h + (l & 3);
            f.o[t] = (unsigned)at(ca, cb, 4 * h + t) << 2;
            f.yr[t] = (unsigned)at(a, 4 * h + t, b) << 2;
            f.zr[t] = (unsigned)at(4 * h + t, a, b) << 2;
            f.yw[t] = (unsigned)at(wa, node, wb) << 2;
            f.zw[t] = (unsigned)at(node, wa, wb) << 2;
        }
        return f;
    }
    __device__ static inline float& lds(unsigned char* smem, unsigned byte)
    {
        return *reinterpret_cast<float*>(smem + byte);
    }

    // Order of the x-pass over the quantities: first those only stored in the tile, then those whose x-derivative
    // feeds few accumulator rows, so that the registers of the lane's values are freed about as fast as the
    // accumulator rows fill (elastic: s_yy s_zz s_yz, s_xx s_xy s_xz, then the velocities, whose x-derivatives
    // feed the stresses; acoustic: v_y v_z, then p and v_x).
    static constexpr int xord(int i)
    {
        if constexpr (PHYS == kElastic) {
            constexpr int t[9] = {4, 5, 7, 3, 6, 8, 0, 1, 2};
            return t[i];
        } else {
            constexpr int t[4] = {2, 3, 0, 1};
            return t[i];
        }
    }

    // For every quantity (in the order xord): store the lane's four values in the tile (if the quantity is
    // differentiated along y or z), and if it is differentiated along x form its x-derivative and apply its
    // pointwise terms.
    template <int I, int R>
    __device__ static inline void xpass(const float (&A)[2][4], unsigned char* smem, const unsigned (&ow)[NL],
                                        const Material<float, PHYS> (&mt)[NL], const float (&v)[M][NL],
                                        float (&r)[R][NL])
    {
        if constexpr (I < M) {
            constexpr int Q = xord(I);
            constexpr int s = S::slot(Q);
            if constexpr (s >= 0) {
#pragma unroll
                for (int t = 0; t < NL; ++t) lds(smem, ow[t] + 4 * (P_OFF + s * SLOT)) = v[Q][t];
            }
            constexpr int k = kx(Q);
            if constexpr (k >= 0) {
                float g[NL];
                deriv4(A, v[Q], g);
                mfma::ncp_cart<PHYS, 0, k>(mt, g, r);
            }
            xpass<I + 1>(A, smem, ow, mt, v, r);
        }
    }

    // y- or z-role: the derivatives along D of the quantities dq(D, k) on the role lines, into their exchange
    // slots or in place (dslot). B[abid][m] = D[4h + l % 4][4 abid + m].
    template <int D>
    __device__ static inline void transposed(const float (&B)[2][4], unsigned char* smem, const Offs& f)
    {
        const unsigned(&rd)[NL] = D == 1 ? f.yr : f.zr;
        const unsigned(&wr)[NL] = D == 1 ? f.yw : f.zw;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int s = S::slot(S::dq(D, k));
            float u[NL];
#pragma unroll
            for (int t = 0; t < NL; ++t) u[t] = lds(smem, rd[t] + 4 * (P_OFF + s * SLOT));
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int m = 0; m < 4; ++m) c = __builtin_amdgcn_mfma_f32_4x4x1f32(u[m], B[0][m], c, 1, 0, 0);
#pragma unroll
            for (int m = 0; m < 4; ++m) c = __builtin_amdgcn_mfma_f32_4x4x1f32(u[m], B[1][m], c, 1, 1, 0);
#pragma unroll
            for (int t = 0; t < NL; ++t) lds(smem, wr[t] + 4 * dslot(D, S::dq(D, k))) = c[t];
        }
    }

    template <int D, int K = 0, int R = M>
    __device__ static inline void gather(unsigned char* smem, const unsigned (&ow)[NL],
                                         const Material<float, PHYS> (&mt)[NL], float (&r)[R][NL])
    {
        if constexpr (K < NG) {
            float g[NL];
#pragma unroll
            for (int t = 0; t < NL; ++t) g[t] = lds(smem, ow[t] + 4 * dslot(D, S::dq(D, K)));
            mfma::ncp_cart<PHYS, D, K>(mt, g, r);
            gather<D, K + 1>(smem, ow, mt, r);
        }
    }

    // r = V(v) at the lane's owner nodes: the x-pass from registers (it also stores v in the tile), then the y-
    // and z-derivatives through the tile and the exchange buffers. Ends after the gathers; the caller may rewrite
    // the tile at once (its last reads came before the barrier that precedes the gathers), and the exchange
    // buffers after its next barrier.
    //
    // The y-pass is local to each wave: wave w's owner lines have z2 = w, and so have its y-role lines, which read
    // only tile nodes its own x-pass wrote and write only nodes its own owners gather (the LDS executes a wave's
    // accesses in order). So the y-role pass follows the x-pass without a barrier, and the y-gather shares the
    // phase of the z-role pass (which reads both waves' tile writes: after the first barrier); the z-gather
    // follows the second barrier. Each phase mixes matrix-core and VALU work.
    __device__ static inline void volume(const float (&A)[2][4], const float (&B)[2][4], unsigned char* smem,
                                         const Offs& f, const Material<float, PHYS> (&mt)[NL],
                                         const float (&v)[M][NL], float (&r)[M][NL])
    {
        xpass<0>(A, smem, f.o, mt, v, r);
        transposed<1>(B, smem, f);
        __syncthreads();
        gather<1>(smem, f.o, mt, r);
        transposed<2>(B, smem, f);
        __syncthreads();
        gather<2>(smem, f.o, mt, r);
    }

    // 4 nodes x M quantities = 4M contiguous floats (16-byte aligned when the element block is)
    __device__ static inline void load4(const float* src, bool aligned, float (&v)[M][NL])
    {
        if (aligned) {
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
            for (int w = 0; w < NL * M; ++w) v[w % M][w / M] = src[w];
        }
    }

    // Store one output block (64 lines x 8 nodes x M contiguous floats at `dst`) through per-wave staging areas:
    // wave w's owner lines 32w .. 32w + 31 are 32 x LINE contiguous floats of the block, which the wave stages in its
    // own area (lines padded to SLINE floats) and copies out with 16-byte stores, each store instruction covering
    // 1 KB of consecutive addresses. The LDS executes a wave's accesses in order, so neither the copy nor the wave's
    // next use of its area waits for the other wave; the caller orders the areas against the other wave's use of
    // the same words. Falls back to per-lane stores when misaligned (`aligned` is uniform over the workgroup).
    __device__ static inline void store_wave(float* area, float* dst, const float (&v)[M][NL], int wv, int l,
                                             int line, int h, bool aligned)
    {
        if (!aligned) {
            float* d = dst + (line * n + 4 * h) * M;
#pragma unroll
            for (int w = 0; w < NL * M; ++w) d[w] = v[w % M][w / M];
            return;
        }
        float* my = area + wv * WSTAGE;
        float4* s4 = reinterpret_cast<float4*>(my + (line - 32 * wv) * SLINE + 4 * h * M);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const int w = 4 * i;
            s4[i] = make_float4(v[(w + 0) % M][(w + 0) / M], v[(w + 1) % M][(w + 1) / M],
                                v[(w + 2) % M][(w + 2) / M], v[(w + 3) % M][(w + 3) / M]);
        }
        wave_sync();
        constexpr int L4 = LINE / 4;  // float4 per line
        static_assert((32 * L4) % 64 == 0, "a wave's lines are a whole number of float4 per lane");
        float4* d4 = reinterpret_cast<float4*>(dst + (int64_t)wv * 32 * LINE);
#pragma unroll
        for (int i = 0; i < 32 * L4 / 64; ++i) {
            const int j = l + 64 * i, ln = j / L4, k = j - ln * L4;
            d4[j] = *reinterpret_cast<const float4*>(my + ln * SLINE + 4 * k);
        }
        wave_sync();
    }

    // The faces of direction D (0 x, 1 y, 2 z) from the q-bar values u[s][t] at the lane's nodes along its line in
    // that direction: F[(2D + side) n^2 + line][s], side h. eo and ep are the face vectors l_j(h) and l_j(1 - h)
    // at the lane's nodes: the lane's sum with eo plus its partner's sum with ep (the partner's own other side)
    // is the line's side-h face.
    template <int D>
    __device__ static inline void faces_dir(float* F, const float (&u)[M][NL], const float (&eo)[NL],
                                            const float (&ep)[NL], int line, int h)
    {
#pragma unroll
        for (int s = 0; s < M; ++s) {
            float so = eo[0] * u[s][0], sp = ep[0] * u[s][0];
#pragma unroll
            for (int t = 1; t < NL; ++t) {
                so = fma(eo[t], u[s][t], so);
                sp = fma(ep[t], u[s][t], sp);
            }
            F[((2 * D + h) * n2 + line) * M + s] = so + mirror(sp);
        }
    }

    __device__ static void run(const StpArgs& a)
    {
        extern __shared__ __align__(16) unsigned char smem[];
        const int tid = threadIdx.x;
        const int wv = tid >> 6, l = tid & 63;
        const int h = half(l);
        const int line = 8 * la(wv, l) + lb(l);  // the owner's x-line (z, y)
        const Offs off = offsets(wv, l);
        float* Sg = reinterpret_cast<float*>(smem);
        const bool per_elem = (a.flags & kParamPerElement) != 0;

        float A[2][4];  // chain g: A[g][m] = D[4G + l % 4][4h + m], output group G = h for g = 0, 1 - h for g = 1
        {
            const float* Dm = static_cast<const float*>(a.D);
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int m = 0; m < 4; ++m) A[g][m] = Dm[(4 * (g ^ h) + (l & 3)) * n + 4 * h + m];
        }
        float B[2][4];  // the roles' products: B[abid][m] = D[4h + l % 4][4 abid + m]
        {
            const float* Dm = static_cast<const float*>(a.D);
#pragma unroll
            for (int ab = 0; ab < 2; ++ab)
#pragma unroll
                for (int m = 0; m < 4; ++m) B[ab][m] = Dm[(4 * h + (l & 3)) * n + 4 * ab + m];
        }
        const int64_t cnt = a.count ? (int64_t)*a.count : a.nelem;

        for (int64_t it = blockIdx.x; it < cnt; it += gridDim.x) {
            ElemRef er;
            elem_ref(a, it, er);
            const int64_t node0 = (int64_t)line * n + 4 * h;  // first of the lane's 4 nodes
            const bool al = (er.q & 3) == 0;  // 16-byte aligned element blocks (float offsets)
            float p[M][NL], qb[M][NL];
            Material<float, PHYS> mt[NL];
            load4(static_cast<const float*>(a.Q) + er.q + node0 * M, al, p);
            {
                const float ih = (float)(1.0 / er.h);
                const float* par = static_cast<const float*>(a.params) + er.coef;
#pragma unroll
                for (int t = 0; t < NL; ++t) mt[t].load_f32(per_elem ? par : par + (node0 + t) * NP, ih);
            }
#pragma unroll
            for (int s = 0; s < M; ++s)
#pragma unroll
                for (int t = 0; t < NL; ++t) qb[s][t] = p[s][t];
            float w = 1.f;
            const float dt = (float)er.dt;
#pragma unroll 1
            for (int o = 1; o <= N; ++o) {
                float r[M][NL];
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) r[s][t] = 0.f;
                volume(A, B, smem, off, mt, p, r);
                w = w * dt * __builtin_amdgcn_rcpf((float)(o + 1));
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) {
                        p[s][t] = r[s][t];
                        qb[s][t] = fma(w, r[s][t], qb[s][t]);
                    }
                // No barrier here: the next step writes the tile after every lane has passed the barrier that
                // precedes this step's gathers (the tile's last reads come before it), and the exchange buffers
                // after the barrier that follows its own tile writes.
            }
            __syncthreads();  // the last gathers' reads of the tile and exchange slots, which stage the outputs

            // outputs: q-bar, the faces, favg
            const bool fsum = (a.flags & kFavgSum) != 0;
            store_wave(Sg, static_cast<float*>(a.qavg) + er.q, qb, wv, l, line, h, al);
            __syncthreads();  // both waves' copies out of their staging areas, which the face tile overwrites
            // faces (before favg, so that q-bar is no longer live once the favg x-pass has stored it in the tile):
            // the x-faces from the registers, the y- and z-faces from an FP32 q-bar tile. The face values are staged
            // in LDS in the output layout [f][a][b][s] and written with coalesced stores.
            float* PF = Sg;
            float* F = PF + FACE_OFF;
            {
                float eo[NL], ep[NL];  // face vectors l_j(h), l_j(1 - h) at the lane's 4 nodes along a line
#pragma unroll
                for (int t = 0; t < NL; ++t) {
                    eo[t] = ld<float>(h ? a.e1 : a.e0, 4 * h + t);
                    ep[t] = ld<float>(h ? a.e0 : a.e1, 4 * h + t);
                }
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) lds(smem, off.o[t] + 4 * s * SLOT) = qb[s][t];
                faces_dir<0>(F, qb, eo, ep, line, h);
                __syncthreads();
                // the y- and z-faces of the lines (z, x) resp. (y, x) = (la, lb) in the owner's lane layout, whose
                // line partners are DPP mirrors
                const int ca = la(wv, l), cb = lb(l);
                float u[M][NL];
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) u[s][t] = PF[s * SLOT + at(ca, 4 * h + t, cb)];
                faces_dir<1>(F, u, eo, ep, line, h);
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) u[s][t] = PF[s * SLOT + at(4 * h + t, ca, cb)];
                faces_dir<2>(F, u, eo, ep, line, h);
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
            {
                // favg = V_d(q-bar): the x-pass (its tile writes miss the face values still being copied out),
                // then, after a barrier, both transposed passes (which overwrite the face values) and the gathers.
                // The three direction blocks are held in registers and staged once the gathers have read the tile.
                float fx[M][NL], fy[M][NL], fz[M][NL];
#pragma unroll
                for (int s = 0; s < M; ++s)
#pragma unroll
                    for (int t = 0; t < NL; ++t) fx[s][t] = fy[s][t] = fz[s][t] = 0.f;
                xpass<0>(A, smem, off.o, mt, qb, fx);
                __syncthreads();
                transposed<1>(B, smem, off);
                transposed<2>(B, smem, off);
                __syncthreads();
                float* fav = static_cast<float*>(a.favg) + (fsum ? er.q : 3 * er.q);
                if (!fsum) {
                    gather<1>(smem, off.o, mt, fy);
                    gather<2>(smem, off.o, mt, fz);
                    __syncthreads();  // the gathers' reads, before the staging overwrites the tile
                    store_wave(Sg, fav, fx, wv, l, line, h, al);
                    store_wave(Sg, fav + (int64_t)n3 * M, fy, wv, l, line, h, al);
                    store_wave(Sg, fav + 2 * (int64_t)n3 * M, fz, wv, l, line, h, al);
                } else {
                    gather<1>(smem, off.o, mt, fx);
                    gather<2>(smem, off.o, mt, fx);
                    __syncthreads();  // the gathers' reads, before the staging overwrites the tile
                    store_wave(Sg, fav, fx, wv, l, line, h, al);
                }
            }
            __syncthreads();  // both waves' staging copies, before the next element's x-pass writes the tile
        }
    }
};

template <int PHYS>
__global__ void __launch_bounds__(128) stp_mfma32_kernel(StpArgs a)
{
    MfmaF<PHYS>::run(a);
}

template <int PHYS>
KernelInfo mfma32_info()
{
    using K = MfmaF<PHYS>;
    KernelInfo ki;
    ki.fn = reinterpret_cast<const void*>(&stp_mfma32_kernel<PHYS>);
    ki.block = K::WG;
    ki.mb = K::M;
    ki.elems_per_block = 1;
    ki.lds = [](int, bool) -> size_t { return sizeof(float) * (size_t)K::LDS_FLOATS; };
    ki.aux = KernelInfo::kAuxNone;
    return ki;
}

}  // namespace mfma32
}  // namespace stp
