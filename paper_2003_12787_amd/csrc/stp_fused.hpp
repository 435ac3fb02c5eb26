// stp_fused.hpp -- fused predictor kernel for the physics presets (acoustic, elastic).
//
// Same mathematics as the plain kernel (Sec. II-A, Eq. (4), Fig. 5 recompute of favg, Sec. II-B faces), with
// the element's work mapped onto lanes so that most data stays in registers:
//   - each lane owns one x-line (z, y) of an element: its n nodes x all m quantities of the current Taylor
//     term p, the accumulator q-bar, and the material coefficients of those nodes;
//   - derivatives along x are computed from the lane's own registers;
//   - derivatives along y and z read the lines through an LDS tile of p (only the quantities the physics
//     differentiates in y or z) in the transposed roles (lane = (z, x) resp. (y, x)), and the results come
//     back to the owning lanes through an LDS exchange buffer of the quantities differentiated per direction;
//   - every 1D derivative uses the centro-antisymmetry of D on the symmetric Gauss-Legendre nodes
//     (D[n-1-i][n-1-j] = -D[i][j]): even/odd parts of the line halve the multiply-adds (n^2/2 instead of n^2);
//   - the pointwise terms are the sparse preset products (8 FMAs per node and direction for elastic);
//   - the SplitCK footprint (Fig. 5): one p, one q-bar, no stored Taylor terms or fluxes.
// Several elements share a workgroup when n^2 is small (lanes = elements x n^2 lines).
#pragma once
#include "stp_device.hpp"
#include "stp_kernels.hpp"

namespace stp {
namespace fused {

template <int PHYS>
struct Sets;

template <>
struct Sets<kElastic> {
    static constexpr int NPS = 8;  // LDS tile slots: every quantity except s_xx (only differentiated in x)
    static constexpr int NG = 6;   // quantities differentiated per direction: v_x, v_y, v_z, s_{d,x}, s_{d,y}, s_{d,z}
    __host__ __device__ static constexpr int slot(int q) { return q < 3 ? q : (q == 3 ? -1 : q - 1); }
    __host__ __device__ static constexpr int dq(int d, int k) { return k < 3 ? k : PhysTraits<kElastic>::sig(d, k - 3); }
};

// curvilinear elastic: every quantity is differentiated in every direction (used by the MFMA kernel)
template <>
struct Sets<kElasticCurv> {
    static constexpr int NPS = 9;
    static constexpr int NG = 9;
    __host__ __device__ static constexpr int slot(int q) { return q; }
    __host__ __device__ static constexpr int dq(int, int k) { return k; }
};

template <>
struct Sets<kAcoustic> {
    static constexpr int NPS = 3;  // p, v_y, v_z
    static constexpr int NG = 2;   // p and v_d
    __host__ __device__ static constexpr int slot(int q) { return q == 0 ? 0 : (q == 2 ? 1 : (q == 3 ? 2 : -1)); }
    __host__ __device__ static constexpr int dq(int d, int k) { return k == 0 ? 0 : 1 + d; }
};

// LDS strides (words): y-stride n, z-stride chosen so that the three access patterns (owner lanes (z,y),
// y-role lanes (z,x), z-role lanes (y,x)) are at most 2-way bank conflicted.
__host__ __device__ constexpr int zstride(int n)
{
    return n == 2 ? 4 : n == 3 ? 9 : n == 4 ? 19 : n == 5 ? 25 : n == 6 ? 36 : n == 7 ? 51 : 69;
}

// Workgroup size per order: elements are packed so that few lanes idle (lanes = EPB * n^2).
__host__ __device__ constexpr int wg_size(int n) { return n == 5 ? 128 : (n == 6 || n == 7) ? 128 : 64; }

template <typename T, int N, int PHYS>
struct Fused {
    static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n, h = n / 2;
    static constexpr bool odd = (n % 2) != 0;
    static constexpr int M = PhysTraits<PHYS>::m;
    static constexpr int NP = PhysTraits<PHYS>::np;
    static constexpr int WG = wg_size(n);
    static constexpr int EPB = WG / n2;  // elements per workgroup
    // n = 8: a 512-word XOR-swizzled tile (at()); other orders: padded linear tile, y-stride n, z-stride ZS
    static constexpr bool kSwz = n == 8;
    static constexpr int YS = n, ZS = zstride(n), SLOT = kSwz ? n3 : n * ZS;
    using S = Sets<PHYS>;
    static constexpr int NPS = S::NPS, NG = S::NG;
    static constexpr int ELDS = (NPS + NG) * SLOT;  // words of LDS per element
    static_assert(NPS + NG >= M, "face pass reuses the tile for all quantities");
    static_assert(n2 <= 64, "fused kernel covers n <= 8");

    // Tile address of node (z, y, x). For n = 8 the address is Lz(z) ^ Ly(y) ^ x, which puts the bank bits at
    //   b0 = x0 ^ z0, b1 = x1 ^ z1, b2 = x2 ^ y2, b3 = y0 ^ z0, b4 = y1 ^ z1
    // and z0, z1, z2, y2 in the four group bits. The 32 lanes of a half-wave vary in z0, z1, y0, y1, y2
    // (owner lines), z0, z1 and x (y-role lines) or y0, y1 and x (z-role lines), and the bank bits are
    // independent over each of these sets, so every access pattern hits 32 distinct banks. The padded linear
    // layout leaves 2-way conflicts.
    __host__ __device__ static constexpr int at(int z, int y, int x)
    {
        if constexpr (kSwz) {
            const int lz = (z & 1) * (1 | 8 | 32) ^ ((z >> 1) & 1) * (2 | 16 | 64) ^ ((z >> 2) & 1) * 128;
            const int ly = (y & 3) * 8 ^ ((y >> 2) & 1) * (4 | 256);
            return lz ^ ly ^ x;
        } else {
            return z * ZS + y * YS + x;
        }
    }
    static constexpr bool at_is_permutation()
    {
        bool seen[n * n * n] = {};
        for (int z = 0; z < n; ++z)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) {
                    const int v = at(z, y, x);
                    if (v < 0 || v >= n3 || seen[v]) return false;
                    seen[v] = true;
                }
        return true;
    }
    static_assert(!kSwz || at_is_permutation(), "the swizzled tile covers [0, n^3) once");

    // even/odd derivative tables: A[i][j], B[i][j] (i, j < h), Cm[i] (odd n), Am[j] (odd n)
    struct Tab {
        T A[h][h], B[h][h], Cm[h > 0 ? h : 1], Am[h > 0 ? h : 1];
    };

    // out = D u with the centro-antisymmetric split.
    __device__ static inline void deriv(const Tab& tb, const T (&u)[n], T (&out)[n])
    {
        T ue[h > 0 ? h : 1], uo[h > 0 ? h : 1];
#pragma unroll
        for (int j = 0; j < h; ++j) {
            ue[j] = u[j] + u[n - 1 - j];
            uo[j] = u[j] - u[n - 1 - j];
        }
#pragma unroll
        for (int i = 0; i < h; ++i) {
            T sa = 0, sb = 0;
#pragma unroll
            for (int j = 0; j < h; ++j) {
                sa = fma(tb.A[i][j], uo[j], sa);
                sb = fma(tb.B[i][j], ue[j], sb);
            }
            if constexpr (odd) sb = fma(tb.Cm[i], u[h], sb);
            out[i] = sa + sb;
            out[n - 1 - i] = sa - sb;
        }
        if constexpr (odd) {
            T sm = 0;
#pragma unroll
            for (int j = 0; j < h; ++j) sm = fma(tb.Am[j], uo[j], sm);
            out[h] = sm;
        }
        if constexpr (n == 1) out[0] = 0;
    }

    // r[.][x] += contribution of g = d/dxi_d of quantity dq(d, k) at the n nodes of the owner line.
    template <int D, int K>
    __device__ static inline void ncp(const Material<T, PHYS> (&mt)[n], const T (&g)[n], T (&r)[M][n])
    {
        if constexpr (PHYS == kElastic) {
            using P = PhysTraits<kElastic>;
            if constexpr (K < 3) {
                if constexpr (K == D) {
#pragma unroll
                    for (int x = 0; x < n; ++x) {
                        r[3 + D][x] = fma(mt[x].c[3], g[x], r[3 + D][x]);                 // s_dd <- (lam+2mu) dv_d
                        r[3 + (D + 1) % 3][x] = fma(mt[x].c[1], g[x], r[3 + (D + 1) % 3][x]);  // s_ii <- lam dv_d
                        r[3 + (D + 2) % 3][x] = fma(mt[x].c[1], g[x], r[3 + (D + 2) % 3][x]);
                    }
                } else {
                    constexpr int q = P::sig(D, K);
#pragma unroll
                    for (int x = 0; x < n; ++x) r[q][x] = fma(mt[x].c[2], g[x], r[q][x]);  // s_dk <- mu dv_k
                }
            } else {
                constexpr int i = K - 3;  // g = d s_{i,d}
#pragma unroll
                for (int x = 0; x < n; ++x) r[i][x] = fma(mt[x].c[0], g[x], r[i][x]);  // v_i <- (1/rho) ds_id
            }
        } else {
            if constexpr (K == 0) {
#pragma unroll
                for (int x = 0; x < n; ++x) r[1 + D][x] = fma(mt[x].c[1], g[x], r[1 + D][x]);  // v_d <- -(1/rho) dp
            } else {
#pragma unroll
                for (int x = 0; x < n; ++x) r[0][x] = fma(mt[x].c[0], g[x], r[0][x]);  // p <- -K dv_d
            }
        }
    }

    template <int D, int K>
    __device__ static inline void xpass_k(const Tab& tb, const Material<T, PHYS> (&mt)[n], const T (&p)[M][n],
                                          T (&r)[M][n])
    {
        T g[n];
        deriv(tb, p[S::dq(D, K)], g);
        ncp<D, K>(mt, g, r);
    }

    // x-direction: from the owner's registers
    template <int K = 0>
    __device__ static inline void xpass(const Tab& tb, const Material<T, PHYS> (&mt)[n], const T (&p)[M][n],
                                        T (&r)[M][n])
    {
        if constexpr (K < NG) {
            xpass_k<0, K>(tb, mt, p, r);
            xpass<K + 1>(tb, mt, p, r);
        }
    }

    // y or z role: derivative lines read from the tile, results written to the exchange buffer.
    // Role lane (a, b): y-role (a, b) = (z, x), lines (a, j, b); z-role (a, b) = (y, x), lines (j, a, b).
    template <int D>
    __device__ static inline void transposed(const Tab& tb, const T* P, T* G, int a, int b)
    {
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int s = S::slot(S::dq(D, k));
            T u[n], g[n];
#pragma unroll
            for (int j = 0; j < n; ++j)
                u[j] = D == 1 ? P[s * SLOT + at(a, j, b)] : P[s * SLOT + at(j, a, b)];
            deriv(tb, u, g);
#pragma unroll
            for (int i = 0; i < n; ++i) {
                if (D == 1) G[k * SLOT + at(a, i, b)] = g[i];
                else G[k * SLOT + at(i, a, b)] = g[i];
            }
        }
    }

    template <int D, int K = 0>
    __device__ static inline void gather(const T* G, int z, int y, const Material<T, PHYS> (&mt)[n], T (&r)[M][n])
    {
        if constexpr (K < NG) {
            T g[n];
#pragma unroll
            for (int x = 0; x < n; ++x) g[x] = G[K * SLOT + at(z, y, x)];
            ncp<D, K>(mt, g, r);
            gather<D, K + 1>(G, z, y, mt, r);
        }
    }

    // r = V(p) at the owner's line (contributions of all three directions); P already holds p.
    __device__ static inline void volume(const Tab& tb, T* P, T* G, int la, int lb, bool act,
                                         const Material<T, PHYS> (&mt)[n], const T (&p)[M][n], T (&r)[M][n])
    {
        if (act) transposed<1>(tb, P, G, la, lb);
#pragma unroll
        for (int q = 0; q < M; ++q)
#pragma unroll
            for (int x = 0; x < n; ++x) r[q][x] = 0;
        xpass(tb, mt, p, r);
        __syncthreads();
        if (act) gather<1>(G, la, lb, mt, r);
        __syncthreads();
        if (act) transposed<2>(tb, P, G, la, lb);
        __syncthreads();
        if (act) gather<2>(G, la, lb, mt, r);
    }

    __device__ static inline void write_tile(T* P, int z, int y, const T (&v)[M][n])
    {
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const int s = S::slot(q);
            if (s < 0) continue;
#pragma unroll
            for (int x = 0; x < n; ++x) P[s * SLOT + at(z, y, x)] = v[q][x];
        }
    }

    // contiguous line of n*M values (the x-line of all quantities) between global memory and registers
    __device__ static inline void load_line(const T* src, T (&v)[M][n])
    {
        if constexpr (sizeof(T) == 4 && (n * M) % 4 == 0) {
            if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
                const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
                for (int i = 0; i < n * M / 4; ++i) {
                    float4 t = s4[i];
                    const int w = 4 * i;
                    v[(w + 0) % M][(w + 0) / M] = t.x;
                    v[(w + 1) % M][(w + 1) / M] = t.y;
                    v[(w + 2) % M][(w + 2) / M] = t.z;
                    v[(w + 3) % M][(w + 3) / M] = t.w;
                }
                return;
            }
        }
#pragma unroll
        for (int w = 0; w < n * M; ++w) v[w % M][w / M] = src[w];
    }

    __device__ static inline void store_line(T* dst, const T (&v)[M][n])
    {
        if constexpr (sizeof(T) == 4 && (n * M) % 4 == 0) {
            if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
                for (int i = 0; i < n * M / 4; ++i) {
                    const int w = 4 * i;
                    d4[i] = make_float4(v[(w + 0) % M][(w + 0) / M], v[(w + 1) % M][(w + 1) / M],
                                        v[(w + 2) % M][(w + 2) / M], v[(w + 3) % M][(w + 3) / M]);
                }
                return;
            }
        }
#pragma unroll
        for (int w = 0; w < n * M; ++w) dst[w] = v[w % M][w / M];
    }

    // Store one output block of the element (n^2 lines x n nodes x M contiguous values at `dst`) through the
    // LDS scratch `S` of `cap` values, as many lines per round as fit, so that consecutive lanes of the
    // element store consecutive words. Starts with a barrier (the scratch may still be read) and ends with
    // one. Unaligned blocks are stored line by line from registers.
    __device__ static inline void store_block(T* S, int cap, T* dst, const T (&v)[M][n], int li, bool act, bool aligned)
    {
        constexpr int LV = n * M;
        const int R = cap / LV;
        __syncthreads();
        for (int r0 = 0; r0 < n2; r0 += R) {
            if (aligned && li >= r0 && li < r0 + R) {
#pragma unroll
                for (int w = 0; w < LV; ++w) S[(li - r0) * LV + w] = v[w % M][w / M];
            }
            __syncthreads();
            if (aligned) {
                const int nv = (n2 - r0 < R ? n2 - r0 : R) * LV;
                T* d = dst + (int64_t)r0 * LV;
                if constexpr (sizeof(T) == 4 && (LV % 4) == 0) {
                    for (int i = li; i < nv / 4; i += n2)
                        reinterpret_cast<float4*>(d)[i] = reinterpret_cast<const float4*>(S)[i];
                } else {
                    for (int i = li; i < nv; i += n2) d[i] = S[i];
                }
            }
            __syncthreads();
        }
        if (act && !aligned) store_line(dst + (int64_t)li * LV, v);
    }

    __device__ static void run(const StpArgs& a)
    {
        extern __shared__ __align__(16) unsigned char smem[];
        const int tid = threadIdx.x;
        const int es = tid / n2;         // element slot in the workgroup
        const int li = tid - es * n2;    // line index
        const int la = li / n, lb = li - la * n;  // owner (z, y); y-role (z, x); z-role (y, x)
        T* P = reinterpret_cast<T*>(smem) + (es < EPB ? es : 0) * ELDS;
        T* G = P + NPS * SLOT;
        const bool per_elem = (a.flags & kParamPerElement) != 0;

        Tab tb;
        {
            const T* t = static_cast<const T*>(a.D);  // even/odd tables in the compute precision
#pragma unroll
            for (int i = 0; i < h; ++i)
#pragma unroll
                for (int j = 0; j < h; ++j) {
                    tb.A[i][j] = t[i * h + j];
                    tb.B[i][j] = t[h * h + i * h + j];
                }
#pragma unroll
            for (int i = 0; i < h; ++i) {
                tb.Cm[i] = t[2 * h * h + i];
                tb.Am[i] = t[2 * h * h + h + i];
            }
        }
        T e0[n], e1[n];
#pragma unroll
        for (int j = 0; j < n; ++j) {
            e0[j] = ld<T>(a.e0, j);
            e1[j] = ld<T>(a.e1, j);
        }
        const int64_t cnt = a.count ? (int64_t)*a.count : a.nelem;

        for (int64_t base = (int64_t)blockIdx.x * EPB; base < cnt; base += (int64_t)gridDim.x * EPB) {
            ElemRef er;
            const bool act = es < EPB && elem_ref(a, base + es, er);
            T p[M][n], qb[M][n];
            Material<T, PHYS> mt[n];
            if (act) {
                load_line(static_cast<const T*>(a.Q) + er.q + (int64_t)li * n * M, p);
                const double inv_h = 1.0 / er.h;
                const T* par = static_cast<const T*>(a.params) + er.coef;
#pragma unroll
                for (int x = 0; x < n; ++x) mt[x].load(per_elem ? par : par + ((int64_t)li * n + x) * NP, inv_h);
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int x = 0; x < n; ++x) qb[q][x] = p[q][x];
            }
            T w = 1;
            const T dt = act ? (T)er.dt : T(0);
            for (int o = 1; o <= N; ++o) {
                if (act) write_tile(P, la, lb, p);
                __syncthreads();
                T r[M][n];
                volume(tb, P, G, la, lb, act, mt, p, r);
                w = w * dt * __builtin_amdgcn_rcpf((T)(o + 1));
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int x = 0; x < n; ++x) {
                        p[q][x] = r[q][x];
                        qb[q][x] = fma(w, r[q][x], qb[q][x]);
                    }
                __syncthreads();
            }

            // outputs: q-bar, favg[d] = V_d(q-bar), faces. Output blocks are staged through the element's LDS
            // region so that consecutive lanes store consecutive words.
            const bool fsum = (a.flags & kFavgSum) != 0;
            const bool al = act && ((er.q & 3) == 0);
            store_block(P, ELDS, act ? static_cast<T*>(a.qavg) + er.q : nullptr, qb, li, act, al);
            {
                T fx[M][n];
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int x = 0; x < n; ++x) fx[q][x] = 0;
                xpass(tb, mt, qb, fx);
                T* fav = act ? static_cast<T*>(a.favg) + (fsum ? er.q : 3 * er.q) : nullptr;
                if (!fsum) {
                    store_block(P, ELDS, fav, fx, li, act, al);
#pragma unroll
                    for (int q = 0; q < M; ++q)
#pragma unroll
                        for (int x = 0; x < n; ++x) fx[q][x] = 0;
                }
                if (act) write_tile(P, la, lb, qb);
                __syncthreads();
                if (act) transposed<1>(tb, P, G, la, lb);
                __syncthreads();
                if (act) gather<1>(G, la, lb, mt, fx);
                if (!fsum) {
                    store_block(G, NG * SLOT, act ? fav + (int64_t)n3 * M : nullptr, fx, li, act, al);
#pragma unroll
                    for (int q = 0; q < M; ++q)
#pragma unroll
                        for (int x = 0; x < n; ++x) fx[q][x] = 0;
                }
                __syncthreads();
                if (act) transposed<2>(tb, P, G, la, lb);
                __syncthreads();
                if (act) gather<2>(G, la, lb, mt, fx);
                store_block(P, ELDS, act ? (fsum ? fav : fav + 2 * (int64_t)n3 * M) : nullptr, fx, li, act, al);
            }
            // faces: x-faces from the owner's line; y- and z-faces from the full tile of q-bar
            T* qf = static_cast<T*>(a.qface) + er.face;
            if (act) {
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    T s0 = 0, s1 = 0;
#pragma unroll
                    for (int x = 0; x < n; ++x) {
                        s0 = fma(e0[x], qb[q][x], s0);
                        s1 = fma(e1[x], qb[q][x], s1);
                    }
                    qf[(int64_t)li * M + q] = s0;
                    qf[(int64_t)(n2 + li) * M + q] = s1;
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int x = 0; x < n; ++x) P[q * SLOT + at(la, lb, x)] = qb[q][x];
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    T y0 = 0, y1 = 0, z0 = 0, z1 = 0;
#pragma unroll
                    for (int j = 0; j < n; ++j) {
                        const T vy = P[q * SLOT + at(la, j, lb)];  // y-role (z, x)
                        const T vz = P[q * SLOT + at(j, la, lb)];  // z-role (y, x)
                        y0 = fma(e0[j], vy, y0);
                        y1 = fma(e1[j], vy, y1);
                        z0 = fma(e0[j], vz, z0);
                        z1 = fma(e1[j], vz, z1);
                    }
                    qf[(int64_t)(2 * n2 + li) * M + q] = y0;
                    qf[(int64_t)(3 * n2 + li) * M + q] = y1;
                    qf[(int64_t)(4 * n2 + li) * M + q] = z0;
                    qf[(int64_t)(5 * n2 + li) * M + q] = z1;
                }
            }
            __syncthreads();
        }
    }
};

// Waves per SIMD the register allocation must allow. The elastic kernel at N = 5, 6 needs 282 and 315
// registers (VGPRs plus AGPRs), one wave per SIMD; bounded to two waves it spills 92 resp. 128 bytes per lane
// and runs 22% faster, with the same results. Acoustic N = 6 (179 registers) bounded to three waves spills
// 44 bytes and gains 3%. Tighter bounds elsewhere measured slower (elastic N = 7 at two waves: 536 bytes of
// spills, 1.7x the time; elastic N = 3, 4 and acoustic N = 7 at three waves: 1.2-1.5x), so those keep the
// compiler's choice.
template <typename T, int N, int PHYS>
struct FusedWaves {
    static constexpr int v = PHYS == kElastic ? ((N == 5 || N == 6) ? 2 : 1) : (PHYS == kAcoustic && N == 6) ? 3 : 1;
};

template <typename T, int N, int PHYS>
__global__ void __launch_bounds__(wg_size(N + 1)) __attribute__((amdgpu_waves_per_eu(FusedWaves<T, N, PHYS>::v)))
stp_fused_kernel(StpArgs a)
{
    Fused<T, N, PHYS>::run(a);
}

template <typename T, int N, int PHYS>
KernelInfo fused_info()
{
    using K = Fused<T, N, PHYS>;
    KernelInfo ki;
    ki.fn = reinterpret_cast<const void*>(&stp_fused_kernel<T, N, PHYS>);
    ki.block = K::WG;
    ki.mb = K::M;
    ki.elems_per_block = K::EPB;
    ki.lds = [](int, bool) -> size_t { return sizeof(T) * (size_t)K::EPB * K::ELDS; };
    ki.aux = KernelInfo::kAuxEvenOdd;
    return ki;
}

template <typename T, int PHYS>
KernelInfo fused_by_order(int N)
{
    switch (N) {
    case 1: return fused_info<T, 1, PHYS>();
    case 2: return fused_info<T, 2, PHYS>();
    case 3: return fused_info<T, 3, PHYS>();
    case 4: return fused_info<T, 4, PHYS>();
    case 5: return fused_info<T, 5, PHYS>();
    case 6: return fused_info<T, 6, PHYS>();
    case 7: return fused_info<T, 7, PHYS>();
    default: return KernelInfo{};
    }
}

}  // namespace fused
}  // namespace stp
