// stp_resident.hpp -- STP kernel for generic classes with dense per-node B_d at high orders (no A, no point
// source; FP32 I/O and arithmetic), with part or all of the element's B_d held on chip for the whole Taylor loop.
//
// The operator of Eq. (4) applies B_d pointwise: a node's three m x m blocks (3 m^2 words) are used once per
// application of V, i.e. N + 1 times per element (N Taylor steps, then the time-averaged fluxes of Fig. 5).
// The plain kernel reads them from memory at each application; for m = 9 the element's B_d (3 n^3 m^2 words:
// 498 KB at N = 7, 972 KB at N = 9) is then read N + 1 times, several times the algorithmic traffic, and the
// re-reads set the kernel's time. Here each thread owns K nodes (node tid + k NT) and keeps the first KR words
// of each node's B_d in registers and the next KL words in LDS, all loaded once per element; only the words
// beyond KR + KL are streamed at each application. Word e of a node's B_d is the entry (s, q) of B_d with
// e = d m^2 + q m + s: the Taylor step forms one derivative (D x_d u)_q at a time and adds column q of B_d
// times it to the node's m accumulators (the column form of the plain kernel at orders 8 and 9, whose
// arithmetic this kernel repeats operation for operation). With G = 4 the derivatives of four quantities are
// formed together from 16-byte LDS reads of a tile padded to a multiple of four words per node; the sums keep
// their order, so the results are the same bits.
//
// Per element (Sec. II-A, Eq. (4); Sec. II-B outputs):
//   p_0 = Q;  for o = 1..N:  p_o = V(p_{o-1});  qavg += dt^o/(o+1)! p_o
//   favg[d] = V_d(qavg);  qface[f] = sum_j l_j(0 or 1) qavg along the face normal
// with V_d(u) = -(1/h) B_d (D x_d u) (no conservative flux: A = 0 for the classes this kernel takes).
#pragma once

#include "stp_device.hpp"
#include "stp_kernels.hpp"

namespace stp {
namespace resident {

template <int N, int MB, int NT, int K, int KR, int KL, int G, bool PF>
struct Res {
    static constexpr int n = N + 1;
    static constexpr int n2 = n * n;
    static constexpr int nn = n * n2;
    static constexpr int m = MB;
    static constexpr int NE = 3 * m * m;  // words of B_d per node
    // G = 4: the tile's node stride is padded to a multiple of 4 words, so that the four quantities q0..q0 + 3 of
    // a line node come in one 16-byte LDS read and four derivatives are formed together (G = 1: one at a time)
    static_assert(G == 1 || G == 4, "derivative group");
    static constexpr int MP = G == 4 ? (m + 3) / 4 * 4 : m;
    static_assert(NT % 64 == 0 && NT * K >= nn && NT * (K - 1) < nn, "the K nodes per thread tile the element");
    static_assert(KR >= 0 && KL >= 0 && KR + KL <= NE, "resident words within a node's B_d");

    // LDS: D [n][n], l(0) [n], l(1) [n]; the Taylor term [nn][MP] (padding words zero); the LDS-resident words
    // [KL][nn]
    static constexpr size_t al16(size_t b) { return (b + 15) & ~size_t(15); }
    static constexpr size_t kP = al16(sizeof(float) * (n * n + 2 * n));
    static constexpr size_t kB = al16(kP + sizeof(float) * nn * MP);
    static constexpr size_t kLds = kB + sizeof(float) * (size_t)KL * nn;
    static_assert(kLds <= 160 * 1024, "LDS of one workgroup");

    // Offset of word e of node 0 in the element's B block [d][s][q][node] (node-fastest).
    __host__ __device__ static constexpr int64_t goff(int e)
    {
        return (int64_t)(e / (m * m)) * m * m * nn + (int64_t)((e % m) * m + (e / m) % m) * nn;
    }

    // (D x_d u)_s at a node with coordinates (z, y, x); u is the LDS tile [node][MP]
    template <int D>
    __device__ static inline float dline(const float* Ds, const float* u, int node, int z, int y, int x, int s)
    {
        const int kd = D == 0 ? x : (D == 1 ? y : z);
        const int base = D == 0 ? node - x : (D == 1 ? node - y * n : node - z * n2);
        constexpr int stride = D == 0 ? 1 : (D == 1 ? n : n2);
        float acc = 0;
#pragma unroll
        for (int j = 0; j < n; ++j) acc = fmaf(Ds[kd * n + j], u[(base + j * stride) * MP + s], acc);
        return acc;
    }

    // (D x_d u)_{q0..q0+3} with the sums in the order of dline (bit-identical per quantity)
    template <int D>
    __device__ static inline void dline4(const float* Ds, const float* u, int node, int z, int y, int x, int q0,
                                         float (&g)[4])
    {
        const int kd = D == 0 ? x : (D == 1 ? y : z);
        const int base = D == 0 ? node - x : (D == 1 ? node - y * n : node - z * n2);
        constexpr int stride = D == 0 ? 1 : (D == 1 ? n : n2);
        g[0] = g[1] = g[2] = g[3] = 0;
#pragma unroll
        for (int j = 0; j < n; ++j) {
            const float dj = Ds[kd * n + j];
            const float4 v = *reinterpret_cast<const float4*>(u + (base + j * stride) * MP + q0);
            g[0] = fmaf(dj, v.x, g[0]);
            g[1] = fmaf(dj, v.y, g[1]);
            g[2] = fmaf(dj, v.z, g[2]);
            g[3] = fmaf(dj, v.w, g[3]);
        }
    }

    struct Nodes {
        int node[K], z[K], y[K], x[K];
        bool own[K];
    };

    // Word e of the thread's node k: registers, LDS or memory
    __device__ static inline float word(int e, int k, const float (&breg)[K][KR > 0 ? KR : 1], const float* bres,
                                        const float* const (&bg)[K], const Nodes& nd)
    {
        if (e < KR) return breg[k][e < KR ? e : 0];
        if (e < KR + KL) return bres[(e - KR) * nn + nd.node[k]];
        return bg[k][goff(e)];
    }

    // r[k] += V_D(u) at the thread's nodes: -(1/h) sum_q B_D[:, q] (D x_D u)_q, column by column. bg[k] points
    // at word 0 of node k's B_d in memory (streamed words), bres at the LDS-resident words.
    template <int D>
    __device__ static inline void apply(const float* Ds, const float* u, const float (&breg)[K][KR > 0 ? KR : 1],
                                        const float* bres, const float* const (&bg)[K], const Nodes& nd,
                                        float ninv_h, float (&r)[K][MB])
    {
        // column q: r[k][s] += B_D[s][q] (-(1/h) g_q) in the order s = 0..m-1, then the accumulators are pinned:
        // they are stored only for owned nodes, and without the pin the compiler sinks the column's arithmetic
        // into that conditional store, past the step's barrier, and keeps every loaded word of the step live
        auto column = [&](const float (&b)[K][MB], const float (&gq)[K]) {
#pragma unroll
            for (int s = 0; s < m; ++s)
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    r[k][s] = fmaf(b[k][s], gq[k], r[k][s]);
                    asm volatile("" : "+v"(r[k][s]));
                }
        };
        if constexpr (G == 1 && PF) {
            // PF: column q + 1's words are loaded before column q's derivative and FMAs, so that two columns of
            // streamed loads are in flight
            float b[K][MB];
#pragma unroll
            for (int s = 0; s < m; ++s)
#pragma unroll
                for (int k = 0; k < K; ++k) b[k][s] = word(D * m * m + s, k, breg, bres, bg, nd);
#pragma unroll
            for (int q = 0; q < m; ++q) {
                float bn[K][MB];
                if (q + 1 < m) {
#pragma unroll
                    for (int s = 0; s < m; ++s)
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            bn[k][s] = word(D * m * m + (q + 1) * m + s, k, breg, bres, bg, nd);
                }
                float g[K];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    g[k] = ninv_h * dline<D>(Ds, u, nd.node[k], nd.z[k], nd.y[k], nd.x[k], q);
                column(b, g);
                __builtin_amdgcn_sched_barrier(0);
                if (q + 1 < m) {
#pragma unroll
                    for (int s = 0; s < m; ++s)
#pragma unroll
                        for (int k = 0; k < K; ++k) b[k][s] = bn[k][s];
                }
            }
        } else if constexpr (G == 1) {
#pragma unroll
            for (int q = 0; q < m; ++q) {
                float b[K][MB];
#pragma unroll
                for (int s = 0; s < m; ++s)
#pragma unroll
                    for (int k = 0; k < K; ++k) b[k][s] = word(D * m * m + q * m + s, k, breg, bres, bg, nd);
                float g[K];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    g[k] = ninv_h * dline<D>(Ds, u, nd.node[k], nd.z[k], nd.y[k], nd.x[k], q);
                column(b, g);
                // one column's loads and derivative at a time: bounds the registers they hold
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int q0 = 0; q0 < m; q0 += 4) {
                float g4[K][4];
#pragma unroll
                for (int k = 0; k < K; ++k) dline4<D>(Ds, u, nd.node[k], nd.z[k], nd.y[k], nd.x[k], q0, g4[k]);
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const int q = q0 + qq;
                    if (q >= m) break;
                    float b[K][MB], g[K];
#pragma unroll
                    for (int s = 0; s < m; ++s)
#pragma unroll
                        for (int k = 0; k < K; ++k) b[k][s] = word(D * m * m + q * m + s, k, breg, bres, bg, nd);
#pragma unroll
                    for (int k = 0; k < K; ++k) g[k] = ninv_h * g4[k][qq];
                    column(b, g);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    // One element by the NT threads of the workgroup (tid in [0, NT)); every thread must call it (barriers).
    __device__ static void element(const StpArgs& a, const ElemRef& er, unsigned char* smem, int tid)
    {
        float* Ds = reinterpret_cast<float*>(smem);
        float* e0s = Ds + n * n;
        float* e1s = e0s + n;
        float* pbuf = reinterpret_cast<float*>(smem + kP);
        float* bres = reinterpret_cast<float*>(smem + kB);
        const float* Bel = static_cast<const float*>(a.B) + er.coef;

        // the thread's nodes; a slot beyond the element works on its last node and writes nothing
        Nodes nd;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int t = tid + k * NT;
            nd.own[k] = t < nn;
            nd.node[k] = nd.own[k] ? t : nn - 1;
            nd.x[k] = nd.node[k] % n;
            nd.y[k] = (nd.node[k] / n) % n;
            nd.z[k] = nd.node[k] / n2;
        }

        for (int i = tid; i < n * n; i += NT) Ds[i] = ld<float>(a.D, i);
        for (int i = tid; i < n; i += NT) {
            e0s[i] = ld<float>(a.e0, i);
            e1s[i] = ld<float>(a.e1, i);
        }
        const float* Q = static_cast<const float*>(a.Q) + er.q;
        for (int i = tid; i < nn * MP; i += NT) {
            const int node = i / MP, s = i - node * MP;
            pbuf[i] = s < m ? Q[node * m + s] : 0.f;
        }
        // LDS-resident words: word KR + j of node t at bres[j nn + t] (consecutive lanes, consecutive banks)
        for (int i = tid; i < KL * nn; i += NT) {
            const int j = i / nn, t = i - j * nn;
            bres[i] = Bel[goff(KR + j) + t];
        }
        float breg[K][KR > 0 ? KR : 1];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < KR; ++e) breg[k][e] = Bel[goff(e) + nd.node[k]];
        __syncthreads();

        const float ninv_h = -(float)(1.0 / er.h);
        float qb[K][MB], r[K][MB];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int s = 0; s < m; ++s) qb[k][s] = pbuf[nd.node[k] * MP + s];
        float w = 1;
        const float dt = (float)er.dt;
        for (int o = 1; o <= N; ++o) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int s = 0; s < m; ++s) r[k][s] = 0;
            // the laundered offset keeps the streamed loads inside the loop (re-read at every step)
            const int oz = opaque_zero();
            const float* bg[K];
#pragma unroll
            for (int k = 0; k < K; ++k) bg[k] = Bel + nd.node[k] + oz;
            apply<0>(Ds, pbuf, breg, bres, bg, nd, ninv_h, r);
            apply<1>(Ds, pbuf, breg, bres, bg, nd, ninv_h, r);
            apply<2>(Ds, pbuf, breg, bres, bg, nd, ninv_h, r);
            __syncthreads();
            w = w * dt / (float)(o + 1);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!nd.own[k]) continue;
#pragma unroll
                for (int s = 0; s < m; ++s) {
                    pbuf[nd.node[k] * MP + s] = r[k][s];
                    qb[k][s] = fmaf(w, r[k][s], qb[k][s]);
                }
            }
            __syncthreads();
        }

        // q-bar: into the tile, then stored whole
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!nd.own[k]) continue;
#pragma unroll
            for (int s = 0; s < m; ++s) pbuf[nd.node[k] * MP + s] = qb[k][s];
        }
        __syncthreads();
        float* qavg = static_cast<float*>(a.qavg) + er.q;
        for (int i = tid; i < nn * m; i += NT) qavg[i] = pbuf[(i / m) * MP + i % m];

        // faces of q-bar: [f][a][b][s], f = 2 axis + side
        float* qface = static_cast<float*>(a.qface) + er.face;
        for (int i = tid; i < 6 * n2 * m; i += NT) {
            const int s = i % m, t = i / m, bb = t % n, aa = (t / n) % n, f = t / n2;
            const int axis = f >> 1;
            const float* ev = (f & 1) ? e1s : e0s;
            float acc = 0;
#pragma unroll
            for (int j = 0; j < n; ++j) {
                const int node = axis == 0 ? (aa * n + bb) * n + j
                                           : (axis == 1 ? (aa * n + j) * n + bb : (j * n + aa) * n + bb);
                acc = fmaf(ev[j], pbuf[node * MP + s], acc);
            }
            qface[i] = acc;
        }

        // time-averaged fluxes favg[d] = V_d(q-bar), stored from the registers (each lane its nodes' m words)
        const bool fsum = (a.flags & kFavgSum) != 0;
        float* favg = static_cast<float*>(a.favg) + (fsum ? er.q : 3 * er.q);
        const int oz = opaque_zero();
        const float* bg[K];
#pragma unroll
        for (int k = 0; k < K; ++k) bg[k] = Bel + nd.node[k] + oz;
        float fv[K][MB];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int s = 0; s < m; ++s) fv[k][s] = 0;
        auto store = [&](float* dst) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!nd.own[k]) continue;
#pragma unroll
                for (int s = 0; s < m; ++s) {
                    dst[nd.node[k] * m + s] = fv[k][s];
                    fv[k][s] = 0;
                }
            }
        };
        apply<0>(Ds, pbuf, breg, bres, bg, nd, ninv_h, fv);
        if (!fsum) store(favg);
        apply<1>(Ds, pbuf, breg, bres, bg, nd, ninv_h, fv);
        if (!fsum) store(favg + nn * m);
        apply<2>(Ds, pbuf, breg, bres, bg, nd, ninv_h, fv);
        store(fsum ? favg : favg + 2 * nn * m);
        __syncthreads();  // the next element overwrites the tiles
    }
};

template <int N, int MB, int NT, int K, int KR, int KL, int G, bool PF>
__global__ void __launch_bounds__(NT) stp_resident_kernel(StpArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    for (int64_t it = blockIdx.x;; it += gridDim.x) {
        ElemRef er;
        if (!elem_ref(a, it, er)) break;
        Res<N, MB, NT, K, KR, KL, G, PF>::element(a, er, smem, threadIdx.x);
    }
}

template <int N, int MB, int NT, int K, int KR, int KL, int G = 1, bool PF = false>
KernelInfo resident_info()
{
    KernelInfo ki;
    ki.fn = reinterpret_cast<const void*>(&stp_resident_kernel<N, MB, NT, K, KR, KL, G, PF>);
    ki.block = NT;
    ki.mb = MB;
    ki.lds = [](int, bool) -> size_t { return Res<N, MB, NT, K, KR, KL, G, PF>::kLds; };
    return ki;
}

}  // namespace resident
}  // namespace stp
