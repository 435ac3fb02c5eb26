// stp_plain.hpp -- plain STP kernel: one element per workgroup, one thread per node, the element's
// current Taylor term p_o staged in LDS.
//
// Per element (Sec. II-A, Eq. (4) and the recursion below it; Sec. II-B outputs):
//   p_0 = Q;  for o = 1..N:  p_o = V(p_{o-1}) (+ S_{o-1});  qavg += dt^o/(o+1)! p_o
//   favg[d] = V_d(qavg)  (time-averaged fluxes recomputed from qavg by linearity, Fig. 5)
//   qface[f] = sum_j l_j(0 or 1) qavg along the face normal; fface[f] likewise for A_{d_f} qavg.
// with V_d(u) = -(1/h)[ D x_d (A_d u) + B_d (D x_d u) ].
//
// This is the straightforward GPU formulation (the generic algorithm's structure with the SplitCK
// footprint): each thread owns one node, keeps its qavg (accumulator precision) and its next Taylor term
// in registers, and reads the n values along each of the three lines through its node from LDS. It
// supports every class (presets and generic, optional A and point source), and the FP64 instantiation is
// the plain FP64 GPU baseline.
#pragma once
#include <type_traits>

#include "stp_device.hpp"
#include "stp_kernels.hpp"

namespace stp {
namespace plain {

template <typename T, typename ACC, int N, int PHYS, int MB, bool EX = false>
struct Plain {
    static constexpr int n = N + 1;
    static constexpr int n2 = n * n;
    static constexpr int nn = n * n * n;
    static constexpr int NT = ((nn + 63) / 64) * 64;
    static constexpr bool kPreset = PHYS != kGeneric;
    // Rows of a per-node B_d product issued between scheduling barriers (FP32, generic orders up to 7): three
    // rows (27 loads in flight at m = 9) for the wider buckets, no barrier for m <= 4. Chosen by timing each
    // class of the mixed 16384-element workload.
    static constexpr int kNcpGroup = MB >= 9 ? 3 : 0;
    // Orders 8 and 9 of the generic physics form B_d g one column at a time: the loads of column q are in
    // flight while the derivative of quantity q is formed from LDS, and only one derivative is live. In the
    // row form (all m derivatives, then the rows of B_d) the waves of those large blocks sit idle on the
    // B_d loads after each direction's LDS work; the column form runs their classes about twice as fast. At
    // orders 7 and below the row form is as fast or faster.
    static constexpr bool kColumnNcp = !kPreset && N >= 8;
    // Presets: the tile's node stride is padded to a multiple of 16 bytes, so the quantities a direction reads
    // come in 16-byte LDS reads (four floats or two doubles; the sums keep their order: the same bits). Taken
    // where it measured faster. FP32: acoustic (one group, 0.20 -> 0.16 ms for 4096 elements at order 7),
    // curvilinear elastic (every quantity is read, 3 groups for 9) and Cartesian elastic at orders 8 and 9
    // (10-20%; one workgroup per CU, latency-bound); below order 8 the elastic kernel reads 12 words for the 6 it
    // needs at more waves per CU, and order 7 measured 13% slower. FP64: curvilinear elastic (order 7 10.99 ->
    // 10.50 ms); the Cartesian elastic kernel at order 7 measured 6.49 -> 8.15 ms, acoustic at order 5 the same.
    static constexpr bool kGroupLds =
        kPreset && (sizeof(T) == 4 ? (PHYS != kElastic || N >= 8) : PHYS == kElasticCurv);
    static constexpr int GS = 16 / (int)sizeof(T);  // values per 16-byte read
    static constexpr int MPS = kGroupLds ? (MB + GS - 1) / GS * GS : 1;
    __host__ __device__ static constexpr int mp(int m) { return kGroupLds ? MPS : m; }
    __host__ __device__ static constexpr bool group_needed(int D, int g)
    {
        for (int s = GS * g; s < GS * g + GS && s < MB; ++s)
            if (PhysTraits<PHYS == kGeneric ? kElastic : PHYS>::needs(D, s)) return true;
        return false;
    }

    // Byte offsets of the LDS regions, each 16-byte aligned; `total` is the dynamic LDS size.
    struct Layout {
        size_t coefs, pbuf, fbuf, qacc, total;
    };
    __host__ __device__ static constexpr size_t al16(size_t b) { return (b + 15) & ~size_t(15); }
    __host__ __device__ static Layout layout(int m, bool hasA)
    {
        Layout L{};
        L.coefs = al16(sizeof(T) * (n * n + 2 * n));
        L.pbuf = al16(L.coefs + (kPreset ? 0 : sizeof(T) * 6 * MB * MB));
        L.fbuf = al16(L.pbuf + sizeof(T) * nn * mp(m));
        L.qacc = al16(L.fbuf + (hasA ? sizeof(T) * nn * m : 0));
        L.total = L.qacc + (std::is_same<ACC, T>::value ? 0 : sizeof(ACC) * nn * m);
        return L;
    }

    // D x_d u at node (z, y, x) for quantity s; u is the LDS tile [node][m].
    template <int D>
    __device__ static inline T dline(const T* Ds, const T* u, int m, int tid, int z, int y, int x, int s)
    {
        const int kd = D == 0 ? x : (D == 1 ? y : z);
        const int base = D == 0 ? tid - x : (D == 1 ? tid - y * n : tid - z * n2);
        constexpr int stride = D == 0 ? 1 : (D == 1 ? n : n2);
        T acc = 0;
#pragma unroll
        for (int j = 0; j < n; ++j) acc = fma(Ds[kd * n + j], u[(base + j * stride) * m + s], acc);
        return acc;
    }

    // r += V_d(u) at the thread's node. Must be called by every thread of the block (barriers when A is
    // present). fbuf: LDS scratch [nn][m] for the conservative flux A_d u.
    template <int D>
    __device__ static inline void accum_Vd(const StpArgs& a, const ElemRef& er, const T* Ds, const T* u,
                                           T* fbuf, const T* coefs, const Material<T, PHYS>& mt, int m,
                                           T inv_h, int tid, int z, int y, int x, bool own, bool hasA, T* r)
    {
        const bool per_elem = (a.flags & kCoefPerElement) != 0;
        if constexpr (!kPreset) {
            if (hasA) {
                // flux F_d = A_d u at every node, then its derivative along d
                if (own) {
                    // Ad: the matrix in LDS (per element, stride 1) or in global memory (per node, stored
                    // node-fastest so that lanes read consecutive words: stride n^3). The two cases stay
                    // separate code paths (one pointer for both address spaces miscompiles on gfx950).
                    auto flux = [&](const T* Ad, int cs) {
#pragma unroll
                        for (int s = 0; s < MB; ++s) {
                            if (s >= m) break;
                            T acc = 0;
#pragma unroll
                            for (int q = 0; q < MB; ++q) {
                                if (q >= m) break;
                                acc = fma(Ad[(s * m + q) * cs], u[tid * m + q], acc);
                            }
                            fbuf[tid * m + s] = acc;
                            if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
                        }
                    };
                    if (per_elem)
                        flux(coefs + (3 + D) * m * m, 1);
                    else  // re-read every Taylor step: the laundered offset keeps the loads inside the loop
                        flux(static_cast<const T*>(a.A) + er.coef + (int64_t)D * m * m * nn + tid + opaque_zero(), nn);
                }
                __syncthreads();
                if (own) {
#pragma unroll
                    for (int s = 0; s < MB; ++s) {
                        if (s >= m) break;
                        r[s] = fma(-inv_h, dline<D>(Ds, fbuf, m, tid, z, y, x, s), r[s]);
                        if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
                    }
                }
                __syncthreads();
            }
        }
        if (!own) return;
        if constexpr (kColumnNcp) {
            // r += -(1/h) sum_q B_d[:, q] (D x_d u)_q
            auto ncp_cols = [&](const T* Bd, int cs) {
#pragma unroll
                for (int q = 0; q < MB; ++q) {
                    if (q >= m) break;
                    T b[MB];
#pragma unroll
                    for (int s = 0; s < MB; ++s) b[s] = s < m ? Bd[(s * m + q) * cs] : T(0);
                    const T gq = -inv_h * dline<D>(Ds, u, m, tid, z, y, x, q);
#pragma unroll
                    for (int s = 0; s < MB; ++s)
                        if (s < m) r[s] = fma(b[s], gq, r[s]);
                    if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
                }
            };
            if (per_elem)
                ncp_cols(coefs + D * m * m, 1);
            else  // re-read every Taylor step: the laundered offset keeps the loads inside the loop
                ncp_cols(static_cast<const T*>(a.B) + er.coef + (int64_t)D * m * m * nn + tid + opaque_zero(), nn);
            return;
        }
        T g[MB];
        if constexpr (kGroupLds) {
            // every quantity B_d reads, from 16-byte reads of the line's nodes (sums in dline's order)
            const int kd = D == 0 ? x : (D == 1 ? y : z);
            const int base = D == 0 ? tid - x : (D == 1 ? tid - y * n : tid - z * n2);
            constexpr int stride = D == 0 ? 1 : (D == 1 ? n : n2);
#pragma unroll
            for (int s = 0; s < MB; ++s) g[s] = 0;
#pragma unroll
            for (int j = 0; j < n; ++j) {
                const T dj = Ds[kd * n + j];
#pragma unroll
                for (int gr = 0; gr < MPS / GS; ++gr) {
                    if (!group_needed(D, gr)) continue;
                    T vv[GS];
                    if constexpr (GS == 4) {
                        const float4 v = *reinterpret_cast<const float4*>(u + (base + j * stride) * MPS + 4 * gr);
                        vv[0] = v.x; vv[1] = v.y; vv[2] = v.z; vv[3] = v.w;
                    } else {
                        const double2 v = *reinterpret_cast<const double2*>(u + (base + j * stride) * MPS + 2 * gr);
                        vv[0] = v.x; vv[1] = v.y;
                    }
#pragma unroll
                    for (int t = 0; t < GS; ++t) {
                        const int s = GS * gr + t;
                        if (s < MB && PhysTraits<PHYS>::needs(D, s)) g[s] = fma(dj, vv[t], g[s]);
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < MB; ++s) {
            if constexpr (kGroupLds) {
                break;
            } else if constexpr (kPreset) {
                g[s] = PhysTraits<PHYS>::needs(D, s) ? dline<D>(Ds, u, MB, tid, z, y, x, s) : T(0);
            } else {
                g[s] = s < m ? dline<D>(Ds, u, m, tid, z, y, x, s) : T(0);
            }
            // one quantity's line at a time: bounds the LDS reads in flight (and the registers they hold).
            // Curvilinear elements up to order 7 take two at a time (5.71 -> 5.04 ms at N = 7); for the
            // other classes two cost the persistent elastic bucket a wave per SIMD. FP32 only: with FP64
            // data this barrier makes the gfx950 back end emit an illegal instruction.
            if constexpr (sizeof(T) == 4) {
                if (N > 7 || PHYS != kElasticCurv || (s & 1) == 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
        if constexpr (kPreset) {
            apply_ncp<T, PHYS, D>(mt, g, r);
        } else {
            // B_d from LDS (per element) or global memory (per node, node-fastest), as for A_d above
            auto ncp = [&](const T* Bd, int cs) {
#pragma unroll
                for (int s = 0; s < MB; ++s) {
                    if (s >= m) break;
                    T acc = 0;
#pragma unroll
                    for (int q = 0; q < MB; ++q) {
                        if (q >= m) break;
                        acc = fma(Bd[(s * m + q) * cs], g[q], acc);
                    }
                    r[s] = fma(-inv_h, acc, r[s]);
                    if constexpr (sizeof(T) == 4 && kNcpGroup > 0)
                        if ((s + 1) % kNcpGroup == 0) __builtin_amdgcn_sched_barrier(0);
                }
            };
            if (per_elem)
                ncp(coefs + D * m * m, 1);
            else  // re-read every Taylor step: the laundered offset keeps the loads inside the loop
                ncp(static_cast<const T*>(a.B) + er.coef + (int64_t)D * m * m * nn + tid + opaque_zero(), nn);
        }
    }

    // One element processed by `stride` threads with local ids tid in [0, stride) (stride >= n^3) and the LDS
    // region `smem` (layout()). Every thread of the workgroup must call it (barriers); `valid` is false for
    // threads of an empty slot, which then touch no memory.
    __device__ static void element(const StpArgs& a, const ElemRef& er, bool valid, unsigned char* smem, int tid,
                                   int stride)
    {
        const int NT = stride;
        const int m = kPreset ? PhysTraits<PHYS>::m : (EX ? MB : a.m);  // EX: generic with m == MB
        const bool own = valid && tid < nn;
        const int x = tid % n, y = (tid / n) % n, z = tid / n2;
        const bool hasA = !kPreset && (a.flags & kAPresent);
        const bool hasSrc = (a.flags & kSrcPoint) != 0;
        const bool per_elem = (a.flags & (kPreset ? kParamPerElement : kCoefPerElement)) != 0;

        // LDS carve-up: tables, coefficient block (generic per element), p tile, flux tile, FP64 qavg tile
        const Layout L = layout(m, hasA);
        T* Ds = reinterpret_cast<T*>(smem);
        T* e0s = Ds + n * n;
        T* e1s = e0s + n;
        T* coefs = reinterpret_cast<T*>(smem + L.coefs);  // [6][m][m]: B_0..B_2 then A_0..A_2
        T* pbuf = reinterpret_cast<T*>(smem + L.pbuf);
        T* fbuf = reinterpret_cast<T*>(smem + L.fbuf);    // only touched when A is present
        ACC* qacc = reinterpret_cast<ACC*>(smem + L.qacc);

        {
            if (valid) {
                for (int i = tid; i < n * n; i += NT) Ds[i] = ld<T>(a.D, i);
                for (int i = tid; i < n; i += NT) {
                    e0s[i] = ld<T>(a.e0, i);
                    e1s[i] = ld<T>(a.e1, i);
                }
            }
            const T inv_h = (T)(1.0 / er.h);
            const T* Q = static_cast<const T*>(a.Q) + er.q;
            if (valid)
                for (int i = tid; i < nn * m; i += NT) pbuf[(i / m) * mp(m) + i % m] = Q[i];
            Material<T, PHYS> mt;
            if constexpr (kPreset) {
                constexpr int np = PhysTraits<PHYS>::np;
                const T* par = static_cast<const T*>(a.params) + er.coef + (per_elem ? 0 : tid * np);
                if (own) mt.load(par, 1.0 / er.h);
            } else if (per_elem && valid) {
                const T* Bsrc = static_cast<const T*>(a.B) + er.coef;
                for (int i = tid; i < 3 * m * m; i += NT) coefs[i] = Bsrc[i];
                if (hasA) {
                    const T* Asrc = static_cast<const T*>(a.A) + er.coef;
                    for (int i = tid; i < 3 * m * m; i += NT) coefs[3 * m * m + i] = Asrc[i];
                }
            }
            // point source [P (n^3)][a (m)][sigma derivatives (N)]: P and a held in registers. (Re-reading them
            // at each step instead made the order-2, m = 9 kernel 3.6 times slower.)
            T srcP = 0, srca[MB];
            const T* src = static_cast<const T*>(a.src) + er.src;
            if (hasSrc && own) {
                srcP = src[tid];
#pragma unroll
                for (int s = 0; s < MB; ++s) srca[s] = s < m ? src[nn + s] : T(0);
            }
            __syncthreads();

            ACC qb[MB];
            T r[MB];
#pragma unroll
            for (int s = 0; s < MB; ++s) qb[s] = (own && s < m) ? (ACC)pbuf[tid * mp(m) + s] : ACC(0);
            ACC w = 1;
            const ACC dt = (ACC)er.dt;
            for (int o = 1; o <= N; ++o) {
#pragma unroll
                for (int s = 0; s < MB; ++s) r[s] = 0;
                accum_Vd<0>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, r);
                accum_Vd<1>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, r);
                accum_Vd<2>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, r);
                if (hasSrc && own) {
                    const T sg = src[nn + m + (o - 1)];
#pragma unroll
                    for (int s = 0; s < MB; ++s) r[s] = fma(srcP * srca[s], sg, r[s]);
                }
                __syncthreads();
                w = w * dt / (ACC)(o + 1);
                if (own) {
#pragma unroll
                    for (int s = 0; s < MB; ++s) {
                        if (s >= m) break;
                        pbuf[tid * mp(m) + s] = r[s];
                        qb[s] = fma(w, (ACC)r[s], qb[s]);
                    }
                }
                __syncthreads();
            }

            // q-bar into LDS (I/O precision, plus the accumulator precision for the faces)
            if (own) {
#pragma unroll
                for (int s = 0; s < MB; ++s) {
                    if (s >= m) break;
                    pbuf[tid * mp(m) + s] = (T)qb[s];
                    if constexpr (!std::is_same<ACC, T>::value) qacc[tid * m + s] = qb[s];
                }
            }
            __syncthreads();
            T* qavg = static_cast<T*>(a.qavg) + er.q;
            if (valid)
                for (int i = tid; i < nn * m; i += NT) qavg[i] = pbuf[(i / m) * mp(m) + i % m];

            // faces of q-bar, in the accumulator precision
            T* qface = static_cast<T*>(a.qface) + er.face;
            for (int i = valid ? tid : 6 * n2 * m; i < 6 * n2 * m; i += NT) {
                const int s = i % m, t = i / m, b = t % n, aa = (t / n) % n, f = t / n2;
                const int axis = f >> 1;
                const T* ev = (f & 1) ? e1s : e0s;
                ACC acc = 0;
#pragma unroll
                for (int j = 0; j < n; ++j) {
                    const int node = axis == 0 ? (aa * n + b) * n + j
                                               : (axis == 1 ? (aa * n + j) * n + b : (j * n + aa) * n + b);
                    if constexpr (std::is_same<ACC, T>::value)
                        acc = fma((ACC)ev[j], pbuf[node * mp(m) + s], acc);
                    else
                        acc = fma((ACC)ev[j], qacc[node * m + s], acc);
                }
                qface[i] = (T)acc;
            }
            if (hasA) {
                // extrapolated conservative flux A_{d_f} q-bar
                T* fface = static_cast<T*>(a.fface) + er.face;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (own) {
                        auto flux = [&](const T* Ad, int cs) {
                            for (int s = 0; s < m; ++s) {
                                T acc = 0;
                                for (int q = 0; q < m; ++q) acc = fma(Ad[(s * m + q) * cs], pbuf[tid * m + q], acc);
                                fbuf[tid * m + s] = acc;
                            }
                        };
                        if (per_elem)
                            flux(coefs + (3 + d) * m * m, 1);
                        else
                            flux(static_cast<const T*>(a.A) + er.coef + (int64_t)d * m * m * nn + tid, nn);
                    }
                    __syncthreads();
                    for (int i = valid ? tid : 2 * n2 * m; i < 2 * n2 * m; i += NT) {
                        const int s = i % m, t = i / m, b = t % n, aa = (t / n) % n, side = t / n2;
                        const T* ev = side ? e1s : e0s;
                        T acc = 0;
                        for (int j = 0; j < n; ++j) {
                            const int node = d == 0 ? (aa * n + b) * n + j
                                                    : (d == 1 ? (aa * n + j) * n + b : (j * n + aa) * n + b);
                            acc = fma(ev[j], fbuf[node * m + s], acc);
                        }
                        fface[(2 * d) * n2 * m + i] = acc;
                    }
                    __syncthreads();
                }
            }

            // time-averaged fluxes favg[d] = V_d(q-bar)
            if constexpr (sizeof(T) == 8) {
                // FP64: one direction at a time, stored from the registers (each thread its node's m words,
                // consecutive threads consecutive nodes), so that the three directions' fluxes (3 m doubles) are
                // never live together
                const bool fsum = (a.flags & kFavgSum) != 0;
                T* favg = static_cast<T*>(a.favg) + (fsum ? er.q : 3 * er.q);
                T fv[MB];
#pragma unroll
                for (int s = 0; s < MB; ++s) fv[s] = 0;
                auto put = [&](T* dst) {
                    if (own) {
#pragma unroll
                        for (int s = 0; s < MB; ++s) {
                            if (s >= m) break;
                            dst[tid * m + s] = fv[s];
                            fv[s] = 0;
                        }
                    }
                };
                accum_Vd<0>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, fv);
                if (!fsum) put(favg);
                accum_Vd<1>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, fv);
                if (!fsum) put(favg + nn * m);
                accum_Vd<2>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, fv);
                put(fsum ? favg : favg + 2 * nn * m);
                __syncthreads();  // the next element overwrites the tiles
                return;
            }
            T fv[3][MB];
#pragma unroll
            for (int s = 0; s < MB; ++s) fv[0][s] = fv[1][s] = fv[2][s] = 0;
            accum_Vd<0>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, fv[0]);
            accum_Vd<1>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, fv[1]);
            accum_Vd<2>(a, er, Ds, pbuf, fbuf, coefs, mt, m, inv_h, tid, z, y, x, own, hasA, fv[2]);
            __syncthreads();
            const bool fsum = (a.flags & kFavgSum) != 0;
            T* favg = static_cast<T*>(a.favg) + (fsum ? er.q : 3 * er.q);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (fsum && d > 0) break;
                if (own) {
#pragma unroll
                    for (int s = 0; s < MB; ++s) {
                        if (s >= m) break;
                        pbuf[tid * mp(m) + s] = fsum ? fv[0][s] + fv[1][s] + fv[2][s] : fv[d][s];
                    }
                }
                __syncthreads();
                if (valid)
                    for (int i = tid; i < nn * m; i += NT) favg[d * nn * m + i] = pbuf[(i / m) * mp(m) + i % m];
                __syncthreads();
            }
        }
    }

    __device__ static void run(const StpArgs& a)
    {
        extern __shared__ __align__(16) unsigned char smem[];
        for (int64_t it = blockIdx.x;; it += gridDim.x) {
            ElemRef er;
            if (!elem_ref(a, it, er)) break;
            element(a, er, true, smem, threadIdx.x, NT);
        }
    }
};

// Waves per SIMD the compiler must allow (registers <= 512 / waves), so that one more workgroup fits a CU. Each
// bound below measured faster with the same bits (batches of about 2 GB of traffic):
//   - FP64 elastic, order 7: 189 registers, one 512-thread workgroup per CU; at 128 (two) it spills 108 bytes per
//     lane and runs 30% faster. Curvilinear: 231 registers, 272 bytes of spills, 4% faster.
//   - FP32 elastic, order 8: 114 registers, one 729-thread workgroup; at 80 (two) 28 bytes of spills, 22% faster.
//   - FP32 acoustic, order 9: 89 registers, one 1000-thread workgroup; at 64 (two) 52 bytes, 21% faster.
//   - FP32 I/O with FP64 accumulation, elastic order 6: at 96 registers (three 343-thread workgroups instead of
//     two) 16% faster.
// The same bound made FP32 elastic order 7 4% slower and, with FP64 accumulation, elastic orders 7 and 8 and
// curvilinear order 7 10-50% slower. With FP64 accumulation, acoustic orders 8 and 9 ran 20-27% faster bounded
// to two workgroups per CU on whole-GPU batches, but the serving path's mixed batches launch these classes with
// a few dozen elements, where the longer workgroups cost 4% of its batch rate; they, and the rest, keep the
// compiler's choice.
template <typename T, typename ACC, int N, int PHYS>
struct PlainWaves {
    static constexpr bool f32 = sizeof(T) == 4 && sizeof(ACC) == 4;  // FP32 I/O and accumulation
    static constexpr bool a64 = sizeof(T) == 4 && sizeof(ACC) == 8;  // FP32 I/O, FP64 accumulation
    static constexpr int v = (sizeof(T) == 8 && N == 7 && (PHYS == kElastic || PHYS == kElasticCurv)) ? 4
                             : (f32 && PHYS == kElastic && N == 8) ? 6
                             : (f32 && PHYS == kAcoustic && N == 9) ? 8
                             : (a64 && PHYS == kElastic && N == 6) ? 5
                                                                    : 1;
};

template <typename T, typename ACC, int N, int PHYS, int MB, bool EX>
__global__ void __launch_bounds__(((N + 1) * (N + 1) * (N + 1) + 63) / 64 * 64)
    __attribute__((amdgpu_waves_per_eu(PlainWaves<T, ACC, N, PHYS>::v))) stp_plain_kernel(StpArgs a)
{
    Plain<T, ACC, N, PHYS, MB, EX>::run(a);
}

template <typename T, typename ACC, int N, int PHYS, int MB, bool EX>
KernelInfo plain_info()
{
    using K = Plain<T, ACC, N, PHYS, MB, EX>;
    KernelInfo ki;
    ki.fn = reinterpret_cast<const void*>(&stp_plain_kernel<T, ACC, N, PHYS, MB, EX>);
    ki.block = K::NT;
    ki.mb = MB;
    ki.lds = [](int m, bool hasA) -> size_t { return K::layout(m, hasA).total; };
    return ki;
}

template <typename T, typename ACC, int PHYS, int MB, bool EX = false>
KernelInfo plain_by_order(int N)
{
    switch (N) {
    case 1: return plain_info<T, ACC, 1, PHYS, MB, EX>();
    case 2: return plain_info<T, ACC, 2, PHYS, MB, EX>();
    case 3: return plain_info<T, ACC, 3, PHYS, MB, EX>();
    case 4: return plain_info<T, ACC, 4, PHYS, MB, EX>();
    case 5: return plain_info<T, ACC, 5, PHYS, MB, EX>();
    case 6: return plain_info<T, ACC, 6, PHYS, MB, EX>();
    case 7: return plain_info<T, ACC, 7, PHYS, MB, EX>();
    case 8: return plain_info<T, ACC, 8, PHYS, MB, EX>();
    case 9: return plain_info<T, ACC, 9, PHYS, MB, EX>();
    default: return KernelInfo{};
    }
}

// Presets (acoustic, elastic, curvilinear elastic) and the generic classes with m = 4 or m = 9 (compiled with
// m fixed). The generic classes with
// another m use a run-time quantity count bounded by 4, 9 or 16 (plain_generic_rt), instantiated in
// translation units of their own so that the library builds in parallel.
template <typename T, typename ACC>
KernelInfo plain_by_physics(int N, int physics, int m)
{
    if (physics == kAcoustic) return plain_by_order<T, ACC, kAcoustic, 4>(N);
    if (physics == kElastic) return plain_by_order<T, ACC, kElastic, 9>(N);
    if (physics == kElasticCurv) return plain_by_order<T, ACC, kElasticCurv, 9>(N);
    if (m == 4) return plain_by_order<T, ACC, kGeneric, 4, true>(N);
    if (m == 9) return plain_by_order<T, ACC, kGeneric, 9, true>(N);
    return KernelInfo{};
}

template <typename T, typename ACC, int MB>
KernelInfo plain_generic_rt(int N)
{
    return plain_by_order<T, ACC, kGeneric, MB>(N);
}

}  // namespace plain
}  // namespace stp
