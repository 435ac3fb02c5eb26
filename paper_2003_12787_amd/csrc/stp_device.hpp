// stp_device.hpp -- definitions shared by the predictor's HIP kernels: the launch argument block, element
// addressing, and the pointwise PDE terms of the physics presets.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace stp {

enum Physics : int { kAcoustic = 0, kElastic = 1, kGeneric = 2, kElasticCurv = 3 };

// Class flags (mirror the STP_* flags of stp.h).
constexpr unsigned kParamPerElement = 1u << 0;
constexpr unsigned kAPresent = 1u << 1;
constexpr unsigned kCoefPerElement = 1u << 2;
constexpr unsigned kFavgSum = 1u << 3;
constexpr unsigned kSrcPoint = 1u << 4;

// Launch argument block (passed by value). Pointers are device pointers.
struct StpArgs {
    int64_t nelem;             // elements handled by this launch
    const int32_t* list;       // element ids of this launch (NULL: 0..nelem-1)
    const int32_t* count;      // device element count of `list` (NULL: nelem)
    const int64_t* off_q;      // per-element offsets (NULL: contiguous with the strides below)
    const int64_t* off_coef;
    const int64_t* off_face;
    const int64_t* off_src;
    int64_t stride_q, stride_coef, stride_face, stride_src;
    const double* dt;          // per element (NULL: dt_s)
    const double* h;           // per element (NULL: h_s)
    double dt_s, h_s;
    const void* Q;
    const void* params;
    const void* A;
    const void* B;
    const void* src;
    void* qavg;
    void* favg;
    void* qface;
    void* fface;
    const void* D;             // [n][n] derivative matrix in the compute precision
    const void* e0;            // [n] l_j(0)
    const void* e1;            // [n] l_j(1)
    const void* Dsplit;        // BF16 tables for the MFMA variant (layout owned by that kernel)
    int m;                     // quantity count (generic; presets use their fixed m)
    unsigned flags;
};

struct ElemRef {
    int64_t e, q, coef, face, src;
    double dt, h;
};

// A zero the compiler cannot see through. Addresses offset by it count as loop-variant, so loads and address
// arithmetic inside a loop stay there instead of being hoisted out and kept live across all iterations.
__device__ inline int opaque_zero()
{
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
}

__device__ inline bool elem_ref(const StpArgs& a, int64_t i, ElemRef& r)
{
    int64_t cnt = a.count ? (int64_t)*a.count : a.nelem;
    if (i >= cnt) return false;
    int64_t e = a.list ? (int64_t)a.list[i] : i;
    r.e = e;
    r.q = a.off_q ? a.off_q[e] : e * a.stride_q;
    r.coef = a.off_coef ? a.off_coef[e] : e * a.stride_coef;
    r.face = a.off_face ? a.off_face[e] : e * a.stride_face;
    r.src = a.off_src ? a.off_src[e] : e * a.stride_src;
    r.dt = a.dt ? a.dt[e] : a.dt_s;
    r.h = a.h ? a.h[e] : a.h_s;
    return true;
}

template <int PHYS>
struct PhysTraits;
template <>
struct PhysTraits<kAcoustic> {
    static constexpr int m = 4;
    static constexpr int np = 2;
    // quantities that B_d reads in direction d: p (0) and v_d (1+d)
    __host__ __device__ static constexpr bool needs(int d, int s) { return s == 0 || s == 1 + d; }
};
template <>
struct PhysTraits<kElastic> {
    static constexpr int m = 9;
    static constexpr int np = 3;
    // stress index of the symmetric pair (i, j): xx,yy,zz = 3,4,5; xy = 6, yz = 7, xz = 8
    __host__ __device__ static constexpr int sig(int i, int j)
    {
        return i == j ? 3 + i : ((i + j == 1) ? 6 : ((i + j == 3) ? 7 : 8));
    }
    // quantities that B_d reads in direction d: the three velocities and the stresses s_{d,i}
    __host__ __device__ static constexpr bool needs(int d, int s)
    {
        return s < 3 || s == sig(d, 0) || s == sig(d, 1) || s == sig(d, 2);
    }
};

// Elastic on a curvilinear element: B_d = sum_j G[d][j] M_j mixes every quantity into every direction.
template <>
struct PhysTraits<kElasticCurv> {
    static constexpr int m = 9;
    static constexpr int np = 12;  // rho, lambda, mu, G[3][3]
    __host__ __device__ static constexpr bool needs(int, int) { return true; }
};

template <>
struct PhysTraits<kGeneric> {
    static constexpr int m = 0;   // runtime
    static constexpr int np = 0;  // no material parameters: A_d, B_d are given
    __host__ __device__ static constexpr bool needs(int, int) { return true; }
};

// Per-node material coefficients with -1/h folded in, in the compute precision.
//   acoustic: c0 = -K/h, c1 = -1/(rho h)
//   elastic : c0 = 1/(rho h), c1 = lambda/h, c2 = mu/h, c3 = (lambda + 2 mu)/h
template <typename T, int PHYS>
struct Material {
    T c[4];
    __device__ inline void load(const T* par, double inv_h)
    {
        if constexpr (PHYS == kAcoustic) {
            double rho = (double)par[0], K = (double)par[1];
            c[0] = (T)(-K * inv_h);
            c[1] = (T)(-inv_h / rho);
            c[2] = c[3] = (T)0;
        } else if constexpr (PHYS == kElastic) {
            double rho = (double)par[0], lam = (double)par[1], mu = (double)par[2];
            c[0] = (T)(inv_h / rho);
            c[1] = (T)(lam * inv_h);
            c[2] = (T)(mu * inv_h);
            c[3] = (T)((lam + 2.0 * mu) * inv_h);
        }
    }
    // The same coefficients from FP32 arithmetic (a reciprocal within 1 ulp for 1/rho): the matrix-core kernels,
    // whose BF16 products are accurate to about FP32, spend no FP64 instructions on them.
    __device__ inline void load_f32(const float* par, float ih)
    {
        if constexpr (PHYS == kAcoustic) {
            c[0] = -par[1] * ih;
            c[1] = -ih * __builtin_amdgcn_rcpf(par[0]);
            c[2] = c[3] = 0.f;
        } else if constexpr (PHYS == kElastic) {
            const float lam = par[1], mu = par[2];
            c[0] = ih * __builtin_amdgcn_rcpf(par[0]);
            c[1] = lam * ih;
            c[2] = mu * ih;
            c[3] = fmaf(2.f, mu, lam) * ih;
        }
    }
};

// Curvilinear elastic: the elastic coefficients plus the metric terms G[d][j] = h dxi_d/dx_j of the node.
template <typename T>
struct Material<T, kElasticCurv> {
    T c[4];  // as elastic: 1/(rho h), lambda/h, mu/h, (lambda + 2 mu)/h
    T G[9];
    __device__ inline void load(const T* par, double inv_h)
    {
        double rho = (double)par[0], lam = (double)par[1], mu = (double)par[2];
        c[0] = (T)(inv_h / rho);
        c[1] = (T)(lam * inv_h);
        c[2] = (T)(mu * inv_h);
        c[3] = (T)((lam + 2.0 * mu) * inv_h);
#pragma unroll
        for (int k = 0; k < 9; ++k) G[k] = par[3 + k];
    }
    __device__ inline void load_f32(const T* par, float ih)
    {
        const float lam = par[1], mu = par[2];
        c[0] = ih * __builtin_amdgcn_rcpf(par[0]);
        c[1] = lam * ih;
        c[2] = mu * ih;
        c[3] = fmaf(2.f, mu, lam) * ih;
#pragma unroll
        for (int k = 0; k < 9; ++k) G[k] = par[3 + k];
    }
};

// r += -(1/h) B_d g  for a preset, with g the reference derivative along d of the quantities B_d reads.
template <typename T, int PHYS, int D>
__device__ inline void apply_ncp(const Material<T, PHYS>& mt, const T* g, T* r)
{
    if constexpr (PHYS == kAcoustic) {
        r[0] = fma(mt.c[0], g[1 + D], r[0]);  // p_t = -K dv_d/dx_d
        r[1 + D] = fma(mt.c[1], g[0], r[1 + D]);  // v_d,t = -(1/rho) dp/dx_d
    } else if constexpr (PHYS == kElasticCurv) {
        // The reference derivative g along xi_d contributes G[d][j] g / h to the physical derivative along
        // x_j; r += the elastic operator of that gradient (1/h is folded into c).
        using P = PhysTraits<kElastic>;
        const T G0 = mt.G[3 * D], G1 = mt.G[3 * D + 1], G2 = mt.G[3 * D + 2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {  // rho v_i,t = sum_j d s_ij / dx_j
            T t = G0 * g[P::sig(i, 0)];
            t = fma(G1, g[P::sig(i, 1)], t);
            t = fma(G2, g[P::sig(i, 2)], t);
            r[i] = fma(mt.c[0], t, r[i]);
        }
        T dv = G0 * g[0];  // div v
        dv = fma(G1, g[1], dv);
        dv = fma(G2, g[2], dv);
        const T Gd[3] = {G0, G1, G2};
        const T mu2 = mt.c[3] - mt.c[1];
#pragma unroll
        for (int i = 0; i < 3; ++i) {  // s_ii,t = lambda div v + 2 mu dv_i/dx_i
            r[3 + i] = fma(mt.c[1], dv, r[3 + i]);
            r[3 + i] = fma(mu2 * Gd[i], g[i], r[3 + i]);
        }
        // s_ij,t = mu (dv_i/dx_j + dv_j/dx_i) for (i, j) = (x, y), (y, z), (x, z)
        r[6] = fma(mt.c[2], fma(G1, g[0], G0 * g[1]), r[6]);
        r[7] = fma(mt.c[2], fma(G2, g[1], G1 * g[2]), r[7]);
        r[8] = fma(mt.c[2], fma(G2, g[0], G0 * g[2]), r[8]);
    } else {
        using P = PhysTraits<kElastic>;
#pragma unroll
        for (int i = 0; i < 3; ++i) r[i] = fma(mt.c[0], g[P::sig(i, D)], r[i]);  // rho v_i,t = d s_id / dx_d
#pragma unroll
        for (int i = 0; i < 3; ++i) r[3 + i] = fma(i == D ? mt.c[3] : mt.c[1], g[D], r[3 + i]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (i != D) r[P::sig(D, i)] = fma(mt.c[2], g[i], r[P::sig(D, i)]);  // s_di,t = mu dv_i/dx_d
    }
}

template <typename T>
__device__ inline T ld(const void* p, int64_t i)
{
    return static_cast<const T*>(p)[i];
}

}  // namespace stp
