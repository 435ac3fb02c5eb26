// stp_correct.hip -- the corrector of the ADER-DG step (Sec. II-A, Eq. (5)) on a periodic Cartesian mesh.
//
// Given q(t_n) and the predictor's outputs of every element (time-averaged volume term favg[d] = V_d(q-bar),
// face projections of q-bar and of A_d q-bar), the corrector adds the time integral of the volume term and
// of the face terms. The numerical flux is a linear Rusanov flux in fluctuation form: at the face f of an
// element with outward normal s e_d (s = -1 lower, +1 upper), with q- / F- the element's own face values and
// q+ / F+ the neighbour's values on the same face,
//     C_f = 1/2 alpha (q+ - q-) - 1/2 s (F+ - F-) - 1/2 s Bbar_d (q+ - q-),
// Bbar_d the mean of the two elements' B_d and alpha the larger of their fastest wave speeds (acoustic
// sqrt(K/rho), elastic sqrt((lambda + 2 mu)/rho), generic max_d ||A_d + B_d||_inf). With Gauss-Legendre
// collocation and the diagonal mass matrix the node k of the element receives
//     q(t_{n+1})_k = q(t_n)_k + dt sum_d favg[d]_k + dt sum_f l_{k_d}(x_f) / (h w_{k_d}) C_f(face node of k).
// One workgroup per element: the face corrections of all six faces go to LDS, then every node is updated.
// Coefficients are per element (presets: rho, K or rho, lambda, mu; generic: A_d, B_d [3][m][m]). Curvilinear
// elastic elements with affine geometry carry rho, lambda, mu and the constant metric G[d][j] = h dxi_d/dx_j
// (12 values): B_d = sum_j G[d][j] M_j with M_j the Cartesian elastic matrices, and alpha = sqrt((lambda +
// 2 mu)/rho) max_d |G[d][:]|_2; the scheme is the Cartesian one in the reference coordinates of the mesh.
// Curved elements carry the 12 parameters per node: at every face point each side's parameters are
// extrapolated from its nodes along the normal with the face vectors, and B_d and alpha are those of the
// extrapolated parameters (mean of the two sides' B_d, larger alpha). Those face values do not change between
// steps: stp_face_params forms them once (same arithmetic), and the corrector then reads them per face point.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "stp_plan.hpp"

namespace stp {

namespace {

constexpr int kCorrThreads = 256;
// Kernel instantiation tag of curved curvilinear elements (parameters per node [e][n^3][12]); the affine ones
// (per element) use kElasticCurv.
constexpr int kCurvNode = 4;
// ... and of curved elements whose face-point parameters [e][6][n^2][12] are given (stp_face_params).
constexpr int kCurvFace = 5;
constexpr int kCorrMaxM = 16;

struct CorrArgs {
    int nx, ny, nz;
    int N, m, physics, favg_sum, hasA;
    double dt, h;
    const void* Q;
    const void* coef;  // presets: params [e][np]; generic: B [e][3][m][m]
    const void* A;     // generic with A: [e][3][m][m]
    const void* favg;
    const void* qface;
    const void* fface;
    void* Qnew;
    const void* fparams;  // curved elements: parameters at the face points [e][6][n^2][12], or NULL
    const void* e0;  // face vectors l_j(0), l_j(1) and quadrature weights on [0, 1] (compute precision)
    const void* e1;
    const void* w;
};

__device__ inline int64_t neighbour_of(const CorrArgs& a, int64_t e, int d, int s)
{
    int64_t ix = e % a.nx, iy = (e / a.nx) % a.ny, iz = e / ((int64_t)a.nx * a.ny);
    if (d == 0) ix = (ix + s + a.nx) % a.nx;
    else if (d == 1) iy = (iy + s + a.ny) % a.ny;
    else iz = (iz + s + a.nz) % a.nz;
    return (iz * a.ny + iy) * a.nx + ix;
}

// (Bbar_d j) for a preset, from the face's averaged coefficients c = (1/rho, K) or (1/rho, lambda, mu): the
// entries of the presets' B_d are linear in these, so the mean of two elements' B_d is B_d of the means.
// The direction is a template parameter so that every quantity index is a constant (no indexed register
// arrays).
template <typename T, int PHYS, int D>
__device__ inline void preset_Bj(const T* c, const T* j, T* out)
{
    if constexpr (PHYS == kAcoustic) {
        out[0] = c[1] * j[1 + D];  // p <- K d_d v_d
#pragma unroll
        for (int i = 0; i < 3; ++i) out[1 + i] = i == D ? c[0] * j[0] : T(0);  // v_d <- d_d p / rho
    } else {
        constexpr auto sig = [](int i, int k) { return i == k ? 3 + i : (i + k == 1 ? 6 : (i + k == 3 ? 7 : 8)); };
#pragma unroll
        for (int i = 0; i < 3; ++i) out[i] = -c[0] * j[sig(i, D)];                          // v_i <- d_d s_id
#pragma unroll
        for (int i = 0; i < 3; ++i) out[3 + i] = i == D ? -(c[1] + 2 * c[2]) * j[D] : -c[1] * j[D];  // s_ii <- v_d
        out[6] = out[7] = out[8] = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (i != D) out[sig(D, i)] = -c[2] * j[i];                                       // s_di <- v_i
    }
}

// (Bbar_d j) for curvilinear elements: B_d = sum_j G[d][j] M_j is bilinear in the metric and the material,
// so the mean over the two elements of the face is taken of the products, side by side. p0, p1: the 12
// parameters (rho, lambda, mu, G) of the element and of its neighbour.
template <typename T, int K>
__device__ inline void curv_term(const T* c, T g, const T* j, T* out)
{
    T t[9];
    preset_Bj<T, kElastic, K>(c, j, t);
#pragma unroll
    for (int r = 0; r < 9; ++r) out[r] = fma(g, t[r], out[r]);
}

template <typename T, int D>
__device__ inline void curv_Bj(const T* p0, const T* p1, const T* j, T* out)
{
#pragma unroll
    for (int r = 0; r < 9; ++r) out[r] = 0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const T* p = side ? p1 : p0;
        const T c[3] = {(T)1 / p[0], p[1], p[2]};
        curv_term<T, 0>(c, (T)0.5 * p[3 + 3 * D], j, out);
        curv_term<T, 1>(c, (T)0.5 * p[4 + 3 * D], j, out);
        curv_term<T, 2>(c, (T)0.5 * p[5 + 3 * D], j, out);
    }
}

// The node of the line along d through face node (fa, fb) (the two other axes, slower first), at index j.
template <int n>
__device__ inline int line_node(int d, int fa, int fb, int j)
{
    return d == 0 ? (fa * n + fb) * n + j : (d == 1 ? (fa * n + j) * n + fb : (j * n + fa) * n + fb);
}

// The 12 parameters of element nodes par [n^3][12] extrapolated to face node (fa, fb) of a face normal to d,
// with that face's vector ev (l_j(0) or l_j(1)).
template <typename T, int n>
__device__ inline void face_extrapolate(const T* par, const T* ev, int d, int fa, int fb, T* ext)
{
#pragma unroll
    for (int i = 0; i < 12; ++i) ext[i] = 0;
#pragma unroll 1  // unrolled, the loads of all n nodes are hoisted and the corrector loses occupancy
    for (int j = 0; j < n; ++j) {
        const T* p = par + line_node<n>(d, fa, fb, j) * 12;
        const T w = ev[j];
#pragma unroll
        for (int i = 0; i < 12; ++i) ext[i] = fma(w, p[i], ext[i]);
    }
}

// alpha of curvilinear parameters (rho, lambda, mu, G)
template <typename T>
__device__ inline T curv_speed(const T* p)
{
    T g = 0;
    for (int d = 0; d < 3; ++d) {
        const T r = sqrt(p[3 + 3 * d] * p[3 + 3 * d] + p[4 + 3 * d] * p[4 + 3 * d] + p[5 + 3 * d] * p[5 + 3 * d]);
        g = r > g ? r : g;
    }
    return sqrt((p[1] + 2 * p[2]) / p[0]) * g;
}

template <typename T>
__device__ T wave_speed(const CorrArgs& a, int64_t e)
{
    if (a.physics == kAcoustic) {
        const T* p = static_cast<const T*>(a.coef) + e * 2;
        return sqrt(p[1] / p[0]);
    }
    if (a.physics == kElastic) {
        const T* p = static_cast<const T*>(a.coef) + e * 3;
        return sqrt((p[1] + 2 * p[2]) / p[0]);
    }
    if (a.physics == kElasticCurv) return curv_speed(static_cast<const T*>(a.coef) + e * 12);
    const int m = a.m;
    const T* B = static_cast<const T*>(a.coef) + e * 3 * m * m;
    const T* A = a.hasA ? static_cast<const T*>(a.A) + e * 3 * m * m : nullptr;
    T best = 0;
    for (int d = 0; d < 3; ++d)
        for (int r = 0; r < m; ++r) {
            T row = 0;
            for (int c = 0; c < m; ++c) row += fabs(B[(d * m + r) * m + c] + (A ? A[(d * m + r) * m + c] : T(0)));
            best = row > best ? row : best;
        }
    return best;
}

// Instantiated per order and physics, so that the index arithmetic divides by constants (with a run-time
// order and quantity count, integer divisions dominated the kernel).
template <typename T, int N, int PHYS>
__global__ void __launch_bounds__(kCorrThreads) stp_correct_kernel(CorrArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
    const int m = PHYS == kAcoustic ? 4 : (PHYS == kGeneric ? a.m : 9);
    constexpr bool preset = PHYS != kGeneric;
    constexpr bool curv = PHYS == kElasticCurv || PHYS == kCurvNode || PHYS == kCurvFace;
    constexpr bool per_node = PHYS == kCurvNode;
    constexpr bool pointwise = per_node || PHYS == kCurvFace;  // parameters differ between face points
    T* Bbar = reinterpret_cast<T*>(smem);  // generic: [6][m][m] mean B_d of the element and its neighbour
    T* cbar = Bbar + (preset ? 0 : 6 * m * m);  // presets: [6][4] mean (1/rho, K) or (1/rho, lambda, mu);
                                               // curvilinear: [6][2][12] parameters of both elements
    T* Cf = cbar + (curv ? 144 : 24);      // [6][n^2][m] face corrections
    T* alpha = Cf + 6 * n2 * m;            // [6]
    T* lift0 = alpha + 8;                  // [n] l_j(0) / (h w_j)
    T* lift1 = lift0 + n;                  // [n] l_j(1) / (h w_j)
    T* ev0 = lift1 + n;                    // [n] l_j(0)
    T* ev1 = ev0 + n;                      // [n] l_j(1)
    const int64_t nelem = (int64_t)a.nx * a.ny * a.nz;
    const int tid = threadIdx.x;
    if (tid < n) {
        const T* w = static_cast<const T*>(a.w);
        lift0[tid] = static_cast<const T*>(a.e0)[tid] / ((T)a.h * w[tid]);
        lift1[tid] = static_cast<const T*>(a.e1)[tid] / ((T)a.h * w[tid]);
        ev0[tid] = static_cast<const T*>(a.e0)[tid];
        ev1[tid] = static_cast<const T*>(a.e1)[tid];
    }
    for (int64_t e = blockIdx.x; e < nelem; e += gridDim.x) {
        // per-face mean coefficients and Rusanov speeds
        if (tid < 6 && !pointwise) {
            const int d = tid >> 1, s = (tid & 1) ? 1 : -1;
            const int64_t nb = neighbour_of(a, e, d, s);
            if constexpr (curv) {
                const T* p0 = static_cast<const T*>(a.coef) + e * 12;
                const T* p1 = static_cast<const T*>(a.coef) + nb * 12;
                for (int i = 0; i < 12; ++i) {
                    cbar[tid * 24 + i] = p0[i];
                    cbar[tid * 24 + 12 + i] = p1[i];
                }
            } else if constexpr (preset) {
                const int np = PHYS == kAcoustic ? 2 : 3;
                const T* p0 = static_cast<const T*>(a.coef) + e * np;
                const T* p1 = static_cast<const T*>(a.coef) + nb * np;
                cbar[tid * 4 + 0] = (T)0.5 * ((T)1 / p0[0] + (T)1 / p1[0]);
                for (int i = 1; i < np; ++i) cbar[tid * 4 + i] = (T)0.5 * (p0[i] + p1[i]);
            }
            const T a0 = wave_speed<T>(a, e), a1 = wave_speed<T>(a, nb);
            alpha[tid] = a0 > a1 ? a0 : a1;
        }
        if constexpr (!preset) {
            for (int i = tid; i < 6 * m * m; i += kCorrThreads) {
                const int f = i / (m * m), r = i - f * m * m, d = f >> 1;
                const int64_t nb = neighbour_of(a, e, d, (f & 1) ? 1 : -1);
                const T* B = static_cast<const T*>(a.coef);
                Bbar[i] = (T)0.5 * (B[(e * 3 + d) * m * m + r] + B[(nb * 3 + d) * m * m + r]);
            }
        }
        __syncthreads();
        // face corrections: one face point (all quantities) per work item; the preset products are dispatched on
        // the direction so that they index registers with constants
        const T* qf = static_cast<const T*>(a.qface);
        const T* ff = static_cast<const T*>(a.fface);
        for (int it = tid; it < 6 * n2; it += kCorrThreads) {
            const int f = it / n2, pt = it - f * n2, d = f >> 1, side = f & 1;
            const T s = side ? T(1) : T(-1);
            const int64_t nb = neighbour_of(a, e, d, side ? 1 : -1);
            const int fo = 2 * d + (1 - side);
            const T* qm = qf + ((e * 6 + f) * n2 + pt) * m;
            const T* qp = qf + ((nb * 6 + fo) * n2 + pt) * m;
            T jump[kCorrMaxM], bj[kCorrMaxM];
            for (int r = 0; r < m; ++r) jump[r] = qp[r] - qm[r];
            T al = 0;
            if constexpr (curv) {
                if constexpr (pointwise) {  // curved: both sides' parameters at the face point
                    T ext[24];
                    if constexpr (per_node) {  // extrapolated from the nodes: own face vector, the neighbour's
                        const T* par = static_cast<const T*>(a.coef);  // opposite one
                        const int fa = pt / n, fb = pt - fa * n;
                        face_extrapolate<T, n>(par + e * n3 * 12, side ? ev1 : ev0, d, fa, fb, ext);
                        face_extrapolate<T, n>(par + nb * n3 * 12, side ? ev0 : ev1, d, fa, fb, ext + 12);
                    } else {
                        const T* fp = static_cast<const T*>(a.fparams);
                        const T* pm = fp + ((e * 6 + f) * n2 + pt) * 12;
                        const T* pp = fp + ((nb * 6 + fo) * n2 + pt) * 12;
#pragma unroll
                        for (int i = 0; i < 12; ++i) {
                            ext[i] = pm[i];
                            ext[12 + i] = pp[i];
                        }
                    }
                    const T a0 = curv_speed(ext), a1 = curv_speed(ext + 12);
                    al = a0 > a1 ? a0 : a1;
                    if (d == 0) curv_Bj<T, 0>(ext, ext + 12, jump, bj);
                    else if (d == 1) curv_Bj<T, 1>(ext, ext + 12, jump, bj);
                    else curv_Bj<T, 2>(ext, ext + 12, jump, bj);
                } else {  // affine: the two elements' parameters staged in LDS
                    const T* c = cbar + f * 24;
                    al = alpha[f];
                    if (d == 0) curv_Bj<T, 0>(c, c + 12, jump, bj);
                    else if (d == 1) curv_Bj<T, 1>(c, c + 12, jump, bj);
                    else curv_Bj<T, 2>(c, c + 12, jump, bj);
                }
            } else if constexpr (preset) {
                if (d == 0) preset_Bj<T, PHYS, 0>(cbar + f * 4, jump, bj);
                else if (d == 1) preset_Bj<T, PHYS, 1>(cbar + f * 4, jump, bj);
                else preset_Bj<T, PHYS, 2>(cbar + f * 4, jump, bj);
            } else {
                const T* Bf = Bbar + f * m * m;
                for (int r = 0; r < m; ++r) {
                    T acc = 0;
                    for (int c = 0; c < m; ++c) acc = fma(Bf[r * m + c], jump[c], acc);
                    bj[r] = acc;
                }
            }
            if constexpr (!curv) al = alpha[f];
            for (int r = 0; r < m; ++r) {
                T v = (T)0.5 * al * jump[r] - (T)0.5 * s * bj[r];
                if (a.hasA) {
                    const T Fm = ff[((e * 6 + f) * n2 + pt) * m + r];
                    const T Fp = ff[((nb * 6 + fo) * n2 + pt) * m + r];
                    v -= (T)0.5 * s * (Fp - Fm);
                }
                Cf[(f * n2 + pt) * m + r] = v;
            }
        }
        __syncthreads();
        // node updates
        const T dt = (T)a.dt;
        const T* Q = static_cast<const T*>(a.Q) + e * n3 * m;
        const T* fa = static_cast<const T*>(a.favg) + (a.favg_sum ? e * n3 * m : e * 3 * n3 * m);
        T* out = static_cast<T*>(a.Qnew) + e * n3 * m;
        for (int it = tid; it < n3 * m; it += kCorrThreads) {
            const int r = it % m, k = it / m;
            const int kx = k % n, ky = (k / n) % n, kz = k / n2;
            T vol = fa[it];
            if (!a.favg_sum) vol += fa[n3 * m + it] + fa[2 * n3 * m + it];
            T face = lift0[kx] * Cf[((0 * n2) + kz * n + ky) * m + r] + lift1[kx] * Cf[((1 * n2) + kz * n + ky) * m + r];
            face += lift0[ky] * Cf[((2 * n2) + kz * n + kx) * m + r] + lift1[ky] * Cf[((3 * n2) + kz * n + kx) * m + r];
            face += lift0[kz] * Cf[((4 * n2) + ky * n + kx) * m + r] + lift1[kz] * Cf[((5 * n2) + ky * n + kx) * m + r];
            out[it] = Q[it] + dt * (vol + face);
        }
        __syncthreads();
    }
}

template <typename T, int PHYS>
const void* corr_kernel_by_order(int N)
{
    switch (N) {
    case 1: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 1, PHYS>);
    case 2: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 2, PHYS>);
    case 3: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 3, PHYS>);
    case 4: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 4, PHYS>);
    case 5: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 5, PHYS>);
    case 6: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 6, PHYS>);
    case 7: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 7, PHYS>);
    case 8: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 8, PHYS>);
    default: return reinterpret_cast<const void*>(&stp_correct_kernel<T, 9, PHYS>);
    }
}

template <typename T>
const void* corr_kernel(int N, int physics, bool per_node, bool face_params)
{
    if (physics == kAcoustic) return corr_kernel_by_order<T, kAcoustic>(N);
    if (physics == kElastic) return corr_kernel_by_order<T, kElastic>(N);
    if (physics == kElasticCurv) {
        if (!per_node) return corr_kernel_by_order<T, kElasticCurv>(N);
        return face_params ? corr_kernel_by_order<T, kCurvFace>(N) : corr_kernel_by_order<T, kCurvNode>(N);
    }
    return corr_kernel_by_order<T, kGeneric>(N);
}

size_t corr_lds(int N, int m, size_t io)
{
    const int n = N + 1;
    return io * (size_t)(6 * m * m + 144 + 6 * n * n * m + 8 + 4 * n);
}

constexpr int kFaceThreads = 256;

// One work item per face point of an element: fp[e][f][pt][12] from par[e][n^3][12].
template <typename T, int N>
__global__ void __launch_bounds__(kFaceThreads) stp_face_params_kernel(int64_t nelem, const T* __restrict__ par,
                                                                        T* __restrict__ fp, const T* e0, const T* e1)
{
    constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
    const int64_t total = nelem * 6 * n2;
    for (int64_t it = blockIdx.x * (int64_t)kFaceThreads + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * kFaceThreads) {
        const int64_t e = it / (6 * n2);
        const int r = (int)(it - e * (6 * n2)), f = r / n2, pt = r - f * n2, fa = pt / n;
        T ext[12];
        face_extrapolate<T, n>(par + e * n3 * 12, (f & 1) ? e1 : e0, f >> 1, fa, pt - fa * n, ext);
#pragma unroll
        for (int i = 0; i < 12; ++i) fp[it * 12 + i] = ext[i];
    }
}

template <typename T>
const void* face_params_kernel(int N)
{
    switch (N) {
    case 1: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 1>);
    case 2: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 2>);
    case 3: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 3>);
    case 4: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 4>);
    case 5: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 5>);
    case 6: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 6>);
    case 7: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 7>);
    case 8: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 8>);
    default: return reinterpret_cast<const void*>(&stp_face_params_kernel<T, 9>);
    }
}

}  // namespace

}  // namespace stp

using namespace stp;

extern "C" stp_status stp_correct(stp_plan_t p, const stp_step* st, void* stream)
{
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    if (!st) return fail(STP_E_INVAL, "step is NULL");
    if (p->classes.size() != 1) return fail(STP_E_UNSUPPORTED, "the corrector takes a single-class plan");
    const ClassState& cs = p->classes[0];
    const stp_class& c = cs.cls;
    const bool generic = c.physics == STP_GENERIC;
    const bool curv = c.physics == STP_ELASTIC_CURV;  // affine (per element) or curved (per node)
    if (!curv && (generic ? !(c.flags & STP_COEF_PER_ELEMENT) : !(c.flags & STP_PARAM_PER_ELEMENT)))
        return fail(STP_E_UNSUPPORTED, "the corrector needs per-element coefficients (STP_PARAM_PER_ELEMENT or "
                                       "STP_COEF_PER_ELEMENT)");
    if (c.flags & STP_SRC_POINT) return fail(STP_E_UNSUPPORTED, "point sources are not supported by the corrector");
    if (st->nx < 1 || st->ny < 1 || st->nz < 1) return fail(STP_E_INVAL, "mesh %d x %d x %d", st->nx, st->ny, st->nz);
    if ((int64_t)st->nx * st->ny * st->nz > (int64_t)INT32_MAX) return fail(STP_E_INVAL, "mesh too large");
    if (!(st->h > 0) || !std::isfinite(st->h)) return fail(STP_E_INVAL, "h must be > 0 (got %g)", st->h);
    if (!(st->dt >= 0) || !std::isfinite(st->dt)) return fail(STP_E_INVAL, "dt must be >= 0 (got %g)", st->dt);
    const bool hasA = generic && (c.flags & STP_A_PRESENT);
    if (!st->Q || !st->favg || !st->qface || !st->Qnew) return fail(STP_E_INVAL, "Q / favg / qface / Qnew is NULL");
    if (generic ? !st->B : !st->params) return fail(STP_E_INVAL, "coefficients are NULL");
    if (hasA && (!st->A || !st->fface)) return fail(STP_E_INVAL, "A / fface is NULL for a class with A present");
    const bool per_node = curv && !(c.flags & STP_PARAM_PER_ELEMENT);
    if (st->fparams && !per_node)
        return fail(STP_E_INVAL, "fparams is for curved curvilinear elements (parameters per node) only");
    const int64_t E = (int64_t)st->nx * st->ny * st->nz;
    const size_t io = p->prec == STP_FP64 ? 8 : 4;
    {
        const uintptr_t o0 = (uintptr_t)st->Qnew, o1 = o0 + (size_t)E * cs.size_q * io;
        const size_t fmul = (c.flags & STP_FAVG_SUM) ? 1 : 3;
        struct R { const void* q; size_t bytes; const char* name; };
        const R ins[] = {{st->Q, (size_t)E * cs.size_q * io, "Q"}, {st->favg, (size_t)E * fmul * cs.size_q * io, "favg"},
                         {st->qface, (size_t)E * cs.size_face * io, "qface"},
                         {st->fparams, (size_t)E * 6 * (c.order + 1) * (c.order + 1) * 12 * io, "fparams"}};
        for (const R& r : ins) {
            if (!r.q) continue;
            const uintptr_t a0 = (uintptr_t)r.q, a1 = a0 + r.bytes;
            if (a0 < o1 && o0 < a1) return fail(STP_E_INVAL, "Qnew aliases %s", r.name);
        }
    }
    if (E == 0) return STP_OK;
    CorrArgs a{};
    a.nx = st->nx;
    a.ny = st->ny;
    a.nz = st->nz;
    a.N = c.order;
    a.m = c.nquant;
    a.physics = c.physics;
    a.favg_sum = (c.flags & STP_FAVG_SUM) ? 1 : 0;
    a.hasA = hasA ? 1 : 0;
    a.dt = st->dt;
    a.h = st->h;
    a.Q = st->Q;
    a.coef = generic ? st->B : st->params;
    a.A = st->A;
    a.favg = st->favg;
    a.qface = st->qface;
    a.fface = st->fface;
    a.Qnew = st->Qnew;
    a.fparams = st->fparams;
    a.e0 = cs.de0;
    a.e1 = cs.de1;
    a.w = cs.dw;
    const size_t lds = corr_lds(c.order, c.nquant, io);
    const bool fpar = st->fparams != nullptr;
    const void* fn = p->prec == STP_FP64 ? corr_kernel<double>(c.order, c.physics, per_node, fpar)
                                         : corr_kernel<float>(c.order, c.physics, per_node, fpar);
    DeviceGuard g(p->device);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(corrector LDS)");
    }
    const unsigned grid = (unsigned)E;  // one workgroup per element: the hardware overlaps their phases
    void* args[] = {&a};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kCorrThreads), args, lds, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipLaunchKernel(corrector)");
    return STP_OK;
}

extern "C" stp_status stp_face_params(stp_plan_t p, int64_t nelem, const void* params, void* fparams, void* stream)
{
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    if (p->classes.size() != 1) return fail(STP_E_UNSUPPORTED, "stp_face_params takes a single-class plan");
    const ClassState& cs = p->classes[0];
    const stp_class& c = cs.cls;
    if (c.physics != STP_ELASTIC_CURV || (c.flags & STP_PARAM_PER_ELEMENT))
        return fail(STP_E_UNSUPPORTED, "stp_face_params is for curved curvilinear elements (STP_ELASTIC_CURV, "
                                       "parameters per node)");
    if (nelem < 0 || nelem > (int64_t)INT32_MAX) return fail(STP_E_INVAL, "nelem %lld", (long long)nelem);
    if (!params || !fparams) return fail(STP_E_INVAL, "params / fparams is NULL");
    const size_t io = p->prec == STP_FP64 ? 8 : 4;
    const int n = c.order + 1;
    {
        const uintptr_t i0 = (uintptr_t)params, i1 = i0 + (size_t)nelem * n * n * n * 12 * io;
        const uintptr_t o0 = (uintptr_t)fparams, o1 = o0 + (size_t)nelem * 6 * n * n * 12 * io;
        if (i0 < o1 && o0 < i1) return fail(STP_E_INVAL, "fparams overlaps params");
    }
    if (nelem == 0) return STP_OK;
    const int64_t items = nelem * 6 * n * n;
    const unsigned grid = (unsigned)std::min<int64_t>((items + kFaceThreads - 1) / kFaceThreads, 1 << 20);
    const void* fn = p->prec == STP_FP64 ? face_params_kernel<double>(c.order) : face_params_kernel<float>(c.order);
    DeviceGuard g(p->device);
    void* args[] = {&nelem, &params, &fparams, const_cast<void**>(&cs.de0), const_cast<void**>(&cs.de1)};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kFaceThreads), args, 0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipLaunchKernel(face parameters)");
    return STP_OK;
}
