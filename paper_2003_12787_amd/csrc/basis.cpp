// basis.cpp -- host-side constant tables of the predictor, built once per plan in FP64/long double:
// Gauss-Legendre nodes on [0,1] (Sec. II-A nodal Lagrange basis), the derivative matrix D[i][j] = l_j'(xi_i)
// (Sec. II-A "discrete derivative operator"), the face vectors l_j(0), l_j(1) (Sec. II-B face projection)
// and the three-piece BF16 split of D used by the split-BF16x3 contraction.
//
// The nodes are the eigenvalues of the symmetric Jacobi matrix of the Legendre recurrence, isolated by
// Sturm-sequence bisection and polished by Newton steps on the recurrence.
#include "basis.hpp"

#include <cmath>
#include <cstdint>
#include <cstring>

namespace stp {

namespace {

// Number of eigenvalues of the n x n Legendre Jacobi matrix (zero diagonal, off-diagonal
// b_k = k / sqrt(4k^2 - 1)) that are smaller than x (Sturm sequence count).
int sturm_count(int n, long double x)
{
    int count = 0;
    long double q = -x;  // first pivot: a_0 - x
    if (q < 0) ++count;
    for (int k = 1; k < n; ++k) {
        long double b2 = (long double)k * k / (4.0L * k * k - 1.0L);
        if (q == 0) q = 1e-30L;
        q = -x - b2 / q;
        if (q < 0) ++count;
    }
    return count;
}

// P_n(x) and P_n'(x)
void legendre(int n, long double x, long double& p, long double& dp)
{
    long double a = 1.0L, b = x;
    if (n == 0) { p = 1; dp = 0; return; }
    for (int k = 2; k <= n; ++k) {
        long double c = ((2.0L * k - 1.0L) * x * b - (k - 1.0L) * a) / k;
        a = b;
        b = c;
    }
    p = b;
    dp = n * (a - x * b) / (1.0L - x * x);
}

}  // namespace

void gauss_legendre_01(int n, double* xi, double* w)
{
    for (int i = 0; i < n; ++i) {
        // i-th smallest eigenvalue of the Jacobi matrix in (-1, 1)
        long double lo = -1.0L, hi = 1.0L;
        for (int it = 0; it < 80; ++it) {
            long double mid = 0.5L * (lo + hi);
            if (sturm_count(n, mid) > i) hi = mid; else lo = mid;
        }
        long double x = 0.5L * (lo + hi), p, dp;
        for (int it = 0; it < 3; ++it) {
            legendre(n, x, p, dp);
            x -= p / dp;
        }
        legendre(n, x, p, dp);
        xi[i] = (double)(0.5L * (1.0L + x));
        w[i] = (double)(1.0L / ((1.0L - x * x) * dp * dp));  // 2/((1-x^2)P'^2) on [-1,1], halved
    }
}

void gauss_lobatto_01(int n, double* xi, double* w)
{
    // The n = N + 1 Lobatto points of [-1, 1] are the zeros of P_{N+1} - P_{N-1} (which is (2N+1)/(N(N+1))
    // times -(1 - x^2) P_N'), with derivative (2N+1) P_N. Newton from the Chebyshev-Lobatto points; the end
    // points are exact. Weights 2 / (N (N+1) P_N(x)^2) on [-1, 1], halved for [0, 1].
    const int N = n - 1;
    auto P = [](int k, long double x, long double* out) {  // out[0..k] = P_0..P_k
        out[0] = 1.0L;
        if (k > 0) out[1] = x;
        for (int j = 2; j <= k; ++j) out[j] = ((2.0L * j - 1.0L) * x * out[j - 1] - (j - 1.0L) * out[j - 2]) / j;
    };
    const long double pi = 3.141592653589793238462643383279502884L;
    long double v[kMaxNodes + 2];
    for (int i = 0; i <= N; ++i) {
        long double x = i == 0 ? -1.0L : (i == N ? 1.0L : -cosl(pi * i / N));
        if (i > 0 && i < N)
            for (int it = 0; it < 60; ++it) {
                P(N + 1, x, v);
                const long double dx = (v[N + 1] - v[N - 1]) / ((2.0L * N + 1.0L) * v[N]);
                x -= dx;
                if (fabsl(dx) < 1e-20L) break;
            }
        P(N, x, v);
        xi[i] = (double)(0.5L * (1.0L + x));
        w[i] = (double)(1.0L / ((long double)N * (N + 1) * v[N] * v[N]));
    }
}

void lagrange_values(int n, const double* xi, double x, double* l)
{
    for (int j = 0; j < n; ++j) {
        long double num = 1.0L, den = 1.0L;
        for (int k = 0; k < n; ++k) {
            if (k == j) continue;
            num *= (long double)x - xi[k];
            den *= (long double)xi[j] - xi[k];
        }
        l[j] = (double)(num / den);
    }
}

void derivative_matrix(int n, const double* xi, double* D)
{
    // l_j'(xi_i) = w_i / (w_j (xi_i - xi_j)) with w_i = prod_{k != i} (xi_i - xi_k)   (i != j)
    long double pw[kMaxNodes];
    for (int i = 0; i < n; ++i) {
        pw[i] = 1.0L;
        for (int k = 0; k < n; ++k)
            if (k != i) pw[i] *= (long double)xi[i] - xi[k];
    }
    for (int i = 0; i < n; ++i) {
        long double diag = 0.0L;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            D[i * n + j] = (double)(pw[i] / (pw[j] * ((long double)xi[i] - xi[j])));
            diag += 1.0L / ((long double)xi[i] - xi[j]);  // l_i'(xi_i) = sum_{k != i} 1/(xi_i - xi_k)
        }
        D[i * n + i] = (double)diag;
    }
}

void derivative_matrix_f32(int n, const double* D, float* Df)
{
    // Off-diagonal entries rounded to FP32; the diagonal is chosen so that every row sums to zero when
    // accumulated in FP32 order, so constants differentiate to (almost exactly) zero in FP32.
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            Df[i * n + j] = (float)D[i * n + j];
            s += (double)Df[i * n + j];
        }
        Df[i * n + i] = (float)(-s);
    }
}

void split3_bf16(int count, const float* x, uint16_t* p0, uint16_t* p1, uint16_t* p2)
{
    // Truncation split: p0 keeps the sign, the exponent and the 7 leading fraction bits of x; the remainder
    // x - p0 is exact in FP32 and has at most 16 significant bits, of which p1 keeps the leading 8; the rest
    // (at most 8 bits) is p2 exactly. So x = p0 + p1 + p2 with no rounding (for finite x of normal range).
    for (int i = 0; i < count; ++i) {
        uint32_t u;
        std::memcpy(&u, &x[i], 4);
        float h, r, m, l;
        const uint32_t hu = u & 0xffff0000u;
        std::memcpy(&h, &hu, 4);
        r = x[i] - h;
        uint32_t ru;
        std::memcpy(&ru, &r, 4);
        const uint32_t mu = ru & 0xffff0000u;
        std::memcpy(&m, &mu, 4);
        l = r - m;
        uint32_t lu;
        std::memcpy(&lu, &l, 4);
        p0[i] = (uint16_t)(hu >> 16);
        p1[i] = (uint16_t)(mu >> 16);
        p2[i] = (uint16_t)(lu >> 16);
    }
}

}  // namespace stp
