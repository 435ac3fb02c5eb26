// basis.hpp -- host-side 1D basis tables of the predictor (see basis.cpp).
#pragma once
#include <cstdint>

namespace stp {

constexpr int kMaxOrder = 9;              // N = 1..9
constexpr int kMaxNodes = kMaxOrder + 1;  // n = N + 1

// n Gauss-Legendre nodes on [0,1], ascending, and weights summing to 1.
void gauss_legendre_01(int n, double* xi, double* w);
// n >= 2 Gauss-Lobatto nodes on [0,1] (0 and 1 included), ascending, and weights summing to 1.
void gauss_lobatto_01(int n, double* xi, double* w);
// Lagrange basis values l_j(x), j = 0..n-1.
void lagrange_values(int n, const double* xi, double x, double* l);
// D[i*n + j] = l_j'(xi_i).
void derivative_matrix(int n, const double* xi, double* D);
// FP32 copy of D with zero row sums in FP32.
void derivative_matrix_f32(int n, const double* D, float* Df);
// Round-to-nearest-even BF16 and the hi/lo split x ~ hi + lo.
// x = p0 + p1 + p2 exactly, each a BF16 bit pattern (truncation split; finite x of normal range).
void split3_bf16(int count, const float* x, uint16_t* p0, uint16_t* p1, uint16_t* p2);

}  // namespace stp
