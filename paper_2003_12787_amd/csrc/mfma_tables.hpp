// mfma_tables.hpp -- host tables of the split-BF16 MFMA predictor kernels.
#pragma once
#include <cstdint>
#include <vector>

namespace stp {

// A operand of the order-7 kernel (v_mfma_f32_16x16x32_bf16), [64 lanes][8 BF16], from the three BF16 pieces
// P0, P1, P2 of the n x n derivative matrix (n = 8, row-major).
std::vector<uint16_t> mfma_table_n8(const uint16_t* P0, const uint16_t* P1, const uint16_t* P2);

// Table of the order 8-9 kernel (n = 9 or 10 nodes): A operands of the two chained v_mfma_f32_32x32x16_bf16
// and the lane-to-line maps of the three lane roles, in the layout of stp_mfma_hi_layout.hpp.
std::vector<uint16_t> mfma_table_hi(int n, const uint16_t* P0, const uint16_t* P1, const uint16_t* P2);

}  // namespace stp
