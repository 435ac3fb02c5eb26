// stp_mfma_hi_layout.hpp -- layout constants of the order 8-9 MFMA kernel shared by the kernel and the host code
// that builds its tables.
#pragma once

namespace stp {
namespace mfma_hi {

// A lane takes five consecutive nodes 5h .. 5h + 4 of a line (h = lane / 32); n = 9 pads the upper half.
constexpr int kNodesPerLane = 5;

// Waves per element: one line per lane column, 32 columns per wave.
constexpr int waves(int n) { return (n * n + 31) / 32; }

// LDS tile of one quantity: node (z, y, x) at word z * zstride(n) + y * n + x. The word address modulo 32 is
// the bank. With the lane-to-line maps of the three roles (built on the host so that the 32 lines of a wave
// fall in distinct banks where the residue counts allow it), the z-stride 103 makes every access pattern of
// n = 10 conflict-free. n = 9 stays dense (729 words) so that three elements share a CU; its y-role pattern
// keeps a few 2- and 3-way conflicts.
constexpr int zstride(int n) { return n == 10 ? 103 : n * n; }
constexpr int slot_words(int n) { return n * zstride(n); }

// Table of the kernel (16-bit entries): the A operands [64 lanes][2 products][8 BF16], then for each role
// (owner x-lines, y-role lines, z-role lines) the line of every lane column [waves][32], with bit 15 set where
// the lane repeats a line that another lane holds (the padding columns of the last wave).
constexpr int kTableA = 64 * 2 * 8;
constexpr int table_entries(int n) { return kTableA + 3 * 32 * waves(n); }
constexpr unsigned kDupBit = 0x8000u;

}  // namespace mfma_hi
}  // namespace stp
