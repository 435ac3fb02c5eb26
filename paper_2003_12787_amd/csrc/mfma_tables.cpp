// mfma_tables.cpp -- host tables of the split-BF16 MFMA predictor kernels: the A operands of the derivative
// products and, for orders 8-9, the lane-to-line maps of the three lane roles.
#include "mfma_tables.hpp"

#include <algorithm>
#include <array>

#include "stp_mfma_hi_layout.hpp"

namespace stp {

std::vector<uint16_t> mfma_table_n8(const uint16_t* P0, const uint16_t* P1, const uint16_t* P2)
{
    // Lane l holds row i = l % 16 and the 8 K entries of lane group q = l / 16, which pair with the B entries of
    // the lanes of that group: the pieces of their nodes 2q and 2q+1 as (hi, mid) of 2q, (hi, mid) of 2q+1, lo of
    // 2q, lo of 2q+1, hi of 2q, hi of 2q+1. Row i belongs to output node 2 (i / 4) + i % 2, part (i / 2) % 2:
    //   part a: D0 on hi, mid and lo, D1 on the second copy of hi;   part b: D2 on hi, D1 on mid.
    // The two parts of a node land in the same lane and sum to D0 (hi + mid + lo) + D1 (hi + mid) + D2 hi.
    constexpr int n = 8;
    std::vector<uint16_t> tab(64 * 8);
    for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
            const int i = l % 16, q = l / 16;
            const int out = 2 * (i / 4) + i % 2, part = (i / 2) % 2;
            // entry e: node 2q + which, piece kind 0 hi, 1 mid, 2 lo, 3 second hi
            const int which = e < 4 ? e / 2 : e % 2;
            const int kind = e < 4 ? e % 2 : (e < 6 ? 2 : 3);
            const int src = out * n + 2 * q + which;
            uint16_t v = 0;
            if (part == 0) v = kind == 3 ? P1[src] : P0[src];
            else if (kind == 0) v = P2[src];
            else if (kind == 1) v = P1[src];
            tab[l * 8 + e] = v;
        }
    return tab;
}

namespace {

// Lines of one role for the W * 32 lane columns. Lane column c of every wave takes a line whose bank residue is
// c, one per wave, so that the 32 lines of a wave hit 32 distinct banks. Residues with more lines than waves
// overflow into free columns, each into the wave where its residue is least frequent (conflicts there). The
// columns still free repeat lines of other waves (bit kDupBit), chosen with residues the wave lacks.
void assign_lines(int n, int W, int (*res)(int n, int line), uint16_t* out)
{
    const int n2 = n * n;
    std::vector<std::vector<int>> bucket(32);
    for (int ln = 0; ln < n2; ++ln) bucket[res(n, ln)].push_back(ln);
    std::vector<int> slot(32 * W, -1), wave_of(n2, -1);
    std::vector<std::array<int, 32>> mult(W);
    for (auto& m : mult) m.fill(0);
    std::vector<int> overflow;
    for (int rho = 0; rho < 32; ++rho)
        for (size_t k = 0; k < bucket[rho].size(); ++k) {
            const int ln = bucket[rho][k];
            if ((int)k < W) {
                slot[32 * k + rho] = ln;
                wave_of[ln] = (int)k;
                mult[k][rho]++;
            } else {
                overflow.push_back(ln);
            }
        }
    for (int ln : overflow) {
        const int rho = res(n, ln);
        int best = -1;
        for (int s = 0; s < 32 * W; ++s) {
            if (slot[s] >= 0) continue;
            const int w = s / 32;
            if (best < 0 || mult[w][rho] < mult[best / 32][rho] ||
                (mult[w][rho] == mult[best / 32][rho] && w > best / 32))
                best = s;
        }
        slot[best] = ln;
        wave_of[ln] = best / 32;
        mult[best / 32][rho]++;
    }
    for (int s = 0; s < 32 * W; ++s) {
        const int w = s / 32;
        if (slot[s] >= 0) {
            out[s] = (uint16_t)slot[s];
            continue;
        }
        int best = -1;
        for (int ln = 0; ln < n2; ++ln) {
            if (wave_of[ln] == w) continue;
            if (best < 0 || mult[w][res(n, ln)] < mult[w][res(n, best)]) best = ln;
        }
        mult[w][res(n, best)]++;
        out[s] = (uint16_t)(best | mfma_hi::kDupBit);
    }
}

// Bank residues of a lane's node 0 in the three roles (word z * PZ + y * PY + x; the node's position along the
// line and the LDS region add the same constant to every lane of a pattern).
int res_owner(int n, int ln) { return ((ln / n) * mfma_hi::zstride(n) + (ln % n) * n) & 31; }     // (z, y)
int res_yrole(int n, int ln) { return ((ln / n) * mfma_hi::zstride(n) + ln % n) & 31; }           // (z, x)
int res_zrole(int n, int ln) { return ((ln / n) * n + ln % n) & 31; }                             // (y, x)

}  // namespace

std::vector<uint16_t> mfma_table_hi(int n, const uint16_t* P0, const uint16_t* P1, const uint16_t* P2)
{
    const int W = mfma_hi::waves(n);
    std::vector<uint16_t> tab(mfma_hi::table_entries(n), 0);
    const uint16_t* piece[3] = {P0, P1, P2};
    for (int l = 0; l < 64; ++l)
        for (int m = 0; m < 2; ++m)
            for (int j = 0; j < 8; ++j) {
                // A row i = l % 32: lane half h' = (i / 4) % 2 receives it as its accumulator row
                // r = 4 (i / 8) + i % 4, which is output node 5h' + r / 3 and piece r % 3 (r = 15 unused)
                const int i = l % 32, hq = (i / 4) % 2, r = 4 * (i / 8) + i % 4;
                // K entry j of lane half hb = l / 32 in product m: product 0 holds (hi, mid) of nodes
                // 5hb .. 5hb + 3, product 1 (hi, mid) of 5hb + 4 then the lo pieces of 5hb .. 5hb + 4 and a zero
                const int hb = l / 32;
                int node;
                if (m == 0) node = 5 * hb + j / 2;
                else node = j < 2 ? 5 * hb + 4 : (j < 7 ? 5 * hb + j - 2 : -1);
                // the pad node of n = 9 (5hq + 4 = 9) gets the rows of node 8, whose values it carries; its
                // own K entries get zero columns
                const int out = std::min(5 * hq + r / 3, n - 1);
                uint16_t v = 0;
                if (r < 15 && node >= 0 && node < n) v = piece[r % 3][out * n + node];
                tab[(l * 2 + m) * 8 + j] = v;
            }
    uint16_t* roles = tab.data() + mfma_hi::kTableA;
    assign_lines(n, W, res_owner, roles);
    assign_lines(n, W, res_yrole, roles + 32 * W);
    assign_lines(n, W, res_zrole, roles + 64 * W);
    // every role holds every line exactly once without the repeat bit (the kernel's outputs rely on it)
    for (int role = 0; role < 3; ++role) {
        std::vector<int> seen(n * n, 0);
        for (int s = 0; s < 32 * W; ++s) {
            const unsigned e = roles[32 * W * role + s];
            if ((e & 0x7fffu) >= (unsigned)(n * n)) return {};
            if (!(e & mfma_hi::kDupBit)) seen[e & 0x7fffu]++;
        }
        for (int v : seen)
            if (v != 1) return {};
    }
    return tab;
}

}  // namespace stp
