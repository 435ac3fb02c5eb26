// Host check of the MFMA kernels' tables (mfma_tables.cpp), built with g++ and no GPU.
//
// The A tables are multiplied, in double precision, with B operands laid out as the kernels lay them out (per
// lane: its nodes' (hi | mid) words, lo pairs, hi pairs), using the lane mappings of the products the kernels
// issue: v_mfma_f32_16x16x32_bf16 (lane l holds A row l % 16 and K entries 8 (l / 16) .. + 7, B column l % 16
// and the same K entries, accumulator rows 4 (l / 16) .. + 3 of column l % 16) and v_mfma_f32_32x32x16_bf16
// (A row l % 32 and K entries 8 (l / 32) .. + 7, B column l % 32, accumulator row 8 (r / 4) + 4 (l / 32) + r % 4
// in register r). The owner's sums of its rows must equal the products the kernels document, exactly in double.
// The lane-to-line maps of the order 8-9 kernel must cover every line once per role, and the banks of each
// wave's accesses are counted.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "mfma_tables.hpp"
#include "stp_mfma_hi_layout.hpp"

static int failures = 0;
#define CHECK(c, ...)                          \
    do {                                       \
        if (!(c)) {                            \
            ++failures;                        \
            std::printf("FAIL: " __VA_ARGS__); \
            std::printf("\n");                 \
        }                                      \
    } while (0)

static float f32(uint32_t b) { float f; std::memcpy(&f, &b, 4); return f; }
static uint32_t bits(float f) { uint32_t b; std::memcpy(&b, &f, 4); return b; }
static double bf(uint16_t h) { return (double)f32((uint32_t)h << 16); }

// truncation split x = p0 + p1 + p2 (the kernels' split of u; the same split gives D's pieces)
static void split3(float x, uint16_t& p0, uint16_t& p1, uint16_t& p2)
{
    const uint32_t xb = bits(x);
    p0 = (uint16_t)(xb >> 16);
    const float r = x - f32(xb & 0xffff0000u);
    p1 = (uint16_t)(bits(r) >> 16);
    const float l = r - f32(bits(r) & 0xffff0000u);
    p2 = (uint16_t)(bits(l) >> 16);
}

static std::vector<float> random_D(int n, std::mt19937& g)
{
    std::normal_distribution<float> N01(0.f, 1.f);
    std::vector<float> D(n * n);
    for (float& v : D) v = 20.f * N01(g);
    return D;
}

static void pieces(const std::vector<float>& D, std::vector<uint16_t> (&P)[3])
{
    for (auto& p : P) p.assign(D.size(), 0);
    for (size_t i = 0; i < D.size(); ++i) split3(D[i], P[0][i], P[1][i], P[2][i]);
}

// order 7 (n = 8): one 16x16x32 product per 16 lines
static void check_n8(std::mt19937& g)
{
    const int n = 8;
    const std::vector<float> D = random_D(n, g);
    std::vector<uint16_t> P[3];
    pieces(D, P);
    const std::vector<uint16_t> tab = stp::mfma_table_n8(P[0].data(), P[1].data(), P[2].data());
    CHECK(tab.size() == 64 * 8, "n8 table size %zu", tab.size());
    std::normal_distribution<float> N01(0.f, 1.f);
    for (int trial = 0; trial < 20; ++trial) {
        float u[16][8];  // 16 lines (columns) x 8 nodes
        uint16_t hi[16][8], mid[16][8], lo[16][8];
        for (int c = 0; c < 16; ++c)
            for (int k = 0; k < n; ++k) {
                u[c][k] = N01(g) * (trial % 2 ? 1e3f : 1.f);
                split3(u[c][k], hi[c][k], mid[c][k], lo[c][k]);
            }
        // B[k][c]: lane (q, c) supplies K entries 8q .. 8q + 7 = hi, mid of 2q; hi, mid of 2q+1; lo of 2q, 2q+1;
        // hi of 2q, 2q+1
        double B[32][16], A[16][32];
        for (int c = 0; c < 16; ++c)
            for (int q = 0; q < 4; ++q) {
                const int a = 2 * q, b = 2 * q + 1;
                const uint16_t e[8] = {hi[c][a], mid[c][a], hi[c][b], mid[c][b], lo[c][a], lo[c][b], hi[c][a], hi[c][b]};
                for (int j = 0; j < 8; ++j) B[8 * q + j][c] = bf(e[j]);
            }
        for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 8; ++j) A[l % 16][8 * (l / 16) + j] = bf(tab[l * 8 + j]);
        for (int c = 0; c < 16; ++c)
            for (int qq = 0; qq < 4; ++qq) {
                double acc[4];
                for (int t = 0; t < 4; ++t) {
                    double s = 0;
                    for (int k = 0; k < 32; ++k) s += A[4 * qq + t][k] * B[k][c];
                    acc[t] = s;
                }
                for (int t = 0; t < 2; ++t) {
                    const int j = 2 * qq + t;  // the lane's node: part a in row t, part b in row t + 2
                    const double got = acc[t] + acc[t + 2];
                    double want = 0;
                    for (int k = 0; k < n; ++k) {
                        const double d0 = bf(P[0][j * n + k]), d1 = bf(P[1][j * n + k]), d2 = bf(P[2][j * n + k]);
                        want += d0 * (bf(hi[c][k]) + bf(mid[c][k]) + bf(lo[c][k])) + d1 * (bf(hi[c][k]) + bf(mid[c][k])) +
                                d2 * bf(hi[c][k]);
                    }
                    CHECK(std::fabs(got - want) <= 1e-9 * (1 + std::fabs(want)), "n8 trial %d col %d node %d: %g vs %g",
                          trial, c, j, got, want);
                }
            }
    }
}

// orders 8-9 (n = 9, 10): two chained 32x32x16 products per 32 lines; all nine products D_P u_Q
static void check_hi(int n, std::mt19937& g)
{
    const std::vector<float> D = random_D(n, g);
    std::vector<uint16_t> P[3];
    pieces(D, P);
    const std::vector<uint16_t> tab = stp::mfma_table_hi(n, P[0].data(), P[1].data(), P[2].data());
    CHECK((int)tab.size() == stp::mfma_hi::table_entries(n), "n%d table size %zu", n, tab.size());
    if ((int)tab.size() != stp::mfma_hi::table_entries(n)) return;
    std::normal_distribution<float> N01(0.f, 1.f);
    double A[2][32][16];
    for (int l = 0; l < 64; ++l)
        for (int m = 0; m < 2; ++m)
            for (int j = 0; j < 8; ++j) A[m][l % 32][8 * (l / 32) + j] = bf(tab[(l * 2 + m) * 8 + j]);
    for (int trial = 0; trial < 10; ++trial) {
        // 32 lines; node 9 of n = 9 is the stand-in, a copy of node 8
        float u[32][10];
        uint16_t hi[32][10], mid[32][10], lo[32][10];
        for (int c = 0; c < 32; ++c) {
            for (int k = 0; k < n; ++k) u[c][k] = N01(g) * (trial % 2 ? 1e3f : 1.f);
            if (n == 9) u[c][9] = u[c][8];
            for (int k = 0; k < 10; ++k) split3(u[c][k], hi[c][k], mid[c][k], lo[c][k]);
        }
        double B[2][16][32];
        for (int c = 0; c < 32; ++c)
            for (int h = 0; h < 2; ++h) {
                const int k0 = 5 * h;
                const uint16_t e0[8] = {hi[c][k0], mid[c][k0], hi[c][k0 + 1], mid[c][k0 + 1],
                                        hi[c][k0 + 2], mid[c][k0 + 2], hi[c][k0 + 3], mid[c][k0 + 3]};
                const uint16_t e1[8] = {hi[c][k0 + 4], mid[c][k0 + 4], lo[c][k0], lo[c][k0 + 1],
                                        lo[c][k0 + 2], lo[c][k0 + 3], lo[c][k0 + 4], 0};
                for (int j = 0; j < 8; ++j) {
                    B[0][8 * h + j][c] = bf(e0[j]);
                    B[1][8 * h + j][c] = bf(e1[j]);
                }
            }
        for (int c = 0; c < 32; ++c)
            for (int hq = 0; hq < 2; ++hq) {
                double reg[16];
                for (int r = 0; r < 16; ++r) {
                    const int row = 8 * (r / 4) + 4 * hq + r % 4;
                    double s = 0;
                    for (int m = 0; m < 2; ++m)
                        for (int k = 0; k < 16; ++k) s += A[m][row][k] * B[m][k][c];
                    reg[r] = s;
                }
                for (int t = 0; t < 5; ++t) {
                    const int j = 5 * hq + t;
                    const int jr = j < n ? j : n - 1;  // the stand-in's rows are node n - 1's
                    const double got = reg[3 * t] + reg[3 * t + 1] + reg[3 * t + 2];
                    double want = 0;
                    for (int k = 0; k < n; ++k) {
                        const double d = bf(P[0][jr * n + k]) + bf(P[1][jr * n + k]) + bf(P[2][jr * n + k]);
                        want += d * (bf(hi[c][k]) + bf(mid[c][k]) + bf(lo[c][k]));
                    }
                    CHECK(std::fabs(got - want) <= 1e-9 * (1 + std::fabs(want)), "n%d trial %d col %d node %d: %g vs %g",
                          n, trial, c, j, got, want);
                    CHECK(reg[15] == 0.0, "n%d unused row is not zero", n);
                }
            }
    }
    // lane-to-line maps: every line once per role without the repeat bit; bank multiplicity per wave
    const int W = stp::mfma_hi::waves(n), zs = stp::mfma_hi::zstride(n);
    const uint16_t* roles = tab.data() + stp::mfma_hi::kTableA;
    int worst[3] = {0, 0, 0};
    for (int role = 0; role < 3; ++role) {
        std::vector<int> seen(n * n, 0);
        for (int w = 0; w < W; ++w) {
            int mult[32] = {};
            for (int c = 0; c < 32; ++c) {
                const unsigned e = roles[32 * W * role + 32 * w + c];
                const int line = (int)(e & 0x7fffu), a = line / n, b = line % n;
                CHECK(line < n * n, "n%d role %d line %d out of range", n, role, line);
                if (!(e & stp::mfma_hi::kDupBit)) seen[line]++;
                const int word = role == 0 ? a * zs + b * n : (role == 1 ? a * zs + b : a * n + b);
                mult[word & 31]++;
            }
            for (int k = 0; k < 32; ++k) worst[role] = worst[role] > mult[k] ? worst[role] : mult[k];
        }
        for (int v : seen) CHECK(v == 1, "n%d role %d: a line held %d times", n, role, v);
    }
    std::printf("n=%d: worst bank multiplicity per wave: owner %d, y-role %d, z-role %d\n", n, worst[0], worst[1],
                worst[2]);
    if (n == 10) CHECK(worst[0] == 1 && worst[1] == 1 && worst[2] == 1, "n=10 patterns are not conflict-free");
    if (n == 9) CHECK(worst[0] == 1 && worst[2] == 1 && worst[1] <= 3, "n=9 bank multiplicities");
}

int main()
{
    std::mt19937 g(2003);
    check_n8(g);
    check_hi(9, g);
    check_hi(10, g);
    std::printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
