// Sanitizer driver for the library's host-only logic
// (paper_1110_6745_amd/csrc/host_logic.cpp), built with it under
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py:
// slope-field validation of canonical bytes and of packed (rotated) bit
// planes, checkpoint parsing, and the measurement times of Sec. III.
// Prints "host logic ok".
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "host_logic.h"

using namespace okpz::host;

static int fails = 0;
#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                               \
        }                                                                          \
    } while (0)

// A valid field: h(x,y) = a(x) + b(y) with a, b closed walks of +-1 steps
// (a(x) = x, b(y) = y mod 2), then some local extrema moved by +-2.
static std::vector<uint8_t> valid_field(int64_t Lx, int64_t Ly, uint32_t seed)
{
    std::mt19937 g(seed);
    auto walk = [&](int64_t L) {
        std::vector<int> st(L);
        for (int64_t i = 0; i < L; ++i) st[i] = (i < L / 2) ? 1 : -1;
        std::shuffle(st.begin(), st.end(), g);
        return st;
    };
    const std::vector<int> sa = walk(Lx), sb = walk(Ly);
    std::vector<int64_t> h(Lx * Ly);
    int64_t ay = 0;
    for (int64_t y = 0; y < Ly; ++y) {
        int64_t ax = 0;
        for (int64_t x = 0; x < Lx; ++x) {
            h[y * Lx + x] = ax + ay;
            ax += sa[x];
        }
        ay += sb[y];
    }
    auto H = [&](int64_t x, int64_t y) -> int64_t & { return h[((y + Ly) % Ly) * Lx + (x + Lx) % Lx]; };
    for (int k = 0; k < 4 * Lx * Ly; ++k) {
        const int64_t x = g() % Lx, y = g() % Ly;
        const int64_t c = H(x, y);
        const bool mn = H(x - 1, y) > c && H(x + 1, y) > c && H(x, y - 1) > c && H(x, y + 1) > c;
        const bool mx = H(x - 1, y) < c && H(x + 1, y) < c && H(x, y - 1) < c && H(x, y + 1) < c;
        if (mn) H(x, y) += 2;
        else if (mx) H(x, y) -= 2;
    }
    std::vector<uint8_t> lat(Lx * Ly);
    for (int64_t y = 0; y < Ly; ++y)
        for (int64_t x = 0; x < Lx; ++x)
            lat[y * Lx + x] = (uint8_t)((H(x + 1, y) > H(x, y) ? 1 : 0) | (H(x, y + 1) > H(x, y) ? 2 : 0));
    return lat;
}

static std::vector<uint32_t> pack(const std::vector<uint8_t> &lat, int64_t Lx, int64_t Ly, int64_t ox)
{
    const int64_t W = Lx / 32;
    std::vector<uint32_t> p(2 * Ly * W, 0u);
    for (int64_t y = 0; y < Ly; ++y)
        for (int64_t x = 0; x < Lx; ++x) {
            const int64_t c = ((x - ox) % Lx + Lx) % Lx;  // stored column
            const uint8_t b = lat[y * Lx + x];
            if (b & 1) p[y * W + c / 32] |= 1u << (c % 32);
            if (b & 2) p[(Ly + y) * W + c / 32] |= 1u << (c % 32);
        }
    return p;
}

static std::vector<char> checkpoint(const std::vector<uint32_t> &planes, int64_t Lx, int64_t Ly,
                                    int64_t H0, int32_t ox, size_t lead = 0)
{
    CkptHeader h{};
    std::memcpy(h.magic, "OKPZCKP1", 8);
    h.version = 1;
    h.Lx = Lx;
    h.Ly = Ly;
    h.p = 1.0;
    h.t = 3;
    h.H0 = H0;
    h.ox = ox;
    h.copies = 2;
    std::vector<char> buf(lead + sizeof h + planes.size() * 4);
    std::memcpy(buf.data() + lead, &h, sizeof h);
    std::memcpy(buf.data() + lead + sizeof h, planes.data(), planes.size() * 4);
    return buf;
}

int main()
{
    std::string why;
    const int64_t shapes[][2] = {{32, 32}, {64, 32}, {96, 160}, {256, 64}};
    for (auto &sh : shapes) {
        const int64_t Lx = sh[0], Ly = sh[1];
        for (uint32_t seed = 1; seed <= 3; ++seed) {
            std::vector<uint8_t> lat = valid_field(Lx, Ly, seed);
            CHECK(valid_slope_field(lat.data(), Lx, Ly, why));
            for (int64_t ox : {int64_t(0), int64_t(5), Lx - 1}) {
                std::vector<uint32_t> pl = pack(lat, Lx, Ly, ox);
                CHECK(valid_packed_planes(pl.data(), Lx, Ly, why));
                // one flipped bit anywhere: both validators reject
                std::mt19937 g(seed);
                for (int k = 0; k < 20; ++k) {
                    const size_t w = g() % pl.size();
                    const uint32_t bit = 1u << (g() % 32);
                    pl[w] ^= bit;
                    CHECK(!valid_packed_planes(pl.data(), Lx, Ly, why));
                    pl[w] ^= bit;
                }
                // checkpoints: good, odd H0, truncated, bad fields, unaligned
                const CkptHeader *hp = nullptr;
                CkptHeader h;
                const uint32_t *planes = nullptr;
                std::vector<char> ck = checkpoint(pl, Lx, Ly, 4, (int32_t)ox);
                CHECK(parse_checkpoint(ck.data(), ck.size(), &h, &planes, why));
                CHECK(planes != nullptr && h.Lx == Lx && h.H0 == 4);
                (void)hp;
                CHECK(!parse_checkpoint(ck.data(), ck.size() - 1, &h, &planes, why));
                CHECK(!parse_checkpoint(ck.data(), 10, &h, &planes, why));
                std::vector<char> odd = checkpoint(pl, Lx, Ly, -3, (int32_t)ox);
                CHECK(!parse_checkpoint(odd.data(), odd.size(), &h, &planes, why));
                std::vector<char> una = checkpoint(pl, Lx, Ly, 0, (int32_t)ox, 1);
                CHECK(parse_checkpoint(una.data() + 1, una.size() - 1, &h, &planes, why));
                std::vector<char> badox = checkpoint(pl, Lx, Ly, 0, (int32_t)Lx);
                CHECK(!parse_checkpoint(badox.data(), badox.size(), &h, &planes, why));
            }
            // a byte above 3 and a flipped canonical bit
            lat[7] |= 4;
            CHECK(!valid_slope_field(lat.data(), Lx, Ly, why));
            lat[7] &= 3;
            lat[Lx + 3] ^= 2;
            CHECK(!valid_slope_field(lat.data(), Lx, Ly, why));
        }
    }
    CHECK(!valid_packed_planes(nullptr, 33, 32, why));

    // measurement times: t_{i+1} = (t_i + 10) e^m, rounded up (by hand for m = 0.01)
    const std::vector<int64_t> t = sample_times(52, 0.01);
    CHECK((t == std::vector<int64_t>{11, 21, 31, 42, 52}));
    CHECK(sample_times(0, 0.01).empty());
    CHECK(sample_times(100, 0.0).empty());
    CHECK(sample_times(100, -1.0).empty());
    const std::vector<int64_t> big = sample_times(1310720, 0.001);
    CHECK(big.back() == 1310720);
    for (size_t i = 1; i < big.size(); ++i) CHECK(big[i] > big[i - 1]);

    if (fails) return 1;
    std::printf("host logic ok\n");
    return 0;
}
