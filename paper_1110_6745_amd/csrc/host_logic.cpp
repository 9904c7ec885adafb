// Host-only logic of the okpz library (see host_logic.h).
#include "host_logic.h"

#include <cmath>
#include <cstring>

namespace okpz {
namespace host {

bool valid_slope_field(const uint8_t *h, int64_t Lx, int64_t Ly, std::string &why)
{
    for (int64_t i = 0; i < Lx * Ly; ++i)
        if (h[i] > 3) {
            why = "byte > 3";
            return false;
        }
    for (int64_t y = 0; y < Ly; ++y) {
        int64_t sum = 0;
        for (int64_t x = 0; x < Lx; ++x) sum += (h[y * Lx + x] & 1) ? 1 : -1;
        if (sum) {
            why = "sigma_x row sum not zero";
            return false;
        }
    }
    for (int64_t x = 0; x < Lx; ++x) {
        int64_t sum = 0;
        for (int64_t y = 0; y < Ly; ++y) sum += (h[y * Lx + x] & 2) ? 1 : -1;
        if (sum) {
            why = "sigma_y column sum not zero";
            return false;
        }
    }
    for (int64_t y = 0; y < Ly; ++y)
        for (int64_t x = 0; x < Lx; ++x) {
            const int64_t x1 = (x + 1) % Lx, y1 = (y + 1) % Ly;
            const int a = (h[y * Lx + x] & 1) ? 1 : -1;
            const int b = (h[y * Lx + x1] & 2) ? 1 : -1;
            const int c = (h[y1 * Lx + x] & 1) ? 1 : -1;
            const int d = (h[y * Lx + x] & 2) ? 1 : -1;
            if (a + b - c - d != 0) {
                why = "plaquette not closed";
                return false;
            }
        }
    return true;
}

bool valid_packed_planes(const uint32_t *planes, int64_t Lx, int64_t Ly, std::string &why)
{
    if (!side_ok(Lx) || !side_ok(Ly)) {
        why = "lattice side out of range";
        return false;
    }
    const int64_t W = Lx / 32;
    const uint32_t *px = planes, *py = planes + (size_t)Ly * W;
    // plaquettes: bits a = sx(x,y), b = sy(x+1,y), c = sx(x,y+1), d = sy(x,y);
    // a + b = c + d as bit counts <=> (a ^ b) == (c ^ d) and (a & b) == (c & d)
    for (int64_t y = 0; y < Ly; ++y) {
        const uint32_t *rx = px + (size_t)y * W, *ry = py + (size_t)y * W;
        const uint32_t *rx1 = px + (size_t)((y + 1) % Ly) * W;
        for (int64_t w = 0; w < W; ++w) {
            const uint32_t nxt = ry[(w + 1) % W];
            const uint32_t a = rx[w], d = ry[w], c = rx1[w];
            const uint32_t b = (d >> 1) | (nxt << 31);
            if (((a ^ b) != (c ^ d)) || ((a & b) != (c & d))) {
                why = "plaquette not closed";
                return false;
            }
        }
    }
    int64_t ones = 0;
    for (int64_t w = 0; w < W; ++w) ones += __builtin_popcount(px[w]);
    if (2 * ones != Lx) {
        why = "sigma_x row sum not zero";
        return false;
    }
    ones = 0;
    for (int64_t y = 0; y < Ly; ++y) ones += py[(size_t)y * W] & 1u;
    if (2 * ones != Ly) {
        why = "sigma_y column sum not zero";
        return false;
    }
    return true;
}

size_t packed_plane_bytes(int64_t Lx, int64_t Ly) { return 2 * (size_t)Ly * (size_t)(Lx / 32) * 4; }

bool parse_checkpoint(const void *buf, size_t bytes, CkptHeader *h, const uint32_t **planes,
                      std::string &why)
{
    if (bytes < sizeof(CkptHeader)) {
        why = "checkpoint truncated";
        return false;
    }
    std::memcpy(h, buf, sizeof(CkptHeader));
    if (std::memcmp(h->magic, "OKPZCKP1", 8) != 0 || h->version != 1) {
        why = "not an okpz checkpoint";
        return false;
    }
    if (!side_ok(h->Lx) || !side_ok(h->Ly) || h->ox < 0 || h->ox >= h->Lx || h->t < 0 ||
        h->t >= (int64_t(1) << 32) || h->cell_borders > 1 || h->copies < 0 || h->copies > 2 ||
        !(h->p >= 0.0 && h->p <= 1.0) || !(h->q >= 0.0 && h->q <= 1.0)) {
        why = "corrupt checkpoint header";
        return false;
    }
    if (!valid_h0(h->H0)) {
        why = "odd height at site (0,0)";
        return false;
    }
    const size_t pb = packed_plane_bytes(h->Lx, h->Ly);
    if (bytes - sizeof(CkptHeader) < pb) {
        why = "checkpoint truncated";
        return false;
    }
    // the planes follow the header; an unaligned buffer is checked on a copy
    const char *p = static_cast<const char *>(buf) + sizeof(CkptHeader);
    *planes = reinterpret_cast<const uint32_t *>(p);
    std::vector<uint32_t> copy;
    const uint32_t *view = *planes;
    if (reinterpret_cast<uintptr_t>(p) % alignof(uint32_t)) {
        copy.resize(pb / 4);
        std::memcpy(copy.data(), p, pb);
        view = copy.data();
    }
    std::string w;
    if (!valid_packed_planes(view, h->Lx, h->Ly, w)) {
        why = "checkpoint lattice is not a valid slope field: " + w;
        return false;
    }
    return true;
}

std::vector<int64_t> sample_times(int64_t t_max, double m)
{
    std::vector<int64_t> out;
    if (t_max <= 0 || !(m > 0.0)) return out;  // m <= 0 never reaches t_max
    double t = 0.0;
    while (true) {
        t = (t + 10.0) * std::exp(m);
        if (t > (double)t_max) break;
        const int64_t c = (int64_t)std::ceil(t);
        if (out.empty() || out.back() != c) out.push_back(c);
    }
    if (out.empty() || out.back() != t_max) out.push_back(t_max);
    return out;
}

}  // namespace host
}  // namespace okpz
