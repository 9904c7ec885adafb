// Host-only logic of the okpz library: validation of slope fields and
// checkpoint headers, and the measurement times.  Plain C++ with no HIP
// types, so it is also built on its own (with sanitizers) for CPU checks.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace okpz {
namespace host {

// A canonical host lattice (one byte per site, bit 0 = [sigma_x = +1],
// bit 1 = [sigma_y = +1], row-major) is the slope field of a single-valued
// periodic height function iff every byte is < 4, every plaquette closes
// (sigma_x(x,y) + sigma_y(x+1,y) = sigma_x(x,y+1) + sigma_y(x,y)) and the
// sigma_x sums of the rows and sigma_y sums of the columns vanish.
bool valid_slope_field(const uint8_t *lat, int64_t Lx, int64_t Ly, std::string &why);

// The same test on two packed bit planes [plane][Ly][Lx/32] of uint32 (plane
// 0 = sigma_x bits, plane 1 = sigma_y bits; bit j of word w of row y is
// column 32w + j).  A cyclic rotation of the columns keeps a field valid,
// so stored (rotated) planes can be tested as they are.  With every
// plaquette closed, all row sums are equal and all column sums are equal,
// so row 0 and column 0 stand for the rest.
bool valid_packed_planes(const uint32_t *planes, int64_t Lx, int64_t Ly, std::string &why);

// Heights satisfy h(x,y) = x + y (mod 2) (flat start h = (x+y) mod 2, every
// move changes one height by 2), so the height of site (0,0) is even.
inline bool valid_h0(int64_t H0) { return (H0 & 1) == 0; }

// Lattice sides the library takes: multiples of 32 in [32, 2^20].
inline bool side_ok(int64_t L) { return L >= 32 && L <= (int64_t(1) << 20) && L % 32 == 0; }

// Checkpoint header (fixed layout, host byte order), followed by the packed
// bit planes of the current copy (2 * Ly * Lx/32 words).
struct CkptHeader {
    char magic[8];          // "OKPZCKP1"
    uint32_t version;       // 1
    uint32_t cell_borders;  // 0 dead, 1 delayed
    int64_t Lx, Ly;
    double p, q;
    uint64_t seed;
    int64_t t, H0;
    int32_t ox;      // stored column rotation of the planes
    int32_t copies;  // 1 for a lattice updated in place; 0 or 2 otherwise
};

size_t packed_plane_bytes(int64_t Lx, int64_t Ly);

// Parse and check a checkpoint buffer: header fields in range, size, even
// H0 and a valid slope field in the stored planes.  On success *h holds the
// header and *planes points at the stored planes inside buf (which need not
// be aligned: read them with memcpy or copy them as bytes).
bool parse_checkpoint(const void *buf, size_t bytes, CkptHeader *h, const uint32_t **planes,
                      std::string &why);

// Measurement times of Sec. III: t_{i+1} = (t_i + 10) e^m from t_0 = 0, each
// rounded up to a whole MCS, repeats dropped, and t_max itself last (empty
// for t_max <= 0 or m <= 0).  The one implementation the library, its binding and the
// benchmark use.
std::vector<int64_t> sample_times(int64_t t_max, double m);

}  // namespace host
}  // namespace okpz
