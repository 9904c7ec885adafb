// Internal declarations of the spectrum pass (not part of the C ABI).
#pragma once

#include "okpz_internal.h"

namespace okpz {

// Power spectrum along the lattice axes: scratch layout
// (byte offsets into one device allocation of `bytes`) and launch.  Needs the
// rows of launch_width_rows; leaves S along x (Lx/2+1 doubles) followed by S
// along y (Ly/2+1 doubles) at off_spec.
struct PsdPlan {
    int32_t R, nch;  // rows per column-count chunk, number of chunks
    size_t off_cnt, off_zx, off_zy, off_spec, off_blk, off_conv, bytes;
    int64_t conv_len;  // Bluestein transform length (0: both sides powers of two)
};
PsdPlan psd_plan(int64_t Lx, int64_t Ly);
// The same with taller column-count chunks, as few as needed to bring the
// scratch down to max_bytes if possible (check .bytes against the cap).
PsdPlan psd_plan_capped(int64_t Lx, int64_t Ly, size_t max_bytes);
hipError_t launch_psd(const LatticeView &v, const PsdPlan &p, const int64_t *rows, void *scratch,
                      hipStream_t st);

}  // namespace okpz
