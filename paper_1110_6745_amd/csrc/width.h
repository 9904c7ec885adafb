// Internal declarations of the width pass (not part of the C ABI).
#pragma once

#include "okpz_internal.h"

namespace okpz {

// Width: per-row partial sums into `rows` scratch (width_scratch_words(Ly)
// int64: 3 Ly row values, then per-block records), then a two-level combine
// into out[0..3] = {S1' lo, S1' hi, S2' lo, S2' hi} (128-bit two's
// complement halves of the sums relative to H0).
hipError_t launch_width(const LatticeView &v, int64_t *rows, int64_t *out, hipStream_t st);

size_t width_scratch_words(int64_t Ly);
// The per-row pass alone (rows[0..3 Ly) as above, no combine).
hipError_t launch_width_rows(const LatticeView &v, int64_t *rows, hipStream_t st);

}  // namespace okpz
