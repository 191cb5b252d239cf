// Detection epilogue of the matrix-core kernels: the offers of one lane's
// four consecutive outputs, out of line.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ols_variants.hpp"

namespace fdas {

// The offers of a lane's four consecutive outputs o0 .. o0 + 3 of a segment
// (plane columns r0 .., powers v), out of line: the wave calls it together,
// and only when one of its lanes has a power at or above the threshold, so
// the registers the offers need are not held across a template loop (the
// caller's live registers are saved around the call, on that rare path).
typedef float cand_f4 __attribute__((ext_vector_type(4)));
static __device__ __attribute__((noinline)) void offer4(CandOut cd, cand_f4 v, bool active, int o0,
                                                        int half, int U, int64_t r0, int64_t nbins,
                                                        int row) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = o0 + i;
    const bool hit = active && o >= half && o < half + U && r0 + i < nbins && v[i] >= cd.thr;
    cand_offer(cd, hit, row, r0 + i, v[i]);
  }
}

}  // namespace fdas
