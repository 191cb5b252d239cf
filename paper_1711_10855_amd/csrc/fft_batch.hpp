// Compiled forms of the standalone batched FFT (fft_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_radix.hpp"

namespace fdas {

struct FftVariant {
  const char *name;
  int L;          // transform length
  int E;          // elements per thread
  int T;          // threads per transform
  int G;          // transforms per block
  hipError_t (*launch)(const void *in, void *out, int64_t batch, int dir, const c32 *tw,
                       hipStream_t s);
};

const FftVariant *fft_variants(int *count);

}  // namespace fdas
