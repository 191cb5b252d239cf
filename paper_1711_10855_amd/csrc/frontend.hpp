// Device front end (frontend.hip): series -> normalised spectrum.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_batch.hpp"
#include "fft_radix.hpp"

namespace fdas {

// How an M-point transform is split: one transform of length N1 (N2 == 1),
// or the four-step N1 x N2 with both lengths compiled.
struct FrontendGeom {
  int64_t M;
  int N1, N2;
  const FftVariant *f1, *f2;
  const c32 *tw1, *tw2;  // twiddle tables of lengths N1 and N2
};

size_t frontend_sel_bytes();
hipError_t launch_frontend(const FrontendGeom &g, const float *series, c32 *spectrum, c32 *work,
                           float *pw, void *sel, float *stats, hipStream_t s);

}  // namespace fdas
