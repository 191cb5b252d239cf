// Allocation-free batched path: sizes of the device scratch array and the
// descriptor upload that fills it (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "fdas.h"
#include "ols_variants.hpp"

namespace fdas {

constexpr int kNoAllocMaxSeries = FDAS_NOALLOC_MAX_SERIES;
// descriptor table, then the 8-byte work counter of the persistent form
constexpr size_t kNoAllocDescBytes = (size_t)kNoAllocMaxSeries * sizeof(SeriesDesc);
constexpr size_t kNoAllocScratchBytes = kNoAllocDescBytes + 256;

// Descriptors travel to the device as kernel arguments (copied by the
// runtime at launch), kDescChunk per launch, so no host buffer has to outlive
// the call and nothing is allocated.
constexpr int kDescChunk = 64;
struct DescChunk {
  int n;      // descriptors in this chunk
  int first;  // index of d[0] in the table
  SeriesDesc d[kDescChunk];
};
static_assert(sizeof(DescChunk) <= 4000, "a chunk fits the kernel-argument limit");
static_assert(sizeof(SeriesDesc) == 56 && kNoAllocScratchBytes == FDAS_NOALLOC_SCRATCH_BYTES,
              "the scratch size stated in fdas.h");

// Device address of the scratch array on `device` (which must be current),
// looked up once per device.
int noalloc_scratch(int device, void **out);
hipError_t launch_desc_upload(const DescChunk &c, SeriesDesc *dst, hipStream_t s);

}  // namespace fdas
