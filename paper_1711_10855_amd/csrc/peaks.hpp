// Peak picking over the candidates of the detection epilogue (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ols_variants.hpp"

namespace fdas {

// Workspace of fdas_convolve_peaks for `cand_capacity` candidates: the
// candidate list (16 B each), then a hash table of cells (8-byte keys, then
// 4-byte candidate indices) with at least twice as many slots.
int64_t peaks_table_slots(int64_t cand_capacity);
size_t peaks_workspace_bytes(int64_t cand_capacity);

// counts[0] (candidates) and counts[1] (peaks) set to zero on the stream.
hipError_t launch_peaks_reset(unsigned long long *counts, hipStream_t s);
// Clear the table, insert the min(counts[0], cand_capacity) listed
// candidates, and append every one that outranks its eight grid neighbours to
// `peaks` (counted on counts[1]; stored while the slot is below peak_cap).
hipError_t launch_peaks(const Cand *cands, int64_t cand_capacity, void *table,
                        unsigned long long *counts, int interbin, Cand *peaks, int64_t peak_cap,
                        hipStream_t s);

}  // namespace fdas
