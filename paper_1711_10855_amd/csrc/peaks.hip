// Peak picking over the thresholded plane: the candidate search that
// follows the plane in the FDAS pipeline (Section 3 names it; the rule is a
// reading, stated in fdas.h). The correlation kernel's epilogue lists every
// plane point at or above the threshold; these kernels keep the points that
// outrank all eight neighbours of their (z, r) grid cell. A neighbour under
// the threshold is under every candidate, so the candidates alone decide:
// they are hashed by grid cell, and each one looks its neighbours up.
//
// Grid: without interbinning row i is z_i and column c is bin r; with it,
// plane row 2i + h (z_i at r + h/2) is grid row i, column 2r + h, so that
// neighbouring columns are half a bin apart. Order: p outranks q when
// P_p > P_q, or P_p == P_q and (row, column) of p comes first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "peaks.hpp"

namespace fdas {

namespace {

constexpr unsigned long long kEmpty = ~0ull;
constexpr int kColBits = 36;  // grid column < 2^36, grid row < 2^27

__device__ __forceinline__ unsigned long long cell_key(int row, int64_t r, int interbin) {
  const unsigned long long gi = interbin ? (unsigned)row >> 1 : (unsigned)row;
  const unsigned long long gc = interbin ? 2ull * (unsigned long long)r + (row & 1)
                                         : (unsigned long long)r;
  return (gi << kColBits) | gc;
}

// 64-bit finaliser of the splitmix64 generator (Steele, Lea & Flood 2014) as
// the hash of a cell key.
__device__ __forceinline__ unsigned long long mix(unsigned long long x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ int64_t stored(const unsigned long long *counts, int64_t cap) {
  const unsigned long long n = counts[0];
  return n < (unsigned long long)cap ? (int64_t)n : cap;
}

__global__ void peaks_reset_kernel(unsigned long long *counts) {
  if (threadIdx.x < 2) counts[threadIdx.x] = 0ull;
}

__global__ void peaks_clear_kernel(unsigned long long *keys, int64_t slots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < slots) keys[i] = kEmpty;
}

__global__ void peaks_insert_kernel(const Cand *__restrict__ cands,
                                    const unsigned long long *__restrict__ counts, int64_t cap,
                                    unsigned long long *keys, int *vals, int64_t mask,
                                    int interbin) {
  const int64_t n = stored(counts, cap);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Cand c = cands[i];
    const unsigned long long k = cell_key(c.row, c.r, interbin);
    // the table holds at least twice the candidates, so a free slot is reached
    for (int64_t h = (int64_t)(mix(k) & (unsigned long long)mask);; h = (h + 1) & mask) {
      const unsigned long long prev = atomicCAS(keys + h, kEmpty, k);
      if (prev == kEmpty || prev == k) {  // a cell appears once; equal keys cannot race
        vals[h] = (int)i;
        break;
      }
    }
  }
}

__global__ void peaks_probe_kernel(const Cand *__restrict__ cands, unsigned long long *counts,
                                   int64_t cap, const unsigned long long *__restrict__ keys,
                                   const int *__restrict__ vals, int64_t mask, int interbin,
                                   Cand *__restrict__ peaks, int64_t peak_cap) {
  const int64_t n = stored(counts, cap);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Cand c = cands[i];
    const unsigned long long k = cell_key(c.row, c.r, interbin);
    const long long gi = (long long)(k >> kColBits);
    const long long gc = (long long)(k & ((1ull << kColBits) - 1));
    bool peak = true;
    for (int d = 0; d < 9 && peak; ++d) {
      if (d == 4) continue;
      const long long ni = gi + d / 3 - 1, nc = gc + d % 3 - 1;
      if (ni < 0 || nc < 0) continue;  // outside the grid: no such neighbour
      const unsigned long long nk = ((unsigned long long)ni << kColBits) | (unsigned long long)nc;
      for (int64_t h = (int64_t)(mix(nk) & (unsigned long long)mask);; h = (h + 1) & mask) {
        const unsigned long long kk = keys[h];
        if (kk == kEmpty) break;  // not a candidate: below the threshold
        if (kk == nk) {
          const float q = cands[vals[h]].power;
          if (q > c.power || (q == c.power && nk < k)) peak = false;
          break;
        }
      }
    }
    if (peak) {
      const unsigned long long slot = atomicAdd(counts + 1, 1ull);
      if (slot < (unsigned long long)peak_cap) peaks[slot] = c;
    }
  }
}

}  // namespace

int64_t peaks_table_slots(int64_t cand_capacity) {
  int64_t s = 64;
  while (s < 2 * cand_capacity) s <<= 1;
  return s;
}

size_t peaks_workspace_bytes(int64_t cand_capacity) {
  const int64_t slots = peaks_table_slots(cand_capacity);
  return (size_t)cand_capacity * sizeof(Cand) + (size_t)slots * (8 + 4);
}

hipError_t launch_peaks_reset(unsigned long long *counts, hipStream_t s) {
  hipLaunchKernelGGL(peaks_reset_kernel, dim3(1), dim3(64), 0, s, counts);
  return hipGetLastError();
}

hipError_t launch_peaks(const Cand *cands, int64_t cand_capacity, void *table,
                        unsigned long long *counts, int interbin, Cand *peaks, int64_t peak_cap,
                        hipStream_t s) {
  const int64_t slots = peaks_table_slots(cand_capacity);
  unsigned long long *keys = static_cast<unsigned long long *>(table);
  int *vals = reinterpret_cast<int *>(keys + slots);
  constexpr int kT = 256;
  hipLaunchKernelGGL(peaks_clear_kernel, dim3((unsigned)((slots + kT - 1) / kT)), dim3(kT), 0, s,
                     keys, slots);
  if (cand_capacity > 0) {
    // threads stride over the listed candidates, whose number only the
    // device knows; 2048 blocks cover the chip several times over
    const dim3 grid((unsigned)std::min<int64_t>((cand_capacity + kT - 1) / kT, 2048));
    hipLaunchKernelGGL(peaks_insert_kernel, grid, dim3(kT), 0, s, cands, counts, cand_capacity,
                       keys, vals, slots - 1, interbin);
    hipLaunchKernelGGL(peaks_probe_kernel, grid, dim3(kT), 0, s, cands, counts, cand_capacity,
                       keys, vals, slots - 1, interbin, peaks, peak_cap);
  }
  return hipGetLastError();
}

}  // namespace fdas
