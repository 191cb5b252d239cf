// Registry of compiled hot-kernel variants (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_radix.hpp"
#include "layout.hpp"

namespace fdas {

// Detection epilogue: with `count` set, plane points whose power is at least
// `thr` are counted on `count` and written to `list` while the slot is below
// `cap` (list may be null when cap is 0), instead of the plane being stored.
struct Cand {
  int row;
  float power;
  int64_t r;
};
static_assert(sizeof(Cand) == 16, "candidate record is 16 bytes");
struct CandOut {
  Cand *list;
  unsigned long long *count;
  int64_t cap;
  float thr;
};

// Called by every lane of the wave together (not under divergent control
// flow); lanes with `hit` set append (row, r, p). One atomic per wave that has
// any hit: lanes take consecutive slots in lane order.
__device__ __forceinline__ void cand_offer(const CandOut &cd, bool hit, int row, int64_t r,
                                           float p) {
  typedef int i4v __attribute__((ext_vector_type(4)));
  const unsigned long long mask = __builtin_amdgcn_ballot_w64(hit);
  if (mask == 0ull) return;
  const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  const int first = __builtin_ctzll(mask);
  unsigned long long base = 0ull;
  if (lane == first) base = atomicAdd(cd.count, (unsigned long long)__builtin_popcountll(mask));
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)base, first);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(base >> 32), first);
  base = ((unsigned long long)hi << 32) | lo;
  if (hit) {
    const unsigned long long i =
        base + (unsigned long long)__builtin_popcountll(mask & ((1ull << lane) - 1ull));
    if (i < (unsigned long long)cd.cap) {
      const i4v v = {row, __builtin_bit_cast(int, p), (int)(uint64_t)r, (int)((uint64_t)r >> 32)};
      *(gptr<i4v>)(cd.list + i) = v;  // one 16-byte store
    }
  }
}

struct OlsArgs {
  const void *spec;  // complex64 [nbins]
  int64_t nbins;
  const void *bank;  // slot-ordered bank [nz][L]
  const void *tw;    // twiddles W_L^j, complex64 [L]
  float *power;      // [nz][ld]
  int64_t ld;
  int nseg;          // ceil(nbins / U)
  int U;             // L - m
  int half;          // m / 2
  int nz;            // rows to produce
  int zpb;           // templates per work unit
  int bank_log2;     // mixed precision: the bank is stored times 2^bank_log2
  const void *consts;  // mixed precision: per-lane constants table
  CandOut cand;        // detection epilogue (count == nullptr: store the plane)
};

// One series of a batch as the persistent kernel sees it.
struct SeriesDesc {
  const void *spec;     // complex64 [nbins]
  float *power;         // [nz][ld]
  int64_t nbins;
  int64_t ld;
  int64_t item_begin;   // first work item of this series
  int nseg;             // segments
  int nz;               // rows of this series' plane
  int row_off;          // first bank row used by this series
  int zpb;              // templates per work item of this series
};

struct BatchArgs {
  const SeriesDesc *desc;
  int nseries;
  int64_t total;        // work items
  unsigned long long *counter;
  const void *bank;
  const void *tw;
  int U, half, zpb;
  int grid;             // persistent blocks
  int bank_log2;        // mixed precision: bank scale
  const void *consts;   // mixed precision: per-lane constants
};

struct OlsVariant {
  const char *name;
  int L, T, G, nbuf;
  int precision;     // FDAS_FP32 (0), FDAS_MIXED_FP16 (1), FDAS_MIXED_BF16 (2)
  int split;         // 1: hi + lo split products (FDAS_FLAG_SPLIT)
  int zpb_target;    // > 0: templates per work unit fixed near this (balanced
                     // groups); 0: chosen per launch from the grid's rounds
  LayoutDesc lay;
  int lds_bytes;
  hipError_t (*launch)(const OlsArgs &, hipStream_t);
  hipError_t (*launch_batch)(const BatchArgs &, hipStream_t);
  int (*batch_blocks_per_cu)();
  int (*grid_blocks_per_cu)();  // occupancy of the single-spectrum kernel
};

const OlsVariant *fp32_variants(int *count);
const OlsVariant *mixed_variants(int *count);
hipError_t launch_bank_mixed(void *bank, const void *h, int nz, int m, int L, int precision,
                             int split, hipStream_t s);
size_t mixed_consts_bytes(int L, int split);
hipError_t launch_mixed_consts(void *out, int L, int precision, int split, hipStream_t s);
hipError_t launch_bank_mixed_natural(c32 *dst, const void *bank, int nz, int L, int precision,
                                     int split, hipStream_t s);

// The 2048-point matrix-core kernel (FP16 and BF16, no split form).
const OlsVariant *mixed2048_variants(int *count);
size_t mixed2048_consts_bytes();
hipError_t launch_mixed2048_consts(void *out, int precision, hipStream_t s);
hipError_t launch_bank_mixed2048(void *bank, const void *h, int nz, int m, int precision,
                                 hipStream_t s);
hipError_t launch_bank_mixed2048_natural(c32 *dst, const void *bank, int nz, int precision,
                                         hipStream_t s);

hipError_t launch_reset_counter(unsigned long long *counter, hipStream_t s);
hipError_t launch_templates(void *out, int rows, int m, double zmax, double dz, int interbin,
                            hipStream_t s);
hipError_t launch_twiddles(c32 *tw, int L, hipStream_t s);
hipError_t launch_bank(c32 *bank, const void *h, int nz, int m, const LayoutDesc &lay,
                       hipStream_t s);
hipError_t launch_bank_natural(c32 *dst, const c32 *bank, int nz,
                               const LayoutDesc &lay, hipStream_t s);

}  // namespace fdas
