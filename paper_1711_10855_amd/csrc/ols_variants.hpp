// Registry of compiled hot-kernel variants (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_radix.hpp"
#include "layout.hpp"

namespace fdas {

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
};

struct OlsVariant {
  const char *name;
  int L, T, G, nbuf;
  LayoutDesc lay;
  int lds_bytes;
  hipError_t (*launch)(const OlsArgs &, hipStream_t);
};

const OlsVariant *fp32_variants(int *count);

hipError_t launch_templates(void *out, int nz, int m, double zmax, double dz, hipStream_t s);
hipError_t launch_twiddles(c32 *tw, int L, hipStream_t s);
hipError_t launch_bank(c32 *bank, const void *h, int nz, int m, const LayoutDesc &lay,
                       hipStream_t s);
hipError_t launch_bank_natural(c32 *dst, const c32 *bank, int nz,
                               const LayoutDesc &lay, hipStream_t s);

}  // namespace fdas
