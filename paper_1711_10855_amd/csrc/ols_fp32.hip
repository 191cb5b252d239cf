// Fused FP32 overlap-and-save correlation kernel for gfx950.
//
// One work unit = (segment s, group of templates). For its segment the kernel
//   1. loads x_j = A[s U - m/2 + j], j in [0, L), zero outside [0, nbins)
//      (the overlap-and-save segment, Section 2), coalesced;
//   2. runs the forward FFT (eq. 3 sign) once, decimation in frequency, with
//      radix-R butterflies in registers and LDS exchanges between stages; the
//      result stays in registers in digit-reversed slot order;
//   3. for every template of its group: multiplies by the bank row (stored in
//      the same slot order, so no reorder), runs the inverse FFT (decimation
//      in time, natural-order output; the 1/L is folded into the bank), keeps
//      outputs j in [m/2, m/2 + U) and writes |y|^2 straight to the power
//      plane with non-temporal stores.
// The paper runs the per-template inverse FFT on shared-memory-resident data
// inside one thread block (Section 3); here each thread holds E = L / T
// elements in VGPRs, the first inverse stage consumes the forward result
// without touching LDS, and only the remaining P - 1 stages exchange
// through a padded LDS buffer.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "fft_block.hpp"
#include "fft_radix.hpp"
#include "layout.hpp"
#include "ols_variants.hpp"

namespace fdas {

// A pointer that is the same in every lane, moved to scalar registers (a
// buffer resource built from it then needs no per-lane loop).
template <class T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}

// One work unit: segment s of a spectrum, bank rows [z0, z1), plane rows
// (iz - row_base). The unit starts on LDS buffer 0: its caller guarantees a
// block barrier since any earlier unit's last LDS read.
template <class Gm, bool TWREG, bool PF, bool CAND>
__device__ __forceinline__ void ols_unit(const c32 *__restrict__ spec_, int64_t nbins,
                                         const c32 *__restrict__ bank_, const c32 *__restrict__ tw_,
                                         float *__restrict__ power_, int64_t ld, int s, bool active,
                                         int U, int half, int z0, int z1, int row_base, c32 *buf0,
                                         c32 *buf1, int t, const CandOut &cd) {
  const auto spec = to_global(spec_);
  const auto bank = to_global(bank_);
  const auto tw = to_global(tw_);
  const auto power = to_global(power_);
  constexpr int L = Gm::L, T = Gm::T, E = Gm::E, P = Gm::P;
  const int64_t seg0 = (int64_t)s * U - half;

  c32 x[E];
  // stage 0 input: element n of butterfly b = t + j T sits at n * S0 + b
  {
    constexpr int S0 = Gm::S(0), R0 = Gm::R[0];
#pragma unroll
    for (int j = 0; j < Gm::B(0); ++j)
#pragma unroll
      for (int n = 0; n < R0; ++n) {
        const int64_t g = seg0 + n * S0 + t + j * T;
        c32 v = {0.f, 0.f};
        if (active && g >= 0 && g < nbins) v = ldg(spec + g);
        x[j * R0 + n] = v;
      }
  }
  // Bank rows are read through a buffer resource over the row (a wave-uniform
  // base): the lane's byte offset t * 8 in its offset register, the element's
  // e T * 8 as a scalar offset, so one register serves every element and no
  // 64-bit address is formed per element and template.
  auto bank_row = [&](int iz) {
    return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(const_cast<c32 *>(bank_) + (int64_t)iz * L),
                                             (short)0, L * 8, 0x00020000);
  };
  const int boff = t * 8;
  auto bank_elem = [&](const __amdgpu_buffer_rsrc_t &rs, int e) {
    const f2v v = __builtin_bit_cast(
        f2v, __builtin_amdgcn_raw_buffer_load_b64(rs, boff, e * T * 8, 0));
    return c32{v.x, v.y};
  };

  c32 bnext[PF ? E : 1];
  if constexpr (PF) {
    const auto rs = bank_row(z0);
#pragma unroll
    for (int e = 0; e < E; ++e) bnext[e] = bank_elem(rs, e);
  }

  // forward, decimation in frequency
  static_for_up<0, P>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int R = Gm::R[I];
    if constexpr (I > 0) exchange<Gm, I - 1, I, flips<Gm>(0, I - 1) & 1>(x, buf0, buf1, t);
#pragma unroll
    for (int j = 0; j < Gm::B(I); ++j) {
      dft<-1, R>(&x[j * R]);
      if constexpr (I < P - 1) {
        constexpr int N = R * Gm::S(I);
        const int mi = stage_suffix<Gm, I>(t, j);
#pragma unroll
        for (int k = 1; k < R; ++k) x[j * R + k] = cmul(x[j * R + k], ldg(tw + (k * mi) * (L / N)));
      }
    }
  });

  // inverse twiddles, reused by every template
  c32 itw[TWREG && Gm::NTW > 0 ? Gm::NTW : 1];
  if constexpr (TWREG) {
    static_for_up<0, P - 1>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      constexpr int R = Gm::R[I];
      constexpr int N = R * Gm::S(I);
#pragma unroll
      for (int j = 0; j < Gm::B(I); ++j) {
        const int mi = stage_suffix<Gm, I>(t, j);
#pragma unroll
        for (int k = 1; k < R; ++k)
          itw[Gm::TWOFF(I) + j * (R - 1) + k - 1] = ldg(tw + (k * mi) * (L / N));
      }
    });
  }

  // Byte offsets of the outputs in the store resource (see the stores), one
  // per output slot, computed once per unit; each passes through an empty
  // asm statement so that it reaches the store whole in the lane's offset
  // register (no constant part is moved into the immediate field).
  constexpr bool kBufStore = !CAND && T >= 64;
  int soff[kBufStore ? E : 1];
  if constexpr (kBufStore) {
    constexpr int S0 = Gm::S(0), R0 = Gm::R[0];
#pragma unroll
    for (int j = 0; j < Gm::B(0); ++j)
#pragma unroll
      for (int n = 0; n < R0; ++n) {
        int off = (n * S0 + t + j * T - half) * 4;
        asm volatile("" : "+v"(off));
        soff[j * R0 + n] = off;
      }
  }

  // one template; P0 is the buffer parity at its start
  auto one = [&](int iz, auto p0c) {
    constexpr int P0 = decltype(p0c)::value;
    // The product Y = X T goes into the first inverse stage's butterflies:
    // its first layer forms x_a T_a + x_c T_c with fused multiply-adds (as it
    // would apply twiddles), two operations fewer per pair than multiplying
    // first. (The detection epilogue computes the same way, so that its
    // powers equal the plane's bit for bit.)
    c32 y[E], bt[E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = x[e];
    if constexpr (PF) {
#pragma unroll
      for (int e = 0; e < E; ++e) bt[e] = bnext[e];
      // the last template reloads its own row: an unconditional load keeps
      // one register set for the bank (a conditional one makes the compiler
      // copy the prefetched values across the loop edge)
      const auto rs = bank_row(iz + 1 < z1 ? iz + 1 : iz);
#pragma unroll
      for (int e = 0; e < E; ++e) bnext[e] = bank_elem(rs, e);
    } else {
      const auto rs = bank_row(iz);
#pragma unroll
      for (int e = 0; e < E; ++e) bt[e] = bank_elem(rs, e);
    }

    // inverse, decimation in time: stages P-1 .. 0
    static_for_down<P - 1, 0>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      constexpr int R = Gm::R[I];
      if constexpr (I == P - 1) {
#pragma unroll
        for (int j = 0; j < Gm::B(I); ++j) dft_tw<+1, false, R, true>(&y[j * R], &bt[j * R]);
      } else {
        exchange<Gm, I + 1, I, (P0 + flips<Gm>(I + 1, P - 1)) & 1>(y, buf0, buf1, t);
        constexpr int N = R * Gm::S(I);
#pragma unroll
        for (int j = 0; j < Gm::B(I); ++j) {
          const int mi = stage_suffix<Gm, I>(t, j);
          c32 w[R];
#pragma unroll
          for (int k = 1; k < R; ++k)
            w[k] = TWREG ? itw[Gm::TWOFF(I) + j * (R - 1) + k - 1] : ldg(tw + (k * mi) * (L / N));
          dft_tw<+1, true, R>(&y[j * R], w);  // conj twiddles folded into the butterfly
        }
      }
    });

    // outputs: slot j*R0 + n holds index n * S0 + t + j T of the segment
    if constexpr (CAND) {
      // detection epilogue: the powers first (the transform's registers are
      // then free), one ballot to skip a wave with no hit at all (the common
      // case), else every lane takes part in each offer (one atomic per wave
      // that has a hit)
      constexpr int S0 = Gm::S(0), R0 = Gm::R[0];
      float pw[E];
      bool any = false;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        pw[e] = __builtin_fmaf(y[e].x, y[e].x, y[e].y * y[e].y);
        any |= pw[e] >= cd.thr;
      }
      if (__builtin_amdgcn_ballot_w64(active && any) != 0ull) {
#pragma unroll
        for (int j = 0; j < Gm::B(0); ++j)
#pragma unroll
          for (int n = 0; n < R0; ++n) {
            const int o = n * S0 + t + j * T;
            const int64_t r = (int64_t)s * U + o - half;
            const float p = pw[j * R0 + n];
            const bool hit = active && o >= half && o < half + U && r < nbins && p >= cd.thr;
            cand_offer(cd, hit, iz - row_base, r, p);
          }
      }
    } else if (kBufStore && active) {
      // Stores through a buffer resource that starts at plane column s U
      // (segment output `half`) and spans the segment's kept outputs: output
      // o goes to byte offset (o - half) * 4, which is negative (so, taken as
      // unsigned, past the end) for o < half and at or past the end for
      // o >= half + U or beyond nbins, and the hardware drops those lanes.
      // (With T >= 64 a wave holds one segment, so s is the same in every
      // lane and the resource is wave-uniform.)
      constexpr int S0 = Gm::S(0), R0 = Gm::R[0];
      const int su = __builtin_amdgcn_readfirstlane(s);
      const int64_t left = nbins - (int64_t)su * U;
      const int nkeep = (int)(left < U ? left : U);
      const auto rs = __builtin_amdgcn_make_buffer_rsrc(
          uniform_ptr(power_ + (int64_t)(iz - row_base) * ld + (int64_t)su * U), (short)0, nkeep * 4,
          0x00020000);
#pragma unroll
      for (int j = 0; j < Gm::B(0); ++j)
#pragma unroll
        for (int n = 0; n < R0; ++n) {
          const c32 v = y[j * R0 + n];
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(__builtin_fmaf(v.x, v.x, v.y * v.y)),
                                                rs, soff[j * R0 + n], 0, 2 /* nontemporal */);
        }
    } else if (active) {  // segments narrower than a wave: per-lane addresses
      constexpr int S0 = Gm::S(0), R0 = Gm::R[0];
      const auto prow = power + (int64_t)(iz - row_base) * ld;
#pragma unroll
      for (int j = 0; j < Gm::B(0); ++j)
#pragma unroll
        for (int n = 0; n < R0; ++n) {
          const int o = n * S0 + t + j * T;
          const int64_t r = (int64_t)s * U + o - half;
          if (o >= half && o < half + U && r < nbins) {
            const c32 v = y[j * R0 + n];
            __builtin_nontemporal_store(__builtin_fmaf(v.x, v.x, v.y * v.y), prow + r);
          }
        }
    }
  };
  constexpr int PF0 = flips<Gm>(0, P - 1) & 1;  // after the forward transform
  if constexpr ((flips<Gm>(0, P - 1) & 1) == 0) {
    for (int iz = z0; iz < z1; ++iz) one(iz, std::integral_constant<int, PF0>{});
  } else {
    // an odd number of flips per template: alternate the two parities
    int iz = z0;
    for (; iz + 1 < z1; iz += 2) {
      one(iz, std::integral_constant<int, PF0>{});
      one(iz + 1, std::integral_constant<int, PF0 ^ 1>{});
    }
    if (iz < z1) one(iz, std::integral_constant<int, PF0>{});
  }
}

// Single spectrum: block -> (segment group, template group), template-group
// major so concurrently running blocks share bank rows in L2.
template <class Gm, int G, bool TWREG, bool PF, int WPE, bool CAND>
__global__ void __launch_bounds__(Gm::T *G) __attribute__((amdgpu_waves_per_eu(WPE)))
    ols_fp32_kernel(const c32 *__restrict__ spec, int64_t nbins, const c32 *__restrict__ bank,
                    const c32 *__restrict__ tw, float *__restrict__ power, int64_t ld, int nseg,
                    int U, int half, int nz, int zpb, int nsb, CandOut cand) {
  constexpr int T = Gm::T, NB = Gm::NBUF;
  __shared__ c32 lds[NB][G][Gm::LP];
  const int tid = threadIdx.x;
  const int sg = tid / T;
  const int t = tid % T;
  const int sb = blockIdx.x % nsb;
  const int zg = blockIdx.x / nsb;
  const int s = sb * G + sg;
  const int z0 = zg * zpb;
  const int z1 = min(nz, z0 + zpb);
  ols_unit<Gm, TWREG, PF, CAND>(spec, nbins, bank, tw, power, ld, s, s < nseg, U, half, z0, z1, 0,
                          lds[0][sg], lds[NB - 1][sg], t, cand);
}

// Batch: persistent blocks take work items (series, template group, segment
// group) from a device counter until the list is exhausted. Items are
// numbered series by series (largest first on the host), template-group major
// inside a series.
template <class Gm, int G, bool TWREG, bool PF, int WPE>
__global__ void __launch_bounds__(Gm::T *G) __attribute__((amdgpu_waves_per_eu(WPE)))
    ols_fp32_batch_kernel(const SeriesDesc *__restrict__ desc, int nseries, int64_t total,
                          unsigned long long *__restrict__ counter, const c32 *__restrict__ bank,
                          const c32 *__restrict__ tw, int U, int half, int zpb) {
  constexpr int T = Gm::T, NB = Gm::NBUF;
  __shared__ c32 lds[NB][G][Gm::LP];
  __shared__ long long s_item[2];
  const int tid = threadIdx.x;
  int par = 0;
  for (;;) {
    if (tid == 0) s_item[par] = (long long)atomicAdd(counter, 1ULL);
    __syncthreads();
    const long long item = s_item[par];
    par ^= 1;
    if (item >= total) break;
    // series k: the last with item_begin <= item
    int lo = 0, hi = nseries - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (desc[mid].item_begin <= item) lo = mid;
      else hi = mid - 1;
    }
    const SeriesDesc d = desc[lo];
    const long long local = item - d.item_begin;
    const int nsb = (d.nseg + G - 1) / G;
    const int zg = (int)(local / nsb);
    const int sb = (int)(local % nsb);
    // The thread index passes through an empty asm statement on every item, so
    // that nothing computed from it is hoisted out of this loop (held across
    // it, one unit's addresses spilled: the loop measured twice as slow).
    int tid_i;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid_i) : "v"(tid));
    const int sg = tid_i / T;
    const int t = tid_i % T;
    const int s = sb * G + sg;
    const int z0 = d.row_off + zg * d.zpb;
    const int z1 = min(d.row_off + d.nz, z0 + d.zpb);
    const CandOut none{};
    ols_unit<Gm, TWREG, PF, false>(static_cast<const c32 *>(d.spec), d.nbins, opaque_ptr(bank),
                            opaque_ptr(tw), d.power, d.ld, s, s < d.nseg, U, half, z0, z1,
                            d.row_off, lds[0][sg], lds[NB - 1][sg], t, none);
  }
}

// Batch as one flat launch: block b takes work item b (same numbering), so
// the hardware dispatcher hands out items in order as blocks retire
// (FDAS_BATCH_PERSISTENT=0; the persistent loop above is the default, 1%
// faster on the batched workloads).
template <class Gm, int G, bool TWREG, bool PF, int WPE>
__global__ void __launch_bounds__(Gm::T *G) __attribute__((amdgpu_waves_per_eu(WPE)))
    ols_fp32_items_kernel(const SeriesDesc *__restrict__ desc, int nseries,
                          const c32 *__restrict__ bank, const c32 *__restrict__ tw, int U,
                          int half, int zpb) {
  constexpr int T = Gm::T, NB = Gm::NBUF;
  __shared__ c32 lds[NB][G][Gm::LP];
  const int tid = threadIdx.x;
  const int sg = tid / T;
  const int t = tid % T;
  const long long item = blockIdx.x;
  int lo = 0, hi = nseries - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].item_begin <= item) lo = mid;
    else hi = mid - 1;
  }
  const SeriesDesc d = desc[lo];
  const long long local = item - d.item_begin;
  const int nsb = (d.nseg + G - 1) / G;
  const int zg = (int)(local / nsb);
  const int sb = (int)(local % nsb);
  const int s = sb * G + sg;
  const int z0 = d.row_off + zg * d.zpb;
  const int z1 = min(d.row_off + d.nz, z0 + d.zpb);
  const CandOut none{};
  ols_unit<Gm, TWREG, PF, false>(static_cast<const c32 *>(d.spec), d.nbins, bank, tw, d.power, d.ld, s,
                          s < d.nseg, U, half, z0, z1, d.row_off, lds[0][sg], lds[NB - 1][sg],
                          t, none);
}

__global__ void reset_counter_kernel(unsigned long long *counter) { *counter = 0ULL; }

hipError_t launch_reset_counter(unsigned long long *counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

static bool batch_persistent() {
  const char *e = std::getenv("FDAS_BATCH_PERSISTENT");
  return !(e && *e == '0');  // the flat item grid with FDAS_BATCH_PERSISTENT=0
}

// ---- variant registry ------------------------------------------------------

template <class Gm, int G, bool TWREG, bool PF, int WPE>
static hipError_t launch_variant(const OlsArgs &a, hipStream_t st) {
  const int nsb = (a.nseg + G - 1) / G;
  const int nzg = (a.nz + a.zpb - 1) / a.zpb;
  const long blocks = (long)nsb * nzg;
  if (a.cand.count)
    hipLaunchKernelGGL((ols_fp32_kernel<Gm, G, TWREG, PF, WPE, true>), dim3((unsigned)blocks),
                       dim3(Gm::T * G), 0, st, static_cast<const c32 *>(a.spec), a.nbins,
                       static_cast<const c32 *>(a.bank), static_cast<const c32 *>(a.tw), a.power,
                       a.ld, a.nseg, a.U, a.half, a.nz, a.zpb, nsb, a.cand);
  else
    hipLaunchKernelGGL((ols_fp32_kernel<Gm, G, TWREG, PF, WPE, false>), dim3((unsigned)blocks),
                       dim3(Gm::T * G), 0, st, static_cast<const c32 *>(a.spec), a.nbins,
                       static_cast<const c32 *>(a.bank), static_cast<const c32 *>(a.tw), a.power,
                       a.ld, a.nseg, a.U, a.half, a.nz, a.zpb, nsb, a.cand);
  return hipGetLastError();
}

template <class Gm, int G, bool TWREG, bool PF, int WPE>
static hipError_t launch_batch_variant(const BatchArgs &a, hipStream_t st) {
  if (batch_persistent()) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, a.counter);
    hipLaunchKernelGGL((ols_fp32_batch_kernel<Gm, G, TWREG, PF, WPE>), dim3((unsigned)a.grid),
                       dim3(Gm::T * G), 0, st, a.desc, a.nseries, a.total, a.counter,
                       static_cast<const c32 *>(a.bank), static_cast<const c32 *>(a.tw), a.U,
                       a.half, a.zpb);
  } else {
    if (a.total > (int64_t)0xffffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((ols_fp32_items_kernel<Gm, G, TWREG, PF, WPE>), dim3((unsigned)a.total),
                       dim3(Gm::T * G), 0, st, a.desc, a.nseries,
                       static_cast<const c32 *>(a.bank), static_cast<const c32 *>(a.tw), a.U,
                       a.half, a.zpb);
  }
  return hipGetLastError();
}

template <class Gm, int G, bool TWREG, bool PF, int WPE>
static int batch_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void *>(&ols_fp32_batch_kernel<Gm, G, TWREG, PF, WPE>),
          Gm::T * G, 0) != hipSuccess)
    return 0;
  return nb;
}

template <class Gm, int G, bool TWREG, bool PF, int WPE>
static int grid_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void *>(&ols_fp32_kernel<Gm, G, TWREG, PF, WPE, false>), Gm::T * G,
          0) != hipSuccess)
    return 0;
  return nb;
}

template <class Gm, int G, bool TWREG, bool PF, int WPE = 1>
static constexpr OlsVariant make_variant(const char *name) {
  OlsVariant v{};
  v.name = name;
  v.L = Gm::L;
  v.T = Gm::T;
  v.G = G;
  v.nbuf = Gm::NBUF;
  v.precision = 0;
  v.lay.L = Gm::L;
  v.lay.T = Gm::T;
  v.lay.E = Gm::E;
  v.lay.P = Gm::P;
  for (int i = 0; i < kMaxStages; ++i) v.lay.R[i] = i < Gm::P ? Gm::R[i] : 1;
  v.lds_bytes = Gm::NBUF * G * Gm::LP * 8;
  v.launch = &launch_variant<Gm, G, TWREG, PF, WPE>;
  v.launch_batch = &launch_batch_variant<Gm, G, TWREG, PF, WPE>;
  v.batch_blocks_per_cu = &batch_blocks_per_cu<Gm, G, TWREG, PF, WPE>;
  v.grid_blocks_per_cu = &grid_blocks_per_cu<Gm, G, TWREG, PF, WPE>;
  return v;
}

// Name: fp32_L<len>_t<threads per segment>[x<segments per block>]_r<radices>
//       [_tg: twiddles re-read from the table | _np: no bank prefetch]
//       [_o<n>: registers capped for n waves per SIMD]
static const OlsVariant kFp32Variants[] = {
    // the first entry for each length is the default for that length
    make_variant<Geo<256, 32, 4, 8, 8>, 2, true, true, 4>("fp32_L256_t32x2_r4.8.8"),
    make_variant<Geo<256, 16, 16, 16>, 4, true, true>("fp32_L256_t16x4_r16.16"),
    make_variant<Geo<512, 64, 8, 8, 8>, 1, true, true, 4>("fp32_L512_t64_r8.8.8"),
    make_variant<Geo<512, 32, 2, 16, 16>, 2, false, true>("fp32_L512_t32x2_r2.16.16_tg"),
    make_variant<Geo<1024, 128, 2, 8, 8, 8>, 1, true, true, 4>("fp32_L1024_t128_r2.8.8.8"),
    make_variant<Geo<1024, 64, 4, 16, 16>, 1, false, true>("fp32_L1024_t64_r4.16.16_tg"),
    make_variant<Geo<1024, 128, 2, 8, 8, 8>, 1, true, true, 3>("fp32_L1024_t128_r2.8.8.8_o3"),
    make_variant<Geo<2048, 128, 8, 16, 16>, 1, true, true, 2>("fp32_L2048_t128_r8.16.16_o2"),
    make_variant<Geo<2048, 128, 8, 16, 16>, 1, true, false>("fp32_L2048_t128_r8.16.16_np"),
    make_variant<Geo<2048, 128, 8, 16, 16>, 1, false, true, 2>("fp32_L2048_t128_r8.16.16_tg_o2"),
    make_variant<Geo<2048, 256, 4, 8, 8, 8>, 1, true, true, 3>("fp32_L2048_t256_r4.8.8.8"),
    make_variant<Geo<2048, 256, 4, 8, 8, 8>, 1, false, true, 3>("fp32_L2048_t256_r4.8.8.8_tg"),
    make_variant<Geo<4096, 256, 16, 16, 16>, 1, true, true, 2>("fp32_L4096_t256_r16.16.16_o2"),
    make_variant<Geo<4096, 256, 16, 16, 16>, 1, true, false, 2>("fp32_L4096_t256_r16.16.16_np"),
    make_variant<Geo<4096, 256, 16, 16, 16>, 1, false, true, 2>("fp32_L4096_t256_r16.16.16_tg_o2"),
    make_variant<Geo<4096, 512, 8, 8, 8, 8>, 1, false, true>("fp32_L4096_t512_r8.8.8.8_tg"),
    make_variant<Geo<4096, 512, 8, 8, 8, 8>, 1, true, true, 2>("fp32_L4096_t512_r8.8.8.8_o2"),
    make_variant<Geo<8192, 512, 2, 16, 16, 16>, 1, false, true>("fp32_L8192_t512_r2.16.16.16_tg"),
    make_variant<Geo<8192, 1024, 2, 8, 8, 8, 8>, 1, false, true>("fp32_L8192_t1024_r2.8.8.8.8_tg"),
    make_variant<Geo<16384, 1024, 4, 16, 16, 16>, 1, false, false>("fp32_L16384_t1024_r4.16.16.16_tg"),
};

const OlsVariant *fp32_variants(int *count) {
  *count = (int)(sizeof(kFp32Variants) / sizeof(kFp32Variants[0]));
  return kFp32Variants;
}

}  // namespace fdas
