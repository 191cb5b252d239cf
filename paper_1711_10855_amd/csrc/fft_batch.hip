// Standalone batched complex FFT built from the same in-register butterflies
// and LDS exchanges as the overlap-and-save kernel.
//
// The paper measures its shared-memory FFT on its own, over many transforms
// of one length with 2, 4 or 8 elements per thread, against the vendor FFT
// library (Section 3, Table 1). This file gives the same building blocks a
// plain interface: every block transforms G sequences of length L held
// contiguously in device memory (complex64, natural order in and out,
// unnormalised, sign of eq. 3 for the forward direction). One thread owns
// E = L / T elements; the stages run decimation in frequency exactly as the
// forward transform of the correlation kernel, and one more LDS exchange puts
// the digit-reversed result back in natural order so that the stores are
// coalesced.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_block.hpp"
#include "fft_radix.hpp"
#include "fft_batch.hpp"

namespace fdas {

// LDS address, in the layout of the last stage, of frequency k.
// After the last forward stage address a = sum_i d_i S_i holds frequency
// k = d_0 + R_0 (d_1 + R_1 (d_2 + ...)), so the digits of k, least
// significant first, are d_0, d_1, ...
template <class Gm>
__device__ __forceinline__ int addr_of_freq(int k) {
  int a = 0;
  static_for_up<0, Gm::P>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    a += (k % Gm::R[I]) * Gm::S(I);
    k /= Gm::R[I];
  });
  return a;
}

template <class Gm, int G, int DIR>
__global__ void __launch_bounds__(Gm::T *G)
    fft_batch_kernel(const c32 *__restrict__ in_, c32 *__restrict__ out_, int64_t batch,
                     const c32 *__restrict__ tw_) {
  constexpr int L = Gm::L, T = Gm::T, E = Gm::E, P = Gm::P, NB = Gm::NBUF;
  __shared__ c32 lds[NB][G][Gm::LP];
  const int tid = threadIdx.x;
  const int g = tid / T;
  const int t = tid % T;
  const int64_t f = (int64_t)blockIdx.x * G + g;
  const bool active = f < batch;
  const auto in = to_global(in_);
  const auto out = to_global(out_);
  const auto tw = to_global(tw_);
  c32 *buf0 = lds[0][g];
  c32 *buf1 = lds[NB - 1][g];

  // stage 0 input: element n of butterfly b = t + j T sits at n * S0 + b
  c32 x[E];
  {
    constexpr int S0 = Gm::S(0), R0 = Gm::R[0];
#pragma unroll
    for (int j = 0; j < Gm::B(0); ++j)
#pragma unroll
      for (int n = 0; n < R0; ++n) {
        c32 v = {0.f, 0.f};
        if (active) v = ldg(in + f * L + n * S0 + t + j * T);
        x[j * R0 + n] = v;
      }
  }

  // decimation in frequency: butterfly, then the twiddle W_N^(k mi) (its
  // conjugate for the inverse direction)
  static_for_up<0, P>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int R = Gm::R[I];
    if constexpr (I > 0) exchange<Gm, I - 1, I, flips<Gm>(0, I - 1) & 1>(x, buf0, buf1, t);
#pragma unroll
    for (int j = 0; j < Gm::B(I); ++j) {
      dft<DIR, R>(&x[j * R]);
      if constexpr (I < P - 1) {
        constexpr int N = R * Gm::S(I);
        const int mi = stage_suffix<Gm, I>(t, j);
#pragma unroll
        for (int k = 1; k < R; ++k) {
          const c32 w = ldg(tw + (k * mi) * (L / N));
          x[j * R + k] = DIR < 0 ? cmul(x[j * R + k], w) : cmulc(x[j * R + k], w);
        }
      }
    }
  });

  // back to natural order: every thread writes the addresses it owns in the
  // last stage's layout (the buffer the preceding exchanges leave free for
  // it), then reads consecutive frequencies
  constexpr int PAR = flips<Gm>(0, P - 1) & 1;
  constexpr int RL = Gm::R[P - 1];
  c32 *buf = PAR ? buf1 : buf0;
#pragma unroll
  for (int j = 0; j < Gm::B(P - 1); ++j)
#pragma unroll
    for (int n = 0; n < RL; ++n) buf[pad<Gm>(stage_addr<Gm, P - 1>(t, j, n))] = x[j * RL + n];
  __syncthreads();
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = t + e * T;
      const c32 v = buf[pad<Gm>(addr_of_freq<Gm>(k))];
      *reinterpret_cast<gptr<f2v>>(out + f * L + k) = f2v{v.x, v.y};
    }
  }
}

template <class Gm, int G>
static hipError_t launch_fft(const void *in, void *out, int64_t batch, int dir, const c32 *tw,
                             hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int64_t blocks = (batch + G - 1) / G;
  if (dir < 0)
    hipLaunchKernelGGL((fft_batch_kernel<Gm, G, -1>), dim3((unsigned)blocks), dim3(Gm::T * G), 0,
                       s, static_cast<const c32 *>(in), static_cast<c32 *>(out), batch, tw);
  else
    hipLaunchKernelGGL((fft_batch_kernel<Gm, G, +1>), dim3((unsigned)blocks), dim3(Gm::T * G), 0,
                       s, static_cast<const c32 *>(in), static_cast<c32 *>(out), batch, tw);
  return hipGetLastError();
}

template <class Gm, int G>
static constexpr FftVariant make_fft(const char *name) {
  return FftVariant{name, Gm::L, Gm::E, Gm::T, G, &launch_fft<Gm, G>};
}

// Name: fft_L<length>_e<elements per thread>_r<radices>[x<transforms per block>]
//       [_1b: one LDS buffer]
// The first entry for a length is its default.
static const FftVariant kFftVariants[] = {
    make_fft<Geo<64, 4, 16, 4>, 32>("fft_L64_e16_r16.4x32"),
    make_fft<Geo<128, 8, 8, 16>, 16>("fft_L128_e16_r8.16x16"),
    make_fft<Geo<256, 16, 16, 16>, 4>("fft_L256_e16_r16.16x4"),
    make_fft<Geo<512, 32, 16, 2, 16>, 4>("fft_L512_e16_r16.2.16x4"),
    make_fft<Geo<512, 32, 2, 16, 16>, 4>("fft_L512_e16_r2.16.16x4"),
    make_fft<Geo<1024, 64, 16, 4, 16>, 2>("fft_L1024_e16_r16.4.16x2"),
    make_fft<Geo<1024, 64, 4, 16, 16>, 4>("fft_L1024_e16_r4.16.16x4"),
    make_fft<Geo<1024, 64, 16, 8, 8>, 2>("fft_L1024_e16_r16.8.8x2"),
    make_fft<Geo<1024, 512, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2>, 1>("fft_L1024_e2_r2^10"),
    make_fft<Geo<1024, 256, 4, 4, 4, 4, 4>, 1>("fft_L1024_e4_r4^5"),
    make_fft<Geo<1024, 128, 2, 8, 8, 8>, 2>("fft_L1024_e8_r2.8.8.8x2"),
    make_fft<OneBuf<Geo<2048, 128, 16, 8, 16>>, 1>("fft_L2048_e16_r16.8.16x1_1b"),
    make_fft<OneBuf<Geo<2048, 128, 16, 8, 16>>, 2>("fft_L2048_e16_r16.8.16x2_1b"),
    make_fft<Geo<2048, 128, 8, 16, 16>, 2>("fft_L2048_e16_r8.16.16x2"),
    make_fft<OneBuf<Geo<4096, 256, 16, 16, 16>>, 1>("fft_L4096_e16_r16.16.16_1b"),
    make_fft<Geo<4096, 256, 16, 16, 16>, 1>("fft_L4096_e16_r16.16.16"),
};

const FftVariant *fft_variants(int *count) {
  *count = (int)(sizeof(kFftVariants) / sizeof(kFftVariants[0]));
  return kFftVariants;
}

}  // namespace fdas
