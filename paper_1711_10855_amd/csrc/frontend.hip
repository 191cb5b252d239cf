// Front end on the device: real time series -> normalised complex spectrum.
//
// The correlation (Section 1, eq. 2) runs on the Fourier spectrum of the
// observation. This file produces it from a real series of n = 2M samples
// without leaving the device:
//   1. z[j] = x[2j] + i x[2j+1] (the series read as M complex values) is
//      transformed with the batched shared-memory FFT: one transform when M
//      is a compiled length, else the four-step split M = N1 N2 (transforms
//      of length N1 over one index, the twiddles W_M^(n2 k1), transforms of
//      length N2 over the other) with tiled LDS transposes between;
//   2. the real-input split A[k] = E[k] + W_n^k O[k], with
//      E = (Z[k] + conj Z[M-k]) / 2 and O = (Z[k] - conj Z[M-k]) / 2i,
//      gives bins 0 .. M-1 of the real transform (eq. 3 sign; the Nyquist bin
//      is not formed), and |A[k]|^2;
//   3. the median of |A[k]|^2 over bins 1 .. M-1 (an odd count, M being a
//      power of two) by a three-pass radix select on the bit patterns
//      (non-negative floats order as unsigned integers);
//   4. A[k] *= sqrt(ln 2 / median) (unit mean noise power; unscaled when the
//      median is 0) and A[0] = 0.
// Every step is a kernel on the caller's stream; nothing returns to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "fft_batch.hpp"
#include "fft_radix.hpp"
#include "frontend.hpp"

namespace fdas {

constexpr int kSelBins = 2048;  // widest radix-select digit (11 bits)

struct SelState {
  unsigned prefix;  // selected high bits of the order statistic
  unsigned mask;    // bits fixed so far
  unsigned rank;    // remaining rank inside the current prefix
  unsigned pad;
  unsigned hist[kSelBins];
};

// [rows][cols] -> [cols][rows], with out[c][r] = in[r][c] * W_M^(r c) when TW
// (forward sign). 32 x 32 tiles through LDS; rows and cols are multiples of 32.
template <bool TW>
__global__ void __launch_bounds__(256)
    transpose_kernel(const c32 *__restrict__ in_, c32 *__restrict__ out_, int rows, int cols,
                     float inv_m2) {
  __shared__ c32 tile[32][33];
  const auto in = to_global(in_);
  const auto out = to_global(out_);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
#pragma unroll
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + i, c = c0 + tx;
    if (r < rows && c < cols) tile[i][tx] = ldg(in + (int64_t)r * cols + c);
  }
  __syncthreads();
#pragma unroll
  for (int i = ty; i < 32; i += 8) {
    const int c = c0 + i, r = r0 + tx;
    if (r < rows && c < cols) {
      c32 v = tile[tx][i];
      if constexpr (TW) {
        // r c < M <= 2^24 is exact in FP32, and so is the scaled argument
        float sn, cs;
        sincospif(-(float)(r * c) * inv_m2, &sn, &cs);
        v = cmul(v, c32{cs, sn});
      }
      *reinterpret_cast<gptr<f2v>>(out + (int64_t)c * rows + r) = f2v{v.x, v.y};
    }
  }
}

// Bins 0 .. M-1 of the real transform from the M-point transform Z of the
// packed series, and their powers.
__global__ void __launch_bounds__(256)
    r2c_split_kernel(const c32 *__restrict__ Z_, c32 *__restrict__ A_, float *__restrict__ P_,
                     int64_t M, float inv_m) {
  const auto Z = to_global(Z_);
  const auto A = to_global(A_);
  const auto P = to_global(P_);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const c32 a = ldg(Z + k);
  const c32 bb = ldg(Z + ((M - k) & (M - 1)));
  const c32 b = {bb.x, -bb.y};  // conj Z[M-k]
  const c32 e = {0.5f * (a.x + b.x), 0.5f * (a.y + b.y)};
  const c32 o = {0.5f * (a.y - b.y), -0.5f * (a.x - b.x)};  // (a - b) / 2i
  float sn, cs;
  sincospif(-(float)k * inv_m, &sn, &cs);  // W_n^k = exp(-2 pi i k / 2M), k < 2^24 exact
  const c32 w = cmul(o, c32{cs, sn});
  const c32 r = {e.x + w.x, e.y + w.y};
  *reinterpret_cast<gptr<f2v>>(A + k) = f2v{r.x, r.y};
  P[k] = __builtin_fmaf(r.x, r.x, r.y * r.y);
}

__global__ void __launch_bounds__(256) sel_init_kernel(SelState *st, unsigned rank) {
  for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) st->hist[i] = 0u;
  if (threadIdx.x == 0) {
    st->prefix = 0u;
    st->mask = 0u;
    st->rank = rank;
  }
}

// Histogram of the next digit of the elements that match the prefix.
__global__ void __launch_bounds__(256)
    sel_hist_kernel(const float *__restrict__ P_, int64_t count, SelState *__restrict__ st,
                    int shift, int nb) {
  __shared__ unsigned h[kSelBins];
  const auto P = to_global(reinterpret_cast<const unsigned *>(P_));
  for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const unsigned mask = st->mask, prefix = st->prefix;
  const unsigned dm = (unsigned)nb - 1u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned u = P[i];
    if ((u & mask) == prefix) atomicAdd(&h[(u >> shift) & dm], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    const unsigned v = h[i];
    if (v) atomicAdd(&st->hist[i], v);
  }
}

// Choose the digit that holds the rank; clear the histogram for the next
// pass. One block of 256 threads; the histogram is staged in LDS so the
// serial part of the scan touches LDS only.
__global__ void __launch_bounds__(256) sel_pick_kernel(SelState *st, int shift, int nb) {
  __shared__ unsigned hh[kSelBins];
  __shared__ unsigned part[256];
  const int per = nb / 256;
  const int t = threadIdx.x;
  unsigned sum = 0u;
  for (int j = 0; j < per; ++j) {
    const unsigned v = st->hist[t * per + j];
    hh[t * per + j] = v;
    sum += v;
  }
  part[t] = sum;
  __syncthreads();
  for (int j = 0; j < per; ++j) st->hist[t * per + j] = 0u;
  if (t == 0) {
    const unsigned rank = st->rank;
    unsigned below = 0u;
    int chunk = 0;
    while (chunk < 255 && below + part[chunk] <= rank) below += part[chunk++];
    int d = chunk * per;
    while (d < chunk * per + per - 1 && below + hh[d] <= rank) below += hh[d++];
    st->prefix |= (unsigned)d << shift;
    st->rank = rank - below;
    st->mask |= ((unsigned)nb - 1u) << shift;
  }
}

// A[k] *= sqrt(ln 2 / median), A[0] = 0; stats = (scale, median) if given.
__global__ void __launch_bounds__(256)
    normalise_kernel(c32 *__restrict__ A_, int64_t M, const SelState *__restrict__ st,
                     float *__restrict__ stats) {
  const auto A = to_global(A_);
  const double med = (double)__uint_as_float(st->prefix);
  const float s = med > 0.0 ? (float)sqrt(0.69314718055994530942 / med) : 1.0f;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && stats) {
    stats[0] = s;
    stats[1] = (float)med;
  }
  if (k >= M) return;
  c32 v = ldg(A + k);
  v = k == 0 ? c32{0.f, 0.f} : c32{v.x * s, v.y * s};
  *reinterpret_cast<gptr<f2v>>(A + k) = f2v{v.x, v.y};
}

size_t frontend_sel_bytes() { return sizeof(SelState); }

hipError_t launch_frontend(const FrontendGeom &g, const float *series, c32 *spectrum, c32 *work,
                           float *pw, void *sel_, float *stats, hipStream_t s) {
  SelState *sel = static_cast<SelState *>(sel_);
  const int64_t M = g.M;
  const c32 *z = reinterpret_cast<const c32 *>(series);
  hipError_t e = hipSuccess;
  if (g.N2 == 1) {
    e = g.f1->launch(z, work, 1, -1, g.tw1, s);
  } else {
    // z as [N1][N2] (j = N2 n1 + n2) -> [N2][N1]; transforms over n1
    hipLaunchKernelGGL(transpose_kernel<false>, dim3(g.N2 / 32, g.N1 / 32), dim3(256), 0, s, z,
                       work, g.N1, g.N2, 0.f);
    e = hipGetLastError();
    if (e == hipSuccess) e = g.f1->launch(work, work, g.N2, -1, g.tw1, s);
    // twiddle W_M^(n2 k1), [N2][N1] -> [N1][N2]; transforms over n2
    if (e == hipSuccess) {
      hipLaunchKernelGGL(transpose_kernel<true>, dim3(g.N1 / 32, g.N2 / 32), dim3(256), 0, s,
                         work, spectrum, g.N2, g.N1, 2.0f / (float)M);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = g.f2->launch(spectrum, spectrum, g.N1, -1, g.tw2, s);
    // X[k1 + N1 k2] sits at [k1][k2]: back to natural order
    if (e == hipSuccess) {
      hipLaunchKernelGGL(transpose_kernel<false>, dim3(g.N2 / 32, g.N1 / 32), dim3(256), 0, s,
                         spectrum, work, g.N1, g.N2, 0.f);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((M + 255) / 256);
  hipLaunchKernelGGL(r2c_split_kernel, dim3(blocks), dim3(256), 0, s, work, spectrum, pw, M,
                     1.0f / (float)M);
  // median of bins 1 .. M-1: M is a power of two, so the count is odd and the
  // median is the single middle order statistic
  const int64_t cnt = M - 1;
  hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, s, sel, (unsigned)(cnt / 2));
  const int shifts[3] = {21, 10, 0}, widths[3] = {2048, 2048, 1024};
  const unsigned hblocks = (unsigned)std::min<int64_t>(1024, (cnt + 255) / 256);
  for (int pass = 0; pass < 3; ++pass) {
    hipLaunchKernelGGL(sel_hist_kernel, dim3(hblocks), dim3(256), 0, s, pw + 1, cnt, sel,
                       shifts[pass], widths[pass]);
    hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(256), 0, s, sel, shifts[pass],
                       widths[pass]);
  }
  hipLaunchKernelGGL(normalise_kernel, dim3(blocks), dim3(256), 0, s, spectrum, M, sel, stats);
  return hipGetLastError();
}

}  // namespace fdas
