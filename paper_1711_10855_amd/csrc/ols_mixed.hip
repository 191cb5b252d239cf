// Mixed-precision overlap-and-save correlation kernel for gfx950: 16-bit
// storage (FP16 or BF16), the inverse-FFT stages run as 16 x 16 complex DFT
// matrices on the matrix cores (v_mfma_f32_16x16x32_{f16,bf16}) with FP32
// accumulation, twiddles and |.|^2 in FP32.
//
// Segment length L = 4096 = 16^3. Per segment (one block of four waves):
//   forward FFT in FP32 (radix 16, registers + LDS, as in the FP32 kernel),
//   per-segment power-of-two scale so the largest component is in [4, 8),
//   X stored once in LDS as two 16-bit planes (re, im);
//   per template: Y = X * T' (packed 16-bit arithmetic; T' = L * T, the
//   bank without the 1/L, stored as 16-bit planes), then three inverse
//   radix-16 stages (decimation in time, natural-order output).
// Each stage processes tiles of 16 butterflies. A tile is one MFMA pair
// D = A * B: A holds the butterflies as rows and the 16 input values as K
// (8 real | 8 real | 8 imaginary | 8 imaginary per lane group), B is the DFT
// matrix in real form ([Re F | -Im F] and [Im F | Re F]), D gives each lane
// four consecutive rows of one output column. Rows of stage s are chosen as
// the digit that stage s+1 transforms, so a lane's four outputs are four
// consecutive inputs of the next stage and go to LDS as one 8-byte write.
//
// With digits k = k0 + 16 k1 + 256 k2 (frequency) and n = 256 n0 + 16 n1 + n2
// (output), the inverse DFT (eq. 3 with the opposite sign, unnormalised) is
//   y[n] = sum_k0 w16^(n0 k0) w256^(n1 k0) w4096^(n2 k0)
//          sum_k1 w16^(n1 k1) w256^(n2 k1) sum_k2 w16^(n2 k2) Y[k],
// with wN = exp(+2 pi i / N). Stage 2': tile k0, rows k1, columns n2, then
// twiddle w256^(k1 n2). Stage 1': tile n2, rows k0, columns n1, then
// twiddle w4096^(k0 n2). Stage 0': tile n1, rows n2, columns n0, with the
// factor w256^(n1 k0) folded into that tile's B matrix.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fft_radix.hpp"
#include "ols_variants.hpp"

namespace fdas {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 hf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 hf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

template <class H>
struct Vec;
template <>
struct Vec<_Float16> {
  typedef hf8 v8;
  typedef hf4 v4;
  static __device__ __forceinline__ f4 mfma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Vec<__bf16> {
  typedef bf8 v8;
  typedef bf4 v4;
  static __device__ __forceinline__ f4 mfma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// One LDS buffer: two planes (re, im) of 256 rows x 16 values. Row r starts
// at r*16 + (r/16)*8 halves; the two 8-value chunks of a row are swapped
// when bit 3 of the row is set. Reads of one chunk by 16 consecutive rows and
// writes of 4 values by rows 16 apart are then free of bank conflicts.
constexpr int kPlane = 256 * 16 + 16 * 8;  // halves per plane

__device__ __forceinline__ int lds_idx(int row, int e) {
  return row * 16 + (row >> 4) * 8 + ((((e >> 3) ^ (row >> 3)) & 1) << 3) + (e & 7);
}

// exp(+2 pi i num / den) in FP32 for 0 <= num < den (den a power of two)
__device__ __forceinline__ c32 wpos(int num, int den) {
  float s, c;
  sincospif(2.0f * (float)num / (float)den, &s, &c);
  return {c, s};
}

// Real-form B operand of lane l for the 16-point matrix M[c][k] = exp(2 pi i
// k (16 c + phase) / 256): re (B1 = [Re M | -Im M]) and im (B2 = [Im M | Re M]).
template <class H>
__device__ __forceinline__ void make_b(int lane, int phase, typename Vec<H>::v8 &b1,
                                       typename Vec<H>::v8 &b2) {
  const int c = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kk = kg * 8 + j;  // 0..31
    const int k = kk & 15;
    const c32 w = wpos((k * (16 * c + phase)) & 255, 256);
    if (kk < 16) {
      b1[j] = (H)w.x;
      b2[j] = (H)w.y;
    } else {
      b1[j] = (H)(-w.y);
      b2[j] = (H)w.x;
    }
  }
}

template <class H>
__device__ __forceinline__ void store4(H *plane, int row, int e0, float a, float b, float c,
                                       float d) {
  typename Vec<H>::v4 v = {(H)a, (H)b, (H)c, (H)d};
  *reinterpret_cast<typename Vec<H>::v4 *>(plane + lds_idx(row, e0)) = v;
}

template <class H>
__device__ __forceinline__ typename Vec<H>::v8 load8(const H *plane, int row, int e0) {
  return *reinterpret_cast<const typename Vec<H>::v8 *>(plane + lds_idx(row, e0));
}

// forward FFT geometry: 4096 = 16 * 16 * 16 over 256 threads (as the FP32 kernel)
constexpr int kT = 256;

template <int I>
__device__ __forceinline__ int fwd_addr(int t, int n) {
  constexpr int S = I == 0 ? 256 : (I == 1 ? 16 : 1);
  const int prefix = t / S, mi = t % S;
  return prefix * 16 * S + n * S + mi;
}
__device__ __forceinline__ int fpad(int a) { return a + (a >> 4); }

template <class H, bool PF, bool NT>
__global__ void __launch_bounds__(256)
    ols_mixed4096_kernel(const c32 *__restrict__ spec, int64_t nbins, const H *__restrict__ bank,
                         const c32 *__restrict__ tw, float *__restrict__ power, int64_t ld,
                         int nseg, int U, int half, int nz, int zpb, int nsb, int bank_log2) {
  typedef typename Vec<H>::v8 v8;
  constexpr int L = 4096;
  // LDS: the FP32 forward exchange buffer is dead once X is written, so it
  // shares storage with the three 16-bit buffers (X, Ea, Eb).
  constexpr int kF32 = (L + L / 16) * 8;
  constexpr int k16 = 3 * 2 * kPlane * 2;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kF32 > k16 ? kF32 : k16];
  __shared__ float s_max[4];
  c32 *fbuf = reinterpret_cast<c32 *>(smem);
  H *Xp = reinterpret_cast<H *>(smem);
  H *Ea = Xp + 2 * kPlane;
  H *Eb = Ea + 2 * kPlane;

  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int g = lane >> 4, c = lane & 15, h = g & 1;
  const int sb = blockIdx.x % nsb;
  const int zg = blockIdx.x / nsb;
  const int s = sb;
  const bool active = s < nseg;
  const int64_t seg0 = (int64_t)s * U - half;
  const int z0 = zg * zpb;
  const int z1 = min(nz, z0 + zpb);

  // ---- forward FFT, FP32, decimation in frequency -------------------------
  c32 x[16];
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    const int64_t gi = seg0 + n * 256 + t;
    c32 v = {0.f, 0.f};
    if (active && gi >= 0 && gi < nbins) v = spec[gi];
    x[n] = v;
  }
  dft<-1, 16>(x);
#pragma unroll
  for (int k = 1; k < 16; ++k) x[k] = cmul(x[k], tw[k * t]);  // W_4096^(k m), m = t
#pragma unroll
  for (int n = 0; n < 16; ++n) fbuf[fpad(fwd_addr<0>(t, n))] = x[n];
  __syncthreads();
#pragma unroll
  for (int n = 0; n < 16; ++n) x[n] = fbuf[fpad(fwd_addr<1>(t, n))];
  dft<-1, 16>(x);
  {
    const int mi = t % 16;
#pragma unroll
    for (int k = 1; k < 16; ++k) x[k] = cmul(x[k], tw[(k * mi) * 16]);  // W_256^(k m)
  }
  __syncthreads();
#pragma unroll
  for (int n = 0; n < 16; ++n) fbuf[fpad(fwd_addr<1>(t, n))] = x[n];
  __syncthreads();
#pragma unroll
  for (int n = 0; n < 16; ++n) x[n] = fbuf[fpad(fwd_addr<2>(t, n))];
  dft<-1, 16>(x);
  // thread t now holds X[k0 + 16 k1 + 256 e] with t = 16 k0 + k1

  // per-segment scale: largest component into [4, 8)
  float mx = 0.f;
#pragma unroll
  for (int e = 0; e < 16; ++e) mx = fmaxf(mx, fmaxf(fabsf(x[e].x), fabsf(x[e].y)));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if (lane == 0) s_max[w] = mx;
  __syncthreads();  // also: every forward read of fbuf is complete
  mx = fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
  int ex = 0;
  if (mx > 0.f) (void)frexpf(mx, &ex);
  const float xscale = ldexpf(1.0f, 3 - ex);
  // power = |y'|^2 * 2^(-2 (a + b)) with a = 3 - ex, b = bank_log2
  const float pscale = ldexpf(1.0f, -2 * (3 - ex + bank_log2));
#pragma unroll
  for (int e0 = 0; e0 < 16; e0 += 4) {
    store4<H>(Xp, t, e0, x[e0].x * xscale, x[e0 + 1].x * xscale, x[e0 + 2].x * xscale,
              x[e0 + 3].x * xscale);
    store4<H>(Xp + kPlane, t, e0, x[e0].y * xscale, x[e0 + 1].y * xscale, x[e0 + 2].y * xscale,
              x[e0 + 3].y * xscale);
  }

  // ---- per-lane constants ----------------------------------------------------
  v8 bF1, bF2;  // plain inverse DFT16 (phase 0)
  make_b<H>(lane, 0, bF1, bF2);
  v8 bT1[4], bT2[4];  // stage 0' tiles n1 = 4w + j: factor w256^(n1 k0) folded in
#pragma unroll
  for (int j = 0; j < 4; ++j) make_b<H>(lane, 4 * w + j, bT1[j], bT2[j]);
  c32 tw1[4];     // after stage 2': w256^(k1 n2), k1 = 4g + i, n2 = c
  c32 tw2[4][4];  // after stage 1': w4096^(k0 n2), k0 = 4g + i, n2 = 4w + j
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    tw1[i] = wpos(((4 * g + i) * c) & 255, 256);
#pragma unroll
    for (int j = 0; j < 4; ++j) tw2[j][i] = wpos(((4 * g + i) * (4 * w + j)) & 4095, 4096);
  }
  __syncthreads();  // X complete

  const H *Xre = Xp, *Xim = Xp + kPlane;
  // bank rows are read one template ahead (tiles k0 = 4w + j, rows 16 k0 + c, chunk h)
  v8 btr[4], bti[4];
  auto load_bank = [&](int iz) {
    const H *brow = bank + (int64_t)iz * (2 * L);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 16 * (4 * w + j) + c;
      btr[j] = *reinterpret_cast<const v8 *>(brow + row * 16 + 8 * h);
      bti[j] = *reinterpret_cast<const v8 *>(brow + L + row * 16 + 8 * h);
    }
  };
  if (PF && z0 < z1) load_bank(z0);
  const bool re_lane = g < 2;
  for (int iz = z0; iz < z1; ++iz) {
    if (!PF) load_bank(iz);
    // ---- product + stage 2' (tiles k0 = 4w + j; rows k1 = c; chunk h) ----
    v8 av[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 16 * (4 * w + j) + c;
      const v8 xr = load8<H>(Xre, row, 8 * h);
      const v8 xi = load8<H>(Xim, row, 8 * h);
      // re lanes: xr*tr - xi*ti ; im lanes: xr*ti + xi*tr
      const v8 u = re_lane ? btr[j] : bti[j];
      const v8 v = re_lane ? -bti[j] : btr[j];
      av[j] = xr * u + xi * v;
    }
    if (PF && iz + 1 < z1) load_bank(iz + 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k0 = 4 * w + j;
      f4 zero = {0.f, 0.f, 0.f, 0.f};
      const f4 dr = Vec<H>::mfma(av[j], bF1, zero);
      const f4 di = Vec<H>::mfma(av[j], bF2, zero);
      // lane holds rows k1 = 4g + i, column n2 = c
      float orr[4], oii[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const c32 v = cmul({dr[i], di[i]}, tw1[i]);
        orr[i] = v.x;
        oii[i] = v.y;
      }
      const int orow = 16 * c + k0;  // stage 1' butterfly (k0, n2 = c)
      store4<H>(Ea, orow, 4 * g, orr[0], orr[1], orr[2], orr[3]);
      store4<H>(Ea + kPlane, orow, 4 * g, oii[0], oii[1], oii[2], oii[3]);
    }
    __syncthreads();
    // ---- stage 1' (tiles n2 = 4w + j; rows k0 = c) ---------------------------
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n2 = 4 * w + j;
      const int row = 16 * n2 + c;
      const v8 a = load8<H>(Ea + (g >> 1) * kPlane, row, 8 * h);
      f4 zero = {0.f, 0.f, 0.f, 0.f};
      const f4 dr = Vec<H>::mfma(a, bF1, zero);
      const f4 di = Vec<H>::mfma(a, bF2, zero);
      // lane holds rows k0 = 4g + i, column n1 = c
      float orr[4], oii[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const c32 v = cmul({dr[i], di[i]}, tw2[j][i]);
        orr[i] = v.x;
        oii[i] = v.y;
      }
      const int orow = 16 * c + n2;  // stage 0' butterfly (n1 = c, n2)
      store4<H>(Eb, orow, 4 * g, orr[0], orr[1], orr[2], orr[3]);
      store4<H>(Eb + kPlane, orow, 4 * g, oii[0], oii[1], oii[2], oii[3]);
    }
    __syncthreads();
    // ---- stage 0' (tiles n1 = 4w + j; rows n2 = c) + |.|^2 --------------------
    float *prow = power + (int64_t)iz * ld;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n1 = 4 * w + j;
      const int row = 16 * n1 + c;
      const v8 a = load8<H>(Eb + (g >> 1) * kPlane, row, 8 * h);
      f4 zero = {0.f, 0.f, 0.f, 0.f};
      const f4 dr = Vec<H>::mfma(a, bT1[j], zero);
      const f4 di = Vec<H>::mfma(a, bT2[j], zero);
      // lane holds y[256 c + 16 n1 + 4g + i], i = 0..3: one 16-byte store;
      // the four lane groups of a column write 64 contiguous bytes
      if (active) {
        const int o0 = 256 * c + 16 * n1 + 4 * g;
        const int64_t r0 = (int64_t)s * U + o0 - half;
        f4 pw;
#pragma unroll
        for (int i = 0; i < 4; ++i) pw[i] = (dr[i] * dr[i] + di[i] * di[i]) * pscale;
        if (o0 >= half && o0 + 3 < half + U && r0 + 3 < nbins && ((r0 + iz * ld) & 3) == 0) {
          if constexpr (NT) __builtin_nontemporal_store(pw, reinterpret_cast<f4 *>(prow + r0));
          else *reinterpret_cast<f4 *>(prow + r0) = pw;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int o = o0 + i;
            if (o >= half && o < half + U && r0 + i < nbins) prow[r0 + i] = pw[i];
          }
        }
      }
    }
  }
}

template <class H, bool PF, bool NT>
static hipError_t launch_mixed4096(const OlsArgs &a, hipStream_t st) {
  const int nsb = a.nseg;
  const int nzg = (a.nz + a.zpb - 1) / a.zpb;
  const long blocks = (long)nsb * nzg;
  hipLaunchKernelGGL((ols_mixed4096_kernel<H, PF, NT>), dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const c32 *>(a.spec), a.nbins, static_cast<const H *>(a.bank),
                     static_cast<const c32 *>(a.tw), a.power, a.ld, a.nseg, a.U, a.half, a.nz,
                     a.zpb, nsb, a.bank_log2);
  return hipGetLastError();
}

template <class H, bool PF = false, bool NT = true>
static OlsVariant make_mixed(const char *name, int precision) {
  OlsVariant v{};
  v.name = name;
  v.L = 4096;
  v.T = 256;
  v.G = 1;
  v.nbuf = 1;
  v.precision = precision;
  v.lay.L = 4096;
  v.lay.T = 256;
  v.lay.E = 16;
  v.lay.P = 3;
  v.lay.R[0] = v.lay.R[1] = v.lay.R[2] = 16;
  for (int i = 3; i < kMaxStages; ++i) v.lay.R[i] = 1;
  v.lds_bytes = 0;
  v.launch = &launch_mixed4096<H, PF, NT>;
  v.launch_batch = nullptr;
  v.batch_blocks_per_cu = nullptr;
  return v;
}

static const OlsVariant kMixedVariants[] = {
    make_mixed<_Float16>("fp16_L4096_mfma_r16.16.16", 1),
    make_mixed<_Float16, true, true>("fp16_L4096_mfma_r16.16.16_pf", 1),
    make_mixed<_Float16, false, false>("fp16_L4096_mfma_r16.16.16_ts", 1),
    make_mixed<__bf16>("bf16_L4096_mfma_r16.16.16", 2),
};

const OlsVariant *mixed_variants(int *count) {
  *count = (int)(sizeof(kMixedVariants) / sizeof(kMixedVariants[0]));
  return kMixedVariants;
}

// ---- plan-time: 16-bit planar bank in the X layout ------------------------
// bank[i][plane][row*16 + k2] with row = 16 k0 + k1 for frequency
// k = k0 + 16 k1 + 256 k2; value conj(FFT_L(h_i))[k] (no 1/L; the kernel
// removes the factor 2^bank_log2 = L from the power).
struct c64m {
  double x, y;
};

template <class H>
__global__ void bank_mixed_kernel(H *__restrict__ bank, const c64m *__restrict__ h, int nz, int m,
                                  int L) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nz * L) return;
  const int i = (int)(idx / L);
  const int slot = (int)(idx % L);  // row*16 + k2
  const int row = slot >> 4, k2 = slot & 15;
  const int k = (row >> 4) + 16 * (row & 15) + 256 * k2;
  const c64m *hi = h + (long)i * (m + 1);
  double sr = 0.0, si = 0.0;
  for (int j = 0; j <= m; ++j) {
    const int q = j - m / 2;
    const int qm = ((q % L) + L) % L;
    const long ph = ((long)qm * k) % L;
    double sn, cs;
    sincospi(-2.0 * (double)ph / (double)L, &sn, &cs);
    const c64m v = hi[j];
    sr += v.x * cs - v.y * sn;
    si += v.x * sn + v.y * cs;
  }
  H *row_i = bank + (long)i * 2 * L;
  row_i[slot] = (H)sr;
  row_i[L + slot] = (H)(-si);
}

template <class H>
__global__ void bank_mixed_natural_kernel(c32 *__restrict__ dst, const H *__restrict__ bank,
                                          int nz, int L) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nz * L) return;
  const int i = (int)(idx / L);
  const int slot = (int)(idx % L);
  const int row = slot >> 4, k2 = slot & 15;
  const int k = (row >> 4) + 16 * (row & 15) + 256 * k2;
  const H *row_i = bank + (long)i * 2 * L;
  const float inv = 1.0f / (float)L;
  dst[(long)i * L + k] = {(float)row_i[slot] * inv, (float)row_i[L + slot] * inv};
}

hipError_t launch_bank_mixed(void *bank, const void *h, int nz, int m, int L, int precision,
                             hipStream_t s) {
  const long n = (long)nz * L;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (precision == 2)
    hipLaunchKernelGGL(bank_mixed_kernel<__bf16>, grid, dim3(256), 0, s,
                       static_cast<__bf16 *>(bank), static_cast<const c64m *>(h), nz, m, L);
  else
    hipLaunchKernelGGL(bank_mixed_kernel<_Float16>, grid, dim3(256), 0, s,
                       static_cast<_Float16 *>(bank), static_cast<const c64m *>(h), nz, m, L);
  return hipGetLastError();
}

hipError_t launch_bank_mixed_natural(c32 *dst, const void *bank, int nz, int L, int precision,
                                     hipStream_t s) {
  const long n = (long)nz * L;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (precision == 2)
    hipLaunchKernelGGL(bank_mixed_natural_kernel<__bf16>, grid, dim3(256), 0, s, dst,
                       static_cast<const __bf16 *>(bank), nz, L);
  else
    hipLaunchKernelGGL(bank_mixed_natural_kernel<_Float16>, grid, dim3(256), 0, s, dst,
                       static_cast<const _Float16 *>(bank), nz, L);
  return hipGetLastError();
}

}  // namespace fdas
