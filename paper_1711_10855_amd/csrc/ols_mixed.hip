// Mixed-precision overlap-and-save correlation kernel for gfx950: 16-bit
// storage (FP16 or BF16), the inverse-FFT stages run as 16 x 16 complex DFT
// matrices on the matrix cores (v_mfma_f32_16x16x32_{f16,bf16}) with FP32
// accumulation, |.|^2 in FP32.
//
// Segment length L = 4096 = 16^3. One block of NW waves (TPW = 16 / NW tiles
// per wave and stage) takes one segment and a group of templates:
//   forward FFT in FP32 (radix 16, registers + LDS, as in the FP32 kernel),
//   per-segment power-of-two scale so the largest component is in [4, 8)
//   (FP16; BF16, with FP32's exponent range, takes a fixed scale),
//   X rounded to 16 bits and kept in registers (the lanes' operand chunks);
//   per template: Y = X * T' (packed 16-bit arithmetic; T' = L * T, the
//   bank without the 1/L, stored as 16-bit planes), three inverse radix-16
//   stages (decimation in time, natural-order output) exchanging through
//   LDS, |.|^2 staged in LDS and stored one template later as contiguous
//   1 KB pieces.
// Each stage processes tiles of 16 butterflies. A tile is one MFMA pair
// D = A * B: A holds the butterflies as rows and the 16 input values as K
// (8 real | 8 real | 8 imaginary | 8 imaginary per lane group), B is the DFT
// matrix in real form ([Re F | -Im F] and [Im F | Re F]), D gives each lane
// four consecutive rows of one output column. Rows of stage s are chosen as
// the digit that stage s+1 transforms, so a lane's four outputs are four
// consecutive inputs of the next stage and go to LDS as 8-byte writes.
//
// With digits k = k0 + 16 k1 + 256 k2 (frequency) and n = 256 n0 + 16 n1 + n2
// (output), the inverse DFT (eq. 3 with the opposite sign, unnormalised) is
//   y[n] = sum_k0 w16^(n0 k0) w256^(n1 k0) w4096^(n2 k0)
//          sum_k1 w16^(n1 k1) w256^(n2 k1) sum_k2 w16^(n2 k2) Y[k],
// with wN = exp(+2 pi i / N). Stage 2': tile k0, rows k1, K = k2, columns n2.
// Stage 1': tile n2, rows k0, K = k1, columns n1. Stage 0': tile n1, rows n2,
// K = k0, columns n0. Every twiddle depends on one stage's tile and on either
// its K index or its column, never on its row, so each is folded into that
// tile's B matrix: w4096^(n2 k0) into stage 2' (tile k0, column n2),
// w256^(n2 k1) into stage 1' (tile n2, K k1), w256^(n1 k0) into stage 0'
// (tile n1, K k0). The inverse then has no scalar twiddle multiplies at all.
// Stages 1' and 0' use the same family of matrices, P_p[K k][column c] =
// w256^(k (16 c + p)), with p the tile; stage 2' uses
// Q_t[k][c] = w4096^(c (256 k + t)).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <iterator>
#include <type_traits>
#include <vector>

#include "fft_radix.hpp"
#include "cand4.hpp"
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
// at r*16 + (r/16)*8 halves (16 bytes of padding per 16 rows); its two
// 8-value chunks are swapped when bit 2 of the row is set, and the two
// 4-value halves of each chunk when bit 7 is set. Operand reads take one
// 16-byte chunk from 16 consecutive rows; stage outputs are written as
// 8-byte groups of four values to rows 16 apart. With 128 bytes served per
// LDS cycle neither has a bank conflict. A chunk read from a row with bit 7
// set holds its values in the order 4..7, 0..3; rows 16 t + c of tile t
// share that bit (bit 3 of t), and the tile's B matrix and bank rows are
// stored in the same order.
constexpr int kPlane = 256 * 16 + 16 * 8 + 32;  // halves per plane

// Plan-time constants of the L = 4096 mixed kernel: the B operands of the
// two matrix families, [family Q, P][16 tiles][64 lanes][B1, B2][8 x 16-bit].
constexpr int kConstBytes = 2 * 16 * 64 * 2 * 16;

__device__ __forceinline__ int lds_idx(int row, int e) {
  return row * 16 + (row >> 4) * 8 + ((((e >> 3) ^ (row >> 2)) & 1) << 3) +
         ((((e >> 2) ^ (row >> 7)) & 1) << 2) + (e & 3);
}
// start of the chunk that holds values 8h .. 8h+7 of row r
__device__ __forceinline__ int lds_chunk(int row, int h) {
  return row * 16 + (row >> 4) * 8 + (((h ^ (row >> 2)) & 1) << 3);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Two values a, b as 16-bit pairs hi = (round16(a), round16(b)) and
// lo = (round16(a - hi_a), round16(b - hi_b)); the differences are exact in
// FP32. For BF16 the rounded values come back to FP32 from the packed pair
// itself (a BF16 value is the upper half of an FP32 one): a shift and a mask,
// then two subtractions. For FP16 each difference is one two-term dot
// product of the packed pair with (-1, 0) or (0, -1) accumulated onto a or b
// (products and sum exact, so the instruction's rounding does not enter);
// 6% faster on the FP16 split form than two conversions back and two
// subtractions, while on BF16 it measured no faster than the shift and mask.
// Returns {hi, lo}.
template <class H>
__device__ __forceinline__ u32x2 split2(float a, float b) {
  typedef H h2 __attribute__((ext_vector_type(2)));
  const h2 ph = {(H)a, (H)b};
  unsigned hi = __builtin_bit_cast(unsigned, ph);
  float la, lb;
  if constexpr (std::is_same<H, __bf16>::value) {
    // (opaque, or the compiler converts a a second time for the shift)
    asm("" : "+v"(hi));
    la = a - __uint_as_float(hi << 16);
    lb = b - __uint_as_float(hi & 0xffff0000u);
  } else {
    const h2 m0 = {(H)-1.0f, (H)0.0f}, m1 = {(H)0.0f, (H)-1.0f};
    la = __builtin_amdgcn_fdot2(ph, m0, a, false);
    lb = __builtin_amdgcn_fdot2(ph, m1, b, false);
  }
  const h2 pl = {(H)la, (H)lb};
  return {hi, __builtin_bit_cast(unsigned, pl)};
}

// A lane holds four consecutive values (4g .. 4g+3 of row `row` of the next
// stage) of both planes; each plane's four go out as one 8-byte write. With
// SPLIT the buffer has four planes (re hi, im hi, re lo, im lo): each value
// v is stored as hi = round16(v) and lo = round16(v - hi).
template <class H, bool SPLIT>
__device__ __forceinline__ void store_stage(H *buf, int row, int g, const f4 &re,
                                            const f4 &im) {
  typedef typename Vec<H>::v4 v4;
  const int o = lds_idx(row, 4 * g);
  if constexpr (SPLIT) {
    const u32x2 r0 = split2<H>(re[0], re[1]), r1 = split2<H>(re[2], re[3]);
    const u32x2 i0 = split2<H>(im[0], im[1]), i1 = split2<H>(im[2], im[3]);
    const u32x2 rh = {r0[0], r1[0]}, rl = {r0[1], r1[1]};
    const u32x2 ih = {i0[0], i1[0]}, il = {i0[1], i1[1]};
    *reinterpret_cast<u32x2 *>(buf + o) = rh;
    *reinterpret_cast<u32x2 *>(buf + kPlane + o) = ih;
    *reinterpret_cast<u32x2 *>(buf + 2 * kPlane + o) = rl;
    *reinterpret_cast<u32x2 *>(buf + 3 * kPlane + o) = il;
  } else {
    const v4 rh = {(H)re[0], (H)re[1], (H)re[2], (H)re[3]};
    const v4 ih = {(H)im[0], (H)im[1], (H)im[2], (H)im[3]};
    *reinterpret_cast<v4 *>(buf + o) = rh;
    *reinterpret_cast<v4 *>(buf + kPlane + o) = ih;
  }
}

// D = A B with FP32 accumulation; with SPLIT, A = ah + al and B = bh + bl and
// D = ah bh + ah bl + al bh (the lo x lo term is below the FP32 rounding of
// the sum).
template <class H, bool SPLIT>
__device__ __forceinline__ f4 mma(const typename Vec<H>::v8 &ah, const typename Vec<H>::v8 &al,
                                  const typename Vec<H>::v8 &bh, const typename Vec<H>::v8 &bl) {
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  f4 d = Vec<H>::mfma(ah, bh, zero);
  if constexpr (SPLIT) {
    d = Vec<H>::mfma(ah, bl, d);
    d = Vec<H>::mfma(al, bh, d);
  }
  return d;
}

// Values e0 .. e0+7 of row `row` (one plane), as two 8-byte groups.
template <class H>
__device__ __forceinline__ void store8(H *plane, int row, int e0, const c32 *x, bool imag,
                                       float scale) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    typename Vec<H>::v4 v;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (H)((imag ? x[4 * q + k].y : x[4 * q + k].x) * scale);
    *reinterpret_cast<typename Vec<H>::v4 *>(plane + lds_idx(row, e0 + 4 * q)) = v;
  }
}

template <class H>
__device__ __forceinline__ typename Vec<H>::v8 load8(const H *plane, int row, int h) {
  return *reinterpret_cast<const typename Vec<H>::v8 *>(plane + lds_chunk(row, h));
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

constexpr int kMixF32 = (4096 + 4096 / 16) * 8;
// stage buffers Ea, Eb of 2 (4 with SPLIT) planes; the forward buffer aliases them
template <bool SPLIT>
constexpr int mix_stage_bytes() {
  return 2 * (SPLIT ? 4 : 2) * kPlane * 2 > kMixF32 ? 2 * (SPLIT ? 4 : 2) * kPlane * 2 : kMixF32;
}
// Output staging: 16 blocks of 256 powers, each padded by 16 bytes.
constexpr int kStageF = 16 * 260;
// The skewed schedule (PF == 7, unsplit) double-buffers the stage and
// staging buffers: Ea0, Ea1, Eb0, Eb1, then two staging buffers.
constexpr int kSkewStageBytes = 4 * 2 * kPlane * 2;
static_assert(kSkewStageBytes >= kMixF32, "forward buffer fits the skewed stage buffers");
// PF == 8 (the split form skewed the same way) doubles the stage buffers
// and has no staging buffer: the powers go out straight from the lanes.
template <bool SPLIT>
constexpr int kSkewDirectBytes = 4 * (SPLIT ? 4 : 2) * kPlane * 2;
static_assert(kSkewDirectBytes<false> >= kMixF32, "forward buffer fits");
template <bool SPLIT, int PF = 0>
constexpr int mix_smem() {
  return PF == 7   ? kSkewStageBytes + 2 * kStageF * 4
         : PF == 8 ? (kSkewDirectBytes<SPLIT> > mix_stage_bytes<SPLIT>() + kStageF * 4
                          ? kSkewDirectBytes<SPLIT>
                          : mix_stage_bytes<SPLIT>() + kStageF * 4)
                   : mix_stage_bytes<SPLIT>() + kStageF * 4;
}
// With SPLIT, X goes from the forward FFT to the lanes in FP32: 256 rows of
// 16 values padded to 17, placed at Eb (first written by stage 1').
constexpr int kXF32Bytes = 256 * 17 * 8;
static_assert(2 * kPlane * 2 * 2 + kXF32Bytes <= mix_smem<true>(), "X transfer fits");

// Per-lane constants, loaded once per block from the plan-time table: the B
// operands of the wave's TPW tiles in each family (hi parts; with SPLIT also
// the lo parts, B - round16(B)).
template <class H, int NW, bool SPLIT>
struct MixedConsts {
  static constexpr int TPW = 16 / NW;
  static constexpr int NL = SPLIT ? TPW : 1;
  typename Vec<H>::v8 q1[TPW], q2[TPW];  // stage 2' tiles k0 = TPW w + j
  typename Vec<H>::v8 p1[TPW], p2[TPW];  // stage 1' tiles n2 and stage 0' tiles n1 = TPW w + j
  typename Vec<H>::v8 q1l[NL], q2l[NL], p1l[NL], p2l[NL];
};

template <class H, int NW, bool SPLIT>
__device__ __forceinline__ void load_mixed_consts(MixedConsts<H, NW, SPLIT> &K,
                                                  gptr<const unsigned char> consts, int lane,
                                                  int w) {
  typedef typename Vec<H>::v8 v8;
  constexpr int TPW = 16 / NW;
  const gptr<const v8> cb = reinterpret_cast<gptr<const v8>>(consts);
  constexpr int LO = 2 * 16 * 64 * 2;  // v8 entries per part
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int tile = TPW * w + j;
    K.q1[j] = cb[((0 * 16 + tile) * 64 + lane) * 2];
    K.q2[j] = cb[((0 * 16 + tile) * 64 + lane) * 2 + 1];
    K.p1[j] = cb[((1 * 16 + tile) * 64 + lane) * 2];
    K.p2[j] = cb[((1 * 16 + tile) * 64 + lane) * 2 + 1];
    if constexpr (SPLIT) {
      K.q1l[j] = cb[LO + ((0 * 16 + tile) * 64 + lane) * 2];
      K.q2l[j] = cb[LO + ((0 * 16 + tile) * 64 + lane) * 2 + 1];
      K.p1l[j] = cb[LO + ((1 * 16 + tile) * 64 + lane) * 2];
      K.p2l[j] = cb[LO + ((1 * 16 + tile) * 64 + lane) * 2 + 1];
    }
  }
}

// One work unit of the mixed kernel: segment s, bank rows [z0, z1), plane
// rows iz - row_base. Every thread of the block calls it (barriers inside).
template <class H, int PF, bool NT, int NW, bool SPLIT, bool CAND>
__device__ __forceinline__ void mixed_unit(const unsigned char *__restrict__ consts_,
                                           const c32 *__restrict__ spec_, int64_t nbins,
                                           const H *__restrict__ bank_, const c32 *__restrict__ tw_,
                                           float *__restrict__ power_, int64_t ld, int s,
                                           bool active, int U, int half, int z0, int z1,
                                           int row_base, int bank_log2, unsigned char *smem,
                                           float *s_max, const CandOut &cd, int t_in = -1) {
  typedef typename Vec<H>::v8 v8;
  constexpr int L = 4096;
  constexpr int TPW = 16 / NW;
  const auto consts = to_global(consts_);
  const auto spec = to_global(spec_);
  const auto bank = to_global(bank_);
  const auto tw = to_global(tw_);
  const auto power = to_global(power_);
  constexpr int NP = SPLIT ? 4 : 2;  // planes per stage buffer
  c32 *fbuf = reinterpret_cast<c32 *>(smem);
  H *Ea = reinterpret_cast<H *>(smem);
  H *Eb = Ea + NP * kPlane;
  H *Xp = Eb;  // X passes through Eb once; first overwritten by stage 1' of the first template
  c32 *Xf = reinterpret_cast<c32 *>(Eb);  // (SPLIT) the same, in FP32
  float *stg = reinterpret_cast<float *>(smem + mix_stage_bytes<SPLIT>());
  // (the persistent form passes the thread index in; see there)
  const int t = t_in < 0 ? (int)threadIdx.x : t_in;
  const int lane = t & 63, w = t >> 6;
  const int g = lane >> 4, c = lane & 15, h = g & 1;
  const int64_t seg0 = (int64_t)s * U - half;

  // ---- forward FFT, FP32, decimation in frequency, threads 0..255 ---------
  // (threads above 255 only join the barriers)
  const bool fw = t < kT;
  c32 x[16];
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    const int64_t gi = seg0 + n * 256 + t;
    c32 v = {0.f, 0.f};
    if (fw && active && gi >= 0 && gi < nbins) v = ldg(spec + gi);
    x[n] = v;
  }
  if (fw) {
    dft<-1, 16>(x);
#pragma unroll
    for (int k = 1; k < 16; ++k) x[k] = cmul(x[k], ldg(tw + (k * t)));  // W_4096^(k m), m = t < 256
#pragma unroll
    for (int n = 0; n < 16; ++n) fbuf[fpad(fwd_addr<0>(t, n))] = x[n];
  }
  __syncthreads();
  if (fw) {
#pragma unroll
    for (int n = 0; n < 16; ++n) x[n] = fbuf[fpad(fwd_addr<1>(t, n))];
    dft<-1, 16>(x);
    const int mi = t % 16;
#pragma unroll
    for (int k = 1; k < 16; ++k) x[k] = cmul(x[k], ldg(tw + (k * mi) * 16));  // W_256^(k m)
  }
  __syncthreads();
  if (fw) {
#pragma unroll
    for (int n = 0; n < 16; ++n) fbuf[fpad(fwd_addr<1>(t, n))] = x[n];
  }
  __syncthreads();
  if (fw) {
#pragma unroll
    for (int n = 0; n < 16; ++n) x[n] = fbuf[fpad(fwd_addr<2>(t, n))];
    dft<-1, 16>(x);
  }
  // thread t now holds X[k0 + 16 k1 + 256 e] with t = 16 k0 + k1

  // per-segment scale: largest component into [4, 8) (used by FP16)
  float mx = 0.f;
#pragma unroll
  for (int e = 0; e < 16; ++e) mx = fmaxf(mx, fmaxf(fabsf(x[e].x), fabsf(x[e].y)));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if (lane == 0) s_max[w] = mx;
  __syncthreads();  // also: every forward read of fbuf is complete
  mx = 0.f;
#pragma unroll
  for (int k = 0; k < NW; ++k) mx = fmaxf(mx, s_max[k]);
  int ex = 0;
  if (mx > 0.f) (void)frexpf(mx, &ex);
  // BF16 has the exponent range of FP32: X is scaled by 2^-b only, so that
  // y' = y and the power needs no scale.
  constexpr bool kUnit = std::is_same<H, __bf16>::value;
  const float xscale = kUnit ? ldexpf(1.0f, -bank_log2) : ldexpf(1.0f, 3 - ex);
  // power = |y'|^2 * 2^(-2 (a + b)) with a = 3 - ex, b = bank_log2
  const float pscale = ldexpf(1.0f, -2 * (3 - ex + bank_log2));
  if (fw) {
    if constexpr (SPLIT) {
#pragma unroll
      for (int e = 0; e < 16; ++e) Xf[t * 17 + e] = {x[e].x * xscale, x[e].y * xscale};
    } else {
#pragma unroll
      for (int e0 = 0; e0 < 16; e0 += 8) {
        store8<H>(Xp, t, e0, &x[e0], false, xscale);
        store8<H>(Xp + kPlane, t, e0, &x[e0], true, xscale);
      }
    }
  }
  __syncthreads();  // X complete

  // The B operands are loaded only now, so that they do not hold registers
  // during the forward FFT.
  MixedConsts<H, NW, SPLIT> K;
  load_mixed_consts<H, NW, SPLIT>(K, consts, lane, w);

  // X stays in registers for the whole template loop: rows 16 k0 + c of the
  // wave's tiles k0 = TPW w + j, chunk h, both planes (with SPLIT in FP32,
  // in the order the operand chunks use). Lanes g < 2 form the real part of
  // Y = X T, Re X Re T - Im X Im T, and keep -Im X; lanes g >= 2 form
  // Re X Im T + Im X Re T. Both then compute xr * tu + xi * tv from the bank
  // planes (tu, tv) = (Re, Im) or (Im, Re).
  const bool re_lane = g < 2;
  v8 xr[SPLIT ? 1 : TPW], xi[SPLIT ? 1 : TPW];
  float xrf[SPLIT ? TPW : 1][8], xif[SPLIT ? TPW : 1][8];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int row = 16 * (TPW * w + j) + c;
    if constexpr (SPLIT) {
      const int sw = ((row >> 7) & 1) << 2;  // 4-value halves swapped on rows with bit 7 set
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const c32 v = Xf[row * 17 + 8 * h + (i ^ sw)];
        xrf[j][i] = v.x;
        xif[j][i] = re_lane ? -v.y : v.y;
      }
    } else {
      xr[j] = load8<H>(Xp, row, h);
      xi[j] = load8<H>(Xp + kPlane, row, h);
      if (re_lane) xi[j] = -xi[j];
    }
  }

  // Bank planes Re, Im: 16-bit, or with SPLIT in FP32 (the product is formed
  // in FP32 there), in the same slot order. A lane takes the 8 values of its
  // chunk from plane u (Re on lanes g < 2, else Im) and plane v (the other).
  constexpr int RB = 2 * L * (SPLIT ? 4 : 2);  // bytes per bank row
  const int pu = (re_lane ? 0 : 1) * L, pv = (re_lane ? 1 : 0) * L;
  v8 btr[SPLIT ? 1 : TPW], bti[SPLIT ? 1 : TPW];
  f4 sbr[SPLIT ? 2 * TPW : 1], sbi[SPLIT ? 2 * TPW : 1];  // (SPLIT) values 4q .. 4q+3 of tile j in [2j + q]
  // (PF == 5) the same loads through a buffer resource over the bank row (a
  // wave-uniform base), so the lanes' byte offsets stay fixed and no 64-bit
  // address is formed per lane and template. Tile j adds 256 j values.
  constexpr int EB = SPLIT ? 4 : 2;  // bytes per bank value
  const int boff_u = (pu + (16 * (TPW * w) + c) * 16 + 8 * h) * EB;
  const int boff_v = (pv + (16 * (TPW * w) + c) * 16 + 8 * h) * EB;
  auto load_bank_buf = [&](int iz) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<unsigned char *>(reinterpret_cast<const unsigned char *>(bank_)) + (int64_t)iz * RB,
        (short)0, RB, 0x00020000);
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      if constexpr (SPLIT) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          sbr[2 * j + q] = __builtin_bit_cast(
              f4, __builtin_amdgcn_raw_buffer_load_b128(rs, boff_u + 1024 * j + 16 * q, 0, 0));
          sbi[2 * j + q] = __builtin_bit_cast(
              f4, __builtin_amdgcn_raw_buffer_load_b128(rs, boff_v + 1024 * j + 16 * q, 0, 0));
        }
      } else {
        btr[j] = __builtin_bit_cast(v8, __builtin_amdgcn_raw_buffer_load_b128(rs, boff_u + 512 * j, 0, 0));
        bti[j] = __builtin_bit_cast(v8, __builtin_amdgcn_raw_buffer_load_b128(rs, boff_v + 512 * j, 0, 0));
      }
    }
  };
  auto load_bank = [&](int iz) {
    if constexpr ((PF == 5 || PF == 7 || PF == 8) && !CAND) {
      load_bank_buf(iz);
      return;
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int row = 16 * (TPW * w + j) + c;
      if constexpr (SPLIT) {
        const auto frow = reinterpret_cast<gptr<const float>>(bank) + (int64_t)iz * (2 * L);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          sbr[2 * j + q] = *reinterpret_cast<gptr<const f4>>(frow + pu + row * 16 + 8 * h + 4 * q);
          sbi[2 * j + q] = *reinterpret_cast<gptr<const f4>>(frow + pv + row * 16 + 8 * h + 4 * q);
        }
      } else {
        const auto brow = bank + (int64_t)iz * (2 * L);
        btr[j] = *reinterpret_cast<gptr<const v8>>(brow + pu + row * 16 + 8 * h);
        bti[j] = *reinterpret_cast<gptr<const v8>>(brow + pv + row * 16 + 8 * h);
      }
    }
  };

  // Output staging. Stage 0' gives lane (g, c) of tile n1 the powers
  // y[256 c + 16 n1 + 4 g + i], i < 4; they are staged at float
  // 260 c + 16 n1 + 4 g (conflict-free 16-byte writes), and after the next
  // barrier wave w stores outputs [256 TPW w, 256 TPW (w + 1)) of the
  // segment, 1 KB contiguous per store instruction.
  // A unit whose groups of 4 outputs lie wholly inside or wholly outside
  // [half, half + U), below nbins and 16-byte aligned in every row stores one
  // group per lane under a single predicate; others (the ragged last segment,
  // rows not 16-byte aligned, odd m / 2) store element by element.
  const bool vec_ok = half % 4 == 0 && ((int64_t)s * U - half) % 4 == 0 &&
                      (int64_t)(s + 1) * U <= nbins && ld % 4 == 0 &&
                      (reinterpret_cast<uintptr_t>(power_) & 15) == 0;
  // The staged powers of the wave's TPW output blocks (one 16-byte LDS read
  // each), then their stores (or candidate offers).
  auto read_staged_from = [&](f4 *v, const float *sg) {
#pragma unroll
    for (int q = 0; q < TPW; ++q)
      v[q] = *reinterpret_cast<const f4 *>(sg + 260 * (TPW * w + q) + 4 * lane);
  };
  auto read_staged = [&](f4 *v) { read_staged_from(v, stg); };
  // PF == 5 stores through a buffer resource that spans the segment's kept
  // outputs in plane row izr: every lane issues its 16-byte store, and a lane
  // whose group is not kept passes an offset past the resource's end, which
  // the hardware drops. That store is issued on every path (it writes nothing
  // when `none` is set or the unit takes the per-value stores), so every
  // path has at least one store after the bank row loaded before it.
  constexpr int kPast = (int)0x80000000u;
  // the 16-byte store's offset for each of the lane's groups (past the end
  // unless the unit takes 16-byte stores and the group is kept), computed
  // once per unit; through an empty asm statement, so that the store does
  // not get split into copies under the unit's branch on vec_ok (every path
  // must keep it, see below)
  // (PF == 7; PF == 5 computes it at the store, which measured faster there;
  // PF == 8 stores from the stage-0' lanes, whose group of tile
  // n1 = TPW w + q starts at output 256 c + 16 n1 + 4 g)
  int off4[PF == 7 || PF == 8 ? TPW : 1];
  if constexpr (PF == 7 || PF == 8) {
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int o0 = PF == 7 ? 256 * (TPW * w + q) + 4 * lane : 256 * c + 16 * (TPW * w + q) + 4 * g;
      off4[q] = vec_ok && o0 >= half && o0 < half + U ? (o0 - half) * 4 : kPast;
      asm volatile("" : "+v"(off4[q]));
    }
  }
  auto write_staged_buffer = [&](int izr, const f4 *vv, bool none) {
    const int64_t rbase = (int64_t)s * U;  // plane column of segment output `half`
    const int64_t left = nbins - rbase;
    const int nkeep = (int)(left < U ? left : U);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        power_ + (int64_t)(izr - row_base) * ld + rbase, (short)0, nkeep * 4, 0x00020000);
    constexpr int aux = NT ? 2 : 0;  // nontemporal
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int o0 = 256 * (TPW * w + q) + 4 * lane;
      int off;
      if constexpr (PF == 7) {
        off = none ? kPast : off4[q];
      } else {
        const bool keep4 = !none && vec_ok && o0 >= half && o0 < half + U;
        off = keep4 ? (o0 - half) * 4 : kPast;
      }
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, vv[q]), rs, off, 0, aux);
      if (!vec_ok && !none) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int o = o0 + i;
          const bool keep = !none && o >= half && o < half + U && o - half < nkeep;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(vv[q][i]), rs,
                                                keep ? (o - half) * 4 : kPast, 0, aux);
        }
      }
    }
  };
  // (PF == 8) the powers stored by the stage-0' lanes that formed them:
  // lane (g, c) of tile n1 holds outputs 256 c + 16 n1 + 4 g .. + 3, so one
  // store instruction writes 16 runs of 64 bytes, and the neighbouring wave
  // (tile n1 + 1) writes the other half of each 128-byte line.
  auto write_direct = [&](int izr, const f4 *vv, bool none) {
    const int64_t rbase = (int64_t)s * U;
    const int64_t left = nbins - rbase;
    const int nkeep = (int)(left < U ? left : U);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        power_ + (int64_t)(izr - row_base) * ld + rbase, (short)0, nkeep * 4, 0x00020000);
    constexpr int aux = NT ? 2 : 0;  // nontemporal
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int o0 = 256 * c + 16 * (TPW * w + q) + 4 * g;
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, vv[q]), rs,
                                             none ? kPast : off4[q], 0, aux);
      if (!vec_ok && !none) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int o = o0 + i;
          const bool keep = o >= half && o < half + U && o - half < nkeep;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(vv[q][i]), rs,
                                                keep ? (o - half) * 4 : kPast, 0, aux);
        }
      }
    }
  };
  auto write_staged = [&](int izr, const f4 *vv) {
    if (!CAND && !active) return;
    if constexpr ((PF == 5 || PF == 7) && !CAND) {
      write_staged_buffer(izr, vv, false);
      return;
    }
    const auto prow = power + (int64_t)(izr - row_base) * ld;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int blk = TPW * w + q;  // 256-output block of the segment
      const int o0 = 256 * blk + 4 * lane;
      const f4 v = vv[q];
      const int64_t r0 = (int64_t)s * U + o0 - half;
      if constexpr (CAND) {  // detection epilogue instead of the plane (all lanes offer)
        const bool any = v[0] >= cd.thr || v[1] >= cd.thr || v[2] >= cd.thr || v[3] >= cd.thr;
        if (__builtin_amdgcn_ballot_w64(active && any) == 0ull) continue;  // no hit in the wave
        offer4(cd, v, active, o0, half, U, r0, nbins, izr - row_base);
        continue;
      }
      if (vec_ok) {
        if (o0 >= half && o0 < half + U) {
          if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<gptr<f4>>(prow + r0));
          else *reinterpret_cast<gptr<f4>>(prow + r0) = v;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int o = o0 + i;
          if (o >= half && o < half + U && r0 + i < nbins) prow[r0 + i] = v[i];
        }
      }
    }
  };
  auto store_staged = [&](int izr) {
    f4 v[TPW];
    read_staged(v);
    write_staged(izr, v);
  };

  // ---- product + stage 2' (tiles k0 = TPW w + j; rows k1 = c; chunk h) ----
  auto product_stage2_to = [&](H *ea) {
    v8 av[TPW], avl[SPLIT ? TPW : 1];
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      if constexpr (SPLIT) {
        // Y = X T in FP32 from X and T (both FP32), then Y = hi + lo
        float y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float tr = sbr[2 * j + (i >> 2)][i & 3];
          const float ti = sbi[2 * j + (i >> 2)][i & 3];
          y[i] = __builtin_fmaf(xrf[j][i], tr, xif[j][i] * ti);
        }
        u32x4 hi, lo;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const u32x2 p = split2<H>(y[2 * q], y[2 * q + 1]);
          hi[q] = p[0];
          lo[q] = p[1];
        }
        av[j] = __builtin_bit_cast(v8, hi);
        avl[j] = __builtin_bit_cast(v8, lo);
      } else {
        av[j] = xr[j] * btr[j] + xi[j] * bti[j];
      }
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int k0 = TPW * w + j;
      const f4 dr = mma<H, SPLIT>(av[j], avl[SPLIT ? j : 0], K.q1[j], K.q1l[SPLIT ? j : 0]);
      const f4 di = mma<H, SPLIT>(av[j], avl[SPLIT ? j : 0], K.q2[j], K.q2l[SPLIT ? j : 0]);
      // lane holds rows k1 = 4g + i, column n2 = c
      store_stage<H, SPLIT>(ea, 16 * c + k0, g, dr, di);  // stage 1' butterfly (k0, n2 = c)
    }
  };
  auto product_stage2 = [&]() { product_stage2_to(Ea); };
  // ---- stage 1' (tiles n2 = TPW w + j; rows k0 = c) -------------------------
  auto stage1_from = [&](const H *ea, H *eb) {
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int n2 = TPW * w + j;
      const v8 a = load8<H>(ea + (g >> 1) * kPlane, 16 * n2 + c, h);
      const v8 al = SPLIT ? load8<H>(ea + (2 + (g >> 1)) * kPlane, 16 * n2 + c, h) : a;
      const f4 dr = mma<H, SPLIT>(a, al, K.p1[j], K.p1l[SPLIT ? j : 0]);
      const f4 di = mma<H, SPLIT>(a, al, K.p2[j], K.p2l[SPLIT ? j : 0]);
      // lane holds rows k0 = 4g + i, column n1 = c
      store_stage<H, SPLIT>(eb, 16 * c + n2, g, dr, di);  // stage 0' butterfly (n1 = c, n2)
    }
  };
  auto stage1 = [&]() { stage1_from(Ea, Eb); };
  // ---- stage 0' (tiles n1 = TPW w + j; rows n2 = c) + |.|^2 -> staging ----
  auto stage0_from = [&](const H *eb, float *sg) {
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int n1 = TPW * w + j;
      const v8 a = load8<H>(eb + (g >> 1) * kPlane, 16 * n1 + c, h);
      const v8 al = SPLIT ? load8<H>(eb + (2 + (g >> 1)) * kPlane, 16 * n1 + c, h) : a;
      const f4 dr = mma<H, SPLIT>(a, al, K.p1[j], K.p1l[SPLIT ? j : 0]);
      const f4 di = mma<H, SPLIT>(a, al, K.p2[j], K.p2l[SPLIT ? j : 0]);
      f4 pw;
#pragma unroll
      for (int i = 0; i < 4; ++i) pw[i] = kUnit ? dr[i] * dr[i] + di[i] * di[i] : (dr[i] * dr[i] + di[i] * di[i]) * pscale;
      *reinterpret_cast<f4 *>(sg + 260 * c + 16 * n1 + 4 * g) = pw;
    }
  };
  auto stage0 = [&]() { stage0_from(Eb, stg); };
  // (PF == 8) stage 0' with the powers kept in the lanes
  auto stage0_pw = [&](const H *eb, f4 *pw) {
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int n1 = TPW * w + j;
      const v8 a = load8<H>(eb + (g >> 1) * kPlane, 16 * n1 + c, h);
      const v8 al = SPLIT ? load8<H>(eb + (2 + (g >> 1)) * kPlane, 16 * n1 + c, h) : a;
      const f4 dr = mma<H, SPLIT>(a, al, K.p1[j], K.p1l[SPLIT ? j : 0]);
      const f4 di = mma<H, SPLIT>(a, al, K.p2[j], K.p2l[SPLIT ? j : 0]);
#pragma unroll
      for (int i = 0; i < 4; ++i) pw[j][i] = kUnit ? dr[i] * dr[i] + di[i] * di[i] : (dr[i] * dr[i] + di[i] * di[i]) * pscale;
    }
  };
  // vmcnt(0), expcnt and lgkmcnt at their maxima (no wait on them)
  auto drain_vm = [&]() { __builtin_amdgcn_s_waitcnt(0x0F70); };

  // Per template: product + stage 2' | barrier | stage 1', stores of the
  // previous template's staged powers | barrier | stage 0' into the staging
  // buffer. Vector loads and stores share one counter, and with both kinds
  // outstanding a wait for a load also waits for every store issued before
  // it. PF == 1: the next bank row is loaded after the stores, so the wait
  // for it (at the next product) comes a full phase after both were issued.
  // PF == 2: the next bank row is loaded as soon as the product has read the
  // current one, and everything outstanding is waited for explicitly at the
  // start of the following phase, before the stores are issued: loads get one
  // phase and the stores of the previous template two.
  // PF == 3: as PF == 2, with the loop rotated so that stage 0' of one
  // template and the product and stage 2' of the next share a phase without
  // a branch between them (independent work the compiler can interleave),
  // and the staged powers read before stage 1' (their LDS latency hidden
  // behind it) and stored after it. In the flat batched form this was 1%
  // faster than PF == 2 for FP16; in the persistent form, and with BF16, the
  // rotated loop spills and is slower.
  // PF == 4: loads as PF == 2, no explicit drain: the compiler waits for the
  // bank row at the next product, stores of the same template included. On
  // the unsplit forms 2-3% faster than PF == 2 on the wide batch and the
  // paper-scale plane; on the split form 1% slower.
  // PF == 5: as PF == 4, with the same vector-memory operations on every
  // path: each template loads a bank row (the last template its own row
  // again) and then issues its stores (the first template, which has no
  // previous powers, a store that writes nothing), and the loop is entered
  // after one such store. The stores then always follow the bank row they
  // share the counter with, so the wait for that row at the next product
  // leaves the newest template's stores outstanding: each store has until the
  // product after next, not the next one, to complete.
  // PF == 7 (unsplit, one 16-wave block per CU): a skewed pipeline. Phase
  // k runs product + stage 2' of template k, stage 1' of template k - 1,
  // stage 0' of template k - 2 and the stores of template k - 3, then one
  // barrier; stage and staging buffers alternate between templates (Ea and
  // Eb of template k in buffer k & 1), so every read in a phase is of data
  // the previous phase wrote. One barrier per template instead of two, and
  // each wave has three independent matrix chains per phase. The memory
  // operations are those of PF == 5 (every phase loads a bank row, clamped
  // to the last, and issues its stores, writing nothing when there is no
  // template k - 3).
  if constexpr (PF == 7 && !CAND) {
    static_assert(!SPLIT, "the skewed schedule is unsplit");
    if (z0 < z1 && active) {
      H *const Ea0 = reinterpret_cast<H *>(smem);
      H *const Ea1 = Ea0 + NP * kPlane;
      H *const Eb0 = Ea1 + NP * kPlane;
      H *const Eb1 = Eb0 + NP * kPlane;
      float *const sg0 = reinterpret_cast<float *>(smem + kSkewStageBytes);
      float *const sg1 = sg0 + kStageF;
      const int n = z1 - z0;
      load_bank(z0);
      f4 v[TPW];
#pragma unroll
      for (int q = 0; q < TPW; ++q) v[q] = __builtin_bit_cast(f4, K.q1[0]);  // any live value: nothing is written
      write_staged_buffer(z0, v, true);
      // phase k with compile-time parity P = k & 1; the flags say which
      // templates exist (uniform over the block)
      auto phase = [&](int k, auto pc, bool s2v, bool s1v, bool s0v, bool stv) {
        constexpr int P = decltype(pc)::value;
        H *const ea_w = P ? Ea1 : Ea0;        // stage 2' of template k
        const H *const ea_r = P ? Ea0 : Ea1;  // stage 1' of template k - 1
        H *const eb_w = P ? Eb0 : Eb1;
        const H *const eb_r = P ? Eb1 : Eb0;  // stage 0' of template k - 2
        float *const sg_w = P ? sg1 : sg0;
        const float *const sg_r = P ? sg0 : sg1;  // stores of template k - 3
        f4 vv[TPW];
        read_staged_from(vv, sg_r);
        if (s1v) stage1_from(ea_r, eb_w);
        if (s0v) stage0_from(eb_r, sg_w);
        if (s2v) product_stage2_to(ea_w);
        load_bank(z0 + (k + 1 < n ? k + 1 : n - 1));
        write_staged_buffer(stv ? z0 + k - 3 : z0, vv, !stv);
        __syncthreads();
      };
      const std::integral_constant<int, 0> p0{};
      const std::integral_constant<int, 1> p1{};
      // fill: phases 0, 1, 2
      phase(0, p0, true, false, false, false);
      phase(1, p1, 1 < n, true, false, false);
      phase(2, p0, 2 < n, 2 <= n, true, false);
      // steady state: phases 3 .. n - 1, every part present
      int k = 3;
      for (; k + 1 <= n - 1; k += 2) {
        phase(k, p1, true, true, true, true);
        phase(k + 1, p0, true, true, true, true);
      }
      if (k <= n - 1) {
        phase(k, p1, true, true, true, true);
        ++k;
      }
      // drain: phases up to n + 2
      for (; k <= n + 2; ++k) {
        const bool s2v = k < n, s1v = k <= n, s0v = k <= n + 1;
        if (k & 1) phase(k, p1, s2v, s1v, s0v, true);
        else phase(k, p0, s2v, s1v, s0v, true);
      }
    }
  } else if constexpr (PF == 8 && !CAND) {
    // PF == 8: the skewed pipeline of PF == 7 without the staging buffer
    // (stage 0' of template k - 2 stores its powers in the same phase), so
    // that the doubled stage buffers of the split form fit in LDS. Every
    // phase loads a bank row and then issues one store per tile (writing
    // nothing while there is no template k - 2), so the wait for that row at
    // the next product leaves the stores in flight.
    if (z0 < z1 && active) {
      H *const Ea0 = reinterpret_cast<H *>(smem);
      H *const Ea1 = Ea0 + NP * kPlane;
      H *const Eb0 = Ea1 + NP * kPlane;
      H *const Eb1 = Eb0 + NP * kPlane;
      const int n = z1 - z0;
      load_bank(z0);
      f4 v0[TPW];
#pragma unroll
      for (int q = 0; q < TPW; ++q) v0[q] = __builtin_bit_cast(f4, K.q1[0]);  // any live value: nothing is written
      write_direct(z0, v0, true);
      auto phase = [&](int k, auto pc, bool s2v, bool s1v, bool s0v) {
        constexpr int P = decltype(pc)::value;
        H *const ea_w = P ? Ea1 : Ea0;        // stage 2' of template k
        const H *const ea_r = P ? Ea0 : Ea1;  // stage 1' of template k - 1
        H *const eb_w = P ? Eb0 : Eb1;
        const H *const eb_r = P ? Eb1 : Eb0;  // stage 0' of template k - 2
        f4 vv[TPW];
        if (s1v) stage1_from(ea_r, eb_w);
        if (s0v) {
          stage0_pw(eb_r, vv);
        } else {
#pragma unroll
          for (int q = 0; q < TPW; ++q) vv[q] = __builtin_bit_cast(f4, K.q1[0]);
        }
        if (s2v) product_stage2_to(ea_w);
        load_bank(z0 + (k + 1 < n ? k + 1 : n - 1));
        write_direct(s0v ? z0 + k - 2 : z0, vv, !s0v);
        __syncthreads();
      };
      const std::integral_constant<int, 0> p0{};
      const std::integral_constant<int, 1> p1{};
      // fill: phases 0, 1
      phase(0, p0, true, false, false);
      phase(1, p1, 1 < n, true, false);
      // steady state: phases 2 .. n - 1, every part present
      int k = 2;
      for (; k + 1 <= n - 1; k += 2) {
        phase(k, p0, true, true, true);
        phase(k + 1, p1, true, true, true);
      }
      if (k <= n - 1) {
        phase(k, p0, true, true, true);
        ++k;
      }
      // drain: phases up to n + 1
      for (; k <= n + 1; ++k) {
        const bool s2v = k < n, s1v = k <= n;
        if (k & 1) phase(k, p1, s2v, s1v, true);
        else phase(k, p0, s2v, s1v, true);
      }
    }
  } else if constexpr (PF == 5 && !CAND) {
    if (z0 < z1 && active) {
      load_bank(z0);
      f4 v[TPW];
#pragma unroll
      for (int q = 0; q < TPW; ++q) v[q] = __builtin_bit_cast(f4, K.q1[0]);  // any live value: nothing is written
      write_staged_buffer(z0, v, true);
      for (int iz = z0; iz < z1; ++iz) {
        product_stage2();
        load_bank(iz + 1 < z1 ? iz + 1 : iz);
        __syncthreads();
        stage1();
        read_staged(v);
        write_staged_buffer(iz > z0 ? iz - 1 : iz, v, iz == z0);
        __syncthreads();
        stage0();
      }
      __syncthreads();
      store_staged(z1 - 1);
    }
  } else if constexpr (PF == 3) {  // (the detection epilogue of PF == 5 runs the PF == 4 loop below)
    if (z0 < z1) {
      load_bank(z0);
      drain_vm();  // nothing outstanding on loop entry
      product_stage2();
      if (z0 + 1 < z1) load_bank(z0 + 1);
      __syncthreads();
      drain_vm();
      stage1();
      __syncthreads();
      for (int iz = z0 + 1; iz < z1; ++iz) {
        stage0();          // template iz - 1
        product_stage2();  // template iz
        if (iz + 1 < z1) load_bank(iz + 1);
        __syncthreads();
        drain_vm();
        f4 v[TPW];
        read_staged(v);    // powers of template iz - 1
        stage1();
        write_staged(iz - 1, v);
        __syncthreads();
      }
      stage0();
      __syncthreads();
      store_staged(z1 - 1);
    }
  } else {
    if (PF && z0 < z1) load_bank(z0);
    // (PF == 2: nothing may be outstanding on entry, or the loads of the
    // preheader would make every later wait a full one)
    if constexpr (PF == 2) drain_vm();
    for (int iz = z0; iz < z1; ++iz) {
      if (!PF) load_bank(iz);
      product_stage2();
      if ((PF == 2 || PF >= 4) && iz + 1 < z1) load_bank(iz + 1);
      __syncthreads();
      if constexpr (PF == 2) drain_vm();
      stage1();
      if (iz > z0) store_staged(iz - 1);
      if (PF == 1 && iz + 1 < z1) load_bank(iz + 1);
      __syncthreads();
      stage0();
    }
    if (z0 < z1) {
      __syncthreads();
      store_staged(z1 - 1);
    }
  }
}

template <class H, int PF, bool NT, int NW, int OCC, bool SPLIT, bool CAND>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
    ols_mixed4096_kernel(const c32 *__restrict__ spec, int64_t nbins, const H *__restrict__ bank,
                         const c32 *__restrict__ tw, const unsigned char *__restrict__ consts,
                         float *__restrict__ power, int64_t ld, int nseg, int U, int half, int nz,
                         int zpb, int nsb, int bank_log2, CandOut cand) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[mix_smem<SPLIT, PF>()];
  __shared__ float s_max[NW];
  const int sb = blockIdx.x % nsb;
  const int zg = blockIdx.x / nsb;
  const int z0 = zg * zpb;
  const int z1 = min(nz, z0 + zpb);
  mixed_unit<H, PF, NT, NW, SPLIT, CAND>(consts, spec, nbins, bank, tw, power, ld, sb, sb < nseg,
                                         U, half, z0, z1, 0, bank_log2, smem, s_max, cand);
}

// Batched form as one flat launch: block b takes work item b (items are
// numbered largest series first, template-group major), so the hardware
// dispatcher hands out items in that order as blocks retire. Same body as
// the single-series kernel (FDAS_BATCH_PERSISTENT=0; the persistent form
// below is the default).
template <class H, int PF, bool NT, int NW, int OCC, bool SPLIT>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
    ols_mixed4096_items_kernel(const SeriesDesc *__restrict__ desc, int nseries,
                               const H *__restrict__ bank, const c32 *__restrict__ tw,
                               const unsigned char *__restrict__ consts, int U, int half, int zpb,
                               int bank_log2) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[mix_smem<SPLIT, PF>()];
  __shared__ float s_max[NW];
  const long long item = blockIdx.x;
  int lo = 0, hi = nseries - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].item_begin <= item) lo = mid;
    else hi = mid - 1;
  }
  const SeriesDesc d = desc[lo];
  const long long local = item - d.item_begin;
  const int zg = (int)(local / d.nseg);
  const int sb = (int)(local % d.nseg);
  const int z0 = d.row_off + zg * d.zpb;
  const int z1 = min(d.row_off + d.nz, z0 + d.zpb);
  const CandOut none{};
  mixed_unit<H, PF, NT, NW, SPLIT, false>(consts, static_cast<const c32 *>(d.spec), d.nbins, bank, tw, d.power,
                            d.ld, sb, true, U, half, z0, z1, d.row_off, bank_log2, smem, s_max,
                            none);
}

template <class H, int PF, bool NT, int NW, int OCC, bool SPLIT>
static hipError_t launch_mixed4096(const OlsArgs &a, hipStream_t st) {
  const int nsb = a.nseg;
  const int nzg = (a.nz + a.zpb - 1) / a.zpb;
  const long blocks = (long)nsb * nzg;
  if (a.cand.count)
    hipLaunchKernelGGL((ols_mixed4096_kernel<H, PF, NT, NW, OCC, SPLIT, true>), dim3((unsigned)blocks),
                       dim3(64 * NW), 0, st, static_cast<const c32 *>(a.spec), a.nbins,
                       static_cast<const H *>(a.bank), static_cast<const c32 *>(a.tw),
                       static_cast<const unsigned char *>(a.consts), a.power, a.ld, a.nseg, a.U,
                       a.half, a.nz, a.zpb, nsb, a.bank_log2, a.cand);
  else
    hipLaunchKernelGGL((ols_mixed4096_kernel<H, PF, NT, NW, OCC, SPLIT, false>), dim3((unsigned)blocks),
                       dim3(64 * NW), 0, st, static_cast<const c32 *>(a.spec), a.nbins,
                       static_cast<const H *>(a.bank), static_cast<const c32 *>(a.tw),
                       static_cast<const unsigned char *>(a.consts), a.power, a.ld, a.nseg, a.U,
                       a.half, a.nz, a.zpb, nsb, a.bank_log2, a.cand);
  return hipGetLastError();
}

// Persistent batched form: a grid sized to the resident blocks, each block
// taking work items from a device counter (reset by a kernel launched just
// before) until none is left. The same body as the flat form.
template <class H, int PF, bool NT, int NW, int OCC, bool SPLIT>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
    ols_mixed4096_persistent_kernel(const SeriesDesc *__restrict__ desc, int nseries,
                                    long long total, unsigned long long *counter,
                                    const H *__restrict__ bank, const c32 *__restrict__ tw,
                                    const unsigned char *__restrict__ consts, int U, int half,
                                    int bank_log2) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[mix_smem<SPLIT, PF>()];
  __shared__ float s_max[NW];
  __shared__ long long s_item[2];
  int par = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item[par] = (long long)atomicAdd(counter, 1ULL);
    __syncthreads();
    const long long item = s_item[par];
    par ^= 1;
    if (item >= total) break;  // every wave of the block sees the same item
    int lo = 0, hi = nseries - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (desc[mid].item_begin <= item) lo = mid;
      else hi = mid - 1;
    }
    const SeriesDesc d = desc[lo];
    const long long local = item - d.item_begin;
    const int zg = (int)(local / d.nseg);
    const int sb = (int)(local % d.nseg);
    const int z0 = d.row_off + zg * d.zpb;
    const int z1 = min(d.row_off + d.nz, z0 + d.zpb);
    const CandOut none{};
    // The thread index passes through an empty asm statement on every item, so
    // that nothing computed from it is hoisted out of this loop (held across
    // it, the addresses of one unit would not fit the register budget).
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    mixed_unit<H, PF, NT, NW, SPLIT, false>(consts, static_cast<const c32 *>(d.spec), d.nbins,
                                            bank, tw, d.power, d.ld, sb, true, U, half, z0, z1,
                                            d.row_off, bank_log2, smem, s_max, none, t);
  }
}

static bool mixed_batch_persistent() {
  const char *e = std::getenv("FDAS_BATCH_PERSISTENT");
  return !(e && *e == '0');  // the flat item grid with FDAS_BATCH_PERSISTENT=0
}

template <class H, int PF, bool NT, int NW, int OCC, bool SPLIT>
static hipError_t launch_mixed4096_batch(const BatchArgs &a, hipStream_t st) {
  if (mixed_batch_persistent()) {
    hipError_t e = launch_reset_counter(a.counter, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ols_mixed4096_persistent_kernel<H, PF, NT, NW, OCC, SPLIT>),
                       dim3((unsigned)a.grid), dim3(64 * NW), 0, st, a.desc, a.nseries,
                       (long long)a.total, a.counter, static_cast<const H *>(a.bank),
                       static_cast<const c32 *>(a.tw), static_cast<const unsigned char *>(a.consts),
                       a.U, a.half, a.bank_log2);
    return hipGetLastError();
  }
  if (a.total > (int64_t)0xffffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((ols_mixed4096_items_kernel<H, PF, NT, NW, OCC, SPLIT>), dim3((unsigned)a.total),
                     dim3(64 * NW), 0, st, a.desc, a.nseries, static_cast<const H *>(a.bank),
                     static_cast<const c32 *>(a.tw), static_cast<const unsigned char *>(a.consts),
                     a.U, a.half, a.zpb, a.bank_log2);
  return hipGetLastError();
}

template <class H, int PF, bool NT, int NW, int OCC, bool SPLIT>
static int mixed_batch_blocks_per_cu() {
  if (!mixed_batch_persistent()) return 1;  // flat launch: the grid is the item count
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void *>(&ols_mixed4096_persistent_kernel<H, PF, NT, NW, OCC, SPLIT>),
          64 * NW, 0) != hipSuccess)
    return 1;
  return nb;
}

template <class H, int PF, bool NT, int NW, int OCC, bool SPLIT>
static int mixed_grid_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void *>(&ols_mixed4096_kernel<H, PF, NT, NW, OCC, SPLIT, false>), 64 * NW,
          0) != hipSuccess)
    return 0;
  return nb;
}

template <class H, int PF, bool NT, int NW, int OCC, bool SPLIT>
static OlsVariant make_mixed(const char *name, int precision) {
  OlsVariant v{};
  v.name = name;
  v.L = 4096;
  v.T = 64 * NW;
  v.G = 1;
  v.nbuf = 1;
  v.precision = precision;
  v.split = SPLIT ? 1 : 0;
  // The forward FFT costs several templates' worth of time here; units of
  // up to 72 templates with a shorter last group measured fastest (17 to 101
  // swept on the paper-scale plane).
  v.zpb_target = 72;
  v.lay.L = 4096;
  v.lay.T = 256;
  v.lay.E = 16;
  v.lay.P = 3;
  v.lay.R[0] = v.lay.R[1] = v.lay.R[2] = 16;
  for (int i = 3; i < kMaxStages; ++i) v.lay.R[i] = 1;
  v.lds_bytes = 0;
  v.launch = &launch_mixed4096<H, PF, NT, NW, OCC, SPLIT>;
  v.launch_batch = &launch_mixed4096_batch<H, PF, NT, NW, OCC, SPLIT>;
  v.batch_blocks_per_cu = &mixed_batch_blocks_per_cu<H, PF, NT, NW, OCC, SPLIT>;
  v.grid_blocks_per_cu = &mixed_grid_blocks_per_cu<H, PF, NT, NW, OCC, SPLIT>;
  return v;
}

static const OlsVariant kMixedVariants[] = {
    // the first of each precision and split form is its default
    make_mixed<_Float16, 5, true, 16, 8, false>("fp16_L4096_mfma_w16_pfb", 1),
    make_mixed<_Float16, 7, true, 16, 4, false>("fp16_L4096_mfma_w16_sk", 1),
    make_mixed<_Float16, 4, true, 16, 8, false>("fp16_L4096_mfma_w16_pfn", 1),
    make_mixed<_Float16, 2, true, 16, 8, false>("fp16_L4096_mfma_w16_pfw", 1),
    make_mixed<_Float16, 3, true, 16, 8, false>("fp16_L4096_mfma_w16_rot", 1),
    make_mixed<_Float16, 1, true, 16, 8, false>("fp16_L4096_mfma_w16_pf", 1),
    make_mixed<_Float16, 1, true, 8, 4, false>("fp16_L4096_mfma_w8_pf", 1),
    make_mixed<_Float16, 1, false, 16, 8, false>("fp16_L4096_mfma_w16_pf_ts", 1),
    make_mixed<__bf16, 4, true, 16, 8, false>("bf16_L4096_mfma_w16_pfn", 2),
    make_mixed<__bf16, 2, true, 16, 8, false>("bf16_L4096_mfma_w16_pfw", 2),
    make_mixed<__bf16, 1, true, 8, 4, false>("bf16_L4096_mfma_w8_pf", 2),
    // hi + lo split products (FDAS_FLAG_SPLIT)
    make_mixed<_Float16, 5, true, 16, 4, true>("fp16_L4096_mfma_split_w16_pfb", 1),
    make_mixed<_Float16, 2, true, 16, 4, true>("fp16_L4096_mfma_split_w16_pfw", 1),
    make_mixed<_Float16, 8, true, 16, 4, true>("fp16_L4096_mfma_split_w16_sk", 1),
    make_mixed<__bf16, 5, true, 16, 4, true>("bf16_L4096_mfma_split_w16_pfb", 2),
    make_mixed<__bf16, 8, true, 16, 4, true>("bf16_L4096_mfma_split_w16_sk", 2),
    make_mixed<__bf16, 2, true, 16, 4, true>("bf16_L4096_mfma_split_w16_pfw", 2),
    make_mixed<__bf16, 4, true, 16, 4, true>("bf16_L4096_mfma_split_w16_pfn", 2),
    make_mixed<__bf16, 3, true, 16, 4, true>("bf16_L4096_mfma_split_w16_rot", 2),
    make_mixed<__bf16, 0, true, 16, 4, true>("bf16_L4096_mfma_split_w16", 2),
};

// Every matrix-core variant: the 4096-point ones above, then the 2048-point
// kernel's.
const OlsVariant *mixed_variants(int *count) {
  static const std::vector<OlsVariant> all = [] {
    std::vector<OlsVariant> v(std::begin(kMixedVariants), std::end(kMixedVariants));
    int n = 0;
    const OlsVariant *w = mixed2048_variants(&n);
    v.insert(v.end(), w, w + n);
    return v;
  }();
  *count = (int)all.size();
  return all.data();
}

// ---- plan-time: planar bank in the X layout --------------------------------
// bank[i][plane][row*16 + slot] with row = 16 k0 + k1 for frequency
// k = k0 + 16 k1 + 256 k2 and slot = k2, its two 4-value halves swapped
// when bit 7 of the row is set (the order in which the kernel reads X);
// value conj(FFT_L(h_i))[k] (no 1/L; the kernel removes the factor
// 2^bank_log2 = L from the power). Planes: Re, Im, rounded to 16 bits, or
// with split to FP32 (the split kernel forms the product in FP32 and splits
// it; the same 8 bytes per value as 16-bit hi and lo planes).
struct c64m {
  double x, y;
};

__device__ __forceinline__ int bank_slot_k(int slot) {
  const int row = slot >> 4;
  const int k2 = (slot & 15) ^ (((row >> 7) & 1) << 2);
  return (row >> 4) + 16 * (row & 15) + 256 * k2;
}

template <class H>
__device__ __forceinline__ void put_split(H *hi, H *lo, double v) {
  const H a = (H)v;
  *hi = a;
  if (lo) *lo = (H)(v - (double)(float)a);
}

template <class H>
__global__ void bank_mixed_kernel(H *__restrict__ bank, const c64m *__restrict__ h, int nz, int m,
                                  int L, int split) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nz * L) return;
  const int i = (int)(idx / L);
  const int slot = (int)(idx % L);
  const int k = bank_slot_k(slot);
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
  if (split) {
    float *row_f = reinterpret_cast<float *>(bank) + (long)i * 2 * L;
    row_f[slot] = (float)sr;       // Re T'
    row_f[L + slot] = (float)-si;  // Im T'
    return;
  }
  H *row_i = bank + (long)i * 2 * L;
  row_i[slot] = (H)sr;       // Re T'
  row_i[L + slot] = (H)-si;  // Im T'
}

template <class H>
__global__ void bank_mixed_natural_kernel(c32 *__restrict__ dst, const H *__restrict__ bank,
                                          int nz, int L, int split) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nz * L) return;
  const int i = (int)(idx / L);
  const int slot = (int)(idx % L);
  const int k = bank_slot_k(slot);
  float re, im;
  if (split) {
    const float *row_f = reinterpret_cast<const float *>(bank) + (long)i * 2 * L;
    re = row_f[slot];
    im = row_f[L + slot];
  } else {
    const H *row_i = bank + (long)i * 2 * L;
    re = (float)row_i[slot];
    im = (float)row_i[L + slot];
  }
  const float inv = 1.0f / (float)L;
  dst[(long)i * L + k] = {re * inv, im * inv};
}

// Per-lane B operands of the mixed kernel, generated in FP64 (layout at
// kConstBytes; with split a second table of residuals follows). Lane l holds
// column c = l & 15 and K rows 8 (l >> 4) + j (j ^ 4 for tiles 8..15, the
// order of their operand chunks in LDS); K < 16 are real inputs, K >= 16
// imaginary inputs, so B1 = [Re M | -Im M] gives the real and
// B2 = [Im M | Re M] the imaginary part of M x.
template <class H>
__global__ void mixed_consts_kernel(unsigned char *__restrict__ out, int split) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * 16 * 64) return;
  const double kTwoPi = 6.283185307179586476925;
  const int fam = idx / 1024, tile = (idx / 64) % 16, lane = idx % 64;
  const int c = lane & 15, kg = lane >> 4;
  H *b = reinterpret_cast<H *>(out) + (size_t)idx * 16;
  H *bl = split ? reinterpret_cast<H *>(out + kConstBytes) + (size_t)idx * 16 : nullptr;
  for (int j = 0; j < 8; ++j) {
    const int kk = kg * 8 + (j ^ (((tile >> 3) & 1) << 2)), k = kk & 15;
    // Q_t: w4096^(c (256 k + t)); P_p: w256^(k (16 c + p)) = w4096^(16 k (16 c + p))
    const int e = fam == 0 ? (c * (256 * k + tile)) & 4095 : (16 * k * (16 * c + tile)) & 4095;
    double sn, cs;
    sincos(kTwoPi * (double)e / 4096.0, &sn, &cs);
    put_split(b + j, bl ? bl + j : nullptr, kk < 16 ? cs : -sn);
    put_split(b + 8 + j, bl ? bl + 8 + j : nullptr, kk < 16 ? sn : cs);
  }
}

size_t mixed_consts_bytes(int L, int split) {
  if (L == 2048) return split ? 0 : mixed2048_consts_bytes();
  return L == 4096 ? (size_t)kConstBytes * (split ? 2 : 1) : 0;
}

hipError_t launch_mixed_consts(void *out, int L, int precision, int split, hipStream_t s) {
  if (L == 2048 && !split) return launch_mixed2048_consts(out, precision, s);
  if (L != 4096) return hipErrorInvalidValue;
  if (precision == 2)
    hipLaunchKernelGGL(mixed_consts_kernel<__bf16>, dim3(8), dim3(256), 0, s,
                       static_cast<unsigned char *>(out), split);
  else
    hipLaunchKernelGGL(mixed_consts_kernel<_Float16>, dim3(8), dim3(256), 0, s,
                       static_cast<unsigned char *>(out), split);
  return hipGetLastError();
}

hipError_t launch_bank_mixed(void *bank, const void *h, int nz, int m, int L, int precision,
                             int split, hipStream_t s) {
  if (L == 2048)
    return split ? hipErrorInvalidValue : launch_bank_mixed2048(bank, h, nz, m, precision, s);
  const long n = (long)nz * L;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (precision == 2)
    hipLaunchKernelGGL(bank_mixed_kernel<__bf16>, grid, dim3(256), 0, s,
                       static_cast<__bf16 *>(bank), static_cast<const c64m *>(h), nz, m, L, split);
  else
    hipLaunchKernelGGL(bank_mixed_kernel<_Float16>, grid, dim3(256), 0, s,
                       static_cast<_Float16 *>(bank), static_cast<const c64m *>(h), nz, m, L,
                       split);
  return hipGetLastError();
}

hipError_t launch_bank_mixed_natural(c32 *dst, const void *bank, int nz, int L, int precision,
                                     int split, hipStream_t s) {
  if (L == 2048)
    return split ? hipErrorInvalidValue : launch_bank_mixed2048_natural(dst, bank, nz, precision, s);
  const long n = (long)nz * L;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (precision == 2)
    hipLaunchKernelGGL(bank_mixed_natural_kernel<__bf16>, grid, dim3(256), 0, s, dst,
                       static_cast<const __bf16 *>(bank), nz, L, split);
  else
    hipLaunchKernelGGL(bank_mixed_natural_kernel<_Float16>, grid, dim3(256), 0, s, dst,
                       static_cast<const _Float16 *>(bank), nz, L, split);
  return hipGetLastError();
}

}  // namespace fdas
