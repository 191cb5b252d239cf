// Mixed-precision overlap-and-save correlation kernel for segments of
// L = 2048 points: 16-bit storage (FP16 or BF16), the three inverse-DFT
// stages on the matrix cores (v_mfma_f32_16x16x32_{f16,bf16}) with FP32
// accumulation, |.|^2 in FP32.
//
// Digits: frequency k = k0 + 16 k1 + 256 k2 (k0, k1 < 16, k2 < 8), output
// n = 128 n0 + 8 n1 + n2 (n0, n1 < 16, n2 < 8). With w = exp(+2 pi i / 2048)
// the inverse DFT (eq. 3 with the opposite sign, unnormalised) is
//   y[n] = sum_k0 w16^(n0 k0) w256^(n1 k0) w2048^(n2 k0)
//          sum_k1 w16^(n1 k1) w128^(n2 k1) sum_k2 w8^(n2 k2) Y[k].
//   S2 (radix 8): tile k0, rows k1, K = k2, columns n2; w2048^(n2 k0)
//     depends on the tile and the column and is folded into the matrix.
//   S1 (radix 16): tile n2, rows k0, K = k1, columns n1; w128^(n2 k1)
//     (tile and K) is folded into the matrix.
//   S0 (radix 16): for the same n2, rows n1, K = k0, columns n0; its
//     twiddle w256^(n1 k0) depends on a row and a K index, so it is applied
//     to S1's results in FP32 (four complex products per lane).
// S2 has 8 complex inputs and outputs per butterfly: its A operand holds the
// four plane-pair products of Y = X T over k2 (Re X Re T, Im X Im T,
// Re X Im T, Im X Re T: K 0..31), and one matrix combines them into both
// parts of the output (columns 0..7 real, 8..15 imaginary), so the complex
// product's sums run in the matrix core's FP32 accumulation.
//
// S1 and S0 of one n2 run back to back in one wave: S1 leaves lane (g, c)
// with rows k0 = 4g .. 4g+3 of column n1 = c, and S0 needs in lane (g, c)
// row n1 = c with K = 8 (g & 1) .. +7 of plane g >> 1. That is a fixed
// exchange between the wave's four 16-lane rows, made with one
// v_permlane32_swap and one v_permlane16_swap per register pair, so only S2
// and S1 exchange through LDS.
//
// One block of 16 waves takes one segment and a group of templates:
//   forward FFT in FP32 on 128 threads (radix 16, 16, 8, decimation in
//   frequency, exchanging through LDS; X[k0 + 16 k1 + 256 k2] lands in LDS
//   slot 8 (16 k0 + k1) + k2), per-segment power-of-two scale, X rounded to
//   16 bits and kept in registers as S2's operand chunks;
//   per template, with a single barrier and two roles: waves 8..15 form the
//   products and S2 (two k0 tiles each) into one of two exchange buffers and
//   load the next bank row; waves 0..7 (n2 = wave) run S1, the twiddle and
//   the exchange of this template, S0 of the previous one into one of two
//   staging buffers, and the stores of the one before.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_radix.hpp"
#include "cand4.hpp"
#include "ols_variants.hpp"

namespace fdas {
namespace m2048 {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 hf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 hf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

template <class H>
struct V;
template <>
struct V<_Float16> {
  typedef hf8 v8;
  typedef hf4 v4;
  static __device__ __forceinline__ f4 mfma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct V<__bf16> {
  typedef bf8 v8;
  typedef bf4 v4;
  static __device__ __forceinline__ f4 mfma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

constexpr int L = 2048;
constexpr int NW = 16;  // waves per block: 8 for S2 (two tiles each), 8 for S1-S0 (one n2 each)

// ---- LDS layout (bytes) ----------------------------------------------------
// Forward FFT (FP32): A -> B exchange, rows of 128 values padded to 132;
// B -> C exchange, 256 pairs (k0, k1) of 8 values padded to 9.
constexpr int kFA = 16 * 132 * 8;
constexpr int kFB = 256 * 9 * 8;
// X in 16 bits: plane [k0][k1][k2] (8 values per row), Re then Im.
constexpr int kXPlane = 2048;  // halves
// Exchange buffer S2 -> S1: two planes (Re, Im) of 128 rows of 16 values,
// row R = 128 plane + 16 n2 + k0 (values over k1), 16 bytes of padding per
// 16 rows. The two 8-value chunks of a row are swapped when bit 2 of k0 is
// set, and the two 4-value halves of each chunk in the Im plane. S1's operand
// reads (16 bytes from 8 consecutive rows) and S2's writes (8 bytes to 16
// rows of different n2 and plane) then fall on distinct banks. S1's Im-plane
// lanes read their chunk as values 4..7, 0..3; their B matrix is stored in
// that order.
constexpr int kEaHalves = 256 * 16 + 16 * 8;
__device__ __forceinline__ int ea_idx(int plane, int n2, int k0, int e) {
  const int R = 128 * plane + 16 * n2 + k0;
  return 16 * R + 8 * (R >> 4) + 8 * (((e >> 3) ^ (k0 >> 2)) & 1) + 4 * (((e >> 2) ^ plane) & 1) +
         (e & 3);
}
// start of the chunk holding values 8h .. 8h+7 of a row
__device__ __forceinline__ int ea_chunk(int plane, int n2, int k0, int h) {
  const int R = 128 * plane + 16 * n2 + k0;
  return 16 * R + 8 * (R >> 4) + 8 * ((h ^ (k0 >> 2)) & 1);
}
// Staging of the powers, [n2][n0][n1] with n1 fastest: S0's lanes write four
// consecutive n1 (16 bytes; rows of 16 padded to 20 floats put 8 lanes on
// distinct banks), the storing lanes gather four consecutive outputs (n2
// apart by one; n2 rows 324 floats apart put 32 lanes on distinct banks).
constexpr int kStgN2 = 324, kStgN0 = 20;
constexpr int kStg = 8 * kStgN2;
// Offsets: the forward buffers alias the exchange and staging buffers (used
// only before the first template; a barrier separates them).
constexpr int kOffE = 0;
constexpr int kOffStg = kOffE + 2 * kEaHalves * 2;
constexpr int kLoopBytes = kOffStg + 2 * kStg * 4;
constexpr int kFwdBytes = kFA + kFB;
constexpr int kOffX = (kLoopBytes > kFwdBytes ? kLoopBytes : kFwdBytes);
constexpr int kSmem = kOffX + 2 * kXPlane * 2;
static_assert(kOffStg % 16 == 0 && (kStg * 4) % 16 == 0 && kOffX % 16 == 0, "alignment");

// Plan-time tables, per lane l (column c = l & 15, K rows 8 (l >> 4) + j):
// family Q (S2, 16 tiles, one 8-value operand), family P (S1, 8 tiles, B1
// and B2), family F (S0, one matrix, B1 and B2); then the FP32 twiddles
// w256^(n1 k0) of S0 for the lane's four S1 results (Re, Im pairs).
constexpr int kQOff = 0;  // v8 entries
constexpr int kPOff = kQOff + 16 * 64;
constexpr int kFOff = kPOff + 8 * 64 * 2;
constexpr int kConstV8 = kFOff + 64 * 2;
constexpr int kTwOff = kConstV8 * 16;  // bytes; 64 lanes x 8 floats
constexpr int kConstBytes = kTwOff + 64 * 8 * 4;

// x[k] *= w^k for k = 1..15, with w = tw[step] and w^4 = tw[4 step] the only
// loads (both in flight together) and every other power at most three
// complex products away from them: a few units in the last place, for
// transforms whose results are rounded to 16 bits afterwards. Loading all
// fifteen powers would keep 30 more registers live, and under a 64-register
// budget the compiler then waits for each load before issuing the next.
__device__ __forceinline__ void twiddle16_pow(c32 *x, gptr<const c32> tw, int step) {
  const c32 w1 = ldg(tw + step), w4 = ldg(tw + 4 * step);
  const c32 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
  const c32 w8 = cmul(w4, w4), w12 = cmul(w8, w4);
  const c32 lo[4] = {{1.f, 0.f}, w1, w2, w3};
  const c32 hi[4] = {{1.f, 0.f}, w4, w8, w12};
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    const int a = k >> 2, b = k & 3;
    const c32 w = a == 0 ? lo[b] : (b == 0 ? hi[a] : cmul(hi[a], lo[b]));
    x[k] = cmul(x[k], w);
  }
}

// One work unit: segment s, bank rows [z0, z1), plane rows iz - row_base.
template <class H, bool NT, bool CAND>
__device__ __forceinline__ void unit2048(const unsigned char *__restrict__ consts_,
                                         const c32 *__restrict__ spec_, int64_t nbins,
                                         const H *__restrict__ bank_, const c32 *__restrict__ tw_,
                                         float *__restrict__ power_, int64_t ld, int s,
                                         bool active, int U, int half, int z0, int z1,
                                         int row_base, int bank_log2, unsigned char *smem,
                                         float *s_max, const CandOut &cd, int t_in = -1) {
  typedef typename V<H>::v8 v8;
  typedef typename V<H>::v4 v4;
  const auto consts = to_global(reinterpret_cast<const v8 *>(consts_));
  const auto spec = to_global(spec_);
  const auto bank = to_global(bank_);
  const auto tw = to_global(tw_);
  const auto power = to_global(power_);
  c32 *fa = reinterpret_cast<c32 *>(smem);
  c32 *fb = reinterpret_cast<c32 *>(smem + kFA);
  H *Ea = reinterpret_cast<H *>(smem + kOffE);
  float *stg = reinterpret_cast<float *>(smem + kOffStg);
  H *Xp = reinterpret_cast<H *>(smem + kOffX);
  const int t = t_in < 0 ? (int)threadIdx.x : t_in;
  const int lane = t & 63, w = t >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t seg0 = (int64_t)s * U - half;

  // ---- forward FFT (FP32), threads 0..127 ------------------------------------
  // input j = 128 ja + 8 jb + jc; stage A over ja -> k0 (twiddle
  // W2048^(k0 (8 jb + jc))), stage B over jb -> k1 (twiddle W128^(k1 jc)),
  // stage C over jc -> k2.
  const bool fw = t < 128;
  float mx = 0.f;
  if (fw) {
    c32 x[16];
#pragma unroll
    for (int n = 0; n < 16; ++n) {
      const int64_t gi = seg0 + 128 * n + t;
      c32 v = {0.f, 0.f};
      if (active && gi >= 0 && gi < nbins) v = ldg(spec + gi);
      x[n] = v;
    }
    dft<-1, 16>(x);
    twiddle16_pow(x, tw, t);  // W2048^(k0 t)
#pragma unroll
    for (int k = 0; k < 16; ++k) fa[k * 132 + t] = x[k];
  }
  __syncthreads();
  if (fw) {
    c32 x[16];
    const int k0 = t >> 3, jc = t & 7;
#pragma unroll
    for (int jb = 0; jb < 16; ++jb) x[jb] = fa[k0 * 132 + 8 * jb + jc];
    dft<-1, 16>(x);
    twiddle16_pow(x, tw, 16 * jc);  // W2048^(16 k1 jc)
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) fb[(k0 * 16 + k1) * 9 + jc] = x[k1];
  }
  __syncthreads();
  c32 xc[2][8];
  if (fw) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = 2 * t + q;  // pair (k0, k1) = (p >> 4, p & 15)
#pragma unroll
      for (int jc = 0; jc < 8; ++jc) xc[q][jc] = fb[p * 9 + jc];
      dft<-1, 8>(xc[q]);
#pragma unroll
      for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fmaxf(fabsf(xc[q][e].x), fabsf(xc[q][e].y)));
    }
  }
  // per-segment scale: largest component into [4, 8)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if (lane == 0) s_max[w] = mx;
  __syncthreads();  // also: every read of the forward buffers is complete
  mx = 0.f;
#pragma unroll
  for (int k = 0; k < NW; ++k) mx = fmaxf(mx, s_max[k]);
  int ex = 0;
  if (mx > 0.f) (void)frexpf(mx, &ex);
  const float xscale = ldexpf(1.0f, 3 - ex);
  const float pscale = ldexpf(1.0f, -2 * (3 - ex + bank_log2));
  if (fw) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = 2 * t + q;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        v4 re, im;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          re[i] = (H)(xc[q][4 * hh + i].x * xscale);
          im[i] = (H)(xc[q][4 * hh + i].y * xscale);
        }
        *reinterpret_cast<v4 *>(Xp + p * 8 + 4 * hh) = re;
        *reinterpret_cast<v4 *>(Xp + kXPlane + p * 8 + 4 * hh) = im;
      }
    }
  }
  __syncthreads();  // X complete

  // Per template, one barrier, two roles in wave-uniform branches (each
  // loop holds only its own operands, so the two share registers):
  //   waves 8..15: S2 of tiles k0 = 2 (w - 8) and 2 (w - 8) + 1 of template
  //     iz into exchange buffer iz & 1, then the next bank row's loads;
  //   waves 0..7 (n2 = w), software-pipelined: S1, the twiddle and the
  //     exchange of template iz, S0 and |.|^2 of template iz - 1 (its S0
  //     operand kept in registers) into staging buffer (iz - 1) & 1, and the
  //     stores of template iz - 2 from staging buffer iz & 1.
  // S2 of template iz + 1 thus runs while S1 of template iz does, and S1 and
  // S0 in one iteration are independent. Both roles pass z1 - z0 + 2
  // barriers. The S2 waves issue only loads and the S1-S0 waves only
  // stores, so no wait for a bank row waits for a store.
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  if (w >= 8) {
    // S2, tile k0 (row k1 = c): lane group g supplies the products over
    // k2 = 0..7 of one pair of planes, g = 0: Re X Re T, 1: Im X Im T,
    // 2: Re X Im T, 3: Im X Re T, and the matrix combines them
    // (Re Y = g0 - g1, Im Y = g2 + g3) in FP32; a lane holds one plane of X
    // and loads one plane of each bank row. Lane (g, c) receives rows
    // k1 = 4g + i of column c (c < 8: Re of n2 = c, else Im of n2 = c - 8).
    const int ka = 2 * (w - 8), kb = ka + 1;
    const int xplane = (g == 0 || g == 2) ? 0 : kXPlane;
    const v8 xa = *reinterpret_cast<const v8 *>(Xp + xplane + (ka * 16 + c) * 8);
    const v8 xb = *reinterpret_cast<const v8 *>(Xp + xplane + (kb * 16 + c) * 8);
    const v8 qa = consts[kQOff + ka * 64 + lane];
    const v8 qb = consts[kQOff + kb * 64 + lane];
    const auto brow0 = bank + ((g == 0 || g == 3) ? 0 : L) + (ka * 16 + c) * 8;
    v8 ta, tb;
    auto load_bank = [&](int iz) {
      const auto r = brow0 + (int64_t)iz * (2 * L);
      ta = *reinterpret_cast<gptr<const v8>>(r);
      tb = *reinterpret_cast<gptr<const v8>>(r + 128);  // tile kb: 16 rows of 8 further
    };
    auto put = [&](H *e, int k0, const f4 &d) {
      v4 o;
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = (H)d[i];
      *reinterpret_cast<v4 *>(e + ea_idx(c >> 3, c & 7, k0, 4 * g)) = o;
    };
    if (z0 < z1) load_bank(z0);
    for (int iz = z0; iz < z1; ++iz) {
      H *e = Ea + ((iz - z0) & 1) * kEaHalves;
      const f4 da = V<H>::mfma(xa * ta, qa, zero);
      const f4 db = V<H>::mfma(xb * tb, qb, zero);
      if (iz + 1 < z1) load_bank(iz + 1);
      put(e, ka, da);
      put(e, kb, db);
      __syncthreads();
    }
    __syncthreads();
    __syncthreads();
    return;
  }

  // S1 (tile n2 = w): both parts, rows k0 = 4g + i of column n1 = c; the
  // lane's four twiddles w256^(k0 n1); S0's DFT-16 matrix.
  const int n2 = w;
  const v8 bp1 = consts[kPOff + (n2 * 64 + lane) * 2];
  const v8 bp2 = consts[kPOff + (n2 * 64 + lane) * 2 + 1];
  // S0's matrix and the lane's twiddles: held in registers, or in the
  // detection form, whose offers need registers of their own, read again
  // from the table at each use (through a pointer the compiler cannot hoist
  // the loads out of the loop with; these waves issue no other loads, so
  // the waits are short).
  const v8 bf1_r = consts[kFOff + lane * 2];
  const v8 bf2_r = consts[kFOff + lane * 2 + 1];
  const f4 twr_r = *to_global(reinterpret_cast<const f4 *>(consts_ + kTwOff) + lane * 2);
  const f4 twi_r = *to_global(reinterpret_cast<const f4 *>(consts_ + kTwOff) + lane * 2 + 1);
  auto cvec = [&](int i) {  // entry i of the table, as v8
    return to_global(reinterpret_cast<const v8 *>(opaque_ptr(consts_)))[i];
  };
  auto cf4 = [&](int i) {  // f4 entry i past the twiddle offset
    return to_global(reinterpret_cast<const f4 *>(opaque_ptr(consts_) + kTwOff))[i];
  };

  // Stores: wave w writes outputs [256 w, 256 w + 256), a lane four
  // consecutive ones (1 KB per store instruction), gathered from the
  // [n2][n0][n1] staging.
  const bool vec_ok = half % 4 == 0 && ((int64_t)s * U - half) % 4 == 0 &&
                      (int64_t)(s + 1) * U <= nbins && ld % 4 == 0 &&
                      (reinterpret_cast<uintptr_t>(power_) & 15) == 0;
  const int o0 = 256 * w + 4 * lane;
  const int sgi = kStgN2 * (o0 & 7) + kStgN0 * (o0 >> 7) + ((o0 >> 3) & 15);
  const int64_t r0 = (int64_t)s * U + o0 - half;
  auto gather = [&](int b) {
    const float *sb = stg + b * kStg + sgi;
    f4 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = sb[kStgN2 * q];
    return v;
  };
  auto store = [&](int izr, const f4 &v) {
    if (!CAND && !active) return;
    const auto prow = power + (int64_t)(izr - row_base) * ld;
    if constexpr (CAND) {
      const bool any = v[0] >= cd.thr || v[1] >= cd.thr || v[2] >= cd.thr || v[3] >= cd.thr;
      if (__builtin_amdgcn_ballot_w64(active && any) == 0ull) return;
      offer4(cd, v, active, o0, half, U, r0, nbins, izr - row_base);
      return;
    }
    const auto dst = prow + r0;
    if (vec_ok) {
      if (o0 >= half && o0 < half + U) {
        if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<gptr<f4>>(dst));
        else *reinterpret_cast<gptr<f4>>(dst) = v;
      }
    } else {
      // ragged segment: outputs inside [half, half + U) and below nbins
      const int64_t left = nbins - r0;
      const int lim = (int)(left < 4 ? (left < 0 ? 0 : left) : 4);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < lim && o0 + i >= half && o0 + i < half + U) dst[i] = v[i];
    }
  };

  // S1, the twiddle and the exchange from exchange buffer b: S0's operand.
  auto stage1 = [&](int b) {
    const f4 twr = twr_r;
    const f4 twi = twi_r;
    const v8 a =
        *reinterpret_cast<const v8 *>(Ea + b * kEaHalves + ea_chunk(g >> 1, n2, c, g & 1));
    const f4 dr = V<H>::mfma(a, bp1, zero);
    const f4 di = V<H>::mfma(a, bp2, zero);
    unsigned re[2], im[2];
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
      const float x0 = dr[i] * twr[i] - di[i] * twi[i];
      const float y0 = dr[i] * twi[i] + di[i] * twr[i];
      const float x1 = dr[i + 1] * twr[i + 1] - di[i + 1] * twi[i + 1];
      const float y1 = dr[i + 1] * twi[i + 1] + di[i + 1] * twr[i + 1];
      typedef H h2 __attribute__((ext_vector_type(2)));
      re[i >> 1] = __builtin_bit_cast(unsigned, h2{(H)x0, (H)x1});
      im[i >> 1] = __builtin_bit_cast(unsigned, h2{(H)y0, (H)y1});
    }
    // rows 2, 3 of Re <-> rows 0, 1 of Im, then odd rows of the first <->
    // even rows of the second: lane (g, c) ends with the k0 values
    // 8 (g & 1) .. +3 (first) and +4 .. +7 (second) of plane g >> 1 of
    // row n1 = c
    unsigned u[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const auto p32 = __builtin_amdgcn_permlane32_swap(re[h], im[h], false, false);
      const auto p16 = __builtin_amdgcn_permlane16_swap(p32[0], p32[1], false, false);
      u[h] = p16[0];
      u[2 + h] = p16[1];
    }
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 uv = {u[0], u[1], u[2], u[3]};
    return __builtin_bit_cast(v8, uv);
  };
  // S0 and |.|^2 into staging buffer b: rows n1 = 4g + i, column n0 = c.
  auto stage0 = [&](const v8 &a0, int b) {
    const v8 bf1 = bf1_r;
    const v8 bf2 = bf2_r;
    const f4 er = V<H>::mfma(a0, bf1, zero);
    const f4 ei = V<H>::mfma(a0, bf2, zero);
    f4 pw;
#pragma unroll
    for (int i = 0; i < 4; ++i) pw[i] = (er[i] * er[i] + ei[i] * ei[i]) * pscale;
    *reinterpret_cast<f4 *>(stg + b * kStg + kStgN2 * n2 + kStgN0 * c + 4 * g) = pw;
  };

  // Template t's powers go to staging buffer (t - z0) & 1: S0(t) runs in
  // iteration t + 1 and its stores in iteration t + 2, after the barrier
  // that completes every wave's S0(t).
  // (The gather runs every iteration, also before there is anything to
  // store: it stays inside the staging buffer and its values are then
  // unused. Two iterations per trip let the S0 operand alternate between
  // two registers instead of being copied.)
  v8 a0 = {}, a1 = {};
  auto step = [&](int iz, v8 &cur, const v8 &prev) {
    const int b = (iz - z0) & 1;
    __syncthreads();
    const f4 v = gather(b);
    cur = stage1(b);
    if (iz > z0) stage0(prev, b ^ 1);
    if (iz - 2 >= z0) store(iz - 2, v);
  };
  int iz = z0;
  for (; iz + 1 < z1; iz += 2) {
    step(iz, a0, a1);
    step(iz + 1, a1, a0);
  }
  if (iz < z1) step(iz, a0, a1);
  const v8 last = ((z1 - z0) & 1) ? a0 : a1;  // the last template's S0 operand
  // S0 of the last template writes the buffer the last iteration gathered
  // from: after a barrier. The powers of the last two templates follow.
  __syncthreads();
  if (z0 < z1) stage0(last, (z1 - 1 - z0) & 1);
  if (z1 - 2 >= z0) store(z1 - 2, gather((z1 - 2 - z0) & 1));
  __syncthreads();
  if (z1 - 1 >= z0) store(z1 - 1, gather((z1 - 1 - z0) & 1));
}

template <class H, bool NT, int OCC, bool CAND>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
    ols_mixed2048_kernel(const c32 *__restrict__ spec, int64_t nbins, const H *__restrict__ bank,
                         const c32 *__restrict__ tw, const unsigned char *__restrict__ consts,
                         float *__restrict__ power, int64_t ld, int nseg, int U, int half, int nz,
                         int zpb, int nsb, int bank_log2, CandOut cand) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kSmem];
  __shared__ float s_max[NW];
  const int sb = blockIdx.x % nsb;
  const int zg = blockIdx.x / nsb;
  const int z0 = zg * zpb;
  const int z1 = min(nz, z0 + zpb);
  unit2048<H, NT, CAND>(consts, spec, nbins, bank, tw, power, ld, sb, sb < nseg, U, half, z0, z1,
                        0, bank_log2, smem, s_max, cand);
}

// Batched forms: one block per work item (flat), or persistent blocks taking
// items from a device counter (the default).
template <class H, bool NT, int OCC>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
    ols_mixed2048_items_kernel(const SeriesDesc *__restrict__ desc, int nseries,
                               const H *__restrict__ bank, const c32 *__restrict__ tw,
                               const unsigned char *__restrict__ consts, int U, int half,
                               int bank_log2) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kSmem];
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
  unit2048<H, NT, false>(consts, static_cast<const c32 *>(d.spec), d.nbins, bank, tw, d.power,
                         d.ld, sb, true, U, half, z0, z1, d.row_off, bank_log2, smem, s_max, none);
}

template <class H, bool NT, int OCC>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
    ols_mixed2048_persistent_kernel(const SeriesDesc *__restrict__ desc, int nseries,
                                    long long total, unsigned long long *counter,
                                    const H *__restrict__ bank, const c32 *__restrict__ tw,
                                    const unsigned char *__restrict__ consts, int U, int half,
                                    int bank_log2) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kSmem];
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
    // (the thread index passes through an empty asm statement on every item,
    // so that nothing derived from it is hoisted out of this loop)
    int tt;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tt) : "v"((int)threadIdx.x));
    unit2048<H, NT, false>(consts, static_cast<const c32 *>(d.spec), d.nbins, bank, tw, d.power,
                           d.ld, sb, true, U, half, z0, z1, d.row_off, bank_log2, smem, s_max,
                           none, tt);
  }
}

static bool batch_persistent() {
  const char *e = std::getenv("FDAS_BATCH_PERSISTENT");
  return !(e && *e == '0');
}

template <class H, bool NT, int OCC>
static hipError_t launch_single(const OlsArgs &a, hipStream_t st) {
  const int nsb = a.nseg;
  const int nzg = (a.nz + a.zpb - 1) / a.zpb;
  const long blocks = (long)nsb * nzg;
  if (a.cand.count)
    hipLaunchKernelGGL((ols_mixed2048_kernel<H, NT, OCC, true>), dim3((unsigned)blocks),
                       dim3(64 * NW), 0, st, static_cast<const c32 *>(a.spec), a.nbins,
                       static_cast<const H *>(a.bank), static_cast<const c32 *>(a.tw),
                       static_cast<const unsigned char *>(a.consts), a.power, a.ld, a.nseg, a.U,
                       a.half, a.nz, a.zpb, nsb, a.bank_log2, a.cand);
  else
    hipLaunchKernelGGL((ols_mixed2048_kernel<H, NT, OCC, false>), dim3((unsigned)blocks),
                       dim3(64 * NW), 0, st, static_cast<const c32 *>(a.spec), a.nbins,
                       static_cast<const H *>(a.bank), static_cast<const c32 *>(a.tw),
                       static_cast<const unsigned char *>(a.consts), a.power, a.ld, a.nseg, a.U,
                       a.half, a.nz, a.zpb, nsb, a.bank_log2, a.cand);
  return hipGetLastError();
}

template <class H, bool NT, int OCC>
static hipError_t launch_batch(const BatchArgs &a, hipStream_t st) {
  if (batch_persistent()) {
    hipError_t e = launch_reset_counter(a.counter, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ols_mixed2048_persistent_kernel<H, NT, OCC>), dim3((unsigned)a.grid),
                       dim3(64 * NW), 0, st, a.desc, a.nseries, (long long)a.total, a.counter,
                       static_cast<const H *>(a.bank), static_cast<const c32 *>(a.tw),
                       static_cast<const unsigned char *>(a.consts), a.U, a.half, a.bank_log2);
    return hipGetLastError();
  }
  if (a.total > (int64_t)0xffffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((ols_mixed2048_items_kernel<H, NT, OCC>), dim3((unsigned)a.total),
                     dim3(64 * NW), 0, st, a.desc, a.nseries, static_cast<const H *>(a.bank),
                     static_cast<const c32 *>(a.tw), static_cast<const unsigned char *>(a.consts),
                     a.U, a.half, a.bank_log2);
  return hipGetLastError();
}

template <class H, bool NT, int OCC>
static int batch_blocks_per_cu() {
  if (!batch_persistent()) return 1;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void *>(&ols_mixed2048_persistent_kernel<H, NT, OCC>),
          64 * NW, 0) != hipSuccess)
    return 1;
  return nb;
}

template <class H, bool NT, int OCC>
static int grid_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void *>(&ols_mixed2048_kernel<H, NT, OCC, false>), 64 * NW,
          0) != hipSuccess)
    return 0;
  return nb;
}

template <class H, bool NT, int OCC>
static OlsVariant make(const char *name, int precision) {
  OlsVariant v{};
  v.name = name;
  v.L = L;
  v.T = 64 * NW;
  v.G = 1;
  v.nbuf = 1;
  v.precision = precision;
  v.split = 0;
  v.zpb_target = 72;
  v.lay.L = L;
  v.lay.T = 128;
  v.lay.E = 16;
  v.lay.P = 3;
  v.lay.R[0] = 16;
  v.lay.R[1] = 16;
  v.lay.R[2] = 8;
  for (int i = 3; i < kMaxStages; ++i) v.lay.R[i] = 1;
  v.lds_bytes = 0;
  v.launch = &launch_single<H, NT, OCC>;
  v.launch_batch = &launch_batch<H, NT, OCC>;
  v.batch_blocks_per_cu = &batch_blocks_per_cu<H, NT, OCC>;
  v.grid_blocks_per_cu = &grid_blocks_per_cu<H, NT, OCC>;
  return v;
}

// ---- plan-time tables ------------------------------------------------------
struct c64m {
  double x, y;
};

// bank[i][plane][(k0 16 + k1) 8 + k2] = conj(FFT_L(h_i))[k0 + 16 k1 + 256 k2]
// (no 1/L; the kernel removes the factor 2^bank_log2 = L from the power);
// planes Re, Im rounded to 16 bits.
template <class H>
__global__ void bank_kernel(H *__restrict__ bank, const c64m *__restrict__ h, int nz, int m) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nz * L) return;
  const int i = (int)(idx / L);
  const int slot = (int)(idx % L);
  const int k = (slot >> 7) + 16 * ((slot >> 3) & 15) + 256 * (slot & 7);
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
__global__ void bank_natural_kernel(c32 *__restrict__ dst, const H *__restrict__ bank, int nz) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nz * L) return;
  const int i = (int)(idx / L);
  const int slot = (int)(idx % L);
  const int k = (slot >> 7) + 16 * ((slot >> 3) & 15) + 256 * (slot & 7);
  const H *row_i = bank + (long)i * 2 * L;
  const float inv = 1.0f / (float)L;
  dst[(long)i * L + k] = {(float)row_i[slot] * inv, (float)row_i[L + slot] * inv};
}

// Matrix operands, FP64 then rounded: lane l holds column c = l & 15 and K
// rows 8 (l >> 4) + j. Q (S2, tile k0): K 8 g + k2 holds the product of
// plane pair g (Re X Re T, Im X Im T, Re X Im T, Im X Re T); columns 0..7
// Re, 8..15 Im of n2; C = w2048^(n2 (256 k2 + k0)).
// P (S1, tile n2): K 0..15 Re over k1, 16..31 Im; column n1;
// C = w128^(k1 (8 n1 + n2)); the Im-plane K rows in the swapped order of
// their LDS chunks. F (S0): K over k0 as P, column n0, C = w16^(k0 n0).
// B1 = [Re C; -Im C] gives the real part, B2 = [Im C; Re C] the imaginary
// part. Twiddles: lane (g, c) multiplies its S1 results (rows k0 = 4g + i,
// column n1 = c) by w256^(k0 n1), stored as FP32 (Re x4, Im x4).
template <class H>
__global__ void consts_kernel(unsigned char *__restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // one per v8 entry
  const double kTwoPi = 6.283185307179586476925;
  if (idx < 64) {  // twiddles of lane idx
    const int c = idx & 15, g = idx >> 4;
    float *t = reinterpret_cast<float *>(out + kTwOff) + idx * 8;
    for (int i = 0; i < 4; ++i) {
      double sn, cs;
      sincos(kTwoPi * (double)(((4 * g + i) * c) & 255) / 256.0, &sn, &cs);
      t[i] = (float)cs;
      t[4 + i] = (float)sn;
    }
  }
  if (idx >= kConstV8) return;
  H *b = reinterpret_cast<H *>(out) + (size_t)idx * 8;
  if (idx < kPOff) {  // Q
    const int tile = idx / 64, lane = idx % 64;
    const int c = lane & 15, kg = lane >> 4;
    const int n2 = c & 7;
    const bool im_out = c >= 8;
    for (int j = 0; j < 8; ++j) {
      const int e = (n2 * (256 * j + tile)) & 2047;
      double sn, cs;
      sincos(kTwoPi * (double)e / 2048.0, &sn, &cs);
      // Re Y = g0 - g1, Im Y = g2 + g3; out_re = Re Y Cr - Im Y Ci,
      // out_im = Re Y Ci + Im Y Cr
      const double yr = kg == 0 ? 1.0 : (kg == 1 ? -1.0 : 0.0);
      const double yi = kg >= 2 ? 1.0 : 0.0;
      b[j] = (H)(!im_out ? yr * cs - yi * sn : yr * sn + yi * cs);
    }
    return;
  }
  const bool p_fam = idx < kFOff;
  const int rel = p_fam ? idx - kPOff : idx - kFOff;
  const int tile = rel / 128, lane = (rel / 2) % 64, which = rel % 2;
  const int c = lane & 15, kg = lane >> 4;
  for (int j = 0; j < 8; ++j) {
    const int kk = kg * 8 + j;
    const bool im_in = kk >= 16;
    const int k = 8 * (kg & 1) + (j ^ ((p_fam && im_in) ? 4 : 0));
    double sn, cs;
    if (p_fam) {
      const int e = (k * (8 * c + tile)) & 127;
      sincos(kTwoPi * (double)e / 128.0, &sn, &cs);
    } else {
      const int e = (k * c) & 15;
      sincos(kTwoPi * (double)e / 16.0, &sn, &cs);
    }
    const double v = which == 0 ? (!im_in ? cs : -sn) : (!im_in ? sn : cs);
    b[j] = (H)v;
  }
}

}  // namespace m2048

static const OlsVariant kMixed2048Variants[] = {
    m2048::make<_Float16, true, 8>("fp16_L2048_mfma_w16", 1),
    m2048::make<__bf16, true, 8>("bf16_L2048_mfma_w16", 2),
};

const OlsVariant *mixed2048_variants(int *count) {
  *count = (int)(sizeof(kMixed2048Variants) / sizeof(kMixed2048Variants[0]));
  return kMixed2048Variants;
}

size_t mixed2048_consts_bytes() { return (size_t)m2048::kConstBytes; }

hipError_t launch_mixed2048_consts(void *out, int precision, hipStream_t s) {
  const dim3 grid((unsigned)((m2048::kConstV8 + 255) / 256));
  if (precision == 2)
    hipLaunchKernelGGL(m2048::consts_kernel<__bf16>, grid, dim3(256), 0, s,
                       static_cast<unsigned char *>(out));
  else
    hipLaunchKernelGGL(m2048::consts_kernel<_Float16>, grid, dim3(256), 0, s,
                       static_cast<unsigned char *>(out));
  return hipGetLastError();
}

hipError_t launch_bank_mixed2048(void *bank, const void *h, int nz, int m, int precision,
                                 hipStream_t s) {
  const long n = (long)nz * m2048::L;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (precision == 2)
    hipLaunchKernelGGL(m2048::bank_kernel<__bf16>, grid, dim3(256), 0, s,
                       static_cast<__bf16 *>(bank), static_cast<const m2048::c64m *>(h), nz, m);
  else
    hipLaunchKernelGGL(m2048::bank_kernel<_Float16>, grid, dim3(256), 0, s,
                       static_cast<_Float16 *>(bank), static_cast<const m2048::c64m *>(h), nz, m);
  return hipGetLastError();
}

hipError_t launch_bank_mixed2048_natural(c32 *dst, const void *bank, int nz, int precision,
                                         hipStream_t s) {
  const long n = (long)nz * m2048::L;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (precision == 2)
    hipLaunchKernelGGL(m2048::bank_natural_kernel<__bf16>, grid, dim3(256), 0, s, dst,
                       static_cast<const __bf16 *>(bank), nz);
  else
    hipLaunchKernelGGL(m2048::bank_natural_kernel<_Float16>, grid, dim3(256), 0, s, dst,
                       static_cast<const _Float16 *>(bank), nz);
  return hipGetLastError();
}

}  // namespace fdas
