// In-register complex DFT kernels of radix 2, 4, 8 and 16 for gfx950.
//
// The discrete Fourier transform follows eq. 3 of the paper (Section 2):
// X_k = sum_n x_n exp(-i 2 pi n k / N). DIR = -1 is that forward transform,
// DIR = +1 its unnormalised inverse. Inputs and outputs are in natural order
// in a register array; radix 8 and 16 are built from radix-4 butterflies with
// their internal twiddles as compile-time constants, so trivial factors
// (1, -i, (1 -/+ i)/sqrt 2) cost adds only.
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

struct __attribute__((aligned(8))) c32 {
  float x, y;
};

__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  return {__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
__device__ __forceinline__ c32 cmulc(c32 a, c32 b) {
  return {__builtin_fmaf(a.x, b.x, a.y * b.y), __builtin_fmaf(a.y, b.x, -a.x * b.y)};
}

// Multiply by exp(DIR * i pi / 2): -i for the forward transform, +i inverse.
template <int DIR>
__device__ __forceinline__ c32 rot90(c32 v) {
  if constexpr (DIR < 0) return {v.y, -v.x};
  else return {-v.y, v.x};
}

// Multiply by exp(DIR * i 2 pi J / 16) for a compile-time J in [0, 16).
template <int DIR, int J>
__device__ __forceinline__ c32 tw16(c32 v) {
  constexpr float C1 = 0.92387953251128675613f;  // cos(pi/8)
  constexpr float S1 = 0.38268343236508977173f;  // sin(pi/8)
  constexpr float H = 0.70710678118654752440f;   // 1/sqrt(2)
  constexpr int j = J & 15;
  if constexpr (j == 0) {
    return v;
  } else if constexpr (j == 4) {
    return rot90<DIR>(v);
  } else if constexpr (j == 8) {
    return {-v.x, -v.y};
  } else if constexpr (j == 12) {
    return rot90<-DIR>(v);
  } else if constexpr (j == 2 || j == 6 || j == 10 || j == 14) {
    // (1 -/+ i)/sqrt2 rotated by multiples of 90 degrees
    c32 w;
    if constexpr (DIR < 0) w = {(v.x + v.y) * H, (v.y - v.x) * H};  // * (1 - i)/sqrt2
    else w = {(v.x - v.y) * H, (v.x + v.y) * H};                   // * (1 + i)/sqrt2
    if constexpr (j == 2) return w;
    else if constexpr (j == 6) return rot90<DIR>(w);
    else if constexpr (j == 10) return {-w.x, -w.y};
    else return rot90<-DIR>(w);
  } else {
    // odd j: exp(DIR i 2 pi j / 16) = cos(pi j/8) + DIR i sin(pi j/8)
    constexpr int q = j & 3;       // 1 or 3 within the quadrant
    constexpr int quad = j >> 2;   // number of 90 degree turns
    constexpr float c = (q == 1) ? C1 : S1;
    constexpr float s = (q == 1) ? S1 : C1;
    constexpr float sd = (DIR < 0) ? -s : s;
    c32 w = {__builtin_fmaf(v.x, c, -v.y * sd), __builtin_fmaf(v.x, sd, v.y * c)};
    if constexpr (quad == 0) return w;
    else if constexpr (quad == 1) return rot90<DIR>(w);
    else if constexpr (quad == 2) return {-w.x, -w.y};
    else return rot90<-DIR>(w);
  }
}

template <int DIR>
__device__ __forceinline__ void dft2(c32 &a, c32 &b) {
  c32 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(c32 &a, c32 &b, c32 &c, c32 &d) {
  c32 t0 = cadd(a, c), t1 = csub(a, c);
  c32 t2 = cadd(b, d), t3 = rot90<DIR>(csub(b, d));
  a = cadd(t0, t2);
  c = csub(t0, t2);
  b = cadd(t1, t3);
  d = csub(t1, t3);
}

// v[0..8) natural order in and out.
template <int DIR>
__device__ __forceinline__ void dft8(c32 *v) {
  c32 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  c32 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  o1 = tw16<DIR, 2>(o1);
  o2 = tw16<DIR, 4>(o2);
  o3 = tw16<DIR, 6>(o3);
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

// ---- second pass of the 16-point DFT ----------------------------------------
// After the first radix-4 pass v[4 k1 + n2] holds Y[n2][k1]; the second pass
// is, for each k1, a radix-4 DFT over n2 of Y[n2][k1] W16^(n2 k1). The
// twiddles are written as a scale times a cheaper factor,
//   W^1 = C (1 + D i t),  W^3 = C (t + D i),  W^2 = H (1 + D i),
//   W^4 = D i,  W^6 = D i W^2,  W^9 = -W^1
// (D = DIR, C = cos(pi/8), t = tan(pi/8), H = 1/sqrt 2), the cheap factors
// are applied first (two fused multiply-adds or two adds each), and the
// scale moves into the butterfly's last adds, which become fused
// multiply-adds: for a group the two odd twiddles share the scale C and the
// even ones the scale H. 16 operations fewer than twiddle-then-butterfly.

// v * (1 + D i t) and v * (t + D i)
template <int DIR>
__device__ __forceinline__ c32 tw_c1(c32 v) {
  constexpr float T8 = 0.41421356237309504880f;  // tan(pi/8)
  return {__builtin_fmaf(-DIR * T8, v.y, v.x), __builtin_fmaf(DIR * T8, v.x, v.y)};
}
template <int DIR>
__device__ __forceinline__ c32 tw_c3(c32 v) {
  constexpr float T8 = 0.41421356237309504880f;
  return {__builtin_fmaf(T8, v.x, -DIR * v.y), __builtin_fmaf(T8, v.y, DIR * v.x)};
}
// v * (1 + D i)
template <int DIR>
__device__ __forceinline__ c32 tw_h(c32 v) {
  if constexpr (DIR < 0) return {v.x + v.y, v.y - v.x};
  else return {v.x - v.y, v.y + v.x};
}
// a + k b and a - k b for a real scale k
__device__ __forceinline__ c32 caxpy(c32 a, float k, c32 b) {
  return {__builtin_fmaf(k, b.x, a.x), __builtin_fmaf(k, b.y, a.y)};
}

// Radix-4 butterfly over (p0, C a1, p2, C a3) with p2 = H u2 (EVEN_H) or
// p2 given (EVEN_H false), ODD_SIGN = -1 when the third input is -C a3.
template <int DIR, bool EVEN_H, int ODD_SIGN>
__device__ __forceinline__ void bfly_c(c32 &o0, c32 &o1, c32 &o2, c32 &o3, c32 p0, c32 a1, c32 p2,
                                       c32 a3) {
  constexpr float C1 = 0.92387953251128675613f;  // cos(pi/8)
  constexpr float H = 0.70710678118654752440f;
  const c32 t0 = EVEN_H ? caxpy(p0, H, p2) : cadd(p0, p2);
  const c32 t1 = EVEN_H ? caxpy(p0, -H, p2) : csub(p0, p2);
  const c32 s = ODD_SIGN > 0 ? cadd(a1, a3) : csub(a1, a3);   // (p1 + p3) / C
  const c32 d = rot90<DIR>(ODD_SIGN > 0 ? csub(a1, a3) : cadd(a1, a3));  // D i (p1 - p3) / C
  o0 = caxpy(t0, C1, s);
  o2 = caxpy(t0, -C1, s);
  o1 = caxpy(t1, C1, d);
  o3 = caxpy(t1, -C1, d);
}

template <int DIR>
__device__ __forceinline__ void dft16_pass2(c32 *v) {
  constexpr float H = 0.70710678118654752440f;
  dft4<DIR>(v[0], v[1], v[2], v[3]);  // k1 = 0: no twiddles
  {  // k1 = 1: W^1, W^2, W^3
    const c32 p0 = v[4], a1 = tw_c1<DIR>(v[5]), u2 = tw_h<DIR>(v[6]), a3 = tw_c3<DIR>(v[7]);
    bfly_c<DIR, true, +1>(v[4], v[5], v[6], v[7], p0, a1, u2, a3);
  }
  {  // k1 = 2: W^2, W^4, W^6 = D i W^2 (all with the scale H or none)
    const c32 p0 = v[8], p2 = rot90<DIR>(v[10]);
    const c32 u1 = tw_h<DIR>(v[9]), u3 = rot90<DIR>(tw_h<DIR>(v[11]));
    const c32 t0 = cadd(p0, p2), t1 = csub(p0, p2);
    const c32 s = cadd(u1, u3), d = rot90<DIR>(csub(u1, u3));
    v[8] = caxpy(t0, H, s);
    v[10] = caxpy(t0, -H, s);
    v[9] = caxpy(t1, H, d);
    v[11] = caxpy(t1, -H, d);
  }
  {  // k1 = 3: W^3, W^6 = D i W^2, W^9 = -W^1
    const c32 p0 = v[12], a1 = tw_c3<DIR>(v[13]), u2 = rot90<DIR>(tw_h<DIR>(v[14]));
    const c32 a3 = tw_c1<DIR>(v[15]);
    bfly_c<DIR, true, -1>(v[12], v[13], v[14], v[15], p0, a1, u2, a3);
  }
  // now v[4*k1 + k2] holds X[k1 + 4 k2]; transpose to natural order
  c32 t;
  t = v[1]; v[1] = v[4]; v[4] = t;
  t = v[2]; v[2] = v[8]; v[8] = t;
  t = v[3]; v[3] = v[12]; v[12] = t;
  t = v[6]; v[6] = v[9]; v[9] = t;
  t = v[7]; v[7] = v[13]; v[13] = t;
  t = v[11]; v[11] = v[14]; v[14] = t;
}

// v[0..16) natural order in and out: 4 x 4 decomposition n = 4 n1 + n2,
// k = k1 + 4 k2, internal twiddle W16^(n2 k1).
template <int DIR>
__device__ __forceinline__ void dft16(c32 *v) {
  dft4<DIR>(v[0], v[4], v[8], v[12]);
  dft4<DIR>(v[1], v[5], v[9], v[13]);
  dft4<DIR>(v[2], v[6], v[10], v[14]);
  dft4<DIR>(v[3], v[7], v[11], v[15]);
  dft16_pass2<DIR>(v);
}

// ---- twiddled butterflies ---------------------------------------------------
// Radix-R DFT of inputs v[k] * w[k] (w[0] = 1 implied), with the twiddle
// products folded into the first butterfly layer: a + b*w costs four fused
// multiply-adds and a - b*w = 2a - (a + b*w) two more. CONJ selects conj(w).

template <bool CONJ>
__device__ __forceinline__ c32 cfma(c32 a, c32 b, c32 w) {  // a + b * w'
  if constexpr (CONJ)
    return {__builtin_fmaf(b.x, w.x, __builtin_fmaf(b.y, w.y, a.x)),
            __builtin_fmaf(b.y, w.x, __builtin_fmaf(-b.x, w.y, a.y))};
  else
    return {__builtin_fmaf(b.x, w.x, __builtin_fmaf(-b.y, w.y, a.x)),
            __builtin_fmaf(b.y, w.x, __builtin_fmaf(b.x, w.y, a.y))};
}
template <bool CONJ>
__device__ __forceinline__ c32 cmul_t(c32 b, c32 w) {  // b * w'
  return CONJ ? cmulc(b, w) : cmul(b, w);
}
__device__ __forceinline__ c32 twice_minus(c32 a, c32 s) {  // 2a - s
  return {__builtin_fmaf(2.0f, a.x, -s.x), __builtin_fmaf(2.0f, a.y, -s.y)};
}

// First radix-2 layers of a radix-4 butterfly on (a, b, c, d) scaled by
// (wa, wb, wc, wd); TA says whether a carries a twiddle.
template <int DIR, bool CONJ, bool TA>
__device__ __forceinline__ void dft4_tw(c32 &a, c32 &b, c32 &c, c32 &d, c32 wa, c32 wb, c32 wc,
                                        c32 wd) {
  const c32 a1 = TA ? cmul_t<CONJ>(a, wa) : a;
  const c32 t0 = cfma<CONJ>(a1, c, wc);
  const c32 t1 = twice_minus(a1, t0);
  const c32 b1 = cmul_t<CONJ>(b, wb);
  const c32 t2 = cfma<CONJ>(b1, d, wd);
  const c32 t3 = rot90<DIR>(twice_minus(b1, t2));
  a = cadd(t0, t2);
  c = csub(t0, t2);
  b = cadd(t1, t3);
  d = csub(t1, t3);
}

// W0: the first input carries a factor w[0] too (a radix DFT of a pointwise
// product v * w), else w[0] = 1 is implied.
template <int DIR, bool CONJ, bool W0 = false>
__device__ __forceinline__ void dft16_tw(c32 *v, const c32 *w) {
  const c32 one = {1.f, 0.f};
  dft4_tw<DIR, CONJ, W0>(v[0], v[4], v[8], v[12], W0 ? w[0] : one, w[4], w[8], w[12]);
  dft4_tw<DIR, CONJ, true>(v[1], v[5], v[9], v[13], w[1], w[5], w[9], w[13]);
  dft4_tw<DIR, CONJ, true>(v[2], v[6], v[10], v[14], w[2], w[6], w[10], w[14]);
  dft4_tw<DIR, CONJ, true>(v[3], v[7], v[11], v[15], w[3], w[7], w[11], w[15]);
  dft16_pass2<DIR>(v);
}

template <int DIR, bool CONJ, bool W0 = false>
__device__ __forceinline__ void dft8_tw(c32 *v, const c32 *w) {
  const c32 one = {1.f, 0.f};
  c32 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  c32 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4_tw<DIR, CONJ, W0>(e0, e1, e2, e3, W0 ? w[0] : one, w[2], w[4], w[6]);
  dft4_tw<DIR, CONJ, true>(o0, o1, o2, o3, w[1], w[3], w[5], w[7]);
  o1 = tw16<DIR, 2>(o1);
  o2 = tw16<DIR, 4>(o2);
  o3 = tw16<DIR, 6>(o3);
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <int DIR, bool CONJ, int R, bool W0 = false>
__device__ __forceinline__ void dft_tw(c32 *v, const c32 *w) {
  static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
  if constexpr (R == 2) {
    const c32 a = W0 ? cmul_t<CONJ>(v[0], w[0]) : v[0];
    const c32 t0 = cfma<CONJ>(a, v[1], w[1]);
    v[1] = twice_minus(a, t0);
    v[0] = t0;
  } else if constexpr (R == 4) {
    dft4_tw<DIR, CONJ, W0>(v[0], v[1], v[2], v[3], W0 ? w[0] : c32{1.f, 0.f}, w[1], w[2], w[3]);
  } else if constexpr (R == 8) {
    dft8_tw<DIR, CONJ, W0>(v, w);
  } else {
    dft16_tw<DIR, CONJ, W0>(v, w);
  }
}

// The pointer value passes through an empty asm statement, so loads through
// it cannot be hoisted out of the loop the call sits in (keeps loop-invariant
// table reads inside persistent loops instead of pinning them in registers).
template <class T>
__device__ __forceinline__ T *opaque_ptr(T *p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Global-memory view of a pointer. Pointers read from memory (descriptor
// tables) or passed through asm are generic to the compiler, which then emits
// FLAT loads and stores; those also count on the LDS counter, so every LDS
// wait would wait for them too. Through a global pointer the compiler emits
// global_load / global_store.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> to_global(T *p) {
  return (gptr<T>)p;
}

typedef float f2v __attribute__((ext_vector_type(2)));
// one 8-byte global load of a complex value
__device__ __forceinline__ c32 ldg(gptr<const c32> p) {
  const f2v v = *reinterpret_cast<gptr<const f2v>>(p);
  return {v.x, v.y};
}

template <int DIR, int R>
__device__ __forceinline__ void dft(c32 *v) {
  static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
  if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
  else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<DIR>(v);
  else dft16<DIR>(v);
}

}  // namespace fdas
