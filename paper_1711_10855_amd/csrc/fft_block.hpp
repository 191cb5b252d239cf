// Block-level FFT building blocks shared by the overlap-and-save kernel and
// the standalone batched FFT: the stage geometry of an L-point transform
// split over T threads (radices R[0] .. R[P-1], outermost first), the LDS
// addresses of every stage and the register <-> LDS exchanges between stages.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_radix.hpp"

namespace fdas {

template <int Begin, int End, class F>
__device__ __forceinline__ void static_for_up(F &&f) {
  if constexpr (Begin < End) {
    f(std::integral_constant<int, Begin>{});
    static_for_up<Begin + 1, End>(f);
  }
}
template <int Begin, int End, class F>  // Begin, Begin-1, ..., End (inclusive)
__device__ __forceinline__ void static_for_down(F &&f) {
  if constexpr (Begin >= End) {
    f(std::integral_constant<int, Begin>{});
    static_for_down<Begin - 1, End>(f);
  }
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

template <int L_, int T_, int... Rs>
struct Geo {
  static constexpr int L = L_;
  static constexpr int T = T_;
  static constexpr int E = L_ / T_;
  static constexpr int P = sizeof...(Rs);
  static constexpr int R[P] = {Rs...};
  static constexpr int S(int i) {
    int s = 1;
    for (int j = i + 1; j < P; ++j) s *= R[j];
    return s;
  }
  static constexpr int B(int i) { return E / R[i]; }
  static constexpr int PADSH = ilog2(R[P - 1]);
  static constexpr int LP = L + (L >> PADSH);  // padded LDS length per segment
  // offsets of each stage's inverse twiddles in a flat register array
  static constexpr int TWOFF(int i) {
    int o = 0;
    for (int j = 0; j < i; ++j) o += B(j) * (R[j] - 1);
    return o;
  }
  static constexpr int NTW = TWOFF(P - 1);
  // Thread that owns address a in stage i (butterfly b = t + j T).
  static constexpr int owner(int i, int a) {
    const int s = S(i), r = R[i];
    const int prefix = a / (r * s), mi = a % s;
    return (prefix * s + mi) % T;
  }
  // An exchange between stages i and i+1 is wave-local when every address is
  // owned by threads of the same 64-lane wave in both layouts; it then needs
  // no workgroup barrier, only ordering within the wave.
  static constexpr bool local(int i, int waves_per_seg_slot_base = 0) {
    (void)waves_per_seg_slot_base;
    if (T <= 64) return true;  // a segment never straddles a wave
    for (int a = 0; a < L; ++a)
      if (owner(i, a) / 64 != owner(i + 1, a) / 64) return false;
    return true;
  }
  static constexpr bool any_block() {
    for (int i = 0; i + 1 < P; ++i)
      if (!local(i)) return true;
    return false;
  }
  // two buffers when a block-wide exchange exists and they fit in LDS
  static constexpr int NBUF = (any_block() && 2 * LP * 8 <= 80 * 1024) ? 2 : 1;
};

// The same geometry with one LDS buffer (every block-wide exchange then
// ends with a second barrier): half the LDS, so more blocks per CU.
template <class G>
struct OneBuf : G {
  static constexpr int NBUF = 1;
};

template <class Gm>
__device__ __forceinline__ int pad(int a) {
  return a + (a >> Gm::PADSH);
}

// Address of element n of the j-th butterfly of thread t in stage I.
template <class Gm, int I>
__device__ __forceinline__ int stage_addr(int t, int j, int n) {
  constexpr int S = Gm::S(I), R = Gm::R[I];
  const int b = t + j * Gm::T;
  const int prefix = b / S, mi = b % S;
  return prefix * R * S + n * S + mi;
}
template <class Gm, int I>
__device__ __forceinline__ int stage_suffix(int t, int j) {
  return (t + j * Gm::T) % Gm::S(I);
}

// Ordering of LDS traffic inside one wave (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Registers in the layout of stage A -> LDS -> registers in the layout of
// stage Bst, through buffer PAR. Block-wide exchanges alternate between the
// two buffers so that one barrier per exchange suffices; wave-local exchanges
// touch only addresses their own wave owns and use the buffer of the next
// block-wide exchange. The parity is a compile-time value, so every LDS
// address is a loop-invariant register plus an immediate offset.
template <class Gm, int A, int Bst, int PAR>
__device__ __forceinline__ void exchange(c32 (&d)[Gm::E], c32 *buf0, c32 *buf1, int t) {
  constexpr int RA = Gm::R[A], RB = Gm::R[Bst];
  constexpr int lo = A < Bst ? A : Bst;
  constexpr bool loc = Gm::local(lo);
  c32 *buf = PAR ? buf1 : buf0;
#pragma unroll
  for (int j = 0; j < Gm::B(A); ++j)
#pragma unroll
    for (int n = 0; n < RA; ++n) buf[pad<Gm>(stage_addr<Gm, A>(t, j, n))] = d[j * RA + n];
  if constexpr (loc) {
    wave_sync();
  } else {
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < Gm::B(Bst); ++j)
#pragma unroll
    for (int n = 0; n < RB; ++n) d[j * RB + n] = buf[pad<Gm>(stage_addr<Gm, Bst>(t, j, n))];
  if constexpr (loc) {
    wave_sync();
  } else if constexpr (Gm::NBUF == 1) {
    __syncthreads();  // single buffer: every read done before the next write
  }
}

// Buffer parity bookkeeping: the number of block-wide exchanges among the
// exchanges with lower stage index in [a, b) (each flips the buffer when
// there are two).
template <class Gm>
constexpr int flips(int a, int b) {
  int f = 0;
  for (int j = a; j < b; ++j) f += (Gm::NBUF == 2 && !Gm::local(j)) ? 1 : 0;
  return f;
}

}  // namespace fdas
