// Register/slot layout of the overlap-and-save FFTs and its frequency map.
//
// An L-point transform is factored into radices R[0] .. R[P-1] (outermost
// first). Address a = sum_i k_i * S_i with S_i = R[i+1] * ... * R[P-1]. The
// forward FFT is decimation in frequency: stage i transforms digit i in place,
// so after the last stage address a holds frequency
//     k = k_0 + R[0] * (k_1 + R[1] * (k_2 + ...))   (digits reversed).
// The inverse FFT runs the same stages in reverse order (decimation in time)
// and returns natural order, so no reordering pass is ever made.
//
// Thread t of T owns E = L / T elements. In stage i it handles butterflies
// b = t + j*T, j in [0, E/R[i]); butterfly b = prefix * S_i + mi reads the
// addresses prefix * R[i] * S_i + n * S_i + mi, n in [0, R[i]). Register slot
// e = j * R[i] + n. After the last forward stage slot (t, e) of every thread
// is what the bank is laid out against: bank[z][e][t] = T_z[k(t, e)].
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

constexpr int kMaxStages = 6;

struct LayoutDesc {
  int L, T, E, P;
  int R[kMaxStages];
};

__host__ __device__ inline int layout_stride(const LayoutDesc &d, int i) {
  int s = 1;
  for (int j = i + 1; j < d.P; ++j) s *= d.R[j];
  return s;
}

// Frequency held by register slot e of thread t after the last forward stage.
__host__ __device__ inline int layout_slot_freq(const LayoutDesc &d, int t, int e) {
  const int r = d.R[d.P - 1];
  const int j = e / r, n = e % r;
  const int b = t + j * d.T;
  int a = b * r + n;  // S_{P-1} = 1
  int digits[kMaxStages];
  for (int i = d.P - 1; i >= 0; --i) {
    digits[i] = a % d.R[i];
    a /= d.R[i];
  }
  int k = 0;
  for (int i = d.P - 1; i >= 0; --i) k = k * d.R[i] + digits[i];
  return k;
}

}  // namespace fdas
