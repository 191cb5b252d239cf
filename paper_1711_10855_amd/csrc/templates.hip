// Plan-time device kernels, all arithmetic in FP64:
//   * the response templates H_z(q) (Section 1: the predicted, normalised
//     Fourier response used in eq. 2),
//   * the Fourier-domain bank T_z[k] = conj(FFT_L(h_z))[k] / L with
//     h_z[q mod L] = H_z(q) (the per-segment filter of overlap-and-save,
//     Section 2), written in the hot kernel's slot order,
//   * the twiddle table W_L^j = exp(-i 2 pi j / L) of eq. 3.
//
// Template: G_z(q) = int_{-1/2}^{1/2} exp(i pi (z s^2 - 2 q s)) ds and
// H_z(q) = exp(-i pi q) G_z(q). For z > 0, completing the square,
//   G_z(q) = exp(-i pi q^2/z) / sqrt(2z) * [F(t2) - F(t1)],
//   t1 = sqrt(2z)(-1/2 - q/z), t2 = sqrt(2z)(1/2 - q/z),
// with F(x) = C(x) + i S(x) the Fresnel integrals (kernel exp(i pi t^2/2)).
// For x >= 0 write F(x) = (1+i)/2 - a(x) exp(i pi x^2/2); F is odd. Since
// (pi/2) t2^2 = pi (z/4 - q + q^2/z) and (pi/2) t1^2 = pi (z/4 + q + q^2/z),
// exp(-i pi q^2/z) exp(i pi t_{1,2}^2/2) = exp(i pi (z/4 +/- q)) exactly, so
// the only large phase left, exp(-i pi q^2/z), is reduced exactly as
// fmod(q^2, 2z)/z; it appears only when t1 < 0 < t2.
//
// a(x): for small x from the power series
//   F(x) = sum_n (i pi/2)^n x^(2n+1) / (n! (2n+1)),  a = ((1+i)/2 - F) e^{-i pi x^2/2};
// otherwise from F(x) = (1+i)/2 erf(w), w = (sqrt(pi)/2)(1 - i) x, so that
//   a(x) = (1+i)/2 * exp(w^2) erfc(w),
// with exp(w^2) erfc(w) from its Laplace continued fraction
//   sqrt(pi) exp(w^2) erfc(w) = 1/(w + (1/2)/(w + (2/2)/(w + (3/2)/(w + ...))))
// (valid for Re w > 0), evaluated by the modified Lentz method.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fft_radix.hpp"
#include "layout.hpp"

namespace fdas {

struct c64 {
  double x, y;
};

__device__ inline c64 zmul(c64 a, c64 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline c64 zadd(c64 a, c64 b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline c64 zsub(c64 a, c64 b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline c64 zscale(c64 a, double s) { return {a.x * s, a.y * s}; }
__device__ inline c64 zdiv(c64 a, c64 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return {(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return {(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}
__device__ inline double zabs(c64 a) { return hypot(a.x, a.y); }

// exp(i pi u) for a real u (argument given in half-turns).
__device__ inline c64 expipi(double u) {
  double s, c;
  sincospi(u, &s, &c);
  return {c, s};
}

constexpr double kSmallX = 1.8;

// a(x) for x >= 0 (see the file comment).
__device__ c64 fresnel_aux(double x) {
  const double kPi = 3.14159265358979323846;
  if (x < kSmallX) {
    const c64 zz = {0.0, 0.5 * kPi * x * x};  // i pi x^2 / 2
    c64 term = {x, 0.0};                      // (i pi x^2/2)^n x / n!
    c64 f = {0.0, 0.0};
    for (int n = 0; n < 64; ++n) {
      const c64 t = zscale(term, 1.0 / (2 * n + 1));
      f = zadd(f, t);
      if (zabs(t) <= 1e-17 * zabs(f)) break;
      term = zscale(zmul(term, zz), 1.0 / (n + 1));
    }
    const c64 e = expipi(-0.5 * x * x);
    return zmul({0.5 - f.x, 0.5 - f.y}, e);
  }
  const double sp = 0.88622692545275801365;  // sqrt(pi)/2
  const c64 w = {sp * x, -sp * x};
  const double tiny = 1e-300;
  c64 f = {tiny, 0.0}, C = f, D = {0.0, 0.0};
  for (int n = 1; n < 400; ++n) {
    const double an = (n == 1) ? 1.0 : 0.5 * (n - 1);
    D = zadd(w, zscale(D, an));
    if (zabs(D) < tiny) D = {tiny, 0.0};
    D = zdiv({1.0, 0.0}, D);
    C = zadd(w, zdiv({an, 0.0}, C));
    if (zabs(C) < tiny) C = {tiny, 0.0};
    const c64 dl = zmul(C, D);
    f = zmul(f, dl);
    if (fabs(dl.x - 1.0) + fabs(dl.y) < 1e-16) break;
  }
  const double inv_sqrt_pi = 0.56418958354775628695;
  const c64 k = zscale(f, inv_sqrt_pi);
  return zmul({0.5, 0.5}, k);
}

// G_z(q) for z > 0.
__device__ c64 response_g_pos(double z, double q) {
  const double rt = sqrt(2.0 * z);
  const double t1 = rt * (-0.5 - q / z);
  const double t2 = rt * (0.5 - q / z);
  const c64 p2 = expipi(fmod(0.25 * z - q, 2.0));  // e^{-i pi q^2/z} e^{i pi t2^2/2}
  const c64 p1 = expipi(fmod(0.25 * z + q, 2.0));  // e^{-i pi q^2/z} e^{i pi t1^2/2}
  const c64 a2 = zmul(fresnel_aux(fabs(t2)), p2);
  const c64 a1 = zmul(fresnel_aux(fabs(t1)), p1);
  c64 g;
  if (t1 < 0.0 && t2 >= 0.0) {
    // F(t2) - F(t1) = (1+i) - a(t2) E(t2) - a(|t1|) E(t1)
    const c64 p0 = expipi(-fmod(q * q, 2.0 * z) / z);
    g = zsub(zsub(zmul({1.0, 1.0}, p0), a2), a1);
  } else if (t1 >= 0.0) {
    // both arguments >= 0: the (1+i)/2 terms cancel exactly
    g = zsub(a1, a2);
  } else {
    // both < 0: F(t) = -(1+i)/2 + a(|t|) E(t)
    g = zsub(a2, a1);
  }
  return zscale(g, 1.0 / rt);
}

__device__ c64 template_h(double z, double q) {
  c64 g;
  if (z == 0.0) {
    const double s = (q == 0.0) ? 1.0 : sinpi(q) / (3.14159265358979323846 * q);
    g = {s, 0.0};
  } else {
    g = response_g_pos(fabs(z), q);
    if (z < 0.0) g.y = -g.y;
  }
  return zmul(expipi(-fmod(q, 2.0)), g);
}

// H[i][j] = H_{z_i}(j - m/2), z_i = -zmax + i dz. With interbin the rows
// come in pairs: H[2i][j] = H_{z_i}(j - m/2) and H[2i+1][j] = H_{z_i}(j - m/2
// - 1/2), the response at r + 1/2 from the same bins.
__global__ void templates_kernel(c64 *__restrict__ out, int rows, int m, double zmax, double dz,
                                 int interbin) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int taps = m + 1;
  if (idx >= rows * taps) return;
  const int row = idx / taps, j = idx % taps;
  const int i = interbin ? row >> 1 : row;
  const double shift = (interbin && (row & 1)) ? 0.5 : 0.0;
  const double z = -zmax + i * dz;
  out[idx] = template_h(z, (double)(j - m / 2) - shift);
}

// W_L^j = exp(-i 2 pi j / L), rounded to FP32.
__global__ void twiddle_kernel(c32 *__restrict__ tw, int L) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
  double s, c;
  sincospi(-2.0 * (double)j / (double)L, &s, &c);
  tw[j] = {(float)c, (float)s};
}

// bank[i][e][t] = conj(sum_q H_i(q) W_L^{(q mod L) k}) / L with k the
// frequency of slot (t, e). One thread per (i, slot). FP64 throughout.
__global__ void bank_kernel(c32 *__restrict__ bank, const c64 *__restrict__ h, int nz, int m,
                            LayoutDesc lay) {
  const int L = lay.L;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nz * L) return;
  const int i = (int)(idx / L);
  const int slot = (int)(idx % L);
  const int e = slot / lay.T, t = slot % lay.T;
  const int k = layout_slot_freq(lay, t, e);
  const c64 *hi = h + (long)i * (m + 1);
  double sr = 0.0, si = 0.0;
  for (int j = 0; j <= m; ++j) {
    const int q = j - m / 2;
    const int qm = ((q % L) + L) % L;
    const long ph = ((long)qm * k) % L;
    double s, c;
    sincospi(-2.0 * (double)ph / (double)L, &s, &c);
    const c64 v = hi[j];
    sr += v.x * c - v.y * s;
    si += v.x * s + v.y * c;
  }
  const double inv = 1.0 / (double)L;
  bank[idx] = {(float)(sr * inv), (float)(-si * inv)};
}

// Natural-order copy of a slot-ordered bank: dst[i][k(t,e)] = bank[i][e][t].
__global__ void bank_natural_kernel(c32 *__restrict__ dst, const c32 *__restrict__ bank, int nz,
                                    LayoutDesc lay) {
  const int L = lay.L;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nz * L) return;
  const int i = (int)(idx / L);
  const int slot = (int)(idx % L);
  const int e = slot / lay.T, t = slot % lay.T;
  const int k = layout_slot_freq(lay, t, e);
  dst[(long)i * L + k] = bank[idx];
}

hipError_t launch_templates(void *out, int rows, int m, double zmax, double dz, int interbin,
                            hipStream_t s) {
  const int n = rows * (m + 1);
  hipLaunchKernelGGL(templates_kernel, dim3((n + 255) / 256), dim3(256), 0, s,
                     static_cast<c64 *>(out), rows, m, zmax, dz, interbin);
  return hipGetLastError();
}

hipError_t launch_twiddles(c32 *tw, int L, hipStream_t s) {
  hipLaunchKernelGGL(twiddle_kernel, dim3((L + 255) / 256), dim3(256), 0, s, tw, L);
  return hipGetLastError();
}

hipError_t launch_bank(c32 *bank, const void *h, int nz, int m, const LayoutDesc &lay,
                       hipStream_t s) {
  const long n = (long)nz * lay.L;
  hipLaunchKernelGGL(bank_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, bank,
                     static_cast<const c64 *>(h), nz, m, lay);
  return hipGetLastError();
}

hipError_t launch_bank_natural(c32 *dst, const c32 *bank, int nz, const LayoutDesc &lay,
                               hipStream_t s) {
  const long n = (long)nz * lay.L;
  hipLaunchKernelGGL(bank_natural_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     dst, bank, nz, lay);
  return hipGetLastError();
}

}  // namespace fdas
