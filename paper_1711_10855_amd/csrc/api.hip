// Host side of the C ABI declared in include/fdas.h: argument validation
// (always before any HIP call), plan construction and kernel dispatch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "fdas.h"
#include "fft_batch.hpp"
#include "frontend.hpp"
#include "ols_variants.hpp"
#include "peaks.hpp"
#include "plan.hpp"

namespace fdas {

static thread_local std::string g_last_error;

int set_error(int status, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int hip_error(hipError_t e, const char *what) {
  return set_error(FDAS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

static int next_pow2(double v) {
  int p = 1;
  while (p < v && p < (1 << 30)) p <<= 1;
  return p;
}

// Validate the z grid; returns nz or a negative status.
static int validate_grid(double zmax, double dz) {
  if (!std::isfinite(zmax) || !std::isfinite(dz) || zmax < 0.0 || dz <= 0.0)
    return set_error(FDAS_ERR_INVALID, "need finite zmax >= 0 and dz > 0 (zmax=%g dz=%g)", zmax, dz);
  const double span = 2.0 * zmax / dz;
  if (span > 1e6) return set_error(FDAS_ERR_INVALID, "2*zmax/dz = %g is too large", span);
  const double n = std::nearbyint(span);
  if (std::fabs(span - n) > 1e-9)
    return set_error(FDAS_ERR_INVALID, "2*zmax/dz = %.12g is not an integer", span);
  return (int)n + 1;
}

int resolve_params(const fdas_params *in, fdas_params *out, int *nz_out) {
  if (!in || !out) return set_error(FDAS_ERR_INVALID, "null params pointer");
  fdas_params p = *in;
  const int ntz = validate_grid(p.zmax, p.dz);
  if (ntz < 0) return ntz;
  if (p.flags & ~(FDAS_FLAG_SPLIT | FDAS_FLAG_AUTOTUNE | FDAS_FLAG_INTERBIN | FDAS_FLAG_BANK))
    return set_error(FDAS_ERR_INVALID, "unknown flag bits 0x%x", p.flags);
  // bank and plane rows: one per trial drift, two with half-bin rows
  const int nz = (p.flags & FDAS_FLAG_INTERBIN) ? 2 * ntz : ntz;
  if (p.precision != FDAS_FP32 && p.precision != FDAS_MIXED_FP16 &&
      p.precision != FDAS_MIXED_BF16)
    return set_error(FDAS_ERR_INVALID, "unknown precision %d", p.precision);
  if ((p.flags & FDAS_FLAG_SPLIT) && p.precision == FDAS_FP32)
    return set_error(FDAS_ERR_INVALID, "FDAS_FLAG_SPLIT applies to the mixed precisions only");
  if (p.m == 0) {
    p.m = next_pow2(2.0 * p.zmax + 32.0);
    if (p.m < 8) p.m = 8;
  }
  if (p.m < 2 || (p.m & 1)) return set_error(FDAS_ERR_INVALID, "m must be even and >= 2 (m=%d)", p.m);
  if (p.m > 8192) return set_error(FDAS_ERR_UNSUPPORTED, "m=%d exceeds the largest segment", p.m);
  if (p.seg_len < 0) return set_error(FDAS_ERR_INVALID, "seg_len must be >= 0");
  if (p.seg_len == 0 && (p.flags & FDAS_FLAG_AUTOTUNE)) {
    // the autotuner picks a compiled length with L - m >= L / 2
    *out = p;
    if (nz_out) *nz_out = nz;
    return FDAS_OK;
  }
  if (p.seg_len == 0) p.seg_len = default_seg_len(p.m, nz, p.precision);
  if (p.seg_len <= p.m)
    return set_error(FDAS_ERR_INVALID, "seg_len (%d) must exceed m (%d)", p.seg_len, p.m);
  if ((p.seg_len & (p.seg_len - 1)) || p.seg_len < 256 || p.seg_len > 16384)
    return set_error(FDAS_ERR_UNSUPPORTED, "seg_len %d: compiled lengths are powers of two in [256, 16384]",
                     p.seg_len);
  if (p.precision != FDAS_FP32) {
    const int split = (p.flags & FDAS_FLAG_SPLIT) ? 1 : 0;
    if (!mixed_supported(p.seg_len, split))
      return set_error(FDAS_ERR_UNSUPPORTED, "precision %d%s is not available for seg_len %d",
                       p.precision, split ? " with the split form" : "", p.seg_len);
  }
  *out = p;
  if (nz_out) *nz_out = nz;
  return FDAS_OK;
}

int default_seg_len(int m, int nz, int precision) {
  (void)nz;
  if (precision != FDAS_FP32) return 4096;  // the faster matrix-core length
  int L = next_pow2(8.0 * m);
  if (L < 256) L = 256;
  if (L > 16384) L = 16384;
  return L;
}

// Device guard: makes `dev` current for the scope and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace fdas

// Standalone batched FFT: the compiled form and its twiddle table.
struct fdas_fft_s {
  int device;
  const fdas::FftVariant *v;
  fdas::c32 *tw;
};

// Device front end: geometry, twiddle tables and scratch.
struct fdas_frontend_s {
  int device;
  int64_t n;
  fdas::FrontendGeom g;
  fdas::c32 *tw1, *tw2, *work;
  float *pw;
  void *sel;
};

namespace fdas {

// Compiled form for (n, elements per thread); elems 0 picks the default.
// FDAS_FFT_VARIANT names a form that replaces the choice for its length.
static int find_fft(int n, int elems, const FftVariant **out) {
  int count = 0;
  const FftVariant *vs = fft_variants(&count);
  if (const char *force = std::getenv("FDAS_FFT_VARIANT")) {
    for (int i = 0; i < count; ++i)
      if (vs[i].L == n && std::strcmp(vs[i].name, force) == 0 &&
          (elems == 0 || vs[i].E == elems)) {
        *out = &vs[i];
        return FDAS_OK;
      }
  }
  bool length_known = false;
  for (int i = 0; i < count; ++i) {
    if (vs[i].L != n) continue;
    length_known = true;
    if (elems == 0 || vs[i].E == elems) {
      *out = &vs[i];
      return FDAS_OK;
    }
  }
  if (!length_known) return set_error(FDAS_ERR_UNSUPPORTED, "no compiled FFT of length %d", n);
  return set_error(FDAS_ERR_UNSUPPORTED, "no compiled FFT of length %d with %d elements per thread",
                   n, elems);
}

}  // namespace fdas

using namespace fdas;

extern "C" {

const char *fdas_status_string(int status) {
  switch (status) {
    case FDAS_OK: return "ok";
    case FDAS_ERR_INVALID: return "invalid argument";
    case FDAS_ERR_UNSUPPORTED: return "unsupported configuration";
    case FDAS_ERR_NOMEM: return "out of memory";
    case FDAS_ERR_DEVICE: return "device error";
    default: return "unknown status";
  }
}

const char *fdas_last_error(void) { return g_last_error.c_str(); }

int fdas_kernel_variants(int seg_len, int precision, char *buf, size_t len) {
  if (seg_len < 0 || precision < -1 || precision > FDAS_MIXED_BF16)
    return set_error(FDAS_ERR_INVALID, "bad seg_len %d or precision %d", seg_len, precision);
  if (!buf && len) return set_error(FDAS_ERR_INVALID, "null buffer with nonzero length");
  return list_variants(seg_len, precision, buf, len);
}

int fdas_plane_rows(const fdas_params *p) {
  if (!p) return set_error(FDAS_ERR_INVALID, "null params pointer");
  const int nz = validate_grid(p->zmax, p->dz);
  if (nz < 0) return nz;
  return (p->flags & FDAS_FLAG_INTERBIN) ? 2 * nz : nz;
}

int fdas_resolve_params(const fdas_params *in, fdas_params *out) {
  return resolve_params(in, out, nullptr);
}

int fdas_make_templates(const fdas_params *p, void *templates, size_t *bytes, void *stream) {
  fdas_params r;
  int nz = 0;
  int st = resolve_params(p, &r, &nz);
  if (st) return st;
  if (!bytes) return set_error(FDAS_ERR_INVALID, "null bytes pointer");
  const bool bank = (r.flags & FDAS_FLAG_BANK) != 0;
  if (bank && r.seg_len <= r.m)
    return set_error(FDAS_ERR_INVALID, "the bank needs a segment length (not autotuned)");
  const size_t need = bank ? (size_t)nz * (size_t)r.seg_len * 8 : (size_t)nz * (size_t)(r.m + 1) * 16;
  if (!templates) {
    *bytes = need;
    return FDAS_OK;
  }
  if (*bytes < need) {
    const size_t have = *bytes;
    *bytes = need;
    return set_error(FDAS_ERR_INVALID, "templates buffer holds %zu bytes, need %zu", have, need);
  }
  if (reinterpret_cast<uintptr_t>(templates) & 7)
    return set_error(FDAS_ERR_INVALID, "misaligned templates buffer");
  *bytes = need;
  const int interbin = (r.flags & FDAS_FLAG_INTERBIN) ? 1 : 0;
  const hipStream_t s = (hipStream_t)stream;
  if (!bank) {
    const hipError_t e = launch_templates(templates, nz, r.m, r.zmax, r.dz, interbin, s);
    if (e != hipSuccess) return hip_error(e, "template kernel launch");
    return FDAS_OK;
  }
  // natural frequency order: one radix-L "stage" on one thread maps slot e to
  // frequency e
  LayoutDesc nat{};
  nat.L = r.seg_len;
  nat.T = 1;
  nat.E = r.seg_len;
  nat.P = 1;
  nat.R[0] = r.seg_len;
  for (int i = 1; i < kMaxStages; ++i) nat.R[i] = 1;
  void *h = nullptr;
  hipError_t e = hipMalloc(&h, (size_t)nz * (size_t)(r.m + 1) * 16);
  if (e != hipSuccess) return set_error(FDAS_ERR_NOMEM, "template temporary: %s", hipGetErrorString(e));
  e = launch_templates(h, nz, r.m, r.zmax, r.dz, interbin, s);
  if (e == hipSuccess) e = launch_bank(static_cast<c32 *>(templates), h, nz, r.m, nat, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(h);
  if (e != hipSuccess) return hip_error(e, "bank kernel launch");
  if (e2 != hipSuccess) return hip_error(e2, "bank kernels");
  return FDAS_OK;
}

int fdas_plan(fdas_plan_t *out, const fdas_params *p, int device, void *stream) {
  if (!out) return set_error(FDAS_ERR_INVALID, "null plan output pointer");
  *out = nullptr;
  fdas_params r;
  int nz = 0;
  int st = resolve_params(p, &r, &nz);
  if (st) return st;
  if (device < 0) return set_error(FDAS_ERR_INVALID, "device %d < 0", device);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (device >= ndev) return set_error(FDAS_ERR_INVALID, "device %d of %d", device, ndev);
  DeviceGuard guard(device);
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  return build_plan(out, r, nz, device, (hipStream_t)stream);
}

int fdas_plan_get_info(fdas_plan_t plan, fdas_plan_info *info) {
  if (!plan || !info) return set_error(FDAS_ERR_INVALID, "null plan or info pointer");
  plan_info(plan, info);
  return FDAS_OK;
}

int fdas_plan_bank(fdas_plan_t plan, void *dst, size_t bytes, void *stream) {
  if (!plan || !dst) return set_error(FDAS_ERR_INVALID, "null plan or destination");
  const size_t need = (size_t)plan_rows(plan) * (size_t)plan_seg_len(plan) * 8;
  if (bytes < need) return set_error(FDAS_ERR_INVALID, "destination holds %zu bytes, need %zu", bytes, need);
  DeviceGuard guard(plan_device(plan));
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  return plan_bank_natural(plan, dst, (hipStream_t)stream);
}

int fdas_convolve(fdas_plan_t plan, const void *spectrum, int64_t nbins, float *power, int64_t ld,
                  void *stream) {
  if (!plan) return set_error(FDAS_ERR_INVALID, "null plan");
  if (!spectrum || !power) return set_error(FDAS_ERR_INVALID, "null spectrum or power pointer");
  if (nbins < 1) return set_error(FDAS_ERR_INVALID, "nbins must be >= 1 (got %lld)", (long long)nbins);
  if (ld < nbins) return set_error(FDAS_ERR_INVALID, "ld (%lld) < nbins (%lld)", (long long)ld, (long long)nbins);
  if ((reinterpret_cast<uintptr_t>(spectrum) & 7) || (reinterpret_cast<uintptr_t>(power) & 3))
    return set_error(FDAS_ERR_INVALID, "misaligned spectrum or power pointer");
  {  // the plane is written while segments of the spectrum are still being read
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(spectrum), s1 = s0 + (uintptr_t)nbins * 8;
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(power);
    const uintptr_t p1 = p0 + ((uintptr_t)(plan_rows(plan) - 1) * (uintptr_t)ld + (uintptr_t)nbins) * 4;
    if (p0 < s1 && s0 < p1) return set_error(FDAS_ERR_INVALID, "power plane overlaps the spectrum");
  }
  DeviceGuard guard(plan_device(plan));
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  return plan_convolve(plan, spectrum, nbins, power, ld, (hipStream_t)stream);
}

int fdas_convolve_candidates(fdas_plan_t plan, const void *spectrum, int64_t nbins, float threshold,
                             fdas_candidate *cands, int64_t capacity, unsigned long long *count,
                             void *stream) {
  if (!plan) return set_error(FDAS_ERR_INVALID, "null plan");
  if (!spectrum || !count) return set_error(FDAS_ERR_INVALID, "null spectrum or count pointer");
  if (nbins < 1) return set_error(FDAS_ERR_INVALID, "nbins must be >= 1 (got %lld)", (long long)nbins);
  if (capacity < 0 || (capacity > 0 && !cands))
    return set_error(FDAS_ERR_INVALID, "need capacity >= 0 and a list when capacity > 0");
  if (!std::isfinite(threshold)) return set_error(FDAS_ERR_INVALID, "threshold must be finite");
  if ((reinterpret_cast<uintptr_t>(spectrum) & 7) || (reinterpret_cast<uintptr_t>(cands) & 15) ||
      (reinterpret_cast<uintptr_t>(count) & 7))
    return set_error(FDAS_ERR_INVALID, "misaligned spectrum, list or count pointer");
  DeviceGuard guard(plan_device(plan));
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  return plan_convolve_candidates(plan, spectrum, nbins, threshold, cands, capacity, count,
                                  (hipStream_t)stream);
}

size_t fdas_peaks_workspace_bytes(int64_t cand_capacity) {
  if (cand_capacity < 0 || cand_capacity > FDAS_PEAKS_MAX_CANDIDATES) return 0;
  return peaks_workspace_bytes(cand_capacity);
}

int fdas_convolve_peaks(fdas_plan_t plan, const void *spectrum, int64_t nbins, float threshold,
                        void *workspace, size_t workspace_bytes, int64_t cand_capacity,
                        fdas_candidate *peaks, int64_t peak_capacity, unsigned long long *counts,
                        void *stream) {
  if (!plan) return set_error(FDAS_ERR_INVALID, "null plan");
  if (!spectrum || !counts || !workspace)
    return set_error(FDAS_ERR_INVALID, "null spectrum, workspace or counts pointer");
  if (nbins < 1 || nbins > ((int64_t)1 << 34))
    return set_error(FDAS_ERR_INVALID, "nbins must be in [1, 2^34] (got %lld)", (long long)nbins);
  if (cand_capacity < 0 || cand_capacity > FDAS_PEAKS_MAX_CANDIDATES)
    return set_error(FDAS_ERR_INVALID, "candidate capacity %lld outside [0, %d]",
                     (long long)cand_capacity, FDAS_PEAKS_MAX_CANDIDATES);
  const size_t need = peaks_workspace_bytes(cand_capacity);
  if (workspace_bytes < need)
    return set_error(FDAS_ERR_INVALID, "workspace of %zu bytes; %zu needed for %lld candidates",
                     workspace_bytes, need, (long long)cand_capacity);
  if (peak_capacity < 0 || (peak_capacity > 0 && !peaks))
    return set_error(FDAS_ERR_INVALID, "need peak capacity >= 0 and a list when it is > 0");
  if (!std::isfinite(threshold)) return set_error(FDAS_ERR_INVALID, "threshold must be finite");
  if ((reinterpret_cast<uintptr_t>(spectrum) & 7) || (reinterpret_cast<uintptr_t>(workspace) & 15) ||
      (reinterpret_cast<uintptr_t>(peaks) & 15) || (reinterpret_cast<uintptr_t>(counts) & 7))
    return set_error(FDAS_ERR_INVALID, "misaligned spectrum, workspace, peak list or counts");
  if (plan_rows(plan) >= (1 << 27))
    return set_error(FDAS_ERR_UNSUPPORTED, "more plane rows than the peak search indexes");
  DeviceGuard guard(plan_device(plan));
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  return plan_convolve_peaks(plan, spectrum, nbins, threshold, workspace, cand_capacity, peaks,
                             peak_capacity, counts, (hipStream_t)stream);
}

// Argument checks shared by the two batched entry points (host only).
static int check_batch(fdas_plan_t plan, const fdas_series *series, int nseries) {
  if (!plan) return set_error(FDAS_ERR_INVALID, "null plan");
  if (!series || nseries < 1) return set_error(FDAS_ERR_INVALID, "need nseries >= 1 and a series array");
  for (int i = 0; i < nseries; ++i) {
    const fdas_series &s = series[i];
    if (!s.spectrum || !s.power) return set_error(FDAS_ERR_INVALID, "series %d: null pointer", i);
    if (s.nbins < 1) return set_error(FDAS_ERR_INVALID, "series %d: nbins < 1", i);
    if (s.ld < s.nbins) return set_error(FDAS_ERR_INVALID, "series %d: ld < nbins", i);
    if ((reinterpret_cast<uintptr_t>(s.spectrum) & 7) || (reinterpret_cast<uintptr_t>(s.power) & 3))
      return set_error(FDAS_ERR_INVALID, "series %d: misaligned pointer", i);
  }
  return FDAS_OK;
}

int fdas_convolve_batch(fdas_plan_t plan, const fdas_series *series, int nseries, void *stream) {
  const int st = check_batch(plan, series, nseries);
  if (st != FDAS_OK) return st;
  DeviceGuard guard(plan_device(plan));
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  return plan_convolve_batch(plan, series, nseries, (hipStream_t)stream);
}

int fdas_convolve_batch_noalloc(fdas_plan_t plan, const fdas_series *series, int nseries,
                                void *stream) {
  const int st = check_batch(plan, series, nseries);
  if (st != FDAS_OK) return st;
  if (nseries > FDAS_NOALLOC_MAX_SERIES)
    return set_error(FDAS_ERR_INVALID, "%d series exceed FDAS_NOALLOC_MAX_SERIES (%d)", nseries,
                     FDAS_NOALLOC_MAX_SERIES);
  DeviceGuard guard(plan_device(plan));
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  return plan_convolve_batch_noalloc(plan, series, nseries, (hipStream_t)stream);
}

int fdas_destroy(fdas_plan_t plan) {
  if (!plan) return FDAS_OK;
  DeviceGuard guard(plan_device(plan));
  return destroy_plan(plan);
}

int fdas_fft_plan(fdas_fft_t *out, int n, int elems_per_thread, int device, void *stream) {
  if (!out) return set_error(FDAS_ERR_INVALID, "null plan pointer");
  *out = nullptr;
  if (n < 2 || (n & (n - 1)))
    return set_error(FDAS_ERR_INVALID, "FFT length %d is not a power of two >= 2", n);
  if (elems_per_thread < 0 || (elems_per_thread & (elems_per_thread - 1)))
    return set_error(FDAS_ERR_INVALID, "elements per thread %d is not 0 or a power of two",
                     elems_per_thread);
  if (device < 0) return set_error(FDAS_ERR_INVALID, "device %d < 0", device);
  const FftVariant *v = nullptr;
  const int st = find_fft(n, elems_per_thread, &v);
  if (st != FDAS_OK) return st;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (device >= ndev) return set_error(FDAS_ERR_INVALID, "device %d of %d", device, ndev);
  DeviceGuard guard(device);
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  auto *p = new (std::nothrow) fdas_fft_s{device, v, nullptr};
  if (!p) return set_error(FDAS_ERR_NOMEM, "host allocation");
  e = hipMalloc(&p->tw, (size_t)n * sizeof(c32));
  if (e != hipSuccess) {
    delete p;
    return set_error(FDAS_ERR_NOMEM, "twiddle table: %s", hipGetErrorString(e));
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  e = launch_twiddles(p->tw, n, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(p->tw);
    delete p;
    return hip_error(e, "twiddle table");
  }
  *out = p;
  return FDAS_OK;
}

int fdas_fft_get_info(fdas_fft_t plan, fdas_fft_info *info) {
  if (!plan || !info) return set_error(FDAS_ERR_INVALID, "null plan or info");
  info->n = plan->v->L;
  info->elems_per_thread = plan->v->E;
  info->threads = plan->v->T;
  info->transforms_per_block = plan->v->G;
  std::snprintf(info->kernel, sizeof(info->kernel), "%s", plan->v->name);
  return FDAS_OK;
}

int fdas_fft_exec(fdas_fft_t plan, const void *in, void *out, int64_t batch, int direction,
                  void *stream) {
  if (!plan) return set_error(FDAS_ERR_INVALID, "null plan");
  if (direction != -1 && direction != 1)
    return set_error(FDAS_ERR_INVALID, "direction %d is not -1 or +1", direction);
  if (batch < 0) return set_error(FDAS_ERR_INVALID, "batch %lld < 0", (long long)batch);
  if (batch == 0) return FDAS_OK;
  if (!in || !out) return set_error(FDAS_ERR_INVALID, "null sample buffer");
  if (reinterpret_cast<uintptr_t>(in) % 8 || reinterpret_cast<uintptr_t>(out) % 8)
    return set_error(FDAS_ERR_INVALID, "sample buffers must be 8-byte aligned");
  const int64_t blocks = (batch + plan->v->G - 1) / plan->v->G;
  if (blocks > (int64_t)INT_MAX || batch > INT64_MAX / (8 * (int64_t)plan->v->L))
    return set_error(FDAS_ERR_INVALID, "batch %lld too large", (long long)batch);
  const char *a = static_cast<const char *>(in);
  const char *b = static_cast<const char *>(out);
  const int64_t nb = batch * 8 * (int64_t)plan->v->L;
  if (a != b && a < b + nb && b < a + nb)
    return set_error(FDAS_ERR_INVALID, "input and output overlap without being equal");
  DeviceGuard guard(plan->device);
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  const hipError_t e = plan->v->launch(in, out, batch, direction, plan->tw,
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? FDAS_OK : hip_error(e, "FFT launch");
}

int fdas_fft_destroy(fdas_fft_t plan) {
  if (!plan) return FDAS_OK;
  DeviceGuard guard(plan->device);
  hipError_t e = hipDeviceSynchronize();
  const hipError_t f = hipFree(plan->tw);
  delete plan;
  if (e == hipSuccess) e = f;
  return e == hipSuccess ? FDAS_OK : hip_error(e, "fdas_fft_destroy");
}

static void free_frontend(fdas_frontend_t p) {
  if (!p) return;
  if (p->tw1) (void)hipFree(p->tw1);
  if (p->tw2) (void)hipFree(p->tw2);
  if (p->work) (void)hipFree(p->work);
  if (p->pw) (void)hipFree(p->pw);
  if (p->sel) (void)hipFree(p->sel);
  delete p;
}

int fdas_frontend_plan(fdas_frontend_t *out, int64_t n, int device, void *stream) {
  if (!out) return set_error(FDAS_ERR_INVALID, "null plan pointer");
  *out = nullptr;
  if (n < 128 || n > ((int64_t)1 << 25) || (n & (n - 1)))
    return set_error(FDAS_ERR_INVALID, "series length %lld is not a power of two in [128, 2^25]",
                     (long long)n);
  if (device < 0) return set_error(FDAS_ERR_INVALID, "device %d < 0", device);
  const int64_t M = n / 2;
  int lg = 0;
  while (((int64_t)1 << lg) < M) ++lg;
  FrontendGeom g{};
  g.M = M;
  if (M <= 4096) {
    g.N1 = (int)M;
    g.N2 = 1;
  } else {
    g.N1 = 1 << ((lg + 1) / 2);
    g.N2 = 1 << (lg / 2);
  }
  int st = find_fft(g.N1, 0, &g.f1);
  if (st == FDAS_OK && g.N2 > 1) st = find_fft(g.N2, 0, &g.f2);
  if (st != FDAS_OK) return st;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (device >= ndev) return set_error(FDAS_ERR_INVALID, "device %d of %d", device, ndev);
  DeviceGuard guard(device);
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  auto *p = new (std::nothrow) fdas_frontend_s{};
  if (!p) return set_error(FDAS_ERR_NOMEM, "host allocation");
  p->device = device;
  p->n = n;
  e = hipMalloc(&p->tw1, (size_t)g.N1 * sizeof(c32));
  if (e == hipSuccess && g.N2 > 1) e = hipMalloc(&p->tw2, (size_t)g.N2 * sizeof(c32));
  if (e == hipSuccess) e = hipMalloc(&p->work, (size_t)M * sizeof(c32));
  if (e == hipSuccess) e = hipMalloc(&p->pw, (size_t)M * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->sel, frontend_sel_bytes());
  if (e != hipSuccess) {
    free_frontend(p);
    return set_error(FDAS_ERR_NOMEM, "front-end buffers: %s", hipGetErrorString(e));
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  e = launch_twiddles(p->tw1, g.N1, s);
  if (e == hipSuccess && g.N2 > 1) e = launch_twiddles(p->tw2, g.N2, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_frontend(p);
    return hip_error(e, "front-end twiddles");
  }
  g.tw1 = p->tw1;
  g.tw2 = p->tw2;
  p->g = g;
  *out = p;
  return FDAS_OK;
}

int fdas_frontend_exec(fdas_frontend_t plan, const float *series, void *spectrum, float *stats,
                       void *stream) {
  if (!plan) return set_error(FDAS_ERR_INVALID, "null plan");
  if (!series || !spectrum) return set_error(FDAS_ERR_INVALID, "null sample buffer");
  if (reinterpret_cast<uintptr_t>(series) % 8 || reinterpret_cast<uintptr_t>(spectrum) % 8 ||
      reinterpret_cast<uintptr_t>(stats) % 4)
    return set_error(FDAS_ERR_INVALID, "series and spectrum must be 8-byte aligned");
  const char *a = reinterpret_cast<const char *>(series);
  const char *b = reinterpret_cast<const char *>(spectrum);
  const int64_t nb = plan->n * 4;  // both buffers span 4 n bytes
  if (a != b && a < b + nb && b < a + nb)
    return set_error(FDAS_ERR_INVALID, "series and spectrum overlap without being equal");
  DeviceGuard guard(plan->device);
  if (guard.err != hipSuccess) return hip_error(guard.err, "hipSetDevice");
  const hipError_t e = launch_frontend(plan->g, series, static_cast<c32 *>(spectrum), plan->work,
                                       plan->pw, plan->sel, stats,
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? FDAS_OK : hip_error(e, "front-end launch");
}

int fdas_frontend_destroy(fdas_frontend_t plan) {
  if (!plan) return FDAS_OK;
  DeviceGuard guard(plan->device);
  const hipError_t e = hipDeviceSynchronize();
  free_frontend(plan);
  return e == hipSuccess ? FDAS_OK : hip_error(e, "fdas_frontend_destroy");
}

int fdas_fft_variants(int n, char *buf, size_t len) {
  if (n < 0) return set_error(FDAS_ERR_INVALID, "length %d < 0", n);
  if (!buf && len) return set_error(FDAS_ERR_INVALID, "null buffer with nonzero length");
  int count = 0;
  const FftVariant *vs = fft_variants(&count);
  std::string all;
  int k = 0;
  for (int i = 0; i < count; ++i) {
    if (n && vs[i].L != n) continue;
    if (k++) all += "\n";
    all += vs[i].name;
  }
  if (len) {
    const size_t c = all.size() < len - 1 ? all.size() : len - 1;
    std::memcpy(buf, all.data(), c);
    buf[c] = 0;
  }
  return k;
}

}  // extern "C"
