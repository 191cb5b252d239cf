// Plan construction (FP64 templates -> FP64 bank FFT -> storage precision,
// twiddle tables, kernel-variant choice) and single-series dispatch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <string>

#include "plan.hpp"

struct fdas_plan_s {
  int device = 0;
  fdas_params p{};
  int nz = 0, m = 0, L = 0, U = 0;
  const fdas::OlsVariant *var = nullptr;
  int zpb = 1;
  void *bank = nullptr;
  size_t bank_bytes = 0;
  void *tw = nullptr;
  double plan_ms = 0.0;
};

namespace fdas {

bool mixed_supported(int seg_len) {
  (void)seg_len;
  return false;
}

static const OlsVariant *find_variant(int L, const char *want) {
  int n = 0;
  const OlsVariant *v = fp32_variants(&n);
  const OlsVariant *first = nullptr;
  for (int i = 0; i < n; ++i) {
    if (v[i].L != L) continue;
    if (want && *want && std::strcmp(v[i].name, want) == 0) return &v[i];
    if (!first) first = &v[i];
  }
  return (want && *want) ? nullptr : first;
}

// Templates per work unit: split nz into ceil(nz / 32) near-equal groups.
static int default_zpb(int nz) {
  const int groups = (nz + 31) / 32;
  return (nz + groups - 1) / groups;
}

int build_plan(fdas_plan_t *out, const fdas_params &p, int nz, int device, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const char *want = std::getenv("FDAS_VARIANT");
  const OlsVariant *var = find_variant(p.seg_len, want);
  if (!var) {
    if (want && *want)
      return set_error(FDAS_ERR_UNSUPPORTED, "variant '%s' not compiled for seg_len %d", want, p.seg_len);
    return set_error(FDAS_ERR_UNSUPPORTED, "no kernel variant for seg_len %d", p.seg_len);
  }
  fdas_plan_s *pl = new (std::nothrow) fdas_plan_s;
  if (!pl) return set_error(FDAS_ERR_NOMEM, "host allocation of the plan");
  pl->device = device;
  pl->p = p;
  pl->nz = nz;
  pl->m = p.m;
  pl->L = p.seg_len;
  pl->U = p.seg_len - p.m;
  pl->var = var;
  pl->zpb = default_zpb(nz);
  if (const char *z = std::getenv("FDAS_ZPB")) {
    const int v = std::atoi(z);
    if (v > 0) pl->zpb = v;
  }

  void *h = nullptr;
  const size_t hbytes = (size_t)nz * (p.m + 1) * 16;
  pl->bank_bytes = (size_t)nz * p.seg_len * 8;
  hipError_t e = hipMalloc(&h, hbytes);
  if (e == hipSuccess) e = hipMalloc(&pl->bank, pl->bank_bytes);
  if (e == hipSuccess) e = hipMalloc(&pl->tw, (size_t)p.seg_len * 8);
  if (e != hipSuccess) {
    if (h) (void)hipFree(h);
    destroy_plan(pl);
    return set_error(FDAS_ERR_NOMEM, "plan allocation: %s", hipGetErrorString(e));
  }
  e = launch_templates(h, nz, p.m, p.zmax, p.dz, s);
  if (e == hipSuccess) e = launch_bank(static_cast<c32 *>(pl->bank), h, nz, p.m, var->lay, s);
  if (e == hipSuccess) e = launch_twiddles(static_cast<c32 *>(pl->tw), p.seg_len, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(h);
  if (e != hipSuccess) {
    destroy_plan(pl);
    return hip_error(e, "plan kernels");
  }
  pl->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = pl;
  return FDAS_OK;
}

void plan_info(fdas_plan_t pl, fdas_plan_info *info) {
  std::memset(info, 0, sizeof(*info));
  info->nz = pl->nz;
  info->m = pl->m;
  info->seg_len = pl->L;
  info->valid = pl->U;
  info->precision = pl->p.precision;
  info->flags = pl->p.flags;
  info->threads = pl->var->T;
  info->templates_per_block = pl->zpb;
  info->segments_per_block = pl->var->G;
  info->bank_bytes = pl->bank_bytes;
  info->plan_ms = pl->plan_ms;
  std::strncpy(info->kernel, pl->var->name, sizeof(info->kernel) - 1);
}

int list_variants(int seg_len, int precision, char *buf, size_t len) {
  int n = 0, count = 0;
  const OlsVariant *v = fp32_variants(&n);
  std::string out;
  if (precision == -1 || precision == FDAS_FP32) {
    for (int i = 0; i < n; ++i) {
      if (seg_len && v[i].L != seg_len) continue;
      out += v[i].name;
      out += '\n';
      ++count;
    }
  }
  if (buf && len > 0) {
    std::strncpy(buf, out.c_str(), len - 1);
    buf[len - 1] = '\0';
  }
  return count;
}

int plan_rows(fdas_plan_t pl) { return pl->nz; }
int plan_seg_len(fdas_plan_t pl) { return pl->L; }
int plan_device(fdas_plan_t pl) { return pl->device; }

int plan_bank_natural(fdas_plan_t pl, void *dst, hipStream_t s) {
  hipError_t e = launch_bank_natural(static_cast<c32 *>(dst), static_cast<const c32 *>(pl->bank),
                                     pl->nz, pl->var->lay, s);
  if (e != hipSuccess) return hip_error(e, "bank copy kernel");
  return FDAS_OK;
}

int plan_convolve(fdas_plan_t pl, const void *spec, int64_t nbins, float *power, int64_t ld,
                  hipStream_t s) {
  const int64_t nseg = (nbins + pl->U - 1) / pl->U;
  if (nseg > INT_MAX / 2) return set_error(FDAS_ERR_UNSUPPORTED, "nbins %lld too large", (long long)nbins);
  const int64_t nsb = (nseg + pl->var->G - 1) / pl->var->G;
  const int64_t nzg = (pl->nz + pl->zpb - 1) / pl->zpb;
  if (nsb * nzg > (int64_t)UINT_MAX)
    return set_error(FDAS_ERR_UNSUPPORTED, "grid of %lld blocks too large", (long long)(nsb * nzg));
  OlsArgs a;
  a.spec = spec;
  a.nbins = nbins;
  a.bank = pl->bank;
  a.tw = pl->tw;
  a.power = power;
  a.ld = ld;
  a.nseg = (int)nseg;
  a.U = pl->U;
  a.half = pl->m / 2;
  a.nz = pl->nz;
  a.zpb = pl->zpb;
  hipError_t e = pl->var->launch(a, s);
  if (e != hipSuccess) return hip_error(e, "correlation kernel launch");
  return FDAS_OK;
}

int plan_convolve_batch(fdas_plan_t pl, const fdas_series *series, int nseries, hipStream_t s) {
  (void)pl;
  (void)series;
  (void)nseries;
  (void)s;
  return set_error(FDAS_ERR_UNSUPPORTED, "batched correlation is not built yet");
}

int destroy_plan(fdas_plan_t pl) {
  if (!pl) return FDAS_OK;
  hipError_t e = hipSuccess;
  if (pl->bank || pl->tw) e = hipDeviceSynchronize();
  if (pl->bank) (void)hipFree(pl->bank);
  if (pl->tw) (void)hipFree(pl->tw);
  delete pl;
  if (e != hipSuccess) return hip_error(e, "synchronise before destroy");
  return FDAS_OK;
}

}  // namespace fdas
