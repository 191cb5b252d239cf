// Plan construction (FP64 templates -> FP64 bank FFT -> storage precision,
// twiddle tables, kernel-variant choice) and single-series dispatch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

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
  // batched path
  unsigned long long *counter = nullptr;
  fdas::SeriesDesc *d_desc = nullptr;
  size_t desc_cap = 0;
  std::vector<fdas::SeriesDesc> last_desc;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int cus = 0;
};

namespace fdas {

bool mixed_supported(int seg_len) {
  int n = 0;
  const OlsVariant *v = mixed_variants(&n);
  for (int i = 0; i < n; ++i)
    if (v[i].L == seg_len) return true;
  return false;
}

static const OlsVariant *find_variant(int L, int precision, const char *want) {
  int n = 0;
  const OlsVariant *v = precision == FDAS_FP32 ? fp32_variants(&n) : mixed_variants(&n);
  const OlsVariant *first = nullptr;
  for (int i = 0; i < n; ++i) {
    if (v[i].L != L || v[i].precision != precision) continue;
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
  const OlsVariant *var = find_variant(p.seg_len, p.precision, want);
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
  pl->bank_bytes = (size_t)nz * p.seg_len * (p.precision == FDAS_FP32 ? 8 : 4);
  hipError_t e = hipMalloc(&h, hbytes);
  if (e == hipSuccess) e = hipMalloc(&pl->bank, pl->bank_bytes);
  if (e == hipSuccess) e = hipMalloc(&pl->tw, (size_t)p.seg_len * 8);
  if (e != hipSuccess) {
    if (h) (void)hipFree(h);
    destroy_plan(pl);
    return set_error(FDAS_ERR_NOMEM, "plan allocation: %s", hipGetErrorString(e));
  }
  e = hipMalloc(reinterpret_cast<void **>(&pl->counter), 256);
  if (e != hipSuccess) {
    (void)hipFree(h);
    destroy_plan(pl);
    return set_error(FDAS_ERR_NOMEM, "plan allocation: %s", hipGetErrorString(e));
  }
  e = launch_templates(h, nz, p.m, p.zmax, p.dz, s);
  if (e == hipSuccess) {
    if (p.precision == FDAS_FP32)
      e = launch_bank(static_cast<c32 *>(pl->bank), h, nz, p.m, var->lay, s);
    else
      e = launch_bank_mixed(pl->bank, h, nz, p.m, p.seg_len, p.precision, s);
  }
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
  int count = 0;
  std::string out;
  for (int pass = 0; pass < 2; ++pass) {
    int n = 0;
    const OlsVariant *v = pass == 0 ? fp32_variants(&n) : mixed_variants(&n);
    for (int i = 0; i < n; ++i) {
      if (seg_len && v[i].L != seg_len) continue;
      if (precision != -1 && v[i].precision != precision) continue;
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
  hipError_t e = pl->p.precision == FDAS_FP32
                     ? launch_bank_natural(static_cast<c32 *>(dst),
                                           static_cast<const c32 *>(pl->bank), pl->nz,
                                           pl->var->lay, s)
                     : launch_bank_mixed_natural(static_cast<c32 *>(dst), pl->bank, pl->nz, pl->L,
                                                 pl->p.precision, s);
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
  a.bank_log2 = 0;
  while ((1 << a.bank_log2) < pl->L) ++a.bank_log2;
  hipError_t e = pl->var->launch(a, s);
  if (e != hipSuccess) return hip_error(e, "correlation kernel launch");
  return FDAS_OK;
}

// Host side of the batched path: validate and order the series (largest
// first), lay out their work items, upload the descriptors when the batch
// changes, and replay one captured graph (counter reset + persistent kernel).
int plan_convolve_batch(fdas_plan_t pl, const fdas_series *series, int nseries, hipStream_t s) {
  if (!pl->var->launch_batch)
    return set_error(FDAS_ERR_UNSUPPORTED, "kernel %s has no batched form", pl->var->name);
  const int G = pl->var->G;
  const double dz = pl->p.dz;
  std::vector<SeriesDesc> desc(nseries);
  std::vector<double> cost(nseries);
  for (int i = 0; i < nseries; ++i) {
    const fdas_series &x = series[i];
    if (!std::isfinite(x.zmax) || x.zmax < 0.0 || x.zmax > pl->p.zmax * (1.0 + 1e-12) + 1e-12)
      return set_error(FDAS_ERR_INVALID, "series %d: zmax %g outside [0, %g]", i, x.zmax, pl->p.zmax);
    const double off = (pl->p.zmax - x.zmax) / dz;
    const double span = 2.0 * x.zmax / dz;
    if (std::fabs(off - std::nearbyint(off)) > 1e-9 || std::fabs(span - std::nearbyint(span)) > 1e-9)
      return set_error(FDAS_ERR_INVALID, "series %d: zmax %g is not on the plan's z grid", i, x.zmax);
    const int64_t nseg = (x.nbins + pl->U - 1) / pl->U;
    if (nseg > INT_MAX / 2) return set_error(FDAS_ERR_UNSUPPORTED, "series %d too long", i);
    SeriesDesc &d = desc[i];
    d.spec = x.spectrum;
    d.power = x.power;
    d.nbins = x.nbins;
    d.ld = x.ld;
    d.nseg = (int)nseg;
    d.nz = (int)std::nearbyint(span) + 1;
    d.row_off = (int)std::nearbyint(off);
    d.pad_ = 0;
    cost[i] = (double)d.nz * (double)x.nbins;
  }
  std::vector<int> order(nseries);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<SeriesDesc> sorted(nseries);
  int64_t total = 0;
  for (int k = 0; k < nseries; ++k) {
    sorted[k] = desc[order[k]];
    sorted[k].item_begin = total;
    const int64_t nsb = (sorted[k].nseg + G - 1) / G;
    const int64_t nzg = (sorted[k].nz + pl->zpb - 1) / pl->zpb;
    total += nsb * nzg;
  }
  if (total == 0) return FDAS_OK;

  const bool same = pl->graph && sorted.size() == pl->last_desc.size() &&
                    std::memcmp(sorted.data(), pl->last_desc.data(), sorted.size() * sizeof(SeriesDesc)) == 0;
  hipError_t e = hipSuccess;
  if (!same) {
    // new batch layout: upload descriptors and capture a fresh graph
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "synchronise before descriptor upload");
    if (pl->graph) {
      (void)hipGraphExecDestroy(pl->graph);
      pl->graph = nullptr;
    }
    if (pl->desc_cap < sorted.size()) {
      if (pl->d_desc) (void)hipFree(pl->d_desc);
      pl->d_desc = nullptr;
      pl->desc_cap = 0;
      e = hipMalloc(&pl->d_desc, sorted.size() * sizeof(SeriesDesc));
      if (e != hipSuccess) return set_error(FDAS_ERR_NOMEM, "descriptor allocation: %s", hipGetErrorString(e));
      pl->desc_cap = sorted.size();
    }
    e = hipMemcpy(pl->d_desc, sorted.data(), sorted.size() * sizeof(SeriesDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "descriptor upload");
    if (!pl->cap_stream) {
      e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_error(e, "capture stream");
    }
    if (!pl->cus) {
      e = hipDeviceGetAttribute(&pl->cus, hipDeviceAttributeMultiprocessorCount, pl->device);
      if (e != hipSuccess) return hip_error(e, "CU count");
    }
    const int per_cu = std::max(1, pl->var->batch_blocks_per_cu());
    BatchArgs a;
    a.desc = pl->d_desc;
    a.nseries = nseries;
    a.total = total;
    a.counter = pl->counter;
    a.bank = pl->bank;
    a.tw = pl->tw;
    a.U = pl->U;
    a.half = pl->m / 2;
    a.zpb = pl->zpb;
    a.grid = (int)std::min<int64_t>((int64_t)pl->cus * per_cu, total);
    const char *nog = std::getenv("FDAS_NO_GRAPH");
    if (nog && *nog == '1') {
      e = pl->var->launch_batch(a, s);
      if (e != hipSuccess) return hip_error(e, "batch kernel launch");
      return FDAS_OK;  // nothing cached: the next call uploads again
    }
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "begin capture");
    hipError_t le = pl->var->launch_batch(a, pl->cap_stream);
    e = hipStreamEndCapture(pl->cap_stream, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_error(le, "batch kernel capture");
    }
    if (e != hipSuccess) return hip_error(e, "end capture");
    e = hipGraphInstantiate(&pl->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      pl->graph = nullptr;
      return hip_error(e, "graph instantiate");
    }
    pl->last_desc = sorted;
  }
  e = hipGraphLaunch(pl->graph, s);
  if (e != hipSuccess) return hip_error(e, "graph launch");
  return FDAS_OK;
}

int destroy_plan(fdas_plan_t pl) {
  if (!pl) return FDAS_OK;
  hipError_t e = hipSuccess;
  if (pl->bank || pl->tw || pl->counter) e = hipDeviceSynchronize();
  if (pl->graph) (void)hipGraphExecDestroy(pl->graph);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  if (pl->d_desc) (void)hipFree(pl->d_desc);
  if (pl->counter) (void)hipFree(pl->counter);
  if (pl->bank) (void)hipFree(pl->bank);
  if (pl->tw) (void)hipFree(pl->tw);
  delete pl;
  if (e != hipSuccess) return hip_error(e, "synchronise before destroy");
  return FDAS_OK;
}

}  // namespace fdas
