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

#include "noalloc.hpp"
#include "peaks.hpp"
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
  void *consts = nullptr;
  double plan_ms = 0.0;
  // batched path: one captured graph (and descriptor table) per batch layout
  struct GraphEntry {
    std::vector<fdas::SeriesDesc> key;
    fdas::SeriesDesc *d_desc = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
  };
  unsigned long long *counter = nullptr;
  std::vector<GraphEntry> graphs;
  uint64_t use_clock = 0;
  hipStream_t cap_stream = nullptr;
  int cus = 0;
  bool zpb_forced = false;  // FDAS_ZPB or the autotuner fixed it
  int slots = 0;            // concurrently resident blocks of the grid kernel
  int last_zpb = 0;         // templates per unit of the last launch (a batch: its largest)
};

// Captured batch layouts kept per plan (least recently used evicted): enough
// for a workload run in many waves to replay every wave's graph, since a
// re-capture synchronises the stream and uploads the descriptors again.
static constexpr size_t kMaxGraphs = 64;

namespace fdas {

bool mixed_supported(int seg_len, int split) {
  int n = 0;
  const OlsVariant *v = mixed_variants(&n);
  for (int i = 0; i < n; ++i)
    if (v[i].L == seg_len && v[i].split == split) return true;
  return false;
}

// FDAS_FLAG_SPLIT selects the hi + lo split-product kernels (mixed precisions).
static int plan_split(const fdas_params &p) {
  return (p.precision != FDAS_FP32 && (p.flags & FDAS_FLAG_SPLIT)) ? 1 : 0;
}

static const OlsVariant *find_variant(int L, int precision, int split, const char *want) {
  int n = 0;
  const OlsVariant *v = precision == FDAS_FP32 ? fp32_variants(&n) : mixed_variants(&n);
  const OlsVariant *first = nullptr;
  for (int i = 0; i < n; ++i) {
    if (v[i].L != L || v[i].precision != precision || v[i].split != split) continue;
    if (want && *want && std::strcmp(v[i].name, want) == 0) return &v[i];
    if (!first) first = &v[i];
  }
  return (want && *want) ? nullptr : first;
}

constexpr int kFp32UnitTarget = 40;

// Templates per work unit. Without a target (plans that choose per launch;
// batched launches split each series this way), near-equal groups of at
// most 40 (larger groups ran 2.7% faster on the 512-series batch than ~32). With a target: units of `target` templates
// in group order and the remainder last (a remainder under a third of the
// target is spread over the other groups), and fewer rows than the target
// split about 3 : 1; work units are dispatched in group order, so the short
// ones start last and fill the end of the launch (on the 2^21-bin plane this
// measured 3-6% faster than equal groups at 65, 101 and 201 rows).
static int default_zpb(int nz, int target) {
  if (target <= 0) {
    const int groups = (nz + kFp32UnitTarget - 1) / kFp32UnitTarget;
    return (nz + groups - 1) / groups;
  }
  if (nz <= 40) return nz;
  const int full = nz / target, rem = nz % target;
  if (full == 0 || (full == 1 && rem < target / 3)) return (3 * nz + 3) / 4;
  if (rem != 0 && rem < target / 3)  // a unit of little more than its forward FFT:
    return (nz + full - 1) / full;   // spread the remainder over the full groups
  return target;
}

static int build_plan_with(fdas_plan_t *out, const fdas_params &p, int nz, int device,
                           hipStream_t s, const OlsVariant *force_var, int force_zpb);

// Autotuner: time every compiled variant for every admissible segment length
// (U = L - m >= L/2 unless the caller fixed L) and a few template-group sizes
// on a synthetic spectrum, keep the fastest per plane point. Results are
// cached in a text file (FDAS_TUNE_CACHE, one line per key) keyed by device
// architecture, CU count, m, nz, precision, split form and segment length.
struct TuneChoice {
  const OlsVariant *var = nullptr;
  int L = 0, zpb = 0;
  double ns_per_point = 0.0;
};

static std::string tune_key(const fdas_params &p, int nz, int device) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (auto &ch : arch)
    if (ch == ' ' || ch == ':') ch = '_';
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s cu%d m%d nz%d prec%d split%d L%d", arch.c_str(), cus, p.m,
                nz, p.precision, (p.flags & FDAS_FLAG_SPLIT) ? 1 : 0, p.seg_len);
  return buf;
}

static const OlsVariant *variant_by_name(const char *name) {
  for (int pass = 0; pass < 2; ++pass) {
    int n = 0;
    const OlsVariant *v = pass == 0 ? fp32_variants(&n) : mixed_variants(&n);
    for (int i = 0; i < n; ++i)
      if (std::strcmp(v[i].name, name) == 0) return &v[i];
  }
  return nullptr;
}

static bool tune_cache_lookup(const std::string &key, const fdas_params &p, TuneChoice *c) {
  const char *path = std::getenv("FDAS_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    std::string ln(line);
    const size_t bar = ln.find(" | ");
    if (bar == std::string::npos || ln.compare(0, bar, key) != 0) continue;
    char name[128];
    int L = 0, zpb = 0;
    double ns = 0;
    if (std::sscanf(ln.c_str() + bar + 3, "%127s %d %d %lf", name, &L, &zpb, &ns) == 4) {
      const OlsVariant *v = variant_by_name(name);
      // a line only counts for the precision and split form it was timed for
      if (v && v->L == L && v->precision == p.precision &&
          v->split == ((p.flags & FDAS_FLAG_SPLIT) ? 1 : 0)) {
        c->var = v;
        c->L = L;
        c->zpb = zpb;
        c->ns_per_point = ns;
        found = true;
      }
    }
  }
  std::fclose(f);
  return found;
}

static void tune_cache_store(const std::string &key, const TuneChoice &c) {
  const char *path = std::getenv("FDAS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s | %s %d %d %.6f\n", key.c_str(), c.var->name, c.L, c.zpb, c.ns_per_point);
  std::fclose(f);
}

__global__ void tune_fill_kernel(c32 *spec, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) spec[i] = {1.0f + 1e-3f * (float)(i & 1023), 0.5f - 1e-3f * (float)(i & 511)};
}

// Median of `reps` timed calls of one candidate plan, each bracketed by its
// own pair of events, after `warm` untimed calls.
static int time_candidate(fdas_plan_t pl, const void *spec, int64_t nbins, float *power,
                          hipStream_t s, hipEvent_t *ev, int warm, int reps, float *median_ms) {
  int st = FDAS_OK;
  for (int r = 0; r < warm && st == FDAS_OK; ++r) st = plan_convolve(pl, spec, nbins, power, nbins, s);
  for (int r = 0; r < reps && st == FDAS_OK; ++r) {
    (void)hipEventRecord(ev[2 * r], s);
    st = plan_convolve(pl, spec, nbins, power, nbins, s);
    (void)hipEventRecord(ev[2 * r + 1], s);
  }
  if (st != FDAS_OK) return st;
  hipError_t e = hipEventSynchronize(ev[2 * reps - 1]);
  if (e != hipSuccess) return hip_error(e, "autotune timing");
  std::vector<float> ms(reps);
  for (int r = 0; r < reps; ++r) {
    e = hipEventElapsedTime(&ms[r], ev[2 * r], ev[2 * r + 1]);
    if (e != hipSuccess) return hip_error(e, "autotune timing");
  }
  std::sort(ms.begin(), ms.end());
  *median_ms = ms[reps / 2];
  return FDAS_OK;
}

// Autotuner: every compiled variant of the precision and split form, at
// every admissible segment length (L - m >= L/2 unless the caller fixed L),
// with the plan's own per-launch choice of templates per unit and with a
// few fixed group sizes, is timed on a synthetic 2^20-bin spectrum; the
// fastest per plane point wins. The GPU is first kept busy for a fixed time
// so that its clock has settled before anything is compared; each candidate
// then takes the median of several individually timed calls, and the few
// closest to the fastest are timed again before one is chosen.
static int autotune(const fdas_params &p, int nz, int device, hipStream_t s, TuneChoice *best) {
  const int64_t nbins = (int64_t)1 << 20;
  constexpr int kReps = 7;
  constexpr double kHeatMs = 100.0;
  void *spec = nullptr;
  float *power = nullptr;
  hipError_t e = hipMalloc(&spec, nbins * 8);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&power), (size_t)nz * nbins * 4);
  if (e != hipSuccess) {
    if (spec) (void)hipFree(spec);
    return set_error(FDAS_ERR_NOMEM, "autotune buffers: %s", hipGetErrorString(e));
  }
  hipLaunchKernelGGL(tune_fill_kernel, dim3((unsigned)((nbins + 255) / 256)), dim3(256), 0, s,
                     static_cast<c32 *>(spec), nbins);
  hipEvent_t ev[2 * kReps] = {};
  for (auto &x : ev) (void)hipEventCreate(&x);
  int status = FDAS_OK;
  bool heated = false;
  best->var = nullptr;
  std::vector<TuneChoice> timed;  // every candidate's first timing
  for (int pass = 0; pass < 2 && status == FDAS_OK; ++pass) {
    int n = 0;
    const OlsVariant *vs = pass == 0 ? fp32_variants(&n) : mixed_variants(&n);
    for (int i = 0; i < n && status == FDAS_OK; ++i) {
      const OlsVariant *v = &vs[i];
      if (v->precision != p.precision || v->split != plan_split(p)) continue;
      if (p.seg_len ? v->L != p.seg_len : (v->L - p.m) * 2 < v->L) continue;
      // zpb 0: the plan's own choice (units of the variant's target size, or
      // per launch from the grid's rounds); then fixed near-equal groups
      std::vector<int> cands = {0};
      for (int ng : {1, 2, 3, 4, 6, 8, 12}) {
        const int zpb = (nz + ng - 1) / ng;
        if (std::find(cands.begin(), cands.end(), zpb) == cands.end()) cands.push_back(zpb);
      }
      for (int zpb : cands) {
        fdas_params q = p;
        q.seg_len = v->L;
        fdas_plan_t pl = nullptr;
        int st = build_plan_with(&pl, q, nz, device, s, v, zpb);
        if (st != FDAS_OK) {
          status = st;
          break;
        }
        if (!heated) {  // settle the clock before the first comparison
          const auto t0 = std::chrono::steady_clock::now();
          while (st == FDAS_OK &&
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                         .count() < kHeatMs) {
            for (int r = 0; r < 8 && st == FDAS_OK; ++r)
              st = plan_convolve(pl, spec, nbins, power, nbins, s);
            e = hipStreamSynchronize(s);
            if (st == FDAS_OK && e != hipSuccess) st = hip_error(e, "autotune warm-up");
          }
          heated = true;
        }
        float ms = 0.f;
        if (st == FDAS_OK) st = time_candidate(pl, spec, nbins, power, s, ev, 2, kReps, &ms);
        destroy_plan(pl);
        if (st != FDAS_OK) {
          status = st;
          break;
        }
        TuneChoice c;
        c.var = v;
        c.L = v->L;
        c.zpb = zpb;
        c.ns_per_point = (double)ms * 1e6 / ((double)nz * (double)nbins);
        timed.push_back(c);
      }
    }
  }
  // Second look at the close contenders: the candidates within kClose of the
  // fastest (at most kFinal of them) are timed again in kRounds interleaved
  // rounds, so that a transient that favoured one of them in the single first
  // timing does not decide; each keeps the median of its first timing and its
  // re-timings, and the fastest of those wins.
  constexpr double kClose = 1.15;
  constexpr int kFinal = 4, kRounds = 3;
  std::sort(timed.begin(), timed.end(),
            [](const TuneChoice &a, const TuneChoice &b) { return a.ns_per_point < b.ns_per_point; });
  std::vector<TuneChoice> fin;
  for (const TuneChoice &c : timed)
    if ((int)fin.size() < kFinal && c.ns_per_point <= kClose * timed[0].ns_per_point) fin.push_back(c);
  std::vector<std::vector<double>> runs(fin.size());
  for (size_t i = 0; i < fin.size(); ++i) runs[i].push_back(fin[i].ns_per_point);
  for (int round = 0; round < kRounds && status == FDAS_OK && fin.size() > 1; ++round) {
    for (size_t i = 0; i < fin.size() && status == FDAS_OK; ++i) {
      fdas_params q = p;
      q.seg_len = fin[i].L;
      fdas_plan_t pl = nullptr;
      int st = build_plan_with(&pl, q, nz, device, s, fin[i].var, fin[i].zpb);
      float ms = 0.f;
      if (st == FDAS_OK) st = time_candidate(pl, spec, nbins, power, s, ev, 2, kReps, &ms);
      if (pl) destroy_plan(pl);
      if (st != FDAS_OK) status = st;
      else runs[i].push_back((double)ms * 1e6 / ((double)nz * (double)nbins));
    }
  }
  for (size_t i = 0; i < fin.size() && status == FDAS_OK; ++i) {
    std::vector<double> &r = runs[i];
    std::sort(r.begin(), r.end());
    fin[i].ns_per_point = r[r.size() / 2];
    if (!best->var || fin[i].ns_per_point < best->ns_per_point) *best = fin[i];
  }
  for (auto &x : ev) (void)hipEventDestroy(x);
  (void)hipFree(spec);
  (void)hipFree(power);
  if (status == FDAS_OK && !best->var)
    status = set_error(FDAS_ERR_UNSUPPORTED, "no compiled variant admits m=%d", p.m);
  return status;
}

int build_plan(fdas_plan_t *out, const fdas_params &p, int nz, int device, hipStream_t s) {
  if (p.flags & FDAS_FLAG_AUTOTUNE) {
    const auto t0 = std::chrono::steady_clock::now();
    fdas_params q = p;
    const std::string key = tune_key(p, nz, device);
    TuneChoice c;
    if (!tune_cache_lookup(key, p, &c)) {
      int st = autotune(p, nz, device, s, &c);
      if (st != FDAS_OK) return st;
      tune_cache_store(key, c);
    }
    q.seg_len = c.L;
    int st = build_plan_with(out, q, nz, device, s, c.var, c.zpb);
    if (st == FDAS_OK)
      (*out)->plan_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return st;
  }
  return build_plan_with(out, p, nz, device, s, nullptr, 0);
}

static int build_plan_with(fdas_plan_t *out, const fdas_params &p, int nz, int device,
                           hipStream_t s, const OlsVariant *force_var, int force_zpb) {
  const auto t0 = std::chrono::steady_clock::now();
  const char *want = std::getenv("FDAS_VARIANT");
  const OlsVariant *var =
      force_var ? force_var : find_variant(p.seg_len, p.precision, plan_split(p), want);
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
  pl->zpb = default_zpb(nz, var->zpb_target);
  if (const char *z = std::getenv("FDAS_ZPB")) {
    const int v = std::atoi(z);
    if (v > 0) pl->zpb = v;
  }
  if (force_zpb > 0) pl->zpb = force_zpb;
  pl->zpb_forced = force_zpb > 0 || (std::getenv("FDAS_ZPB") && std::atoi(std::getenv("FDAS_ZPB")) > 0);

  void *h = nullptr;
  const size_t hbytes = (size_t)nz * (p.m + 1) * 16;
  const int split = plan_split(p);
  pl->bank_bytes = (size_t)nz * p.seg_len * (p.precision == FDAS_FP32 ? 8 : (split ? 8 : 4));
  hipError_t e = hipMalloc(&h, hbytes);
  if (e == hipSuccess) e = hipMalloc(&pl->bank, pl->bank_bytes);
  if (e == hipSuccess) e = hipMalloc(&pl->tw, (size_t)p.seg_len * 8);
  if (e == hipSuccess && p.precision != FDAS_FP32)
    e = hipMalloc(&pl->consts, mixed_consts_bytes(p.seg_len, split));
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
  e = launch_templates(h, nz, p.m, p.zmax, p.dz, (p.flags & FDAS_FLAG_INTERBIN) ? 1 : 0, s);
  if (e == hipSuccess) {
    if (p.precision == FDAS_FP32)
      e = launch_bank(static_cast<c32 *>(pl->bank), h, nz, p.m, var->lay, s);
    else
      e = launch_bank_mixed(pl->bank, h, nz, p.m, p.seg_len, p.precision, split, s);
  }
  if (e == hipSuccess) e = launch_twiddles(static_cast<c32 *>(pl->tw), p.seg_len, s);
  if (e == hipSuccess && pl->consts)
    e = launch_mixed_consts(pl->consts, p.seg_len, p.precision, split, s);
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
  info->templates_per_block = pl->last_zpb > 0 ? pl->last_zpb : pl->zpb;
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
                                                 pl->p.precision, plan_split(pl->p), s);
  if (e != hipSuccess) return hip_error(e, "bank copy kernel");
  return FDAS_OK;
}

// Templates per work unit for a grid of nsb segment groups: the grid runs in
// ceil(blocks / slots) rounds, each as long as one unit (zpb inverse FFTs plus
// about one forward FFT); pick the group count that minimises that product.
static int launch_zpb(fdas_plan_t pl, int64_t nsb) {
  if (pl->zpb_forced || pl->var->zpb_target > 0) return pl->zpb;
  if (!pl->slots) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess)
      return pl->zpb;
    const int per = pl->var->grid_blocks_per_cu ? pl->var->grid_blocks_per_cu() : 0;
    if (per <= 0 || cus <= 0) return pl->zpb;
    pl->slots = cus * per;
  }
  double best = 0.0;
  int best_zpb = pl->zpb;
  for (int ng = 1; ng <= std::min(pl->nz, 16); ++ng) {
    const int zpb = (pl->nz + ng - 1) / ng;
    const int groups = (pl->nz + zpb - 1) / zpb;
    const double rounds = std::ceil((double)(nsb * groups) / (double)pl->slots);
    const double cost = rounds * (zpb + 1.0);
    if (ng == 1 || cost < best * 0.999) {
      best = cost;
      best_zpb = zpb;
    }
  }
  // On grids of two or more full rounds, units of 40 templates with the
  // remainder last beat equal groups (the short units fill the end of the
  // launch; 2-3% on the 2^21-bin plane at 65 and 101 rows).
  const int tz = default_zpb(pl->nz, kFp32UnitTarget);
  if (nsb * ((pl->nz + tz - 1) / tz) >= 2 * (int64_t)pl->slots) best_zpb = tz;
  return best_zpb;
}

static int plan_launch(fdas_plan_t pl, const void *spec, int64_t nbins, float *power, int64_t ld,
                       const CandOut &cand, hipStream_t s) {
  const int64_t nseg = (nbins + pl->U - 1) / pl->U;
  if (nseg > INT_MAX / 2) return set_error(FDAS_ERR_UNSUPPORTED, "nbins %lld too large", (long long)nbins);
  const int64_t nsb = (nseg + pl->var->G - 1) / pl->var->G;
  const int zpb = launch_zpb(pl, nsb);
  pl->last_zpb = zpb;
  const int64_t nzg = (pl->nz + zpb - 1) / zpb;
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
  a.zpb = zpb;
  a.bank_log2 = 0;
  while ((1 << a.bank_log2) < pl->L) ++a.bank_log2;
  a.consts = pl->consts;
  a.cand = cand;
  hipError_t e = pl->var->launch(a, s);
  if (e != hipSuccess) return hip_error(e, "correlation kernel launch");
  return FDAS_OK;
}

int plan_convolve(fdas_plan_t pl, const void *spec, int64_t nbins, float *power, int64_t ld,
                  hipStream_t s) {
  return plan_launch(pl, spec, nbins, power, ld, CandOut{}, s);
}

// Detection epilogue: the count is cleared on the stream by a kernel (no
// memset node, so the call may be captured), then the correlation kernel
// appends every plane point with power >= thr.
int plan_convolve_candidates(fdas_plan_t pl, const void *spec, int64_t nbins, float thr,
                             void *cands, int64_t cap, unsigned long long *count, hipStream_t s) {
  hipError_t e = launch_reset_counter(count, s);
  if (e != hipSuccess) return hip_error(e, "candidate counter reset");
  CandOut cd;
  cd.list = static_cast<Cand *>(cands);
  cd.count = count;
  cd.cap = cap;
  cd.thr = thr;
  return plan_launch(pl, spec, nbins, nullptr, 0, cd, s);
}

// One series of a batch: check its zmax against the plan's z grid and fill
// its descriptor (all but the first work item); `cost` orders the series.
static int series_desc(fdas_plan_t pl, const fdas_series &x, int i, int zpb, SeriesDesc *d,
                       double *cost) {
  const double dz = pl->p.dz;
  if (!std::isfinite(x.zmax) || x.zmax < 0.0 || x.zmax > pl->p.zmax * (1.0 + 1e-12) + 1e-12)
    return set_error(FDAS_ERR_INVALID, "series %d: zmax %g outside [0, %g]", i, x.zmax, pl->p.zmax);
  const double off = (pl->p.zmax - x.zmax) / dz;
  const double span = 2.0 * x.zmax / dz;
  if (std::fabs(off - std::nearbyint(off)) > 1e-9 || std::fabs(span - std::nearbyint(span)) > 1e-9)
    return set_error(FDAS_ERR_INVALID, "series %d: zmax %g is not on the plan's z grid", i, x.zmax);
  const int64_t nseg = (x.nbins + pl->U - 1) / pl->U;
  if (nseg > INT_MAX / 2) return set_error(FDAS_ERR_UNSUPPORTED, "series %d too long", i);
  const int per = (pl->p.flags & FDAS_FLAG_INTERBIN) ? 2 : 1;  // bank rows per drift
  d->spec = x.spectrum;
  d->power = x.power;
  d->nbins = x.nbins;
  d->ld = x.ld;
  d->item_begin = 0;
  d->nseg = (int)nseg;
  d->nz = per * ((int)std::nearbyint(span) + 1);
  d->row_off = per * (int)std::nearbyint(off);
  // near-equal template groups of at most zpb templates
  const int ng = (d->nz + zpb - 1) / zpb;
  d->zpb = (d->nz + ng - 1) / ng;
  *cost = (double)d->nz * (double)x.nbins;
  return FDAS_OK;
}

// Templates per work item of a batch whose series have `nsb` segment groups
// in all. A batch that fills the grid many times over has no tail to
// balance, and one unit per (series, segment) pays the forward transform
// once per segment: 3-4% faster than units of 40 (FP32) or 72 (matrix cores)
// on 118 series of 2^21 bins at 201 templates. Smaller batches keep the
// plan's unit size, as does a size fixed by FDAS_ZPB or the autotuner.
static int batch_zpb(fdas_plan_t pl, int64_t nsb) {
  if (pl->zpb_forced) return pl->zpb;
  if (!pl->slots) {
    int cus = 0;
    const int per = pl->var->grid_blocks_per_cu ? pl->var->grid_blocks_per_cu() : 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess ||
        per <= 0 || cus <= 0)
      return pl->zpb;
    pl->slots = cus * per;
  }
  return nsb >= 8 * (int64_t)pl->slots ? INT_MAX / 2 : pl->zpb;
}

static int64_t series_items(const SeriesDesc &d, int G) {
  const int64_t nsb = (d.nseg + G - 1) / G;
  const int64_t nzg = (d.nz + d.zpb - 1) / d.zpb;
  return nsb * nzg;
}

// Launch arguments of the batch kernel over a descriptor table on the device.
static int batch_args(fdas_plan_t pl, const SeriesDesc *d_desc, int nseries, int64_t total,
                      unsigned long long *counter, BatchArgs *a) {
  if (!pl->cus) {
    const hipError_t e =
        hipDeviceGetAttribute(&pl->cus, hipDeviceAttributeMultiprocessorCount, pl->device);
    if (e != hipSuccess) return hip_error(e, "CU count");
  }
  const int per_cu = std::max(1, pl->var->batch_blocks_per_cu());
  a->desc = d_desc;
  a->nseries = nseries;
  a->total = total;
  a->counter = counter;
  a->bank = pl->bank;
  a->tw = pl->tw;
  a->U = pl->U;
  a->half = pl->m / 2;
  a->zpb = pl->zpb;
  a->grid = (int)std::min<int64_t>((int64_t)pl->cus * per_cu, total);
  a->bank_log2 = 0;
  while ((1 << a->bank_log2) < pl->L) ++a->bank_log2;
  a->consts = pl->consts;
  return FDAS_OK;
}

// Detection epilogue with peak picking: the candidate list goes to the head
// of the workspace, the hash table of grid cells after it, and the peaks
// kernels run after the correlation on the same stream.
int plan_convolve_peaks(fdas_plan_t pl, const void *spec, int64_t nbins, float thr, void *work,
                        int64_t cand_cap, void *peaks, int64_t peak_cap,
                        unsigned long long *counts, hipStream_t s) {
  hipError_t e = launch_peaks_reset(counts, s);
  if (e != hipSuccess) return hip_error(e, "peak counter reset");
  CandOut cd;
  cd.list = static_cast<Cand *>(work);
  cd.count = counts;
  cd.cap = cand_cap;
  cd.thr = thr;
  const int st = plan_launch(pl, spec, nbins, nullptr, 0, cd, s);
  if (st != FDAS_OK) return st;
  void *table = static_cast<unsigned char *>(work) + (size_t)cand_cap * sizeof(Cand);
  e = launch_peaks(cd.list, cand_cap, table, counts, (pl->p.flags & FDAS_FLAG_INTERBIN) ? 1 : 0,
                   static_cast<Cand *>(peaks), peak_cap, s);
  if (e != hipSuccess) return hip_error(e, "peak kernels");
  return FDAS_OK;
}

// Host side of the batched path: validate and order the series (largest
// first), lay out their work items, upload the descriptors when the batch
// changes, and replay one captured graph of the batch launch.
int plan_convolve_batch(fdas_plan_t pl, const fdas_series *series, int nseries, hipStream_t s) {
  if (!pl->var->launch_batch)
    return set_error(FDAS_ERR_UNSUPPORTED, "kernel %s has no batched form", pl->var->name);
  const int G = pl->var->G;
  std::vector<SeriesDesc> desc(nseries);
  std::vector<double> cost(nseries);
  int64_t nsb = 0;
  for (int i = 0; i < nseries; ++i) {
    const int st = series_desc(pl, series[i], i, pl->zpb, &desc[i], &cost[i]);
    if (st != FDAS_OK) return st;
    nsb += (desc[i].nseg + G - 1) / G;
  }
  const int zpb = batch_zpb(pl, nsb);
  int most = 0;  // templates per unit of the largest unit, for plan info
  for (int i = 0; i < nseries; ++i) {
    const int ng = (desc[i].nz + zpb - 1) / zpb;
    desc[i].zpb = (desc[i].nz + ng - 1) / ng;
    most = std::max(most, desc[i].zpb);
  }
  pl->last_zpb = most;
  std::vector<int> order(nseries);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<SeriesDesc> sorted(nseries);
  int64_t total = 0;
  for (int k = 0; k < nseries; ++k) {
    sorted[k] = desc[order[k]];
    sorted[k].item_begin = total;
    total += series_items(sorted[k], G);
  }
  if (total == 0) return FDAS_OK;

  hipError_t e = hipSuccess;
  auto &graphs = pl->graphs;
  fdas_plan_s::GraphEntry *hit = nullptr;
  for (auto &ge : graphs)
    if (ge.key.size() == sorted.size() &&
        std::memcmp(ge.key.data(), sorted.data(), sorted.size() * sizeof(SeriesDesc)) == 0) {
      hit = &ge;
      break;
    }
  const char *nog = std::getenv("FDAS_NO_GRAPH");
  const bool eager = nog && *nog == '1';
  if (!hit || eager) {
    // new batch layout: upload its descriptors and capture a graph for it
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "synchronise before descriptor upload");
    if (!hit && graphs.size() >= kMaxGraphs) {  // evict the least recently used layout
      size_t old = 0;
      for (size_t i = 1; i < graphs.size(); ++i)
        if (graphs[i].last_use < graphs[old].last_use) old = i;
      if (graphs[old].exec) (void)hipGraphExecDestroy(graphs[old].exec);
      if (graphs[old].d_desc) (void)hipFree(graphs[old].d_desc);
      graphs.erase(graphs.begin() + old);
    }
    fdas_plan_s::GraphEntry ent;
    e = hipMalloc(&ent.d_desc, sorted.size() * sizeof(SeriesDesc));
    if (e != hipSuccess) return set_error(FDAS_ERR_NOMEM, "descriptor allocation: %s", hipGetErrorString(e));
    e = hipMemcpy(ent.d_desc, sorted.data(), sorted.size() * sizeof(SeriesDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(ent.d_desc);
      return hip_error(e, "descriptor upload");
    }
    if (!pl->cap_stream) {
      e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        (void)hipFree(ent.d_desc);
        return hip_error(e, "capture stream");
      }
    }
    BatchArgs a;
    const int st = batch_args(pl, ent.d_desc, nseries, total, pl->counter, &a);
    if (st != FDAS_OK) {
      (void)hipFree(ent.d_desc);
      return st;
    }
    if (eager) {
      e = pl->var->launch_batch(a, s);
      hipError_t e2 = hipStreamSynchronize(s);
      (void)hipFree(ent.d_desc);
      if (e != hipSuccess) return hip_error(e, "batch kernel launch");
      if (e2 != hipSuccess) return hip_error(e2, "batch kernel");
      return FDAS_OK;
    }
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipFree(ent.d_desc);
      return hip_error(e, "begin capture");
    }
    hipError_t le = pl->var->launch_batch(a, pl->cap_stream);
    e = hipStreamEndCapture(pl->cap_stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipFree(ent.d_desc);
      return hip_error(le != hipSuccess ? le : e, "batch kernel capture");
    }
    e = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      (void)hipFree(ent.d_desc);
      return hip_error(e, "graph instantiate");
    }
    ent.key = sorted;
    graphs.push_back(std::move(ent));
    hit = &graphs.back();
  }
  hit->last_use = ++pl->use_clock;
  e = hipGraphLaunch(hit->exec, s);
  if (e != hipSuccess) return hip_error(e, "graph launch");
  return FDAS_OK;
}

// Allocation-free batched path: the same work items and kernels, with the
// descriptor table and the work counter in the library's device scratch
// array (uploaded as kernel arguments) and the launch made directly on the
// stream, without a graph. Host-side state is on the stack.
int plan_convolve_batch_noalloc(fdas_plan_t pl, const fdas_series *series, int nseries,
                                hipStream_t s) {
  if (!pl->var->launch_batch)
    return set_error(FDAS_ERR_UNSUPPORTED, "kernel %s has no batched form", pl->var->name);
  if (nseries > kNoAllocMaxSeries)
    return set_error(FDAS_ERR_INVALID, "%d series exceed the %d the allocation-free batch holds",
                     nseries, kNoAllocMaxSeries);
  const int G = pl->var->G;
  double cost[kNoAllocMaxSeries];
  int order[kNoAllocMaxSeries];
  int64_t nsb = 0;
  for (int i = 0; i < nseries; ++i) {
    SeriesDesc d;
    const int st = series_desc(pl, series[i], i, pl->zpb, &d, &cost[i]);
    if (st != FDAS_OK) return st;
    order[i] = i;
    nsb += (d.nseg + G - 1) / G;
  }
  const int zpb = batch_zpb(pl, nsb);
  // largest first, ties in input order (the order the graph path uses)
  std::sort(order, order + nseries,
            [&](int a, int b) { return cost[a] > cost[b] || (cost[a] == cost[b] && a < b); });
  void *base = nullptr;
  int st = noalloc_scratch(pl->device, &base);
  if (st != FDAS_OK) return st;
  SeriesDesc *table = static_cast<SeriesDesc *>(base);
  unsigned long long *counter =
      reinterpret_cast<unsigned long long *>(static_cast<unsigned char *>(base) + kNoAllocDescBytes);
  DescChunk chunk;
  chunk.n = 0;
  chunk.first = 0;
  int64_t total = 0;
  for (int k = 0; k < nseries; ++k) {
    SeriesDesc &d = chunk.d[chunk.n];
    double c = 0.0;
    (void)series_desc(pl, series[order[k]], order[k], zpb, &d, &c);
    d.item_begin = total;
    total += series_items(d, G);
    if (++chunk.n == kDescChunk || k == nseries - 1) {
      const hipError_t e = launch_desc_upload(chunk, table, s);
      if (e != hipSuccess) return hip_error(e, "descriptor upload kernel");
      chunk.first += chunk.n;
      chunk.n = 0;
    }
  }
  if (total == 0) return FDAS_OK;
  BatchArgs a;
  st = batch_args(pl, table, nseries, total, counter, &a);
  if (st != FDAS_OK) return st;
  const hipError_t e = pl->var->launch_batch(a, s);
  if (e != hipSuccess) return hip_error(e, "batch kernel launch");
  return FDAS_OK;
}

int destroy_plan(fdas_plan_t pl) {
  if (!pl) return FDAS_OK;
  hipError_t e = hipSuccess;
  if (pl->bank || pl->tw || pl->counter || pl->consts) e = hipDeviceSynchronize();
  for (auto &ge : pl->graphs) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    if (ge.d_desc) (void)hipFree(ge.d_desc);
  }
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  if (pl->counter) (void)hipFree(pl->counter);
  if (pl->bank) (void)hipFree(pl->bank);
  if (pl->tw) (void)hipFree(pl->tw);
  if (pl->consts) (void)hipFree(pl->consts);
  delete pl;
  if (e != hipSuccess) return hip_error(e, "synchronise before destroy");
  return FDAS_OK;
}

}  // namespace fdas
