// Plan object shared by the host translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "fdas.h"
#include "ols_variants.hpp"

namespace fdas {

int set_error(int status, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);
int resolve_params(const fdas_params *in, fdas_params *out, int *nz_out);
int default_seg_len(int m, int nz, int precision);
bool mixed_supported(int seg_len, int split);

int build_plan(fdas_plan_t *out, const fdas_params &p, int nz, int device, hipStream_t s);
void plan_info(fdas_plan_t plan, fdas_plan_info *info);
int list_variants(int seg_len, int precision, char *buf, size_t len);
int plan_rows(fdas_plan_t plan);
int plan_seg_len(fdas_plan_t plan);
int plan_device(fdas_plan_t plan);
int plan_bank_natural(fdas_plan_t plan, void *dst, hipStream_t s);
int plan_convolve(fdas_plan_t plan, const void *spec, int64_t nbins, float *power, int64_t ld,
                  hipStream_t s);
int plan_convolve_batch(fdas_plan_t plan, const fdas_series *series, int nseries, hipStream_t s);
int plan_convolve_batch_noalloc(fdas_plan_t plan, const fdas_series *series, int nseries,
                                hipStream_t s);
int plan_convolve_candidates(fdas_plan_t plan, const void *spec, int64_t nbins, float thr,
                             void *cands, int64_t cap, unsigned long long *count, hipStream_t s);
int plan_convolve_peaks(fdas_plan_t plan, const void *spec, int64_t nbins, float thr, void *work,
                        int64_t cand_cap, void *peaks, int64_t peak_cap,
                        unsigned long long *counts, hipStream_t s);
int destroy_plan(fdas_plan_t plan);

}  // namespace fdas
