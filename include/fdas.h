/*
 * fdas.h -- C ABI of the FDAS correlation step on AMD Instinct MI355X (gfx950).
 *
 * What it computes (Adamek, Dimoudi, Giles & Armour, "Improved Acceleration
 * of the GPU Fourier Domain Acceleration Search Algorithm"):
 *
 *   For every trial drift z_i = -zmax + i*dz, i in [0, nz), nz = 2*zmax/dz + 1
 *   (z is the number of bins the signal frequency drifts over the observation,
 *   Section 1, eq. 1), and every bin r in [0, nbins):
 *
 *     B_i(r) = sum_{q=-m/2}^{m/2} A[r+q] * conj(H_{z_i}(q))      (Section 1, eq. 2)
 *     power[i*ld + r] = |B_i(r)|^2
 *
 *   A is the complex spectrum (zero outside [0, nbins)); H_z(q) is the
 *   predicted, normalised Fourier response of a constant-frequency-derivative
 *   signal (Section 1): H_z(q) = exp(-i pi q) * integral_{-1/2}^{1/2}
 *   exp(i pi (z s^2 - 2 q s)) ds, evaluated in FP64 through Fresnel integrals.
 *   The sum is computed by overlap-and-save (Section 2): segments of L bins,
 *   a forward FFT (eq. 3 sign convention) held in on-chip memory, one
 *   pointwise product and one inverse FFT per template (Section 3), discard of
 *   the m wrapped outputs, and |.|^2 written straight to device memory.
 *
 * Conventions for every entry point:
 *   - Sample buffers (spectrum, power, templates, bank copies) are DEVICE
 *     pointers owned by the caller; structs and status are host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is stream-ordered and asynchronous; buffers must stay live until
 *     the stream has synchronised.
 *   - Every call validates its arguments on the host before any HIP call and
 *     returns a status code; nothing is thrown across the ABI. Detail for the
 *     last failure on the calling thread is in fdas_last_error().
 *   - A plan may be used from one stream at a time (it owns scratch state).
 *   - Results are bitwise deterministic for a fixed plan and input.
 */
#ifndef FDAS_H
#define FDAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define FDAS_OK 0
#define FDAS_ERR_INVALID (-1)     /* bad argument (checked before device work) */
#define FDAS_ERR_UNSUPPORTED (-2) /* valid but not compiled in (e.g. seg_len)   */
#define FDAS_ERR_NOMEM (-3)       /* a device or host allocation failed         */
#define FDAS_ERR_DEVICE (-4)      /* a HIP runtime call failed                  */

/* ---- precisions ---------------------------------------------------------- */
#define FDAS_FP32 0        /* FP32 storage and FFTs, FP32 output             */
#define FDAS_MIXED_FP16 1  /* FP16 storage, MFMA DFT stages, FP32 accumulate */
#define FDAS_MIXED_BF16 2  /* BF16 storage, MFMA DFT stages, FP32 accumulate */

/* ---- flags ----------------------------------------------------------------- */
#define FDAS_FLAG_SPLIT 1u    /* mixed: hi+lo split products (3 MFMA per stage;
                                 seg_len 4096) */
#define FDAS_FLAG_AUTOTUNE 2u /* fdas_plan: time the compiled variants (segment
                                 length, radix split, threads, templates per
                                 block) on a synthetic spectrum of 2^20 bins and
                                 keep the fastest per plane point; cached in the
                                 file named by FDAS_TUNE_CACHE when set */
#define FDAS_FLAG_INTERBIN 4u /* also the response half-way between bins (the
                                 corrected response of Section 1 at r + 1/2):
                                 the plane has 2 nz rows, row 2i holding z_i at
                                 integer r and row 2i + 1 the same z_i at
                                 r + 1/2, from the same m + 1 bins
                                 [r - m/2, r + m/2] (offsets q - 1/2) */
#define FDAS_FLAG_BANK 8u     /* fdas_make_templates: the Fourier-domain bank
                                 instead of the templates (ignored elsewhere) */

/* Filter-bank parameters.
 *   zmax, dz  : z grid z_i = -zmax + i*dz; zmax >= 0, dz > 0, 2*zmax/dz an
 *               integer within 1e-9.
 *   m         : even, >= 2; taps q in [-m/2, m/2] (m + 1 bins, eq. 2).
 *               0 selects the default nextpow2(2*zmax + 32), at least 8.
 *   seg_len   : overlap-and-save segment (FFT) length L, a power of two in
 *               [256, 16384] with L > m (mixed precisions: 2048 or 4096,
 *               with FDAS_FLAG_SPLIT 4096; others give
 *               FDAS_ERR_UNSUPPORTED). 0 selects the default (FP32:
 *               nextpow2(8 m) clamped to [256, 16384]; mixed: 4096), or
 *               with FDAS_FLAG_AUTOTUNE lets the tuner choose among
 *               compiled lengths with L - m >= L / 2.
 *   precision : FDAS_FP32 / FDAS_MIXED_FP16 / FDAS_MIXED_BF16.
 *   flags     : FDAS_FLAG_* bits.                                           */
typedef struct {
  double zmax;
  double dz;
  int m;
  int seg_len;
  int precision;
  unsigned flags;
} fdas_params;

/* One series of a batch (fdas_convolve_batch).
 *   spectrum : device complex64 [nbins] (interleaved re, im; 8-byte aligned).
 *   nbins    : >= 1.
 *   zmax     : this series' zmax; <= the plan's zmax and on its grid
 *              ((plan.zmax - zmax)/dz an integer). Its plane has
 *              nz_s = 2*zmax/dz + 1 rows, row j <-> z = -zmax + j*dz
 *              (2 nz_s rows with FDAS_FLAG_INTERBIN, as for the full plane).
 *   power    : device float [nz_s][ld], ld >= nbins.                        */
typedef struct {
  const void *spectrum;
  int64_t nbins;
  double zmax;
  float *power;
  int64_t ld;
} fdas_series;

/* What a plan resolved to (fdas_plan_get_info). */
typedef struct {
  int nz;              /* rows of the plane                                  */
  int m;               /* window (taps -m/2..m/2)                            */
  int seg_len;         /* L                                                  */
  int valid;           /* U = L - m outputs kept per segment                 */
  int precision;
  unsigned flags;
  int threads;         /* threads per segment in the hot kernel              */
  int templates_per_block; /* of the last fdas_convolve launch, or the largest
                              work unit of the last fdas_convolve_batch
                              (before either: the plan's default)         */
  int segments_per_block;
  size_t bank_bytes;   /* device bytes of the Fourier-domain template bank   */
  double plan_ms;      /* wall time of fdas_plan (templates + bank)          */
  char kernel[64];     /* name of the selected hot-kernel variant            */
} fdas_plan_info;

typedef struct fdas_plan_s *fdas_plan_t;

/* Number of plane rows for valid params: nz = 2*zmax/dz + 1, or 2 nz with
 * FDAS_FLAG_INTERBIN; else a negative status. Host only; never touches the
 * device.                                                                    */
int fdas_plane_rows(const fdas_params *p);

/* Fill defaults (m, seg_len) and validate; *out receives the resolved
 * parameters. Host only. Returns FDAS_OK, FDAS_ERR_INVALID or
 * FDAS_ERR_UNSUPPORTED.                                                      */
int fdas_resolve_params(const fdas_params *in, fdas_params *out);

/* Template generation (Section 1, the predicted normalised response H used in
 * eq. 2), in FP64 on the device.
 *   templates : device complex128 [nz][m+1], element [i][j] = H_{z_i}(j - m/2),
 *               or NULL to only query the size.
 *               With FDAS_FLAG_BANK in p->flags: the template bank the
 *               overlap-and-save product multiplies by instead, device
 *               complex64 [nz][L] in natural frequency order,
 *               T_i[k] = conj(sum_q H_{z_i}(q) exp(-2 pi i (q mod L) k / L)) / L
 *               (an FP64 direct sum with exact phase reduction, rounded to
 *               FP32; L = seg_len as resolved, which must not be left to the
 *               autotuner). This form allocates an FP64 temporary of
 *               nz (m+1) 16 bytes and synchronises `stream`.
 *   bytes     : in/out. On return holds the required size in bytes. When
 *               templates != NULL, *bytes on entry must be >= that size.
 * Parameters are resolved as in fdas_resolve_params (nz doubles with
 * FDAS_FLAG_INTERBIN). Otherwise asynchronous on `stream`, no allocation.    */
int fdas_make_templates(const fdas_params *p, void *templates, size_t *bytes,
                        void *stream);

/* Build a plan on `device`: generates the templates (FP64), transforms them
 * to the Fourier-domain bank T_i[k] = conj(FFT_L(h_i))[k] / L with
 * h_i[q mod L] = H_{z_i}(q) (FP64, then rounded to the storage precision and
 * laid out in the hot kernel's register order), builds twiddle tables, and
 * picks the kernel variant (autotuned with FDAS_FLAG_AUTOTUNE). Synchronises
 * `stream` before returning. *out is NULL on failure.                        */
int fdas_plan(fdas_plan_t *out, const fdas_params *p, int device, void *stream);

/* Report the resolved configuration of a plan.                              */
int fdas_plan_get_info(fdas_plan_t plan, fdas_plan_info *info);

/* Copy the plan's bank, in natural frequency order, as complex64 [nz][L]
 * (FP32 plans and mixed plans with FDAS_FLAG_SPLIT: exactly the stored
 * FP32 values; other mixed plans: the 16-bit values widened to FP32) into
 * device memory `dst` of at least nz*L*8 bytes. For testing.               */
int fdas_plan_bank(fdas_plan_t plan, void *dst, size_t bytes, void *stream);

/* The hot path: power[i*ld + r] = |B_i(r)|^2 for one spectrum.
 *   spectrum : device complex64 [nbins]; nbins >= 1.
 *   power    : device float [nz][ld], ld >= nbins; fully overwritten in
 *              columns [0, nbins) of every row.
 * Asynchronous on `stream`; launches only kernels (no allocation, no copy). */
int fdas_convolve(fdas_plan_t plan, const void *spectrum, int64_t nbins,
                  float *power, int64_t ld, void *stream);

/* One detection candidate: plane row (as in the power plane), bin, power. */
typedef struct {
  int32_t row;
  float power;
  int64_t r;
} fdas_candidate;

/* The hot path with a detection epilogue instead of the plane (the step that
 * follows the plane in the FDAS pipeline, Section 3; only the threshold part
 * of it): every plane point with power >= threshold is appended to `cands`.
 *   cands    : device fdas_candidate [capacity] (16-byte aligned); the first
 *              min(*count, capacity) entries are written, in no fixed order.
 *   count    : device uint64; set to the number of plane points at or above
 *              the threshold (also those that did not fit).
 * The count is cleared on `stream` by a kernel before the correlation, so the
 * call can be captured into a graph. Asynchronous; no allocation, no copy.   */
int fdas_convolve_candidates(fdas_plan_t plan, const void *spectrum, int64_t nbins,
                             float threshold, fdas_candidate *cands, int64_t capacity,
                             unsigned long long *count, void *stream);

/* The hot path with the whole detection epilogue: threshold, then peak
 * picking (the candidate search that follows the plane, Section 3, which
 * names it without defining it; the rule below is this library's reading).
 * On the (z, r) grid -- plane row i and bin r, or with FDAS_FLAG_INTERBIN
 * grid row i = plane row >> 1 and column 2 r + (row & 1), so neighbouring
 * columns are half a bin apart -- a peak is a point with power >= threshold
 * that outranks each of its (up to) eight neighbours: p outranks q when
 * P_p > P_q, or P_p == P_q and p's (grid row, column) comes first. A
 * plateau therefore has exactly one peak. No plane is written.
 *   workspace      : device memory of fdas_peaks_workspace_bytes(cand_capacity)
 *                    bytes or more, 16-byte aligned (candidate list and a
 *                    hash table of grid cells).
 *   cand_capacity  : candidates (points >= threshold) the workspace holds,
 *                    0 .. FDAS_PEAKS_MAX_CANDIDATES. When more are found the
 *                    peaks are not valid: compare counts[0] with it.
 *   peaks          : device fdas_candidate [peak_capacity] (16-byte aligned),
 *                    plane row and bin as in the power plane; the first
 *                    min(counts[1], peak_capacity) entries, in no fixed order.
 *   counts         : device uint64 [2]: candidates found, peaks found.
 * Counters are cleared by a kernel on `stream`; kernels only, no allocation,
 * no copy, no synchronisation.                                               */
#define FDAS_PEAKS_MAX_CANDIDATES (1 << 30)
size_t fdas_peaks_workspace_bytes(int64_t cand_capacity); /* 0 if out of range */
int fdas_convolve_peaks(fdas_plan_t plan, const void *spectrum, int64_t nbins, float threshold,
                        void *workspace, size_t workspace_bytes, int64_t cand_capacity,
                        fdas_candidate *peaks, int64_t peak_capacity, unsigned long long *counts,
                        void *stream);

/* Batched hot path: one persistent launch over every (series, template group,
 * segment) work item, largest series first: as many blocks as the GPU holds
 * at once take items from a device counter (reset by a kernel in the same
 * graph) until none is left. FDAS_BATCH_PERSISTENT=0 in the environment
 * selects a flat grid of one block per item instead. Each series uses the
 * central rows of the plan's bank; a batch that fills the GPU many times over
 * gives each (series, segment) one work item for all its templates. The
 * launch is captured once into a HIP graph per distinct batch shape and
 * replayed. `series` is host memory with nseries >= 1 entries.               */
int fdas_convolve_batch(fdas_plan_t plan, const fdas_series *series,
                        int nseries, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batched
 * hot path of fdas_convolve_batch with the same work items, kernels and
 * results, but no allocation, no graph and no host synchronisation. The
 * descriptor table (56 bytes per series) and the work counter live in a
 * device array of the library, one per GPU, FDAS_NOALLOC_SCRATCH_BYTES
 * (229,632) bytes, held until the process ends; descriptors reach it as kernel
 * arguments, so `series` may be reused as soon as the call returns.
 *   nseries : 1 .. FDAS_NOALLOC_MAX_SERIES; more is FDAS_ERR_INVALID.
 * Other arguments, validation and errors are those of fdas_convolve_batch.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams, or different threads without ordering) race and
 * must not be made; calls ordered on one stream are safe.                   */
#define FDAS_NOALLOC_MAX_SERIES 4096
#define FDAS_NOALLOC_SCRATCH_BYTES (FDAS_NOALLOC_MAX_SERIES * 56 + 256)
int fdas_convolve_batch_noalloc(fdas_plan_t plan, const fdas_series *series, int nseries,
                                void *stream);

/* Release a plan and everything it owns. NULL is allowed (returns FDAS_OK).
 * Synchronises the device the plan lives on.                                */
int fdas_destroy(fdas_plan_t plan);

/* Names of the compiled hot-kernel variants for a segment length (0 = all)
 * and precision (-1 = all), newline-separated, into the host buffer `buf` of
 * `len` bytes (truncated, always NUL-terminated when len > 0; buf may be NULL
 * with len 0 to count). Returns the number of variants or a negative status.
 * A variant is forced for new plans by the FDAS_VARIANT environment
 * variable; FDAS_ZPB overrides templates per work unit.                     */
int fdas_kernel_variants(int seg_len, int precision, char *buf, size_t len);

/* ---- standalone batched FFT ---------------------------------------------
 * The shared-memory FFT the correlation kernel is built from, on its own
 * (the FFT the paper measures separately, Section 3 and Table 1): batch
 * transforms of length n, each held in registers and LDS by one group of
 * threads with elems_per_thread elements per thread.
 *   out[b][k] = sum_j in[b][j] exp(direction * 2 pi i j k / n)
 * direction -1 is the forward transform of eq. 3, +1 the inverse (no 1/n).
 * Buffers are device complex64 [batch][n], natural order, 8-byte aligned;
 * in == out (in place) is allowed, other overlap is not.                    */
typedef struct fdas_fft_s *fdas_fft_t;

typedef struct {
  int n;                    /* transform length                              */
  int elems_per_thread;
  int threads;              /* threads per transform                          */
  int transforms_per_block;
  char kernel[64];          /* compiled form                                  */
} fdas_fft_info;

/* Choose the compiled form for n (a power of two) and elems_per_thread (0 =
 * the default for n) and build its FP64-generated twiddle table on `device`
 * (allocates n * 8 bytes; synchronises `stream`). FDAS_ERR_UNSUPPORTED when
 * no form of that length / elements per thread is compiled.                 */
int fdas_fft_plan(fdas_fft_t *out, int n, int elems_per_thread, int device, void *stream);
int fdas_fft_get_info(fdas_fft_t plan, fdas_fft_info *info);
/* batch >= 0 transforms (0 is a no-op); asynchronous on `stream`, one kernel
 * launch, no allocation.                                                     */
int fdas_fft_exec(fdas_fft_t plan, const void *in, void *out, int64_t batch, int direction,
                  void *stream);
/* NULL is allowed. Synchronises the plan's device.                          */
int fdas_fft_destroy(fdas_fft_t plan);
/* Names of the compiled FFT forms of length n (0 = all), as for
 * fdas_kernel_variants. The FDAS_FFT_VARIANT environment variable forces a
 * form (by name) for new plans of its length.                               */
int fdas_fft_variants(int n, char *buf, size_t len);

/* ---- device front end --------------------------------------------------
 * The spectrum the correlation runs on (Section 1), made on the device from
 * a real series x[0 .. n): A[k] = sum_j x[j] exp(-2 pi i j k / n) (eq. 3
 * sign) for k in [0, n/2) (the Nyquist bin is dropped), A[0] = 0, then
 * A *= sqrt(ln 2 / median_{k=1..n/2-1} |A[k]|^2), which gives white noise unit
 * mean power (no scaling when that median is 0; n/2 - 1 is odd, so the
 * median is the middle value). FP32 throughout.                           */
typedef struct fdas_frontend_s *fdas_frontend_t;

/* n: a power of two in [128, 2^25]. Allocates the plan's scratch on `device`
 * (12 n / 2 bytes plus twiddle tables); synchronises `stream`.              */
int fdas_frontend_plan(fdas_frontend_t *out, int64_t n, int device, void *stream);
/* series   : device float [n], 8-byte aligned.
 * spectrum : device complex64 [n/2], 8-byte aligned; may be the series' own
 *            buffer (the series is consumed before the first write); any
 *            other overlap is rejected.
 * stats    : NULL, or device float [2] receiving (scale, median |A|^2).
 * Asynchronous on `stream`; kernels only, no allocation. A plan may be used
 * from one stream at a time (it owns the scratch).                          */
int fdas_frontend_exec(fdas_frontend_t plan, const float *series, void *spectrum, float *stats,
                       void *stream);
/* NULL is allowed. Synchronises the plan's device.                          */
int fdas_frontend_destroy(fdas_frontend_t plan);

/* Static description of a status code.                                      */
const char *fdas_status_string(int status);

/* Detail of the last failure on the calling thread ("" if none).            */
const char *fdas_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDAS_H */
