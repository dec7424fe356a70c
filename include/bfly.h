/*
 * bfly.h -- C ABI of the MI355X butterfly-filtering library (libbfly.so).
 *
 * Butterfly filtering (van Putten, "GPU-accelerated broadband analysis of multi-messenger
 * light curves of GRBs", Sec. 2.1) correlates a series against a large bank of ~1 s
 * ascending and descending chirp templates at every time offset (matched filtering) and
 * reduces the correlations to:
 *   - the butterfly output: per offset tau, m[tau] = max_k |rho(tau,k)| and the template
 *     a[tau] reaching it (its maxima are histogrammed beside a time-randomised control,
 *     Fig. 2 caption and Sec. 2.2);
 *   - the chirp-based spectrogram: per offset and f0 bin, the max |rho| over the fdot
 *     templates of that bin, and its time mean, the broadband spectrum (Sec. 2.1, Fig. 1).
 *
 * Definitions used throughout (the paper states none of them; these are the readings):
 *   template k = (i, j): f0_i = linspace(f0_min, f0_max, n_f0)[i], fdot_j likewise,
 *     k = i*n_fdot + j (f0-major); h_k[n] = cos(2 pi (f0_i t + fdot_j t^2 / 2)), t = n/fs,
 *     n = 0..L-1, with its mean removed and scaled to unit L2 norm.
 *   d(tau,k) = sum_{n<L} h_k[n] x[tau+n],  tau = 0..W-1,  W = n_samples - L + 1.
 *   E_tau = sum_n (x[tau+n] - mean)^2 (centred norm, default) or sum_n x[tau+n]^2 (raw),
 *     from float64 prefix sums; rho = d / sqrt(E_tau).
 *   A window is degenerate when it holds a non-finite sample, when R = sum x^2 is 0, or
 *     when E <= 1e-12 R; then m = 0, a = -1, its spectrogram entries are 0 and it is left
 *     out of the histogram (and counted in n_degenerate).
 *   Ties: the smallest global template index wins.
 *
 * Conventions
 *   - Every call returns a bf_status (0 = BF_OK, negative = error) and never throws; on
 *     error bf_last_error() returns a message for the calling thread.
 *   - Device buffers (bank memory, workspaces, inputs, outputs) are owned by the caller;
 *     sizes come from the *_bytes() queries.  Pointers marked "device" must be device
 *     memory on the current HIP device; "host" pointers are ordinary host memory.
 *   - Work is enqueued on the caller's stream (a hipStream_t passed as bf_stream; NULL is
 *     the default stream) and runs asynchronously; the caller synchronises.
 *   - A bank is immutable once created and may be shared by threads and streams.
 *   - Inputs are float32 series; samples must satisfy |x| <= 1e30 (non-finite samples are
 *     allowed and make their windows degenerate).
 */
#ifndef BFLY_H
#define BFLY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* bf_stream; /* a hipStream_t */

typedef enum {
  BF_OK = 0,
  BF_EINVAL = -1,     /* invalid argument or descriptor */
  BF_ENOMEM = -2,     /* a host or device allocation failed */
  BF_EBUDGET = -3,    /* a request cannot fit the server's HBM budget even alone */
  BF_EAGAIN = -4,     /* result not ready yet */
  BF_ENOTFOUND = -5,  /* unknown ticket */
  BF_EHIP = -6,       /* a HIP runtime call failed */
  BF_ECANCELED = -7   /* the request was cancelled */
} bf_status;

typedef enum {
  BF_FP32 = 0,   /* float32 templates and data, float32 MFMA */
  BF_BF16X3 = 1, /* bf16 hi+lo split of templates and data; hi*hi + hi*lo + lo*hi */
  BF_FP8 = 2     /* e4m3 templates with a per-template power-of-two scale (reserved) */
} bf_precision;

typedef enum { BF_NORM_CENTRED = 0, BF_NORM_RAW = 1 } bf_norm;

/* Template bank descriptor (Sec. 2.1: banks of up to millions of 1 s chirps covering
 * ascending and descending branches).  The grid is f0-major; shard s of S owns the f0
 * index range [s*n_f0/S, (s+1)*n_f0/S) -- (0, 1) is the whole bank.  Requires fs > 0,
 * 1 <= L <= 8192, n_f0 >= 1, n_fdot >= 1, 0 <= shard_index < shard_count <= n_f0,
 * finite bounds with min <= max, and every template must have a non-zero centred norm
 * (BF_EINVAL otherwise). */
typedef struct {
  double fs;
  int32_t L;
  int32_t n_f0;
  int32_t n_fdot;
  int32_t shard_index;
  int32_t shard_count;
  int32_t precision; /* bf_precision */
  double f0_min, f0_max;
  double fdot_min, fdot_max;
} bf_bank_desc;

typedef struct bf_bank bf_bank;

/* Device bytes the caller must provide to bf_bank_create for this descriptor.
 * Returns BF_EINVAL for an invalid descriptor. */
bf_status bf_bank_bytes(const bf_bank_desc* desc, size_t* bytes);

/* Builds the template bank in float64 on the device and stores it, quantised to the
 * descriptor's precision and in the kernel's tile layout, in dev_mem (device, caller-
 * owned, at least bf_bank_bytes(), 256-byte aligned, alive for the bank's lifetime).
 * Runs on stream and synchronises it before returning, to check that every template could
 * be normalised.  *out receives a host handle to free with bf_bank_destroy; the handle
 * records the current device, on which every search with it must run. */
bf_status bf_bank_create(const bf_bank_desc* desc, void* dev_mem, size_t dev_bytes,
                         bf_stream stream, bf_bank** out);

/* Bank shape: number of local templates K, spectrogram bins (local f0 values), the global
 * index of local template 0.  f0 / fdot (host, K entries each) may be NULL. */
bf_status bf_bank_info(const bf_bank* bank, int64_t* K, int32_t* n_bins, int64_t* k_offset,
                       double* f0, double* fdot);

bf_status bf_bank_destroy(bf_bank* bank);

/* Search parameters. */
typedef struct {
  int32_t norm;      /* bf_norm */
  int32_t t_block;   /* spectrogram rows hold the max over blocks of t_block offsets, >= 1 */
  int32_t hist_bins; /* histogram bins over [hist_lo, hist_hi), 1..4096 */
  int32_t reserved;  /* must be 0 */
  double hist_lo, hist_hi; /* hist_lo < hist_hi; values are clamped into the end bins */
} bf_search_params;

/* Outputs of one series (device pointers, caller-owned; NULL = not requested).
 *   max_abs[W]      butterfly output m (float32)
 *   argmax[W]       global template index reaching m; -1 on degenerate windows
 *   spec[R][B]      spectrogram, R = ceil(W / t_block) rows, B = n_bins, float32
 *   spectrum[B]     (1/W) sum_tau S(tau, i) over the undecimated spectrogram (float64)
 *   hist[hist_bins] histogram of m over non-degenerate windows (uint32)
 *   n_degenerate[1] number of degenerate windows (int64) */
typedef struct {
  float* max_abs;
  int32_t* argmax;
  float* spec;
  double* spectrum;
  uint32_t* hist;
  int64_t* n_degenerate;
} bf_result;

/* One series of a batch: x (device, float32, n samples, n >= L) and its outputs. */
typedef struct {
  const float* x;
  int64_t n;
  bf_result out;
} bf_segment;

/* Device workspace bytes for a batch of n_segs series of lengths n[0..n_segs-1] (host
 * array).  Returns BF_EINVAL when a length is below L or n_segs < 1. */
bf_status bf_workspace_bytes(const bf_bank* bank, const int64_t* n, int32_t n_segs,
                             const bf_search_params* params, size_t* bytes);

/* Searches one series: every template at every offset, then the reductions above.
 * workspace: device, at least bf_workspace_bytes() for {n}, 256-byte aligned.
 * Asynchronous on stream; n < L -> BF_EINVAL. */
bf_status bf_search_segment(const bf_bank* bank, const float* x, int64_t n,
                            const bf_search_params* params, const bf_result* out,
                            void* workspace, size_t workspace_bytes, bf_stream stream);

/* Searches n_segs series of uneven lengths in one pass: one launch of each kernel covers
 * all series (a time-randomised control is just another series).  segs is a host array.
 * Results are identical, bit for bit, to searching each series alone. */
bf_status bf_search_batch(const bf_bank* bank, const bf_segment* segs, int32_t n_segs,
                          const bf_search_params* params, void* workspace,
                          size_t workspace_bytes, bf_stream stream);

/* Work decomposition the searches would use for series of lengths n[0..n_segs-1] (host):
 * the bank sweep is split into *n_ranges contiguous ranges of whole f0 bins, and each
 * (series, block of offsets, range) is one work item of the contraction kernel. */
bf_status bf_plan(const bf_bank* bank, const int64_t* n, int32_t n_segs, int32_t* n_ranges,
                  int64_t* n_items);

/* Profiling aid.  With timing enabled, every search records HIP events on its stream
 * around each of its five kernels (clear, prefix sums, window norms, contraction,
 * finalise).  bf_kernel_times waits for the calling thread's last search and writes the
 * five durations in milliseconds to ms[0..4] (host); BF_EAGAIN if no timed search ran. */
bf_status bf_set_timing(int32_t enable);
bf_status bf_kernel_times(double* ms);

/* Message describing the last error on the calling thread ("" if none). */
const char* bf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BFLY_H */
