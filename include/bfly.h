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
  BF_FP8 = 2,    /* OCP e4m3 templates and data with power-of-two scales (per template, per
                    strip), undone by the MFMA scale operands; the rounded templates' sums
                    times the window mean are subtracted.  Bound from the rounding model
                    (e4m3, 2^-4 per operand, six standard deviations): 0.43 of the noise
                    scale 1/sqrt(L) of |rho|; ~1% median relative error */
  BF_F16X2 = 3,  /* fp16 hi+lo split of the templates, fp16 data with a power-of-two strip
                    scale; h_hi*x + h_lo*x (two MFMA products per tap).  The data's fp16
                    rounding (2^-11) bounds the error: 2.4e-3 of the noise scale */
  BF_FFT = 4,    /* FFT correlation (Sec. 2.2): float32 template spectra, overlap-save with
                    real FFTs of length N = 8192 (N - L + 1 valid outputs per block; the
                    environment variable BF_FFT_POINTS = 1024, 2048 or 4096 selects a shorter
                    transform that holds the template, on the general kernel); L <= 4096;
                    the same outputs as the direct forms.
                    Bound 1e-5, growing as 3.2e-6 x (RMS of the loudest transform block
                    near the window / the window's RMS) where that ratio exceeds ~3 */
  BF_F16F8 = 5,  /* fp16 product of the fp16-rounded template and data, plus the two residual
                    products (template residual x data, template x data residual) as e4m3 codes
                    with power-of-two scales (per template, per strip) undone by the MFMA scale
                    operands; the rounded templates' sums times the window mean are
                    subtracted.  Two thirds of BF_BF16X3's MFMA time per tap; ~1e-5 to 3e-5
                    relative error, bound 1e-4; L <= 4224 */
  BF_F16F6 = 6   /* as BF_F16F8 with the residual products in e2m3 (fp6) codes, whose MFMA
                    runs at twice the e4m3 rate: half of BF_BF16X3's MFMA time per tap.
                    Bound 1e-4, growing as 2.8e-5 x (largest sample near the window / the
                    window's RMS) up to BF_F16X2's 2.4e-3: the data residual codes have a
                    fixed quantum within a strip; L <= 4224 */
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
 *   spec[B][R]      spectrogram, bin-major: row i holds f0 bin i over R = ceil(W / t_block)
 *                   time blocks (max over each block of t_block offsets), float32
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

/* The search of bf_search_segment for callers that cannot allocate memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same results, bit for bit, with the workspace taken from a device array of 32 MiB built
 * into the library (one per GPU, held until the process ends) and the batch table written
 * by a kernel from its arguments.  No host or device memory is allocated by the call.
 * Limit: table + bf_workspace_bytes of the series <= 32 MiB (about 540,000 samples at
 * L = 4096 for the direct forms); a larger series returns BF_EINVAL.  The array keeps the
 * last call's contents and is cleared by the search itself where it must start at zero.
 * Calls that overlap on one GPU (two streams, two threads) share the array and race: the
 * caller serialises them.  Timing records (bf_set_timing) are not taken. */
bf_status bf_search_segment_noalloc(const bf_bank* bank, const float* x, int64_t n,
                                    const bf_search_params* params, const bf_result* out,
                                    bf_stream stream);

/* ---- kappa-sigma tails (Sec. 2.2 and the Fig. 5 caption: only correlations above kappa
 * sigma leave the GPU; Fig. 6 caption: pseudo-spectra of their counts) -------------------
 * sigma_k of a series = sqrt(mean over its non-degenerate offsets of rho_k(tau)^2): the
 * spread of template k's matched-filter output (its variance, as a zero-mean template gives
 * a zero-mean output; the paper obtains it from the spectra by Parseval's theorem, here it
 * is summed in the contraction's epilogue).  A tail is an offset-template pair with
 * |rho_k(tau)| > kappa * sigma_k (strict); the pseudo-spectrum counts the tails per f0 bin.
 * Tail outputs of one series (device pointers, caller-owned):
 *   sigma[K]        sigma_k, float32 (0 for every k if all windows are degenerate)
 *   tau, k, rho     [capacity] offset, global template index and signed rho (float32) of
 *                   each tail, in unspecified order; may be NULL when capacity is 0
 *   bin_counts[B]   tails per f0 bin, all tails counted (uint32)
 *   n_tails[1]      the number of tails (int64); when it exceeds capacity the lists hold
 *                   `capacity` of them, which ones is unspecified
 * The set of tails, their values, sigma and the counts are deterministic and, as for the
 * search, identical alone or in a batch. */
typedef struct {
  float* sigma;
  int32_t* tau;
  int32_t* k;
  float* rho;
  uint32_t* bin_counts;
  int64_t* n_tails;
  int64_t capacity;
} bf_tails;

/* One series of a tail search: x and the search outputs as in bf_segment, and its tails. */
typedef struct {
  const float* x;
  int64_t n;
  bf_result out;
  bf_tails tails;
} bf_tail_segment;

/* Device workspace bytes of a tail search: bf_workspace_bytes plus, per series, the rho^2
 * sums and thresholds (K_pad * 16 bytes), the candidate lists of the single pass (12 bytes a
 * candidate, K_pad * W / 16384 of them clamped to [2^16, 2^24]), the locally normalised
 * series and its lag sums (n * 4 + (17 L + 1) * 8 bytes), the predictor's spectrum and,
 * with an FFT bank, rho^2 partial sums per block and wave (tiles * 4 * K_pad * 8 bytes). */
bf_status bf_tails_workspace_bytes(const bf_bank* bank, const int64_t* n, int32_t n_segs,
                                   const bf_search_params* params, size_t* bytes);

/* The search of bf_search_batch plus the kappa-sigma tails of every series, in one pass of
 * the contraction: before it, sigma_k is predicted from the series' own spectrum by
 * Parseval's theorem (Sec. 2.2: the mean square of template k's output is the sum over
 * frequency of |H_k|^2 times the power of the locally normalised series); the pass sums the
 * exact rho^2 per template and keeps every (tau, k) above 0.95 kappa times the prediction.
 * A check then selects the tails against the exact kappa * sigma_k; a series whose exact
 * threshold falls below the kept bound, or whose candidate lists overflow, gets a second
 * pass that extracts its tails directly.  Results are the same bit for bit as with two
 * passes (sums first, extraction second).  With an FFT bank of N < 8192 points the search,
 * the sums and the extraction are three passes of the FFT kernel.  kappa finite and >= 0;
 * sigma, bin_counts and n_tails are required.  segs is a host array. */
bf_status bf_search_tails(const bf_bank* bank, const bf_tail_segment* segs, int32_t n_segs,
                          float kappa, const bf_search_params* params, void* workspace,
                          size_t workspace_bytes, bf_stream stream);

/* ---- Two-detector coincidence (Fig. 6 caption: pseudo-spectra of simultaneous tails in
 * two detectors, counted with frequency pairs within a width) ----------------------------
 * Channels a and b are two simultaneous series of the same length (n_offsets = W offsets),
 * searched with one bank by bf_search_tails.  A tail (tau, k) of a is coincident when b has
 * a tail (tau', k') with |tau - tau'| <= dtau and |f0(k) - f0(k')| <= df (f0 = the
 * template's start frequency on the bank grid); likewise for b.  Outputs (device,
 * caller-owned): counts_a[B] and counts_b[B], the coincident tails of each channel per f0
 * bin, and n_pairs[1] (int64), the coincident pairs.  Only the listed tails count
 * (min(n_tails, capacity) of each list); entries outside the bank share or the offsets are
 * ignored.  dtau >= 0, df >= 0 (+inf allowed).  Asynchronous on stream. */
bf_status bf_coincidence_workspace_bytes(const bf_bank* bank, int64_t n_offsets,
                                         int64_t capacity_b, size_t* bytes);
bf_status bf_coincidence(const bf_bank* bank, const bf_tails* a, const bf_tails* b,
                         int64_t n_offsets, int32_t dtau, double df, uint32_t* counts_a,
                         uint32_t* counts_b, int64_t* n_pairs, void* workspace,
                         size_t workspace_bytes, bf_stream stream);

/* ---- Serving: continuous batching with a device-resident bank --------------------------
 * A server owns a worker thread, `ticks_in_flight` HIP streams and one device allocation of
 * hbm_budget_bytes from which each admitted request takes its buffers (samples, workspace,
 * outputs; bf_server_request_bytes).  bf_submit copies the samples to pinned host memory and
 * returns at once.  Requests are admitted in arrival order while fewer than max_slots hold
 * device memory and their buffers fit the budget; admitted requests are searched in ticks:
 * one batched search per tick over every admitted, not yet launched request, replaying a
 * HIP graph captured at creation (table upload + the five kernels) on a free stream.
 * Requests arriving while ticks run join the next tick, which overlaps the running ones on
 * the device.  A request's results are identical, bit for bit, alone or in any mix.
 * Thread-safe: any thread may submit, poll, fetch and cancel. */
typedef struct bf_server bf_server;

typedef struct {
  size_t hbm_budget_bytes;  /* device bytes for request buffers, >= 1 MiB */
  int32_t max_slots;        /* requests holding device memory at once, 1..1024 */
  int32_t ticks_in_flight;  /* concurrent ticks (streams), 1..4 */
  int32_t reserved;         /* must be 0 */
  int32_t reserved2;        /* must be 0 */
  bf_search_params params;  /* applied to every request */
} bf_server_desc;

typedef enum { BF_QUEUED = 0, BF_RUNNING = 1, BF_DONE = 2, BF_FAILED = 3, BF_CANCELLED = 4 }
    bf_request_state;

/* Creates a server for a bank (which must outlive it) on the current device; allocates the
 * budget and captures one graph per stream.  BF_ENOMEM if the budget cannot be allocated. */
bf_status bf_server_create(const bf_bank* bank, const bf_server_desc* desc, bf_server** out);

/* Device bytes a request of n samples takes from the budget. */
bf_status bf_server_request_bytes(const bf_server* server, int64_t n, size_t* bytes);

/* Queues a search of x_host (host, n float32 samples, copied before returning).  *ticket
 * identifies the request.  BF_EBUDGET if the request cannot fit the budget even alone,
 * BF_EINVAL if n < L. */
bf_status bf_submit(bf_server* server, const float* x_host, int64_t n, uint64_t* ticket);

/* State (bf_request_state) and times in seconds since the server's creation: submitted,
 * launched (0 while queued), finished (0 until done).  Any pointer may be NULL.
 * BF_ENOTFOUND for an unknown or already fetched ticket. */
bf_status bf_poll(bf_server* server, uint64_t ticket, int32_t* state, double* t_submit,
                  double* t_start, double* t_done);

/* Copies a finished request's outputs (host buffers sized as for bf_search_segment; any may
 * be NULL) and forgets the ticket.  BF_EAGAIN while queued or running (the ticket stays);
 * BF_ECANCELED for a cancelled request and BF_EHIP for a failed one (the ticket is
 * forgotten); BF_ENOTFOUND for an unknown ticket. */
bf_status bf_fetch(bf_server* server, uint64_t ticket, float* max_abs, int32_t* argmax,
                   float* spec, double* spectrum, uint32_t* hist, int64_t* n_degenerate);

/* Cancels a request: a queued one is dropped, an admitted or running one completes and its
 * result is discarded (its state becomes BF_CANCELLED).  BF_ENOTFOUND if unknown. */
bf_status bf_cancel(bf_server* server, uint64_t ticket);

/* Counters: requests done, ticks launched, correlations done, requests queued, requests
 * holding device memory.  Any pointer may be NULL. */
bf_status bf_server_stats(bf_server* server, int64_t* done, int64_t* ticks,
                          double* correlations, int32_t* queued, int32_t* on_device);

/* Drops queued requests, waits for running ticks, frees everything.  Unfetched results are
 * lost. */
bf_status bf_server_destroy(bf_server* server);

/* Work decomposition the searches would use for series of lengths n[0..n_segs-1] (host):
 * the bank sweep is split into *n_ranges contiguous ranges of whole f0 bins, and each
 * (series, block of offsets, range) is one work item of the contraction kernel. */
bf_status bf_plan(const bf_bank* bank, const int64_t* n, int32_t n_segs, int32_t* n_ranges,
                  int64_t* n_items);

/* Profiling aid.  With timing enabled, every search records HIP events on its stream
 * around each of its five kernels (clear, prefix sums, window norms, contraction,
 * finalise); the calling thread keeps the records of up to 256 searches.  bf_kernel_times
 * waits for those searches, writes the summed durations in milliseconds per kernel to
 * ms[0..4] (host) and their number to *n_searches (may be NULL), and forgets them.
 * BF_EAGAIN if no timed search ran on this thread since the last collection. */
bf_status bf_set_timing(int32_t enable);
bf_status bf_kernel_times(double* ms, int32_t* n_searches);

/* Message describing the last error on the calling thread ("" if none). */
const char* bf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BFLY_H */
