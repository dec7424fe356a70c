// Internal declarations shared by the host runtime (bfly_api.cpp) and the kernels
// (bfly_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bfly {

// ---- tile geometry of the contraction kernel -------------------------------------------
// A work-group of 4 waves owns 4 * 32 * tn consecutive offsets; each wave owns tn blocks
// of 32 offsets.  All four waves sweep the same templates, tm blocks of 32 per step, and
// the taps in chunks of KCH.  (tm, tn) is a compiled tile shape chosen per search.
constexpr int WAVE = 64;
constexpr int WG_WAVES = 4;
constexpr int WG_THREADS = WAVE * WG_WAVES;
constexpr int TILE_K = 64;                    // K_pad granule (largest template tile)
constexpr int MAX_N_WG = 32 * 8 * WG_WAVES;  // offsets per work item at tn = 8
constexpr int KCH = 16;                       // taps per chunk, FP32 and BF16 forms
constexpr int KCH_FP8 = 64;                   // taps per chunk, FP8 form
constexpr int KCH_F16F8 = 32;                 // taps per chunk, F16F8 form
constexpr int STRIP_SLACK = 16;               // extra strip samples past N_WG + L_pad
constexpr int MAX_L = 8192;
constexpr int MAX_FFT_L = 4096;              // FFT form: N = 2M <= 8192
constexpr int MAX_F16F8_L = 4224;            // F16F8, F16F6: 24-byte strip cells + 36 KB
                                             // fill 160 KB LDS
constexpr int MAX_HIST_BINS = 4096;
// Fixed-point units of the spectrum sums (per offset s <= 1) and of the rho^2 sums per
// template (rho^2 <= 1): 2^-31, so that a sum over the most offsets a series can have
// (< 2^31) stays below 2^63 and a u64 accumulator cannot wrap.
constexpr double SPEC_FIX_SCALE = 2147483648.0;     // 2^31
constexpr double SIGMA_FIX_SCALE = 2147483648.0;    // 2^31
// The FFT form's single pass marks a wave's rho^2 sum with bit 63 (the sums stay below 2^63)
// when one of its correlations is above the kept bound.
constexpr unsigned long long SIG_FLAG = 1ull << 63;
constexpr int64_t MAX_SERIES_SAMPLES = (int64_t)1 << 31;
static_assert((double)MAX_SERIES_SAMPLES * 1.001 * SPEC_FIX_SCALE < 9223372036854775808.0,
              "spectrum sums cannot wrap");
static_assert((double)MAX_SERIES_SAMPLES * 1.001 * SIGMA_FIX_SCALE < 9223372036854775808.0,
              "rho^2 sums cannot wrap");

enum Precision {
  P_FP32 = 0, P_BF16X3 = 1, P_FP8 = 2, P_F16X2 = 3, P_FFT = 4, P_F16F8 = 5, P_F16F6 = 6
};

// F16X2 and F16F8: templates are stored as fp16 (hi + lo) of h * 2^F16_TEMPLATE_EXP.
constexpr int F16_TEMPLATE_EXP = 10;

// F16F8: the e4m3 codes of the template residual are scaled by 2^(e_k + F8_LO_SHIFT), those
// of the data residual by 2^F8_XLO_EXP, and those of the fp16 strip samples by
// 2^-F8_XHI_SHIFT; with these the two correction products share one scale (see k_main).
constexpr int F8_LO_SHIFT = 11;
constexpr int F8_XLO_EXP = 5;
constexpr int F8_XHI_SHIFT = 6;

// F16F6: as F16F8 with e2m3 residual codes (max 7.5).  Template codes: the residual scaled by
// 2^(e_k + 11), the template by 2^e_k (e_k keeps max |h| * 2^e_k <= 7.5); strip codes: the
// fp16 samples scaled by 2^-11 (the strip scale keeps them <= 15360 = 7.5 * 2^11) and the data
// residual unscaled (|y - fp16(y)| <= 4).  Each lane half has its own MFMA scale pair.
constexpr int F6_LO_SHIFT = 11;
constexpr int F6_XHI_SHIFT = 11;
constexpr float F6_STRIP_LIM = 15360.0f;

// Taps per K-loop chunk; L_pad is a multiple of twice this.
constexpr int chunk_taps(int precision) {
  return precision == P_FP8 ? KCH_FP8 : (precision == P_F16F8 || precision == P_F16F6) ? KCH_F16F8 : KCH;
}
// The fp16 + low-precision residual forms (F16F8, F16F6).
constexpr bool is_f16r(int precision) { return precision == P_F16F8 || precision == P_F16F6; }
// Forms whose bank carries per-template exponents and template sums.
constexpr bool has_side_tables(int precision) {
  return precision == P_FP8 || is_f16r(precision);
}

// Per-series table entry, resident in the workspace (device).
struct SegDesc {
  const float* x;
  int64_t n;
  int64_t W;
  int64_t tile0;        // first global offset tile of this series
  int64_t n_tiles;      // ceil(W / n_wg)
  double* pre;          // [n+1][4] prefix sums: S1 (hi, lo), S2 (hi, lo)
  int32_t* cnt;         // [n+1] prefix count of non-finite samples
  double* inv_norm;     // [W] 1/sqrt(E), 0 for degenerate windows
  unsigned long long* mkey;      // [W] packed (|d| bits << 32 | ~k) running maxima
  unsigned long long* spec_acc;  // [n_bins] fixed-point spectrum sums
  float* max_abs;       // outputs (device, may be null)
  int32_t* argmax;
  float* spec;
  double* spectrum;
  uint32_t* hist;
  int64_t* n_degenerate;
  int64_t spec_rows;    // ceil(W / t_block)
  float2* xspec;        // FFT form: [n_tiles][M + 2] spectra of the data blocks
  // kappa-sigma tails (null unless the search extracts them)
  unsigned long long* sig_acc;   // [K_pad] fixed-point sums of rho^2 per template
  unsigned long long* sig_part;  // FFT form at N = 8192: [n_tiles][4][K_pad] the same sums
                                 // per block and wave (one plain store per wave and template,
                                 // no atomics; summed by k_sigma), bit 63 = SIG_FLAG
  unsigned long long* n_ok;      // [1] non-degenerate offsets
  float* thr;                    // [K_pad] kappa * sigma_k (+inf past K)
  float* sigma;                  // [K] output sigma_k
  int32_t* t_tau;                // [tail_cap] tail offsets
  int32_t* t_k;                  // [tail_cap] tail global template indices
  float* t_rho;                  // [tail_cap] tail rho (signed)
  uint32_t* t_bins;              // [n_bins] tails per f0 bin
  unsigned long long* n_tails;   // [1] tails found
  int64_t tail_cap;
  // single-pass tail search (null when the tails are extracted by a second pass): the
  // predicted lower thresholds, the candidates above them and the check of the prediction
  float* thr_lo;                 // [K_pad] kappa * margin * predicted sigma_k (+inf past K)
  int32_t* c_tau;                // [cand_cap] candidate offsets (FFT form: blocks)
  int32_t* c_k;                  // [cand_cap] candidate local template indices
  float* c_rho;                  // [cand_cap] candidate rho (signed; unused by the FFT form)
  unsigned long long* n_cand;    // [CAND_SHARDS] candidates found per shard
  int64_t cand_cap;              // CAND_SHARDS shards of cand_cap / CAND_SHARDS entries
  uint32_t* redo;                // [1] 1: the prediction did not hold, run the tails pass
  float* zloc;                   // [n] the locally normalised series
  double* acf_part;              // [ACF_CHUNKS][L] lag sums over chunks of the series
  double* acf;                   // [L + 1] lag sums, then the non-degenerate offset count
  float* qspec;                  // [pred_n / 2 + 1] their cosine transform
};
constexpr int ACF_CHUNKS = 16;
// Candidates are appended to one of CAND_SHARDS sub-lists (by work-group), each with its own
// counter: appends to one global counter from every work-group contend (device-scope atomics
// on one address serialise across the XCDs).
constexpr int CAND_SHARDS = 256;

// The level subtracted from every staged sample: the mean of the series over its finite
// samples, from its prefix sums, rounded to a multiple of q = 2^floor(log2 sigma), sigma the
// series' standard deviation.  A mean within about one sigma of zero gives 0, so data that the
// forms hold exactly (a run of zeros) stays exact, while a level far above the fluctuations is
// removed.  With zero-mean templates the correlation does not depend on a constant, under
// either normalisation (the window energy comes from the prefix sums of the series itself), so
// each form rounds the fluctuations, not the level.  0 for a series with no finite samples or
// no spread.
__device__ inline float series_offset(const SegDesc& sg) {
  const int64_t good = sg.n - (int64_t)sg.cnt[sg.n];
  if (good <= 0) return 0.0f;
  const double mean = (sg.pre[4 * sg.n] + sg.pre[4 * sg.n + 1]) / (double)good;
  const double var = (sg.pre[4 * sg.n + 2] + sg.pre[4 * sg.n + 3]) / (double)good - mean * mean;
  if (!(var > 0.0)) return 0.0f;
  int e;
  frexp(sqrt(var), &e);             // sigma in [2^(e-1), 2^e)
  const double q = ldexp(1.0, e - 1);
  return (float)(rint(mean / q) * q);
}

// Header of a batch table in device memory: the table is [BatchHdr][SegDesc x n_segs].  The
// kernels read the batch sizes from it, so one captured launch sequence (grids sized for the
// largest batch, the contraction kernel looping over its work items) serves any batch.
struct BatchHdr {
  int32_t n_segs;
  int32_t n_ranges;     // bin ranges the bank sweep is split into
  int64_t total_tiles;  // sum of n_tiles over the series
  int64_t n_items;      // total_tiles * n_ranges
  int64_t reserved[5];
};
static_assert(sizeof(BatchHdr) == 64, "BatchHdr layout");

__host__ __device__ inline const SegDesc* hdr_segs(const BatchHdr* h) {
  return reinterpret_cast<const SegDesc*>(h + 1);
}

// The bank as the kernels see it (passed by value).
struct BankDev {
  const void* data;     // tile layout, see bank_gen
  const int32_t* texp;  // FP8, F16F8: per-template power-of-two exponent e_k (codes hold
                        // h * 2^e_k)
  const float* tsum;    // FP8, F16F8: sum over taps of the rounded template (not exactly 0)
  int64_t K;            // local templates
  int64_t K_pad;        // multiple of TILE_K
  int64_t k_offset;     // global index of local template 0
  int32_t L;
  int32_t L_pad;        // multiple of KCH
  int32_t n_chunks;     // L_pad / chunk_taps(precision)
  int32_t n_fdot;       // templates per spectrogram bin
  int32_t n_bins;
  int32_t precision;
  int32_t fft_m;        // FFT form: complex FFT length M = N / 2 (N = real FFT length)
};

// Grid description for bank generation (float64).
struct GridDev {
  double fs, f0_min, f0_step, f0_max, fdot_min, fdot_step, fdot_max;
  int32_t n_f0, n_fdot, f0_lo;
};

struct SearchDev {
  int32_t norm;
  int32_t t_block;
  int32_t hist_bins;
  int32_t tm;           // 32-template blocks per template tile (1 or 2)
  int32_t tn;           // 32-offset blocks per wave (4 or 8)
  int32_t pipe;         // K-loop schedule: 0 blocked, 1 MFMA/load interleaved
  int32_t n_wg;         // offsets per work item = 4 * 32 * tn
  int32_t mode;         // contraction pass: MODE_SEARCH, MODE_SIGMA or MODE_TAILS
  float kappa;          // tails: search depth
  double hist_lo, hist_hi;
};

// Contraction passes: the search; the search that also sums rho^2 per template; the pass
// that extracts the tails above kappa * sigma_k (and does nothing else); the FFT form's
// single pass (search, rho^2 sums, and the (template, block) pairs holding a correlation
// above the kept bound).
enum MainMode { MODE_SEARCH = 0, MODE_SIGMA = 1, MODE_TAILS = 2, MODE_ONEPASS = 3 };

// Single-pass tail search: the fraction of the predicted sigma below which candidates are
// kept (the prediction is checked against the exact sigma after the pass).  Only the time
// depends on it: the exact sigma stayed within 0.989-1.08 of the prediction on the
// light-curve, strain and batch workloads, and a lower margin keeps (and, in the FFT form,
// transforms again) more: 3.1% of the (block, template) pairs at 0.9, 0.95% at 0.95.
constexpr float TAILS_MARGIN = 0.95f;

// Bytes of the quantised templates, of the per-template side tables, and of the whole bank
// allocation (templates, side tables, then a 256-byte status word).
inline size_t bank_data_bytes(const BankDev& b) {
  if (b.precision == P_FFT) return (size_t)b.K_pad * (size_t)(b.fft_m + 2) * 8;  // spectra
  if (b.precision == P_F16F6) return (size_t)b.K_pad * (size_t)b.L_pad / 2 * 7;  // 3.5 B/tap
  return (size_t)b.K_pad * (size_t)b.L_pad * (b.precision == P_FP8 ? 1 : 4);
}
// FP8 and F16F8 side tables after the codes: int32 exponent e_k [K_pad], then the float sum
// of the rounded template [K_pad].
inline size_t bank_exp_bytes(const BankDev& b) {
  return has_side_tables(b.precision) ? (((size_t)b.K_pad * 8 + 255) & ~(size_t)255) : 0;
}
inline size_t bank_total_bytes(const BankDev& b) {
  return bank_data_bytes(b) + bank_exp_bytes(b) + 256;
}

// ---- launchers (bfly_kernels.hip); each returns the launch's hipError_t ----------------
// Grid sizes: seg_slots = series the grids cover (>= hdr->n_segs), x_blocks = blocks per
// series of the grid-stride kernels, main_blocks = work-groups of the contraction kernel
// (each loops over items blockIdx.x, blockIdx.x + main_blocks, ... < hdr->n_items).
hipError_t launch_bank_gen(const GridDev& g, const BankDev& b, void* dst, hipStream_t s);
hipError_t launch_zero(const BatchHdr* hdr, int32_t seg_slots, int32_t x_blocks,
                       const BankDev& b, const SearchDev& p, hipStream_t s);
hipError_t launch_prefix(const BatchHdr* hdr, int32_t seg_slots, hipStream_t s);
hipError_t launch_norms(const BatchHdr* hdr, int32_t seg_slots, int32_t x_blocks, int L,
                        int norm, hipStream_t s);
hipError_t prepare_main(const BankDev& b, const SearchDev& p);
bool main_variant_exists(int precision, int tm, int tn, int pipe, int mode);
hipError_t launch_main(const BatchHdr* hdr, int64_t main_blocks, const BankDev& b,
                       const SearchDev& p, hipStream_t s);
hipError_t launch_finalize(const BatchHdr* hdr, int32_t seg_slots, int32_t x_blocks,
                           const BankDev& b, const SearchDev& p, hipStream_t s);
// sigma_k = sqrt(sum rho^2 / n_ok) and the tail thresholds kappa * sigma_k (MODE_SIGMA's sums
// and k_finalize's n_ok must be complete).
hipError_t launch_sigma(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                        const SearchDev& p, hipStream_t s);
size_t main_lds_bytes(int precision, int L_pad, int n_wg);

// FFT form (bfly_fft.hip): template spectra at bank creation; a search transforms its data
// blocks and runs the fused correlation/reduction kernel (persistent over hdr's items).
hipError_t launch_fft_bank(const GridDev& g, const BankDev& b, void* dst, hipStream_t s);
hipError_t launch_fft_search(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                             const SearchDev& p, hipStream_t s);
// The sigma or tails pass of a tail search (p.mode), after the search left the data spectra.
// Single-pass tail search (bfly_tails.hip, bfly_fft.hip).  The predictor: lag sums of each
// series' locally normalised samples (k_acf), their cosine transform on pred_n points
// (k_qspec), and per template kappa * margin * sqrt(sum_f |H_k(f)|^2 Q(f) / (n_ok pred_n))
// from the bank's spectra (FFT form) or from spectra made on the fly (direct forms).  After
// the pass that sums rho^2 and keeps candidates above those thresholds: k_tails_check flags
// a series whose exact thresholds fall below the predicted ones (or whose candidates
// overflowed), and k_tails_keep (direct forms) moves the candidates above the exact
// thresholds into the tail lists of every series not flagged, or launch_fft_pairs (FFT form)
// transforms its listed pairs again; the tails pass then runs only for flagged series.
int pred_points(const BankDev& b);
// The FFT form's search kernel has the single-pass mode (N = 8192, fewer than 2^16
// templates per f0 bin).  Its candidates are (block, template) pairs, not correlations: the
// pass flags them in its per-wave rho^2 sums, launch_fft_pair_list lists them per shard (c_tau
// holds the block and c_k the template, n_cand the count), and launch_fft_pairs extracts the
// tails of the listed pairs of every series whose check passed.
bool fft_onepass_available(const BankDev& b);
// Work-groups of the bank's contraction kernel that are resident on one CU (the grid of a
// persistent launch is the CU count times this).
int contraction_wgs_per_cu(const BankDev& b);
hipError_t launch_fft_pair_list(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                                hipStream_t s);
hipError_t launch_fft_pairs(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                            hipStream_t s);
hipError_t launch_acf(const BatchHdr* hdr, int32_t seg_slots, int L, hipStream_t s);
hipError_t launch_qspec(const BatchHdr* hdr, int32_t seg_slots, int L, int pred_n,
                        hipStream_t s);
hipError_t launch_pred(const BatchHdr* hdr, int32_t seg_slots, const GridDev& g,
                       const BankDev& b, float kappa, float margin, hipStream_t s);
hipError_t launch_tails_check(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                              hipStream_t s);
hipError_t launch_tails_keep(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                             hipStream_t s);
hipError_t launch_fft_pass(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                           const SearchDev& p, hipStream_t s);

// Two-detector coincidence (bfly_coinc.hip).  A channel's tail list (device) and its output
// counts per f0 bin; the workspace of the offset buckets of channel B.
struct CoincSide {
  const int32_t* tau;
  const int32_t* k;
  const int64_t* n_tails;
  int64_t capacity;
  uint32_t* counts;
};
struct CoincWork {
  uint32_t* start;     // [W + 1] first bucket slot per offset
  uint32_t* cursor;    // [W] scatter cursors
  uint32_t* order;     // [capacity_b] B tail indices by offset
  uint32_t* flag_b;    // [capacity_b] B tail has a partner
  unsigned long long* n_pairs;
};
hipError_t launch_coincidence(const CoincSide& a, const CoincSide& b, const CoincWork& w,
                              const GridDev& g, int32_t n_bins, int32_t n_fdot, int64_t W,
                              int32_t dtau, double df, hipStream_t s);

}  // namespace bfly
