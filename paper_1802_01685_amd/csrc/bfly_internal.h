// Internal declarations shared by the host runtime (bfly_api.cpp) and the kernels
// (bfly_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bfly {

// ---- tile geometry of the contraction kernel -------------------------------------------
// A work-group of 4 waves owns N_WG consecutive offsets; each wave owns TN blocks of 32
// offsets.  All four waves sweep the same templates, TM blocks of 32 per step, and the
// taps in chunks of KCH.
constexpr int WAVE = 64;
constexpr int WG_WAVES = 4;
constexpr int WG_THREADS = WAVE * WG_WAVES;
constexpr int TM = 2;                         // 32-template blocks per template tile
constexpr int TILE_K = 32 * TM;               // templates per template tile
constexpr int TN = 4;                         // 32-offset blocks per wave
constexpr int N_WAVE = 32 * TN;               // offsets per wave
constexpr int N_WG = N_WAVE * WG_WAVES;       // offsets per work item
constexpr int KCH = 16;                       // taps per chunk (L_pad is a multiple of 2*KCH)
constexpr int STRIP_SLACK = 16;               // extra strip samples past N_WG + L_pad
constexpr int MAX_L = 8192;
constexpr int MAX_HIST_BINS = 4096;
constexpr double SPEC_FIX_SCALE = 1099511627776.0;  // 2^40: fixed-point spectrum sums

enum Precision { P_FP32 = 0, P_BF16X3 = 1, P_FP8 = 2 };

// Per-series table entry, resident in the workspace (device).
struct SegDesc {
  const float* x;
  int64_t n;
  int64_t W;
  int64_t tile0;        // first global offset tile of this series
  int64_t n_tiles;      // ceil(W / N_WG)
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
};

// The bank as the kernels see it (passed by value).
struct BankDev {
  const void* data;     // tile layout, see bank_gen
  int64_t K;            // local templates
  int64_t K_pad;        // multiple of TILE_K
  int64_t k_offset;     // global index of local template 0
  int32_t L;
  int32_t L_pad;        // multiple of KCH
  int32_t n_chunks;     // L_pad / KCH
  int32_t n_fdot;       // templates per spectrogram bin
  int32_t n_bins;
  int32_t precision;
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
  int32_t n_ranges;     // bin ranges the bank sweep is split into
  double hist_lo, hist_hi;
  int64_t total_tiles;  // sum of n_tiles over the series
  int32_t n_segs;
};

// ---- launchers (bfly_kernels.hip); each returns the launch's hipError_t ----------------
hipError_t launch_bank_gen(const GridDev& g, const BankDev& b, void* dst, hipStream_t s);
hipError_t launch_zero(const SegDesc* segs_dev, int32_t n_segs, int64_t max_words,
                       const BankDev& b, const SearchDev& p, hipStream_t s);
hipError_t launch_prefix(const SegDesc* segs_dev, int32_t n_segs, const BankDev& b,
                         const SearchDev& p, hipStream_t s);
hipError_t launch_norms(const SegDesc* segs_dev, int32_t n_segs, int64_t max_W, int L,
                        int norm, hipStream_t s);
hipError_t launch_main(const SegDesc* segs_dev, const BankDev& b, const SearchDev& p,
                       hipStream_t s);
hipError_t launch_finalize(const SegDesc* segs_dev, int32_t n_segs, int64_t max_W,
                           const BankDev& b, const SearchDev& p, hipStream_t s);
size_t main_lds_bytes(int precision, int L_pad);

}  // namespace bfly
