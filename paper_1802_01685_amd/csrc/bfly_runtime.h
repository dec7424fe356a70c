// Host-side runtime pieces shared by the search entry points (bfly_api.cpp) and the server
// (bfly_server.cpp).  Not part of the public ABI.
#pragma once

#include "bfly.h"
#include "bfly_internal.h"

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

struct bf_bank {
  bf_bank_desc desc;
  bfly::GridDev grid;
  bfly::BankDev dev;
  int device;
};

namespace bfly {

bf_status set_error(bf_status code, const char* fmt, ...);
bf_status hip_error(hipError_t e, const char* what);

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Device buffers of one series: its samples, its workspace part, its outputs.
struct SeriesBufs {
  const float* x;
  int64_t n;
  double* pre;
  int32_t* cnt;
  double* inv_norm;
  unsigned long long* mkey;
  unsigned long long* spec_acc;
  bf_result out;
  // tail search only (else null): workspace sums, counts, thresholds, and the outputs
  unsigned long long* sig_acc = nullptr;
  unsigned long long* sig_part = nullptr;
  unsigned long long* n_ok = nullptr;
  float* thr = nullptr;
  const bf_tails* tails = nullptr;
  float2* xspec = nullptr;     // FFT form: data block spectra (workspace)
  // single-pass tail search (workspace; used when the search runs in one pass)
  float* thr_lo = nullptr;
  int32_t* c_tau = nullptr;
  int32_t* c_k = nullptr;
  float* c_rho = nullptr;
  unsigned long long* n_cand = nullptr;
  int64_t cand_cap = 0;
  uint32_t* redo = nullptr;
  float* zloc = nullptr;
  double* acf_part = nullptr;
  double* acf = nullptr;
  float* qspec = nullptr;
  bool onepass = false;        // this search extracts its tails in one pass
};

// Candidates a single-pass tail search keeps room for (per series of W offsets).
int64_t cand_capacity(const BankDev& b, int64_t W);

// Bytes of one series' workspace part (prefix sums, counts, norms, maxima, spectrum sums;
// with tails also the per-template rho^2 sums and thresholds).
size_t series_ws_bytes(const BankDev& b, int64_t n, bool tails = false);
// Assigns the workspace pointers of a series whose workspace part starts at base.
void series_ws_carve(const BankDev& b, int64_t n, char* base, SeriesBufs* s,
                     bool tails = false);
// Bytes of a batch table for n_segs series ([BatchHdr][SegDesc x n_segs], 256-aligned).
inline size_t table_bytes(int32_t n_segs) {
  return align256(sizeof(BatchHdr) + (size_t)n_segs * sizeof(SegDesc));
}

bf_status check_params(const bf_search_params* p);
SearchDev make_search(const BankDev& b, const bf_search_params* p, int mode = MODE_SEARCH,
                      float kappa = 0.0f);
bf_status device_slots(int* slots);
int32_t plan_ranges(const BankDev& b, int64_t total_tiles, int slots, int tm);
int32_t plan_fft_ranges(const BankDev& b, int64_t total_tiles, int slots);
// FFT form: overlap-save blocks of a series with W offsets.
inline int64_t fft_blocks(const BankDev& b, int64_t W) {
  const int64_t v = 2 * (int64_t)b.fft_m - b.L + 1;
  return (W + v - 1) / v;
}

// Fills a host batch table (hdr followed by the SegDescs) for the series s[0..n-1].
struct TableInfo {
  int64_t max_W = 0;
  int64_t max_words = 0;
  int64_t n_items = 0;
};
TableInfo fill_table(const BankDev& b, const SearchDev& sp, const SeriesBufs* s, int32_t n,
                     int slots, BatchHdr* hdr);

// The batch table of a single series, laid out as in the workspace ([BatchHdr][SegDesc]).
struct OneSeriesTable {
  BatchHdr hdr;
  SegDesc seg;
};
static_assert(offsetof(OneSeriesTable, seg) == sizeof(BatchHdr), "table layout");

// How a search's batch table reaches the device: copied from a pinned host staging buffer
// (any batch), or written by a one-work-group kernel that takes the table of a single series
// as its argument (no host or device allocation; bfly_noalloc.hip).
enum class TableUpload { Staging, Kernel };
hipError_t launch_put_table(const OneSeriesTable& t, OneSeriesTable* dst, hipStream_t s);

// Validates a batch, lays it out in the workspace (table first), uploads the table and
// enqueues the search (and, with tails, the tail passes) on stream.  With
// TableUpload::Kernel, n_segs must be 1, the workspace is not checked with the pointer
// query and no timing records are taken.
bf_status run_batch(const bf_bank* bank, const bf_segment* segs, int32_t n_segs,
                    const bf_search_params* prm, void* workspace, size_t ws_bytes,
                    hipStream_t stream, const bf_tails* tails, float kappa,
                    TableUpload upload);

// Per-kernel timing records (optional; see bf_set_timing).
struct TimingSet {
  hipEvent_t ev[6] = {};
  int device = -1;
};
TimingSet* timing_slot(int device, bf_status* st);

// Enqueues the five kernels of a search on `stream`, reading the batch table at table_dev.
// prepare_main(b, sp) must have been called once before (outside any stream capture).
bf_status enqueue_kernels(const BankDev& b, const SearchDev& sp, const BatchHdr* table_dev,
                          int32_t seg_slots, int32_t x_blocks, int64_t main_blocks,
                          hipStream_t stream, TimingSet* te);
// The tail search: the kernels above with the contraction in MODE_SIGMA, then k_sigma and
// the MODE_TAILS contraction (sp_sigma and sp_tails differ only in mode).
// The single-pass tail search: the predictor, one correlation pass that sums rho^2 and keeps
// candidates (sp_pass: MODE_SIGMA for k_main, MODE_ONEPASS for the FFT form), the exact
// thresholds, the check and the selection of the tails, and the tails pass for the series
// whose check failed (its work-groups return at once for the others).
bf_status enqueue_onepass_tail_kernels(const bf_bank* bank, const SearchDev& sp_pass,
                                       const SearchDev& sp_tails, const BatchHdr* table_dev,
                                       int32_t seg_slots, int32_t x_blocks, int64_t main_blocks,
                                       float margin, hipStream_t stream, TimingSet* te);
bf_status enqueue_tail_kernels(const BankDev& b, const SearchDev& sp_sigma,
                               const SearchDev& sp_tails, const BatchHdr* table_dev,
                               int32_t seg_slots, int32_t x_blocks, int64_t main_blocks,
                               hipStream_t stream, TimingSet* te);

}  // namespace bfly
