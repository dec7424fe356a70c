// Host runtime of libbfly.so: the C ABI declared in include/bfly.h.
//
// Validates arguments, builds banks, lays out workspaces, plans the work decomposition,
// stages the per-series table to the device and enqueues the kernels on the caller's
// stream.  No C++ exception crosses the ABI; errors are returned as bf_status with a
// thread-local message.
#include "bfly.h"
#include "bfly_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace bfly;

struct bf_bank {
  bf_bank_desc desc;
  GridDev grid;
  BankDev dev;
  int device;
};

namespace {

thread_local std::string g_err;

bf_status fail(bf_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

bf_status hip_fail(hipError_t e, const char* what) {
  return fail(BF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                     \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

bf_status check_desc(const bf_bank_desc* d) {
  if (!d) return fail(BF_EINVAL, "bank descriptor is NULL");
  if (!(d->fs > 0.0) || !std::isfinite(d->fs)) return fail(BF_EINVAL, "fs must be > 0");
  if (d->L < 1 || d->L > MAX_L) return fail(BF_EINVAL, "L must be in [1, %d]", MAX_L);
  if (d->n_f0 < 1 || d->n_fdot < 1) return fail(BF_EINVAL, "n_f0 and n_fdot must be >= 1");
  if (d->shard_count < 1 || d->shard_index < 0 || d->shard_index >= d->shard_count ||
      d->shard_count > d->n_f0)
    return fail(BF_EINVAL, "need 0 <= shard_index < shard_count <= n_f0");
  if (d->precision != BF_FP32 && d->precision != BF_BF16X3)
    return fail(BF_EINVAL, "precision %d is not available", d->precision);
  const double v[4] = {d->f0_min, d->f0_max, d->fdot_min, d->fdot_max};
  for (double x : v)
    if (!std::isfinite(x)) return fail(BF_EINVAL, "grid bounds must be finite");
  if (d->f0_max < d->f0_min || d->fdot_max < d->fdot_min)
    return fail(BF_EINVAL, "grid bounds must satisfy min <= max");
  const int64_t nb = (int64_t)(d->shard_index + 1) * d->n_f0 / d->shard_count -
                     (int64_t)d->shard_index * d->n_f0 / d->shard_count;
  if (nb * (int64_t)d->n_fdot > (int64_t)0x7FFFFFFF - 4096)
    return fail(BF_EINVAL, "too many templates");
  return BF_OK;
}

void fill_geometry(const bf_bank_desc* d, GridDev* g, BankDev* b) {
  const int64_t f0_lo = (int64_t)d->shard_index * d->n_f0 / d->shard_count;
  const int64_t f0_hi = (int64_t)(d->shard_index + 1) * d->n_f0 / d->shard_count;
  g->fs = d->fs;
  g->f0_min = d->f0_min;
  g->f0_max = d->f0_max;
  g->f0_step = d->n_f0 > 1 ? (d->f0_max - d->f0_min) / (double)(d->n_f0 - 1) : 0.0;
  g->fdot_min = d->fdot_min;
  g->fdot_max = d->fdot_max;
  g->fdot_step = d->n_fdot > 1 ? (d->fdot_max - d->fdot_min) / (double)(d->n_fdot - 1) : 0.0;
  g->n_f0 = d->n_f0;
  g->n_fdot = d->n_fdot;
  g->f0_lo = (int32_t)f0_lo;
  b->data = nullptr;
  b->n_bins = (int32_t)(f0_hi - f0_lo);
  b->n_fdot = d->n_fdot;
  b->K = (int64_t)b->n_bins * d->n_fdot;
  b->K_pad = round_up(b->K, TILE_K);
  b->k_offset = f0_lo * d->n_fdot;
  b->L = d->L;
  b->L_pad = (int32_t)round_up(d->L, 2 * KCH);
  b->n_chunks = b->L_pad / KCH;
  b->precision = d->precision;
}

size_t bank_data_bytes(const BankDev& b) { return (size_t)b.K_pad * (size_t)b.L_pad * 4; }

// The grid value numpy.linspace produces: i*step + start, the last point exactly stop.
double grid_value(double lo, double hi, double step, int n, int64_t i) {
  if (n > 1 && i == n - 1) return hi;
  return (double)i * step + lo;
}

bf_status check_device_ptr(const void* p, const char* name) {
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(BF_EINVAL, "%s is not a device pointer", name);
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return fail(BF_EINVAL, "%s is not device memory", name);
  return BF_OK;
}

// ---- pinned staging buffers for the per-series table ------------------------------------
struct Staging {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
  int device = -1;
  bool busy = false;
  bool recorded = false;
};
std::mutex g_stage_mu;
std::vector<Staging*> g_stage;

// Returns a pinned host buffer of at least `bytes` that no pending copy still reads.
Staging* acquire_staging(size_t bytes, int device, bf_status* st) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  for (Staging* s : g_stage) {
    if (s->busy || s->device != device || s->bytes < bytes) continue;
    if (s->recorded) {
      hipError_t q = hipEventQuery(s->ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
    }
    s->busy = true;
    return s;
  }
  Staging* s = new (std::nothrow) Staging();
  if (!s) {
    *st = fail(BF_ENOMEM, "host allocation failed");
    return nullptr;
  }
  s->bytes = std::max<size_t>(bytes, 64 * 1024);
  s->device = device;
  hipError_t e = hipHostMalloc(&s->host, s->bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete s;
    *st = hip_fail(e, "hipHostMalloc(staging)");
    return nullptr;
  }
  e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipHostFree(s->host);
    delete s;
    *st = hip_fail(e, "hipEventCreate");
    return nullptr;
  }
  s->busy = true;
  g_stage.push_back(s);
  return s;
}

void release_staging(Staging* s, bool recorded) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  s->recorded = recorded;
  s->busy = false;
}

// ---- optional per-kernel timing ---------------------------------------------------------
bool g_timing = false;
struct TimingEvents {
  hipEvent_t ev[6] = {};
  int device = -1;
  bool valid = false;
};
thread_local TimingEvents t_timing;

// ---- workspace layout ------------------------------------------------------------------
struct SegLayout {
  size_t pre, cnt, inv_norm, mkey, spec_acc;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Computes the byte offsets of every series' buffers; returns the total size.
size_t layout(const BankDev& b, const int64_t* n, int32_t n_segs, std::vector<SegLayout>* out) {
  size_t off = align256((size_t)n_segs * sizeof(SegDesc));
  if (out) out->resize((size_t)n_segs);
  for (int32_t i = 0; i < n_segs; ++i) {
    const int64_t W = n[i] - b.L + 1;
    SegLayout s;
    s.pre = off;
    off = align256(off + (size_t)(n[i] + 1) * 4 * sizeof(double));
    s.cnt = off;
    off = align256(off + (size_t)(n[i] + 1) * sizeof(int32_t));
    s.inv_norm = off;
    off = align256(off + (size_t)W * sizeof(double));
    s.mkey = off;
    off = align256(off + (size_t)W * sizeof(unsigned long long));
    s.spec_acc = off;
    off = align256(off + (size_t)b.n_bins * sizeof(unsigned long long));
    if (out) (*out)[(size_t)i] = s;
  }
  return off;
}

bf_status check_params(const bf_search_params* p) {
  if (!p) return fail(BF_EINVAL, "params is NULL");
  if (p->norm != BF_NORM_CENTRED && p->norm != BF_NORM_RAW)
    return fail(BF_EINVAL, "norm must be BF_NORM_CENTRED or BF_NORM_RAW");
  if (p->t_block < 1) return fail(BF_EINVAL, "t_block must be >= 1");
  if (p->hist_bins < 1 || p->hist_bins > MAX_HIST_BINS)
    return fail(BF_EINVAL, "hist_bins must be in [1, %d]", MAX_HIST_BINS);
  if (p->reserved != 0) return fail(BF_EINVAL, "reserved must be 0");
  if (!std::isfinite(p->hist_lo) || !std::isfinite(p->hist_hi) || !(p->hist_lo < p->hist_hi))
    return fail(BF_EINVAL, "need finite hist_lo < hist_hi");
  return BF_OK;
}

// Splits the bank sweep into bin ranges so that the work items fill the device in whole
// waves: estimated makespan = ceil(items / slots) * (tiles of the largest range), plus a
// small per-item cost (strip fill and flushes).
int32_t plan_ranges(const BankDev& b, int64_t total_tiles, int slots) {
  double best_cost = 1e300;
  int32_t best_r = 1;
  const int32_t rmax = std::min<int32_t>(b.n_bins, 4096);
  for (int32_t r = 1; r <= rmax; ++r) {
    const int64_t items = total_tiles * r;
    if (items > (int64_t)0x7FFFFFFF) break;
    int64_t max_tiles = 0;
    // the largest range (ranges differ by at most one bin)
    const int32_t bins = (b.n_bins + r - 1) / r;
    const int64_t k_span = (int64_t)bins * b.n_fdot;
    max_tiles = (k_span + TILE_K - 1) / TILE_K + 1;
    const int64_t waves = (items + slots - 1) / slots;
    const double cost = (double)waves * (double)max_tiles + 0.02 * (double)waves;
    if (cost < best_cost * 0.999) {
      best_cost = cost;
      best_r = r;
    }
    if (items > 64LL * slots) break;
  }
  return best_r;
}

int g_slots = 0;  // concurrent work-groups of the contraction kernel (one per CU)

bf_status device_slots(int* slots) {
  if (g_slots > 0) {
    *slots = g_slots;
    return BF_OK;
  }
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
          "hipDeviceGetAttribute");
  g_slots = cus > 0 ? cus : 1;
  *slots = g_slots;
  return BF_OK;
}

bf_status run_batch(const bf_bank* bank, const bf_segment* segs, int32_t n_segs,
                    const bf_search_params* prm, void* workspace, size_t ws_bytes,
                    hipStream_t stream) {
  if (!bank) return fail(BF_EINVAL, "bank is NULL");
  if (!segs || n_segs < 1) return fail(BF_EINVAL, "need at least one series");
  bf_status st = check_params(prm);
  if (st != BF_OK) return st;
  const BankDev& b = bank->dev;
  std::vector<int64_t> n((size_t)n_segs);
  for (int32_t i = 0; i < n_segs; ++i) {
    if (segs[i].n < b.L)
      return fail(BF_EINVAL, "series %d has %lld samples, fewer than L = %d", i,
                  (long long)segs[i].n, b.L);
    if (segs[i].n > ((int64_t)1 << 31) - N_WG - b.L_pad - STRIP_SLACK)
      return fail(BF_EINVAL, "series %d is too long", i);
    if (!segs[i].x) return fail(BF_EINVAL, "series %d: x is NULL", i);
    n[(size_t)i] = segs[i].n;
  }
  std::vector<SegLayout> lay;
  const size_t need = layout(b, n.data(), n_segs, &lay);
  if (!workspace) return fail(BF_EINVAL, "workspace is NULL");
  if (ws_bytes < need)
    return fail(BF_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  if (((uintptr_t)workspace & 255) != 0) return fail(BF_EINVAL, "workspace not 256-byte aligned");
  if ((st = check_device_ptr(workspace, "workspace")) != BF_OK) return st;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != bank->device) return fail(BF_EINVAL, "bank lives on device %d, current is %d",
                                       bank->device, dev);
  for (int32_t i = 0; i < n_segs; ++i) {
    if ((st = check_device_ptr(segs[i].x, "x")) != BF_OK) return st;
    const bf_result& o = segs[i].out;
    const void* outs[6] = {o.max_abs, o.argmax, o.spec, o.spectrum, o.hist, o.n_degenerate};
    for (const void* q : outs)
      if (q && (st = check_device_ptr(q, "output buffer")) != BF_OK) return st;
  }

  char* ws = (char*)workspace;
  SearchDev sp;
  sp.norm = prm->norm;
  sp.t_block = prm->t_block;
  sp.hist_bins = prm->hist_bins;
  sp.hist_lo = prm->hist_lo;
  sp.hist_hi = prm->hist_hi;
  sp.n_segs = n_segs;

  const size_t table_bytes = (size_t)n_segs * sizeof(SegDesc);
  Staging* stg = acquire_staging(table_bytes, dev, &st);
  if (!stg) return st;
  SegDesc* tab = (SegDesc*)stg->host;
  int64_t tiles = 0, max_W = 0, max_words = 0;
  for (int32_t i = 0; i < n_segs; ++i) {
    SegDesc& d = tab[i];
    const SegLayout& l = lay[(size_t)i];
    d.x = segs[i].x;
    d.n = segs[i].n;
    d.W = segs[i].n - b.L + 1;
    d.n_tiles = (d.W + N_WG - 1) / N_WG;
    d.tile0 = tiles;
    tiles += d.n_tiles;
    d.pre = (double*)(ws + l.pre);
    d.cnt = (int32_t*)(ws + l.cnt);
    d.inv_norm = (double*)(ws + l.inv_norm);
    d.mkey = (unsigned long long*)(ws + l.mkey);
    d.spec_acc = (unsigned long long*)(ws + l.spec_acc);
    d.max_abs = segs[i].out.max_abs;
    d.argmax = segs[i].out.argmax;
    d.spec = segs[i].out.spec;
    d.spectrum = segs[i].out.spectrum;
    d.hist = segs[i].out.hist;
    d.n_degenerate = segs[i].out.n_degenerate;
    d.spec_rows = (d.W + prm->t_block - 1) / prm->t_block;
    max_W = std::max(max_W, d.W);
    max_words = std::max(max_words, std::max(d.W, d.spec ? d.spec_rows * b.n_bins : 0));
  }
  sp.total_tiles = tiles;
  int slots = 0;
  if ((st = device_slots(&slots)) != BF_OK) {
    release_staging(stg, false);
    return st;
  }
  sp.n_ranges = plan_ranges(b, tiles, slots);

  SegDesc* tab_dev = (SegDesc*)ws;
  hipError_t e = hipMemcpyAsync(tab_dev, tab, table_bytes, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) {
    release_staging(stg, false);
    return hip_fail(e, "hipMemcpyAsync(series table)");
  }
  e = hipEventRecord(stg->ev, stream);
  release_staging(stg, e == hipSuccess);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");

  TimingEvents& te = t_timing;
  const bool timing = g_timing;
  if (timing && (te.device != dev || !te.ev[0])) {
    for (auto& ev : te.ev)
      if (ev) (void)hipEventDestroy(ev);
    for (auto& ev : te.ev) HIP_TRY(hipEventCreate(&ev), "hipEventCreate");
    te.device = dev;
  }
  te.valid = false;
  if (timing) HIP_TRY(hipEventRecord(te.ev[0], stream), "hipEventRecord");
  HIP_TRY(launch_zero(tab_dev, n_segs, max_words, b, sp, stream), "k_zero launch");
  if (timing) HIP_TRY(hipEventRecord(te.ev[1], stream), "hipEventRecord");
  HIP_TRY(launch_prefix(tab_dev, n_segs, b, sp, stream), "k_prefix launch");
  if (timing) HIP_TRY(hipEventRecord(te.ev[2], stream), "hipEventRecord");
  HIP_TRY(launch_norms(tab_dev, n_segs, max_W, b.L, sp.norm, stream), "k_norms launch");
  if (timing) HIP_TRY(hipEventRecord(te.ev[3], stream), "hipEventRecord");
  HIP_TRY(launch_main(tab_dev, b, sp, stream), "k_main launch");
  if (timing) HIP_TRY(hipEventRecord(te.ev[4], stream), "hipEventRecord");
  HIP_TRY(launch_finalize(tab_dev, n_segs, max_W, b, sp, stream), "k_finalize launch");
  if (timing) {
    HIP_TRY(hipEventRecord(te.ev[5], stream), "hipEventRecord");
    te.valid = true;
  }
  return BF_OK;
}

}  // namespace

// =======================================================================================
extern "C" {

bf_status bf_bank_bytes(const bf_bank_desc* desc, size_t* bytes) {
  try {
    bf_status st = check_desc(desc);
    if (st != BF_OK) return st;
    if (!bytes) return fail(BF_EINVAL, "bytes is NULL");
    GridDev g;
    BankDev b;
    fill_geometry(desc, &g, &b);
    *bytes = bank_data_bytes(b) + 256;
    return BF_OK;
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_bank_create(const bf_bank_desc* desc, void* dev_mem, size_t dev_bytes,
                         bf_stream stream, bf_bank** out) {
  try {
    bf_status st = check_desc(desc);
    if (st != BF_OK) return st;
    if (!out) return fail(BF_EINVAL, "out is NULL");
    *out = nullptr;
    GridDev g;
    BankDev b;
    fill_geometry(desc, &g, &b);
    const size_t need = bank_data_bytes(b) + 256;
    if (!dev_mem) return fail(BF_EINVAL, "dev_mem is NULL");
    if (dev_bytes < need) return fail(BF_EINVAL, "dev_mem too small: %zu < %zu", dev_bytes, need);
    if (((uintptr_t)dev_mem & 255) != 0) return fail(BF_EINVAL, "dev_mem not 256-byte aligned");
    if ((st = check_device_ptr(dev_mem, "dev_mem")) != BF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_bank_gen(g, b, dev_mem, s), "k_bank_gen launch");
    unsigned int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, (char*)dev_mem + bank_data_bytes(b), sizeof bad,
                           hipMemcpyDeviceToHost, s),
            "hipMemcpyAsync(bank check)");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize(bank)");
    if (bad) return fail(BF_EINVAL, "%u template(s) have a zero centred norm", bad);
    bf_bank* bk = new (std::nothrow) bf_bank();
    if (!bk) return fail(BF_ENOMEM, "host allocation failed");
    bk->desc = *desc;
    bk->grid = g;
    bk->dev = b;
    bk->dev.data = dev_mem;
    HIP_TRY(hipGetDevice(&bk->device), "hipGetDevice");
    *out = bk;
    return BF_OK;
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_bank_info(const bf_bank* bank, int64_t* K, int32_t* n_bins, int64_t* k_offset,
                       double* f0, double* fdot) {
  if (!bank) return fail(BF_EINVAL, "bank is NULL");
  if (K) *K = bank->dev.K;
  if (n_bins) *n_bins = bank->dev.n_bins;
  if (k_offset) *k_offset = bank->dev.k_offset;
  const GridDev& g = bank->grid;
  for (int64_t k = 0; k < bank->dev.K; ++k) {
    const int64_t ig = g.f0_lo + k / g.n_fdot;
    const int64_t j = k % g.n_fdot;
    if (f0) f0[k] = grid_value(g.f0_min, g.f0_max, g.f0_step, g.n_f0, ig);
    if (fdot) fdot[k] = grid_value(g.fdot_min, g.fdot_max, g.fdot_step, g.n_fdot, j);
  }
  return BF_OK;
}

bf_status bf_bank_destroy(bf_bank* bank) {
  delete bank;
  return BF_OK;
}

bf_status bf_workspace_bytes(const bf_bank* bank, const int64_t* n, int32_t n_segs,
                             const bf_search_params* params, size_t* bytes) {
  try {
    if (!bank) return fail(BF_EINVAL, "bank is NULL");
    if (!n || n_segs < 1) return fail(BF_EINVAL, "need at least one series length");
    if (!bytes) return fail(BF_EINVAL, "bytes is NULL");
    bf_status st = check_params(params);
    if (st != BF_OK) return st;
    for (int32_t i = 0; i < n_segs; ++i)
      if (n[i] < bank->dev.L)
        return fail(BF_EINVAL, "series %d has %lld samples, fewer than L = %d", i,
                    (long long)n[i], bank->dev.L);
    *bytes = layout(bank->dev, n, n_segs, nullptr);
    return BF_OK;
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_search_segment(const bf_bank* bank, const float* x, int64_t n,
                            const bf_search_params* params, const bf_result* out,
                            void* workspace, size_t workspace_bytes, bf_stream stream) {
  try {
    if (!out) return fail(BF_EINVAL, "out is NULL");
    bf_segment s;
    s.x = x;
    s.n = n;
    s.out = *out;
    return run_batch(bank, &s, 1, params, workspace, workspace_bytes, (hipStream_t)stream);
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_search_batch(const bf_bank* bank, const bf_segment* segs, int32_t n_segs,
                          const bf_search_params* params, void* workspace,
                          size_t workspace_bytes, bf_stream stream) {
  try {
    return run_batch(bank, segs, n_segs, params, workspace, workspace_bytes,
                     (hipStream_t)stream);
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_set_timing(int32_t enable) {
  g_timing = enable != 0;
  return BF_OK;
}

bf_status bf_kernel_times(double* ms) {
  if (!ms) return fail(BF_EINVAL, "ms is NULL");
  TimingEvents& te = t_timing;
  if (!te.valid) return fail(BF_EAGAIN, "no timed search on this thread");
  HIP_TRY(hipEventSynchronize(te.ev[5]), "hipEventSynchronize");
  for (int i = 0; i < 5; ++i) {
    float v = 0.0f;
    HIP_TRY(hipEventElapsedTime(&v, te.ev[i], te.ev[i + 1]), "hipEventElapsedTime");
    ms[i] = (double)v;
  }
  return BF_OK;
}

bf_status bf_plan(const bf_bank* bank, const int64_t* n, int32_t n_segs, int32_t* n_ranges,
                  int64_t* n_items) {
  if (!bank || !n || n_segs < 1) return fail(BF_EINVAL, "bad arguments");
  int64_t tiles = 0;
  for (int32_t i = 0; i < n_segs; ++i) {
    if (n[i] < bank->dev.L) return fail(BF_EINVAL, "series shorter than L");
    tiles += (n[i] - bank->dev.L + 1 + N_WG - 1) / N_WG;
  }
  int slots = 0;
  bf_status st = device_slots(&slots);
  if (st != BF_OK) return st;
  const int32_t r = plan_ranges(bank->dev, tiles, slots);
  if (n_ranges) *n_ranges = r;
  if (n_items) *n_items = tiles * r;
  return BF_OK;
}

const char* bf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
