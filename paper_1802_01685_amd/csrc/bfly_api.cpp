// Host runtime of libbfly.so: the C ABI declared in include/bfly.h.
//
// Validates arguments, builds banks, lays out workspaces, plans the work decomposition,
// stages the per-series table to the device and enqueues the kernels on the caller's
// stream.  No C++ exception crosses the ABI; errors are returned as bf_status with a
// thread-local message.
#include "bfly.h"
#include "bfly_internal.h"
#include "bfly_runtime.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace bfly;

namespace {
thread_local std::string g_err;
}  // namespace

namespace bfly {

bf_status set_error(bf_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

bf_status hip_error(hipError_t e, const char* what) {
  return set_error(BF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace bfly

namespace {

#define fail ::bfly::set_error
#define hip_fail ::bfly::hip_error

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
  if (d->precision != BF_FP32 && d->precision != BF_BF16X3 && d->precision != BF_FP8 &&
      d->precision != BF_F16X2 && d->precision != BF_FFT && d->precision != BF_F16F8 &&
      d->precision != BF_F16F6)
    return fail(BF_EINVAL, "precision %d is not available", d->precision);
  if (d->precision == BF_FFT && d->L > MAX_FFT_L)
    return fail(BF_EINVAL, "the FFT form needs L <= %d", MAX_FFT_L);
  if ((d->precision == BF_F16F8 || d->precision == BF_F16F6) && d->L > MAX_F16F8_L)
    return fail(BF_EINVAL, "the F16F8 and F16F6 forms need L <= %d", MAX_F16F8_L);
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
  b->texp = nullptr;
  b->tsum = nullptr;
  b->L_pad = (int32_t)round_up(d->L, 2 * chunk_taps(d->precision));
  b->n_chunks = b->L_pad / chunk_taps(d->precision);
  b->precision = d->precision;
  b->fft_m = 0;
  if (d->precision == BF_FFT) {
    // real FFT length N = 2M = 8192 for every L (<= 4096): its kernel (k_fft4k) runs at 1.5
    // to 2.6 times the flop rate of the general one (k_fft_main at N = 4096 and 2048), which
    // outweighs the up to 8% less transform work per valid output, M log2 M / (2M - L + 1),
    // that a shorter transform has for short templates.  BF_FFT_POINTS = 1024, 2048 or 4096
    // selects a shorter transform on the general kernel (a comparison knob, read at each
    // bank description; ignored where 2M - L + 1 < 1).
    b->fft_m = 4096;
    const char* e = getenv("BF_FFT_POINTS");
    if (e && *e) {
      const long v = strtol(e, nullptr, 10);
      if ((v == 1024 || v == 2048 || v == 4096) && v - d->L + 1 >= 1) b->fft_m = (int32_t)(v / 2);
    }
  }
}

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

int g_slots = 0;  // concurrent work-groups of the contraction kernel (one per CU)

// Environment knobs, read at every call (so a test can switch them between calls).
bool env_flag(const char* name) {
  const char* e = getenv(name);
  return e && e[0] == '1';
}
int64_t env_int(const char* name, int64_t dflt) {
  const char* e = getenv(name);
  if (!e || !*e) return dflt;
  char* end = nullptr;
  const long long v = strtoll(e, &end, 10);
  return (end && *end == 0) ? (int64_t)v : dflt;
}
double env_double(const char* name, double dflt) {
  const char* e = getenv(name);
  if (!e || !*e) return dflt;
  char* end = nullptr;
  const double v = strtod(e, &end);
  return (end && *end == 0 && std::isfinite(v) && v > 0.0) ? v : dflt;
}

// Tile shape of the contraction kernel: tm template blocks x tn offset blocks (of 32) per
// wave, and the K-loop schedule.  BF_TILE=<tm>x<tn>[i|p] (e.g. "2x8i"; i = interleaved,
// p = pair streaming) overrides the default -- a tuning knob for experiments; FP32 and BF16 results do not
// depend on it (FP8 does, through its per-strip scales).
void choose_tile(int precision, int mode, int32_t* tm, int32_t* tn, int32_t* pipe) {
  // Defaults from measurement on MI355X: the split forms are fastest with 2 x 8 blocks and
  // the interleaved schedule; FP32 (64-cycle MFMAs) and FP8 with 2 x 4.
  // F16F8 and F16F6 have one shape, 2 x 8 with their pair-streaming schedule.
  const bool split = precision == BF_BF16X3 || precision == BF_F16X2;
  const bool f16r = precision == BF_F16F8 || precision == BF_F16F6;
  *tm = 2;
  *tn = split || f16r ? 8 : 4;
  *pipe = split ? 1 : f16r ? 2 : 0;
  const char* e = getenv("BF_TILE");
  int a = 0, c = 0;
  char il = 0;
  if (e && sscanf(e, "%dx%d%c", &a, &c, &il) >= 2) {
    const int pp = il == 'i' ? 1 : il == 'p' ? 2 : 0;
    if (main_variant_exists(precision, a, c, pp, mode)) {
      *tm = a;
      *tn = c;
      *pipe = pp;
    }
  }
}

// Per-thread pool of timing records, collected by bf_kernel_times.  The events live until
// the process ends: destroying them from a thread-exit destructor could run after the HIP
// runtime has shut down.
bool g_timing = false;
constexpr int MAX_TIMED = 256;
struct TimingLog {
  std::vector<TimingSet> sets;
  int used = 0;
};
thread_local TimingLog t_timing;

}  // namespace

namespace bfly {

// tails: per-series tail outputs for a tail search (else null), with its kappa.
// upload: how the batch table reaches the workspace (see TableUpload).
bf_status run_batch(const bf_bank* bank, const bf_segment* segs, int32_t n_segs,
                    const bf_search_params* prm, void* workspace, size_t ws_bytes,
                    hipStream_t stream, const bf_tails* tails, float kappa,
                    TableUpload upload) {
  if (!bank) return fail(BF_EINVAL, "bank is NULL");
  if (!segs || n_segs < 1) return fail(BF_EINVAL, "need at least one series");
  bf_status st = check_params(prm);
  if (st != BF_OK) return st;
  const BankDev& b = bank->dev;
  for (int32_t i = 0; i < n_segs; ++i) {
    if (segs[i].n < b.L)
      return fail(BF_EINVAL, "series %d has %lld samples, fewer than L = %d", i,
                  (long long)segs[i].n, b.L);
    if (segs[i].n > MAX_SERIES_SAMPLES - MAX_N_WG - b.L_pad - STRIP_SLACK)
      return fail(BF_EINVAL, "series %d is too long", i);
    if (!segs[i].x) return fail(BF_EINVAL, "series %d: x is NULL", i);
  }
  const bool with_tails = tails != nullptr;
  if (with_tails && !(kappa >= 0.0f && std::isfinite(kappa)))
    return fail(BF_EINVAL, "kappa must be finite and >= 0");
  size_t need = table_bytes(n_segs);
  for (int32_t i = 0; i < n_segs; ++i) need += series_ws_bytes(b, segs[i].n, with_tails);
  if (!workspace) return fail(BF_EINVAL, "workspace is NULL");
  if (ws_bytes < need)
    return fail(BF_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  if (((uintptr_t)workspace & 255) != 0) return fail(BF_EINVAL, "workspace not 256-byte aligned");
  if (upload == TableUpload::Kernel && n_segs != 1)
    return fail(BF_EINVAL, "the kernel-written table holds one series");
  if (upload == TableUpload::Staging &&
      (st = check_device_ptr(workspace, "workspace")) != BF_OK)
    return st;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != bank->device)
    return fail(BF_EINVAL, "bank lives on device %d, current is %d", bank->device, dev);
  for (int32_t i = 0; i < n_segs; ++i) {
    if ((st = check_device_ptr(segs[i].x, "x")) != BF_OK) return st;
    const bf_result& o = segs[i].out;
    const void* outs[6] = {o.max_abs, o.argmax, o.spec, o.spectrum, o.hist, o.n_degenerate};
    for (const void* q : outs)
      if (q && (st = check_device_ptr(q, "output buffer")) != BF_OK) return st;
    if (with_tails) {
      const bf_tails& t = tails[i];
      if (!t.sigma || !t.n_tails || !t.bin_counts)
        return fail(BF_EINVAL, "series %d: tails need sigma, bin_counts and n_tails", i);
      if (t.capacity < 0) return fail(BF_EINVAL, "series %d: negative tail capacity", i);
      if (t.capacity > 0 && (!t.tau || !t.k || !t.rho))
        return fail(BF_EINVAL, "series %d: tail lists are NULL with capacity > 0", i);
      const void* touts[6] = {t.sigma, t.n_tails, t.bin_counts, t.tau, t.k, t.rho};
      for (const void* q : touts)
        if (q && (st = check_device_ptr(q, "tail buffer")) != BF_OK) return st;
    }
  }

  // A tail search runs in one pass unless BF_TAILS_TWO_PASS=1 (a comparison knob; the
  // results are the same bit for bit) or the FFT form's kernel lacks the single-pass mode
  // (N < 8192).  In two passes the FFT form's search pass is a plain search and its sigma
  // pass comes after.
  const bool onepass = with_tails && !env_flag("BF_TAILS_TWO_PASS") &&
                       (b.precision != P_FFT || fft_onepass_available(b));
  const int pass_mode = !with_tails ? MODE_SEARCH
                        : b.precision == P_FFT ? (onepass ? MODE_ONEPASS : MODE_SEARCH)
                                               : MODE_SIGMA;
  const SearchDev sp = make_search(b, prm, pass_mode, kappa);
  SeriesBufs one;                 // a single series needs no host allocation
  std::vector<SeriesBufs> many;
  if (n_segs > 1) many.resize((size_t)n_segs);
  SeriesBufs* sb = n_segs > 1 ? many.data() : &one;
  char* ws = (char*)workspace;
  size_t off = table_bytes(n_segs);
  for (int32_t i = 0; i < n_segs; ++i) {
    SeriesBufs& q = sb[i];
    series_ws_carve(b, segs[i].n, ws + off, &q, with_tails);
    off += series_ws_bytes(b, segs[i].n, with_tails);
    q.x = segs[i].x;
    q.n = segs[i].n;
    q.out = segs[i].out;
    if (with_tails) q.tails = &tails[i];
    q.onepass = onepass;
    if (onepass) {
      // BF_TAILS_CAND_CAP lowers the candidate room (a knob that forces the checked path)
      const int64_t cap = env_int("BF_TAILS_CAND_CAP", q.cand_cap);
      if (cap >= 0 && cap < q.cand_cap) q.cand_cap = cap;
    }
  }
  int slots = 0;
  if ((st = device_slots(&slots)) != BF_OK) return st;

  BatchHdr* tab_dev = (BatchHdr*)ws;
  TableInfo ti;
  if (upload == TableUpload::Kernel) {
    OneSeriesTable tab;
    ti = fill_table(b, sp, sb, 1, slots, &tab.hdr);
    HIP_TRY(launch_put_table(tab, (OneSeriesTable*)tab_dev, stream), "k_put_table launch");
  } else {
    Staging* stg = acquire_staging(table_bytes(n_segs), dev, &st);
    if (!stg) return st;
    BatchHdr* hdr = (BatchHdr*)stg->host;
    ti = fill_table(b, sp, sb, n_segs, slots, hdr);
    hipError_t e =
        hipMemcpyAsync(tab_dev, hdr, table_bytes(n_segs), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
      release_staging(stg, false);
      return hip_fail(e, "hipMemcpyAsync(series table)");
    }
    e = hipEventRecord(stg->ev, stream);
    release_staging(stg, e == hipSuccess);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }

  if (b.precision != P_FFT) HIP_TRY(prepare_main(b, sp), "hipFuncSetAttribute(k_main)");
  // the kernel-written table is the no-allocation path: no timing records (they create events)
  TimingSet* te = nullptr;
  if (g_timing && upload == TableUpload::Staging && (te = timing_slot(dev, &st)) == nullptr)
    return st;
  const int32_t xb =
      (int32_t)std::min<int64_t>(std::max<int64_t>((ti.max_words + 255) / 256, 1), 2048);
  if (!with_tails) return enqueue_kernels(b, sp, tab_dev, n_segs, xb, ti.n_items, stream, te);
  SearchDev sp_t = sp;
  sp_t.mode = MODE_TAILS;
  if (b.precision != P_FFT) HIP_TRY(prepare_main(b, sp_t), "hipFuncSetAttribute(k_main)");
  if (onepass) {
    // BF_TAILS_MARGIN overrides the predicted-threshold margin (a knob; above 1 it makes the
    // check fail, which exercises the fallback)
    const float margin = (float)env_double("BF_TAILS_MARGIN", TAILS_MARGIN);
    return enqueue_onepass_tail_kernels(bank, sp, sp_t, tab_dev, n_segs, xb, ti.n_items,
                                        margin, stream, te);
  }
  return enqueue_tail_kernels(b, sp, sp_t, tab_dev, n_segs, xb, ti.n_items, stream, te);
}

size_t series_ws_bytes(const BankDev& b, int64_t n, bool tails) {
  const int64_t W = n - b.L + 1;
  size_t off = 0;
  off = align256(off + (size_t)(n + 1) * 4 * sizeof(double));
  off = align256(off + (size_t)(n + 1) * sizeof(int32_t));
  off = align256(off + (size_t)W * sizeof(double));
  off = align256(off + (size_t)W * sizeof(unsigned long long));
  off = align256(off + (size_t)b.n_bins * sizeof(unsigned long long));
  if (tails) {
    off = align256(off + (size_t)b.K_pad * sizeof(unsigned long long));
    off = align256(off + sizeof(unsigned long long));
    off = align256(off + (size_t)b.K_pad * sizeof(float));
    // single-pass area: thr_lo, n_cand + redo, candidates, zloc, lag sums, Q
    const size_t cap = (size_t)cand_capacity(b, W);
    off = align256(off + (size_t)b.K_pad * sizeof(float));
    off = align256(off + (CAND_SHARDS + 1) * sizeof(unsigned long long));
    off = align256(off + cap * 4);
    off = align256(off + cap * 4);
    off = align256(off + cap * 4);
    off = align256(off + (size_t)n * sizeof(float));
    off = align256(off + (size_t)ACF_CHUNKS * b.L * sizeof(double));
    off = align256(off + (size_t)(b.L + 1) * sizeof(double));
    off = align256(off + (size_t)(pred_points(b) / 2 + 1) * sizeof(float));
    if (b.precision == P_FFT && b.fft_m == 4096)
      off = align256(off + (size_t)fft_blocks(b, W) * 4 * b.K_pad * sizeof(unsigned long long));
  }
  if (b.precision == P_FFT) off = align256(off + fft_blocks(b, W) * (size_t)(b.fft_m + 2) * 8);
  return off;
}

int64_t cand_capacity(const BankDev& b, int64_t W) {
  const int64_t c = b.K_pad * W / 16384;
  return c < 65536 ? 65536 : (c > ((int64_t)1 << 24) ? ((int64_t)1 << 24) : c);
}

void series_ws_carve(const BankDev& b, int64_t n, char* base, SeriesBufs* s, bool tails) {
  const int64_t W = n - b.L + 1;
  size_t off = 0;
  s->pre = (double*)(base + off);
  off = align256(off + (size_t)(n + 1) * 4 * sizeof(double));
  s->cnt = (int32_t*)(base + off);
  off = align256(off + (size_t)(n + 1) * sizeof(int32_t));
  s->inv_norm = (double*)(base + off);
  off = align256(off + (size_t)W * sizeof(double));
  s->mkey = (unsigned long long*)(base + off);
  off = align256(off + (size_t)W * sizeof(unsigned long long));
  s->spec_acc = (unsigned long long*)(base + off);
  off = align256(off + (size_t)b.n_bins * sizeof(unsigned long long));
  if (tails) {
    s->sig_acc = (unsigned long long*)(base + off);
    off = align256(off + (size_t)b.K_pad * sizeof(unsigned long long));
    s->n_ok = (unsigned long long*)(base + off);
    off = align256(off + sizeof(unsigned long long));
    s->thr = (float*)(base + off);
    off = align256(off + (size_t)b.K_pad * sizeof(float));
    const int64_t cap = cand_capacity(b, W);
    s->thr_lo = (float*)(base + off);
    off = align256(off + (size_t)b.K_pad * sizeof(float));
    s->n_cand = (unsigned long long*)(base + off);
    s->redo = (uint32_t*)(base + off + CAND_SHARDS * sizeof(unsigned long long));
    off = align256(off + (CAND_SHARDS + 1) * sizeof(unsigned long long));
    s->c_tau = (int32_t*)(base + off);
    off = align256(off + (size_t)cap * 4);
    s->c_k = (int32_t*)(base + off);
    off = align256(off + (size_t)cap * 4);
    s->c_rho = (float*)(base + off);
    off = align256(off + (size_t)cap * 4);
    s->cand_cap = cap;
    s->zloc = (float*)(base + off);
    off = align256(off + (size_t)n * sizeof(float));
    s->acf_part = (double*)(base + off);
    off = align256(off + (size_t)ACF_CHUNKS * b.L * sizeof(double));
    s->acf = (double*)(base + off);
    off = align256(off + (size_t)(b.L + 1) * sizeof(double));
    s->qspec = (float*)(base + off);
    off = align256(off + (size_t)(pred_points(b) / 2 + 1) * sizeof(float));
    s->sig_part = nullptr;
    if (b.precision == P_FFT && b.fft_m == 4096) {
      s->sig_part = (unsigned long long*)(base + off);
      off = align256(off + (size_t)fft_blocks(b, W) * 4 * b.K_pad * sizeof(unsigned long long));
    }
  }
  s->xspec = nullptr;
  if (b.precision == P_FFT) s->xspec = (float2*)(base + off);
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

SearchDev make_search(const BankDev& b, const bf_search_params* prm, int mode, float kappa) {
  SearchDev sp;
  sp.mode = mode;
  sp.kappa = kappa;
  sp.norm = prm->norm;
  sp.t_block = prm->t_block;
  sp.hist_bins = prm->hist_bins;
  sp.hist_lo = prm->hist_lo;
  sp.hist_hi = prm->hist_hi;
  choose_tile(b.precision, mode, &sp.tm, &sp.tn, &sp.pipe);
  sp.n_wg = 32 * sp.tn * WG_WAVES;
  if (b.precision == P_FFT) {
    sp.tm = sp.tn = sp.pipe = 0;
    sp.n_wg = 2 * b.fft_m - b.L + 1;   // valid outputs per overlap-save block
  }
  return sp;
}

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

// Splits the bank sweep into bin ranges so that the work items fill the device in whole
// waves: estimated makespan = ceil(items / slots) * (tiles of the largest range), plus a
// small per-item cost (strip fill and flushes).  With at least 8 bins the count is a
// multiple of 8, so that each XCD sweeps its own ranges (see the item order in k_main).
// FFT form: items = blocks x ranges of whole f0 bins; two work-groups fit a CU.  Minimises
// waves x (bins per range), preferring fewer ranges (each item transforms its block once).
int32_t plan_fft_ranges(const BankDev& b, int64_t total_tiles, int slots) {
  double best_cost = 1e300;
  int32_t best_r = 1;
  const int64_t conc = 2 * (int64_t)slots;
  if (b.fft_m == 4096 && b.n_bins >= 8) {
    // The N = 8192 kernel (two work-groups per CU) deals each XCD whole ranges when their
    // count is a multiple of 8: cost = the XCD's rounds of items x bins per range.
    const int64_t per_xcd = conc / 8;
    for (int32_t r = 8; r <= b.n_bins; r += 8) {
      const int64_t items = total_tiles * r;
      if (items > (int64_t)0x7FFFFFFF) break;
      const int64_t rounds = (total_tiles * (r / 8) + per_xcd - 1) / per_xcd;
      const double cost = (double)rounds * (double)((b.n_bins + r - 1) / r) + 0.01 * (double)rounds;
      if (cost < best_cost * 0.999) {
        best_cost = cost;
        best_r = r;
      }
      if (items > 16 * conc) break;
    }
    return best_r;
  }
  for (int32_t r = 1; r <= b.n_bins; ++r) {
    const int64_t items = total_tiles * r;
    if (items > (int64_t)0x7FFFFFFF) break;
    const int64_t waves = (items + conc - 1) / conc;
    const double cost = (double)waves * (double)((b.n_bins + r - 1) / r) + 0.01 * (double)waves;
    if (cost < best_cost * 0.999) {
      best_cost = cost;
      best_r = r;
    }
    if (items > 16 * conc) break;
  }
  return best_r;
}

constexpr int XCDS = 8;
int32_t plan_ranges(const BankDev& b, int64_t total_tiles, int slots, int tm) {
  double best_cost = 1e300;
  int32_t best_r = 1;
  const int32_t rmax = std::min<int32_t>(b.n_bins, 4096);
  const int32_t step = b.n_bins >= XCDS ? XCDS : 1;
  for (int32_t r = step; r <= rmax; r += step) {
    const int64_t items = total_tiles * r;
    if (items > (int64_t)0x7FFFFFFF) break;
    // the largest range (ranges differ by at most one bin)
    const int32_t bins = (b.n_bins + r - 1) / r;
    const int64_t k_span = (int64_t)bins * b.n_fdot;
    const int64_t max_tiles = (k_span + 32 * tm - 1) / (32 * tm) + 1;
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

TableInfo fill_table(const BankDev& b, const SearchDev& sp, const SeriesBufs* s, int32_t n,
                     int slots, BatchHdr* hdr) {
  TableInfo ti;
  SegDesc* tab = (SegDesc*)(hdr + 1);
  int64_t tiles = 0;
  for (int32_t i = 0; i < n; ++i) {
    SegDesc& d = tab[i];
    d.x = s[i].x;
    d.n = s[i].n;
    d.W = s[i].n - b.L + 1;
    d.n_tiles = (d.W + sp.n_wg - 1) / sp.n_wg;
    d.tile0 = tiles;
    tiles += d.n_tiles;
    d.pre = s[i].pre;
    d.cnt = s[i].cnt;
    d.inv_norm = s[i].inv_norm;
    d.mkey = s[i].mkey;
    d.spec_acc = s[i].spec_acc;
    d.max_abs = s[i].out.max_abs;
    d.argmax = s[i].out.argmax;
    d.spec = s[i].out.spec;
    d.spectrum = s[i].out.spectrum;
    d.hist = s[i].out.hist;
    d.n_degenerate = s[i].out.n_degenerate;
    d.spec_rows = (d.W + sp.t_block - 1) / sp.t_block;
    d.xspec = s[i].xspec;
    const bf_tails* t = s[i].tails;
    d.sig_acc = t ? s[i].sig_acc : nullptr;
    // per-block sums only where the kernel that writes them runs (k_fft4k)
    d.sig_part = (t && b.precision == P_FFT && fft_onepass_available(b)) ? s[i].sig_part : nullptr;
    d.n_ok = t ? s[i].n_ok : nullptr;
    d.thr = t ? s[i].thr : nullptr;
    d.sigma = t ? t->sigma : nullptr;
    d.t_tau = t ? t->tau : nullptr;
    d.t_k = t ? t->k : nullptr;
    d.t_rho = t ? t->rho : nullptr;
    d.t_bins = t ? t->bin_counts : nullptr;
    d.n_tails = t ? (unsigned long long*)t->n_tails : nullptr;
    d.tail_cap = t ? t->capacity : 0;
    const bool one = t && s[i].onepass;
    d.thr_lo = one ? s[i].thr_lo : nullptr;
    d.c_tau = one ? s[i].c_tau : nullptr;
    d.c_k = one ? s[i].c_k : nullptr;
    d.c_rho = one ? s[i].c_rho : nullptr;
    d.n_cand = one ? s[i].n_cand : nullptr;
    d.cand_cap = one ? s[i].cand_cap : 0;
    d.redo = one ? s[i].redo : nullptr;
    d.zloc = one ? s[i].zloc : nullptr;
    d.acf_part = one ? s[i].acf_part : nullptr;
    d.acf = one ? s[i].acf : nullptr;
    d.qspec = one ? s[i].qspec : nullptr;
    ti.max_W = std::max(ti.max_W, d.W);
    ti.max_words = std::max(ti.max_words, std::max(d.W, d.spec ? d.spec_rows * b.n_bins : 0));
  }
  std::memset(hdr, 0, sizeof(BatchHdr));
  hdr->n_segs = n;
  hdr->total_tiles = tiles;
  hdr->n_ranges = b.precision == P_FFT ? plan_fft_ranges(b, tiles, slots)
                                       : plan_ranges(b, tiles, slots, sp.tm);
  hdr->n_items = tiles * hdr->n_ranges;
  ti.n_items = hdr->n_items;
  return ti;
}

TimingSet* timing_slot(int dev, bf_status* st) {
  TimingLog& log = t_timing;
  if (log.used >= MAX_TIMED) log.used = 0;  // drop the oldest records
  if ((int)log.sets.size() <= log.used) log.sets.emplace_back();
  TimingSet* te = &log.sets[(size_t)log.used];
  if (te->device != dev) {
    for (auto& ev : te->ev) {
      if (ev) (void)hipEventDestroy(ev);
      ev = nullptr;
    }
    for (auto& ev : te->ev) {
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) {
        *st = hip_fail(e, "hipEventCreate");
        te->device = -1;
        return nullptr;
      }
    }
    te->device = dev;
  }
  ++log.used;
  return te;
}

// x_blocks: blocks per series of the grid-stride kernels (any value >= 1 is correct);
// main_blocks: work-groups of the contraction kernel (n_items for one item each).
bf_status enqueue_kernels(const BankDev& b, const SearchDev& sp, const BatchHdr* table_dev,
                          int32_t seg_slots, int32_t x_blocks, int64_t main_blocks,
                          hipStream_t stream, TimingSet* te) {
  const int32_t xb = x_blocks > 0 ? x_blocks : 1;
  if (te) HIP_TRY(hipEventRecord(te->ev[0], stream), "hipEventRecord");
  HIP_TRY(launch_zero(table_dev, seg_slots, xb, b, sp, stream), "k_zero launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[1], stream), "hipEventRecord");
  HIP_TRY(launch_prefix(table_dev, seg_slots, stream), "k_prefix launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[2], stream), "hipEventRecord");
  HIP_TRY(launch_norms(table_dev, seg_slots, xb, b.L, sp.norm, stream), "k_norms launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[3], stream), "hipEventRecord");
  if (b.precision == P_FFT)
    HIP_TRY(launch_fft_search(table_dev, main_blocks, b, sp, stream), "k_fft launch");
  else
    HIP_TRY(launch_main(table_dev, main_blocks, b, sp, stream), "k_main launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[4], stream), "hipEventRecord");
  HIP_TRY(launch_finalize(table_dev, seg_slots, xb, b, sp, stream), "k_finalize launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[5], stream), "hipEventRecord");
  return BF_OK;
}

bf_status enqueue_tail_kernels(const BankDev& b, const SearchDev& sp_sigma,
                               const SearchDev& sp_tails, const BatchHdr* table_dev,
                               int32_t seg_slots, int32_t x_blocks, int64_t main_blocks,
                               hipStream_t stream, TimingSet* te) {
  bf_status st = enqueue_kernels(b, sp_sigma, table_dev, seg_slots, x_blocks, main_blocks,
                                 stream, te);
  if (st != BF_OK) return st;
  if (b.precision == P_FFT) {
    // the FFT form: a sigma pass and a tails pass over the search's data spectra
    SearchDev s1 = sp_tails;
    s1.mode = MODE_SIGMA;
    HIP_TRY(launch_fft_pass(table_dev, main_blocks, b, s1, stream), "k_fft sigma launch");
    HIP_TRY(launch_sigma(table_dev, seg_slots, b, sp_tails, stream), "k_sigma launch");
    HIP_TRY(launch_fft_pass(table_dev, main_blocks, b, sp_tails, stream), "k_fft tails launch");
    return BF_OK;
  }
  HIP_TRY(launch_sigma(table_dev, seg_slots, b, sp_tails, stream), "k_sigma launch");
  HIP_TRY(launch_main(table_dev, main_blocks, b, sp_tails, stream), "k_main launch");
  return BF_OK;
}

bf_status enqueue_onepass_tail_kernels(const bf_bank* bank, const SearchDev& sp_pass,
                                       const SearchDev& sp_tails, const BatchHdr* table_dev,
                                       int32_t seg_slots, int32_t x_blocks, int64_t main_blocks,
                                       float margin, hipStream_t stream, TimingSet* te) {
  const BankDev& b = bank->dev;
  const int32_t xb = x_blocks > 0 ? x_blocks : 1;
  if (te) HIP_TRY(hipEventRecord(te->ev[0], stream), "hipEventRecord");
  HIP_TRY(launch_zero(table_dev, seg_slots, xb, b, sp_pass, stream), "k_zero launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[1], stream), "hipEventRecord");
  HIP_TRY(launch_prefix(table_dev, seg_slots, stream), "k_prefix launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[2], stream), "hipEventRecord");
  HIP_TRY(launch_norms(table_dev, seg_slots, xb, b.L, sp_pass.norm, stream), "k_norms launch");
  // the predictor
  HIP_TRY(launch_acf(table_dev, seg_slots, b.L, stream), "k_acf launch");
  HIP_TRY(launch_qspec(table_dev, seg_slots, b.L, pred_points(b), stream), "k_qspec launch");
  HIP_TRY(launch_pred(table_dev, seg_slots, bank->grid, b, sp_tails.kappa, margin, stream),
          "k_pred launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[3], stream), "hipEventRecord");
  if (b.precision == P_FFT)
    HIP_TRY(launch_fft_search(table_dev, main_blocks, b, sp_pass, stream), "k_fft launch");
  else
    HIP_TRY(launch_main(table_dev, main_blocks, b, sp_pass, stream), "k_main launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[4], stream), "hipEventRecord");
  HIP_TRY(launch_finalize(table_dev, seg_slots, xb, b, sp_pass, stream), "k_finalize launch");
  HIP_TRY(launch_sigma(table_dev, seg_slots, b, sp_tails, stream), "k_sigma launch");
  if (b.precision == P_FFT)
    HIP_TRY(launch_fft_pair_list(table_dev, seg_slots, b, stream), "k_fft_pair_list launch");
  HIP_TRY(launch_tails_check(table_dev, seg_slots, b, stream), "k_tails_check launch");
  // the tails of the series whose check passed: from the kept correlations (direct forms) or
  // by transforming the listed (block, template) pairs again (FFT form)
  if (b.precision == P_FFT)
    HIP_TRY(launch_fft_pairs(table_dev, seg_slots, b, stream), "k_fft4k_pairs launch");
  else
    HIP_TRY(launch_tails_keep(table_dev, seg_slots, b, stream), "k_tails_keep launch");
  // the tails pass: every work item of a series whose check passed returns at once
  if (b.precision == P_FFT)
    HIP_TRY(launch_fft_pass(table_dev, main_blocks, b, sp_tails, stream), "k_fft tails launch");
  else
    HIP_TRY(launch_main(table_dev, main_blocks, b, sp_tails, stream), "k_main launch");
  if (te) HIP_TRY(hipEventRecord(te->ev[5], stream), "hipEventRecord");
  return BF_OK;
}

}  // namespace bfly

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
    *bytes = bank_total_bytes(b);
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
    const size_t need = bank_total_bytes(b);
    if (!dev_mem) return fail(BF_EINVAL, "dev_mem is NULL");
    if (dev_bytes < need) return fail(BF_EINVAL, "dev_mem too small: %zu < %zu", dev_bytes, need);
    if (((uintptr_t)dev_mem & 255) != 0) return fail(BF_EINVAL, "dev_mem not 256-byte aligned");
    if ((st = check_device_ptr(dev_mem, "dev_mem")) != BF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (b.precision == P_FFT)
      HIP_TRY(launch_fft_bank(g, b, dev_mem, s), "k_fft_bank launch");
    else
      HIP_TRY(launch_bank_gen(g, b, dev_mem, s), "k_bank_gen launch");
    unsigned int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, (char*)dev_mem + bank_data_bytes(b) + bank_exp_bytes(b), sizeof bad,
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
    if (has_side_tables(b.precision)) {
      bk->dev.texp = (const int32_t*)((char*)dev_mem + bank_data_bytes(b));
      bk->dev.tsum = (const float*)(bk->dev.texp + b.K_pad);
    }
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
    size_t total = table_bytes(n_segs);
    for (int32_t i = 0; i < n_segs; ++i) total += series_ws_bytes(bank->dev, n[i]);
    *bytes = total;
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
    return run_batch(bank, &s, 1, params, workspace, workspace_bytes, (hipStream_t)stream,
                     nullptr, 0.0f, TableUpload::Staging);
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_search_batch(const bf_bank* bank, const bf_segment* segs, int32_t n_segs,
                          const bf_search_params* params, void* workspace,
                          size_t workspace_bytes, bf_stream stream) {
  try {
    return run_batch(bank, segs, n_segs, params, workspace, workspace_bytes,
                     (hipStream_t)stream, nullptr, 0.0f, TableUpload::Staging);
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_tails_workspace_bytes(const bf_bank* bank, const int64_t* n, int32_t n_segs,
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
    size_t total = table_bytes(n_segs);
    for (int32_t i = 0; i < n_segs; ++i) total += series_ws_bytes(bank->dev, n[i], true);
    *bytes = total;
    return BF_OK;
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_search_tails(const bf_bank* bank, const bf_tail_segment* segs, int32_t n_segs,
                          float kappa, const bf_search_params* params, void* workspace,
                          size_t workspace_bytes, bf_stream stream) {
  try {
    if (!segs || n_segs < 1) return fail(BF_EINVAL, "need at least one series");
    std::vector<bf_segment> ss((size_t)n_segs);
    std::vector<bf_tails> tt((size_t)n_segs);
    for (int32_t i = 0; i < n_segs; ++i) {
      ss[(size_t)i].x = segs[i].x;
      ss[(size_t)i].n = segs[i].n;
      ss[(size_t)i].out = segs[i].out;
      tt[(size_t)i] = segs[i].tails;
    }
    return run_batch(bank, ss.data(), n_segs, params, workspace, workspace_bytes,
                     (hipStream_t)stream, tt.data(), kappa, TableUpload::Staging);
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

namespace {
size_t coinc_ws_bytes(int64_t W, int64_t cap_b) {
  return align256((size_t)(W + 1) * 4) + align256((size_t)W * 4) +
         2 * align256((size_t)cap_b * 4) + 256;
}
}  // namespace

bf_status bf_coincidence_workspace_bytes(const bf_bank* bank, int64_t n_offsets,
                                         int64_t capacity_b, size_t* bytes) {
  if (!bank || !bytes) return fail(BF_EINVAL, "bank or bytes is NULL");
  if (n_offsets < 1 || n_offsets > ((int64_t)1 << 31) - 2)
    return fail(BF_EINVAL, "n_offsets must be in [1, 2^31 - 2]");
  if (capacity_b < 0 || capacity_b > ((int64_t)1 << 32) - 1)
    return fail(BF_EINVAL, "capacity_b must be in [0, 2^32 - 1]");
  *bytes = coinc_ws_bytes(n_offsets, capacity_b);
  return BF_OK;
}

bf_status bf_coincidence(const bf_bank* bank, const bf_tails* a, const bf_tails* b,
                         int64_t n_offsets, int32_t dtau, double df, uint32_t* counts_a,
                         uint32_t* counts_b, int64_t* n_pairs, void* workspace,
                         size_t workspace_bytes, bf_stream stream) {
  try {
    if (!bank || !a || !b) return fail(BF_EINVAL, "bank or tails is NULL");
    if (n_offsets < 1 || n_offsets > ((int64_t)1 << 31) - 2)
      return fail(BF_EINVAL, "n_offsets must be in [1, 2^31 - 2]");
    if (dtau < 0) return fail(BF_EINVAL, "dtau must be >= 0");
    if (!(df >= 0.0)) return fail(BF_EINVAL, "df must be >= 0");
    if (!counts_a || !counts_b || !n_pairs) return fail(BF_EINVAL, "an output is NULL");
    const bf_tails* sides[2] = {a, b};
    for (const bf_tails* t : sides) {
      if (!t->n_tails) return fail(BF_EINVAL, "tails need n_tails");
      if (t->capacity < 0 || t->capacity > ((int64_t)1 << 32) - 1)
        return fail(BF_EINVAL, "tail capacity must be in [0, 2^32 - 1]");
      if (t->capacity > 0 && (!t->tau || !t->k))
        return fail(BF_EINVAL, "tail lists are NULL with capacity > 0");
    }
    const size_t need = coinc_ws_bytes(n_offsets, b->capacity);
    if (!workspace) return fail(BF_EINVAL, "workspace is NULL");
    if (workspace_bytes < need)
      return fail(BF_EINVAL, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
    if (((uintptr_t)workspace & 255) != 0)
      return fail(BF_EINVAL, "workspace not 256-byte aligned");
    bf_status st;
    const void* ptrs[8] = {workspace, counts_a, counts_b, n_pairs, a->n_tails, b->n_tails,
                           a->tau, b->tau};
    for (const void* q : ptrs)
      if (q && (st = check_device_ptr(q, "coincidence buffer")) != BF_OK) return st;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != bank->device)
      return fail(BF_EINVAL, "bank lives on device %d, current is %d", bank->device, dev);
    char* ws = (char*)workspace;
    CoincWork w;
    size_t off = 0;
    w.start = (uint32_t*)(ws + off);
    off += align256((size_t)(n_offsets + 1) * 4);
    w.cursor = (uint32_t*)(ws + off);
    off += align256((size_t)n_offsets * 4);
    w.order = (uint32_t*)(ws + off);
    off += align256((size_t)b->capacity * 4);
    w.flag_b = (uint32_t*)(ws + off);
    off += align256((size_t)b->capacity * 4);
    w.n_pairs = (unsigned long long*)n_pairs;
    const CoincSide sa = {a->tau, a->k, a->n_tails, a->capacity, counts_a};
    const CoincSide sb = {b->tau, b->k, b->n_tails, b->capacity, counts_b};
    HIP_TRY(launch_coincidence(sa, sb, w, bank->grid, bank->dev.n_bins, bank->dev.n_fdot,
                               n_offsets, dtau, df, (hipStream_t)stream),
            "coincidence launch");
    return BF_OK;
  } catch (...) {
    return fail(BF_ENOMEM, "internal error");
  }
}

bf_status bf_set_timing(int32_t enable) {
  g_timing = enable != 0;
  return BF_OK;
}

bf_status bf_kernel_times(double* ms, int32_t* n_searches) {
  if (!ms) return fail(BF_EINVAL, "ms is NULL");
  TimingLog& log = t_timing;
  if (log.used == 0) return fail(BF_EAGAIN, "no timed search on this thread");
  for (int i = 0; i < 5; ++i) ms[i] = 0.0;
  for (int k = 0; k < log.used; ++k) {
    TimingSet& t = log.sets[(size_t)k];
    HIP_TRY(hipEventSynchronize(t.ev[5]), "hipEventSynchronize");
    for (int i = 0; i < 5; ++i) {
      float v = 0.0f;
      HIP_TRY(hipEventElapsedTime(&v, t.ev[i], t.ev[i + 1]), "hipEventElapsedTime");
      ms[i] += (double)v;
    }
  }
  if (n_searches) *n_searches = log.used;
  log.used = 0;
  return BF_OK;
}

bf_status bf_plan(const bf_bank* bank, const int64_t* n, int32_t n_segs, int32_t* n_ranges,
                  int64_t* n_items) {
  if (!bank || !n || n_segs < 1) return fail(BF_EINVAL, "bad arguments");
  int64_t tiles = 0;
  for (int32_t i = 0; i < n_segs; ++i) {
    if (n[i] < bank->dev.L) return fail(BF_EINVAL, "series shorter than L");
    int32_t tm = 0, tn = 0, pp = 0;
    choose_tile(bank->dev.precision, MODE_SEARCH, &tm, &tn, &pp);
    const int64_t n_wg = bank->dev.precision == P_FFT ? 2 * (int64_t)bank->dev.fft_m - bank->dev.L + 1
                                                       : 32 * (int64_t)tn * WG_WAVES;
    tiles += (n[i] - bank->dev.L + 1 + n_wg - 1) / n_wg;
  }
  int slots = 0;
  bf_status st = device_slots(&slots);
  if (st != BF_OK) return st;
  int32_t tm = 0, tn = 0, pp = 0;
  choose_tile(bank->dev.precision, MODE_SEARCH, &tm, &tn, &pp);
  const int32_t r = bank->dev.precision == P_FFT ? plan_fft_ranges(bank->dev, tiles, slots)
                                                 : plan_ranges(bank->dev, tiles, slots, tm);
  if (n_ranges) *n_ranges = r;
  if (n_items) *n_items = tiles * r;
  return BF_OK;
}

const char* bf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
