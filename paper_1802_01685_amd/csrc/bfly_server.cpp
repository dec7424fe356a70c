// Serving: continuous batching of uneven series against a device-resident bank.
//
// A worker thread owns the device side.  Requests are queued by bf_submit (which only copies
// the samples into pinned host memory), admitted in arrival order when a slot is free and
// their device buffers fit the HBM budget (one arena carved from a single allocation), and
// launched in "ticks": each tick is one batched search over every admitted, not yet launched
// request, on one of `ticks_in_flight` streams.  A tick copies the samples in, replays a
// graph captured once per stream at creation (table upload + the five kernels, grids sized
// for max_slots series, the contraction kernel looping over the tick's work items), and
// copies each request's outputs back to pinned host memory.  Requests that arrive while
// ticks run are admitted as slots and memory free up and go into the next tick, whose
// kernels overlap the running ones on the device.  Every result is a pure function of its
// own series (all merges in the kernels are exact), so a request gives the same bits alone
// and in any mix.
#include "bfly.h"
#include "bfly_runtime.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace bfly;

namespace {

// First-fit allocator over [0, size) with coalescing; offsets and sizes are 256-aligned.
class Arena {
 public:
  explicit Arena(size_t size = 0) { reset(size); }
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

enum State { QUEUED = 0, RUNNING = 1, DONE = 2, FAILED = 3, CANCELLED = 4 };

// Per-request result layout, identical in device memory and in the pinned host copy, so one
// device-to-host copy moves all outputs.
struct ResLayout {
  size_t max_abs, argmax, spec, spectrum, hist, ndeg, bytes;
};
ResLayout res_layout(const BankDev& b, const SearchDev& sp, int64_t n) {
  const int64_t W = n - b.L + 1;
  const int64_t rows = (W + sp.t_block - 1) / sp.t_block;
  ResLayout r;
  size_t off = 0;
  r.max_abs = off;
  off = align256(off + (size_t)W * 4);
  r.argmax = off;
  off = align256(off + (size_t)W * 4);
  r.spec = off;
  off = align256(off + (size_t)rows * b.n_bins * 4);
  r.spectrum = off;
  off = align256(off + (size_t)b.n_bins * 8);
  r.hist = off;
  off = align256(off + (size_t)sp.hist_bins * 4);
  r.ndeg = off;
  off = align256(off + 8);
  r.bytes = off;
  return r;
}

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0;
  int state = QUEUED;
  bool cancel = false;
  double t_submit = 0, t_start = 0, t_done = 0;
  float* x_pin = nullptr;   // pinned copy of the samples
  char* res_pin = nullptr;  // pinned results, ResLayout
  ResLayout rl{};
  size_t dev_off = 0, dev_bytes = 0;  // arena block: x | workspace part | results
  bool on_device = false;
  std::string error;
};

struct Tick {
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchHdr* table_dev = nullptr;
  char* table_pin = nullptr;
  hipEvent_t done = nullptr;
  std::vector<Request*> reqs;
  bool busy = false;
};

}  // namespace

struct bf_server {
  const bf_bank* bank = nullptr;
  bf_server_desc desc{};
  SearchDev sp{};
  int device = 0;
  int slots = 1;
  int32_t x_blocks = 256;
  char* arena_dev = nullptr;
  Arena arena;
  std::vector<Tick> ticks;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  std::deque<Request*> queue;   // QUEUED, arrival order
  std::vector<Request*> ready;  // admitted (device memory held), not yet launched
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1;
  int admitted = 0;             // requests holding device memory
  std::chrono::steady_clock::time_point t0;
  // statistics
  int64_t n_done = 0, n_ticks = 0;
  double corr_done = 0.0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

size_t request_dev_bytes(const bf_server* s, int64_t n, ResLayout* rl) {
  *rl = res_layout(s->bank->dev, s->sp, n);
  return align256((size_t)n * 4) + series_ws_bytes(s->bank->dev, n) + rl->bytes;
}

void free_request_host(Request* r) {
  if (r->x_pin) (void)hipHostFree(r->x_pin);
  if (r->res_pin) (void)hipHostFree(r->res_pin);
  r->x_pin = nullptr;
  r->res_pin = nullptr;
}

// Launches one tick on slot t for the requests in s->ready.  Called with s->mu held.
bool launch_tick(bf_server* s, Tick& t) {
  const BankDev& b = s->bank->dev;
  const int32_t nseg = (int32_t)std::min<size_t>(s->ready.size(), (size_t)s->desc.max_slots);
  t.reqs.assign(s->ready.begin(), s->ready.begin() + nseg);
  s->ready.erase(s->ready.begin(), s->ready.begin() + nseg);
  std::vector<SeriesBufs> sb((size_t)nseg);
  for (int32_t i = 0; i < nseg; ++i) {
    Request* r = t.reqs[(size_t)i];
    char* base = s->arena_dev + r->dev_off;
    SeriesBufs& q = sb[(size_t)i];
    q.x = (const float*)base;
    q.n = r->n;
    char* ws = base + align256((size_t)r->n * 4);
    series_ws_carve(b, r->n, ws, &q);
    char* res = ws + series_ws_bytes(b, r->n);
    q.out.max_abs = (float*)(res + r->rl.max_abs);
    q.out.argmax = (int32_t*)(res + r->rl.argmax);
    q.out.spec = (float*)(res + r->rl.spec);
    q.out.spectrum = (double*)(res + r->rl.spectrum);
    q.out.hist = (uint32_t*)(res + r->rl.hist);
    q.out.n_degenerate = (int64_t*)(res + r->rl.ndeg);
  }
  fill_table(b, s->sp, sb.data(), nseg, s->slots, (BatchHdr*)t.table_pin);
  std::string err;
  hipError_t e = hipSuccess;
  for (int32_t i = 0; i < nseg && e == hipSuccess; ++i)
    e = hipMemcpyAsync((void*)sb[(size_t)i].x, t.reqs[(size_t)i]->x_pin,
                       (size_t)t.reqs[(size_t)i]->n * 4, hipMemcpyHostToDevice, t.stream);
  if (e == hipSuccess) e = hipGraphLaunch(t.exec, t.stream);
  for (int32_t i = 0; i < nseg && e == hipSuccess; ++i) {
    Request* r = t.reqs[(size_t)i];
    e = hipMemcpyAsync(r->res_pin, (void*)sb[(size_t)i].out.max_abs, r->rl.bytes,
                       hipMemcpyDeviceToHost, t.stream);
  }
  if (e == hipSuccess) e = hipEventRecord(t.done, t.stream);
  const double now = s->now();
  for (Request* r : t.reqs) {
    r->t_start = now;
    r->state = RUNNING;
  }
  if (e != hipSuccess) {
    // Nothing reliable was enqueued: fail the tick's requests and give their memory back
    // once the stream has drained.
    (void)hipStreamSynchronize(t.stream);
    (void)hipGetLastError();
    for (Request* r : t.reqs) {
      r->state = FAILED;
      r->error = std::string("tick launch failed: ") + hipGetErrorString(e);
      r->t_done = now;
      s->arena.release(r->dev_off, r->dev_bytes);
      r->on_device = false;
      --s->admitted;
    }
    t.reqs.clear();
    return false;
  }
  t.busy = true;
  ++s->n_ticks;
  return true;
}

// Retires finished ticks.  Called with s->mu held.
bool retire(bf_server* s) {
  bool any = false;
  for (Tick& t : s->ticks) {
    if (!t.busy) continue;
    hipError_t q = hipEventQuery(t.done);
    if (q == hipErrorNotReady) continue;
    const double now = s->now();
    for (Request* r : t.reqs) {
      if (q != hipSuccess) {
        r->state = FAILED;
        r->error = std::string("tick failed: ") + hipGetErrorString(q);
      } else if (r->cancel) {
        r->state = CANCELLED;
      } else {
        r->state = DONE;
        ++s->n_done;
        s->corr_done += (double)s->bank->dev.K * (double)(r->n - s->bank->dev.L + 1);
      }
      r->t_done = now;
      s->arena.release(r->dev_off, r->dev_bytes);
      r->on_device = false;
      --s->admitted;
      if (r->state == CANCELLED && r->x_pin) {
        (void)hipHostFree(r->x_pin);
        r->x_pin = nullptr;
      }
    }
    if (q != hipSuccess) (void)hipGetLastError();
    t.reqs.clear();
    t.busy = false;
    any = true;
  }
  return any;
}

// Admits queued requests in arrival order while slots and memory allow.
bool admit(bf_server* s) {
  bool any = false;
  while (!s->queue.empty() && s->admitted < s->desc.max_slots) {
    Request* r = s->queue.front();
    if (r->cancel) {
      s->queue.pop_front();
      r->state = CANCELLED;
      r->t_done = s->now();
      continue;
    }
    size_t off = 0;
    if (!s->arena.alloc(r->dev_bytes, &off)) break;  // wait for memory
    s->queue.pop_front();
    r->dev_off = off;
    r->on_device = true;
    ++s->admitted;
    s->ready.push_back(r);
    any = true;
  }
  return any;
}

void worker_main(bf_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progress = retire(s);
    progress |= admit(s);
    for (Tick& t : s->ticks) {
      if (s->ready.empty()) break;
      if (!t.busy) progress |= launch_tick(s, t);
    }
    bool busy = false;
    for (Tick& t : s->ticks) busy |= t.busy;
    if (s->stop && !busy && s->ready.empty() && s->queue.empty()) break;
    if (progress) continue;
    if (busy)
      s->cv.wait_for(lk, std::chrono::microseconds(100));
    else
      s->cv.wait_for(lk, std::chrono::milliseconds(50));
  }
}

bf_status destroy_ticks(bf_server* s) {
  for (Tick& t : s->ticks) {
    if (t.exec) (void)hipGraphExecDestroy(t.exec);
    if (t.graph) (void)hipGraphDestroy(t.graph);
    if (t.done) (void)hipEventDestroy(t.done);
    if (t.stream) (void)hipStreamDestroy(t.stream);
    if (t.table_pin) (void)hipHostFree(t.table_pin);
    t = Tick();
  }
  return BF_OK;
}

void free_server(bf_server* s) {
  destroy_ticks(s);
  if (s->arena_dev) (void)hipFree(s->arena_dev);
  for (auto& kv : s->reqs) {
    free_request_host(kv.second);
    delete kv.second;
  }
  delete s;
}

}  // namespace

extern "C" {

bf_status bf_server_create(const bf_bank* bank, const bf_server_desc* desc, bf_server** out) {
  try {
    if (!bank || !desc || !out) return set_error(BF_EINVAL, "NULL argument");
    *out = nullptr;
    bf_status st = check_params(&desc->params);
    if (st != BF_OK) return st;
    if (desc->max_slots < 1 || desc->max_slots > 1024)
      return set_error(BF_EINVAL, "max_slots must be in [1, 1024]");
    if (desc->ticks_in_flight < 1 || desc->ticks_in_flight > 4)
      return set_error(BF_EINVAL, "ticks_in_flight must be in [1, 4]");
    if (desc->hbm_budget_bytes < 1024 * 1024)
      return set_error(BF_EINVAL, "hbm_budget_bytes must be at least 1 MiB");
    if (desc->reserved != 0 || desc->reserved2 != 0)
      return set_error(BF_EINVAL, "reserved fields must be 0");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev != bank->device) return set_error(BF_EINVAL, "bank lives on another device");
    bf_server* s = new (std::nothrow) bf_server();
    if (!s) return set_error(BF_ENOMEM, "host allocation failed");
    s->bank = bank;
    s->desc = *desc;
    s->sp = make_search(bank->dev, &desc->params);
    s->device = dev;
    s->t0 = std::chrono::steady_clock::now();
    if ((st = device_slots(&s->slots)) != BF_OK) {
      delete s;
      return st;
    }
    e = hipMalloc((void**)&s->arena_dev, desc->hbm_budget_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      delete s;
      return set_error(BF_ENOMEM, "hipMalloc of the %zu-byte HBM budget failed",
                       desc->hbm_budget_bytes);
    }
    s->arena.reset(desc->hbm_budget_bytes & ~(size_t)255);
    if (bank->dev.precision != P_FFT && (e = prepare_main(bank->dev, s->sp)) != hipSuccess) {
      free_server(s);
      return hip_error(e, "hipFuncSetAttribute(k_main)");
    }
    const size_t tb = table_bytes(desc->max_slots);
    s->ticks.resize((size_t)desc->ticks_in_flight);
    for (Tick& t : s->ticks) {
      if ((e = hipStreamCreateWithFlags(&t.stream, hipStreamNonBlocking)) != hipSuccess ||
          (e = hipEventCreateWithFlags(&t.done, hipEventDisableTiming)) != hipSuccess ||
          (e = hipMalloc((void**)&t.table_dev, tb)) != hipSuccess ||
          (e = hipHostMalloc((void**)&t.table_pin, tb, hipHostMallocDefault)) != hipSuccess) {
        free_server(s);
        return hip_error(e, "server stream/table setup");
      }
      std::memset(t.table_pin, 0, tb);
      // Capture: table upload + the five kernels, grids sized for max_slots series and as
      // many contraction work-groups as the CUs hold at once (they loop over the tick's
      // items).
      if ((e = hipStreamBeginCapture(t.stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        free_server(s);
        return hip_error(e, "hipStreamBeginCapture");
      }
      hipError_t ce = hipMemcpyAsync(t.table_dev, t.table_pin, tb, hipMemcpyHostToDevice,
                                     t.stream);
      bf_status kst = ce == hipSuccess
                          ? enqueue_kernels(bank->dev, s->sp, t.table_dev, desc->max_slots,
                                            s->x_blocks,
                                            (int64_t)s->slots * contraction_wgs_per_cu(bank->dev),
                                            t.stream, nullptr)
                          : hip_error(ce, "hipMemcpyAsync(capture)");
      e = hipStreamEndCapture(t.stream, &t.graph);
      if (kst != BF_OK || e != hipSuccess) {
        free_server(s);
        return kst != BF_OK ? kst : hip_error(e, "hipStreamEndCapture");
      }
      if ((e = hipGraphInstantiate(&t.exec, t.graph, nullptr, nullptr, 0)) != hipSuccess) {
        free_server(s);
        return hip_error(e, "hipGraphInstantiate");
      }
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return BF_OK;
  } catch (...) {
    return set_error(BF_ENOMEM, "internal error");
  }
}

bf_status bf_server_request_bytes(const bf_server* s, int64_t n, size_t* bytes) {
  if (!s || !bytes) return set_error(BF_EINVAL, "NULL argument");
  if (n < s->bank->dev.L) return set_error(BF_EINVAL, "series shorter than L");
  ResLayout rl;
  *bytes = request_dev_bytes(s, n, &rl);
  return BF_OK;
}

bf_status bf_submit(bf_server* s, const float* x_host, int64_t n, uint64_t* ticket) {
  try {
    if (!s || !x_host || !ticket) return set_error(BF_EINVAL, "NULL argument");
    const BankDev& b = s->bank->dev;
    if (n < b.L) return set_error(BF_EINVAL, "series has %lld samples, fewer than L = %d",
                                  (long long)n, b.L);
    if (n > ((int64_t)1 << 31) - MAX_N_WG - b.L_pad - STRIP_SLACK)
      return set_error(BF_EINVAL, "series too long");
    Request* r = new (std::nothrow) Request();
    if (!r) return set_error(BF_ENOMEM, "host allocation failed");
    r->n = n;
    r->dev_bytes = request_dev_bytes(s, n, &r->rl);
    if (r->dev_bytes > (s->desc.hbm_budget_bytes & ~(size_t)255)) {
      const size_t need = r->dev_bytes;
      delete r;
      return set_error(BF_EBUDGET, "request needs %zu device bytes, the budget is %zu", need,
                       s->desc.hbm_budget_bytes);
    }
    hipError_t e = hipHostMalloc((void**)&r->x_pin, (size_t)n * 4, hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&r->res_pin, r->rl.bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      free_request_host(r);
      delete r;
      return set_error(BF_ENOMEM, "pinned host allocation failed");
    }
    std::memcpy(r->x_pin, x_host, (size_t)n * 4);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop) {
        free_request_host(r);
        delete r;
        return set_error(BF_EINVAL, "server is shutting down");
      }
      r->ticket = s->next_ticket++;
      r->t_submit = s->now();
      s->reqs[r->ticket] = r;
      s->queue.push_back(r);
      *ticket = r->ticket;
    }
    s->cv.notify_one();
    return BF_OK;
  } catch (...) {
    return set_error(BF_ENOMEM, "internal error");
  }
}

bf_status bf_poll(bf_server* s, uint64_t ticket, int32_t* state, double* t_submit,
                  double* t_start, double* t_done) {
  if (!s) return set_error(BF_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(BF_ENOTFOUND, "unknown ticket %llu",
                                            (unsigned long long)ticket);
  const Request* r = it->second;
  if (state) *state = r->state;
  if (t_submit) *t_submit = r->t_submit;
  if (t_start) *t_start = r->t_start;
  if (t_done) *t_done = r->t_done;
  return BF_OK;
}

bf_status bf_fetch(bf_server* s, uint64_t ticket, float* max_abs, int32_t* argmax, float* spec,
                   double* spectrum, uint32_t* hist, int64_t* n_degenerate) {
  if (!s) return set_error(BF_EINVAL, "server is NULL");
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
      return set_error(BF_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    r = it->second;
    if (r->state == QUEUED || r->state == RUNNING)
      return set_error(BF_EAGAIN, "ticket %llu is not done", (unsigned long long)ticket);
    s->reqs.erase(it);
  }
  bf_status st = BF_OK;
  if (r->state == DONE) {
    const BankDev& b = s->bank->dev;
    const int64_t W = r->n - b.L + 1;
    const int64_t rows = (W + s->sp.t_block - 1) / s->sp.t_block;
    if (max_abs) std::memcpy(max_abs, r->res_pin + r->rl.max_abs, (size_t)W * 4);
    if (argmax) std::memcpy(argmax, r->res_pin + r->rl.argmax, (size_t)W * 4);
    if (spec) std::memcpy(spec, r->res_pin + r->rl.spec, (size_t)rows * b.n_bins * 4);
    if (spectrum) std::memcpy(spectrum, r->res_pin + r->rl.spectrum, (size_t)b.n_bins * 8);
    if (hist) std::memcpy(hist, r->res_pin + r->rl.hist, (size_t)s->sp.hist_bins * 4);
    if (n_degenerate) std::memcpy(n_degenerate, r->res_pin + r->rl.ndeg, 8);
  } else if (r->state == CANCELLED) {
    st = set_error(BF_ECANCELED, "ticket %llu was cancelled", (unsigned long long)ticket);
  } else {
    st = set_error(BF_EHIP, "ticket %llu failed: %s", (unsigned long long)ticket,
                   r->error.c_str());
  }
  free_request_host(r);
  delete r;
  return st;
}

bf_status bf_cancel(bf_server* s, uint64_t ticket) {
  if (!s) return set_error(BF_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
      return set_error(BF_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second;
    // A queued request is dropped at admission; an admitted or running one finishes and
    // its result is discarded.
    if (r->state == QUEUED || r->state == RUNNING) r->cancel = true;
  }
  s->cv.notify_one();
  return BF_OK;
}

bf_status bf_server_stats(bf_server* s, int64_t* done, int64_t* ticks, double* correlations,
                          int32_t* queued, int32_t* on_device) {
  if (!s) return set_error(BF_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (done) *done = s->n_done;
  if (ticks) *ticks = s->n_ticks;
  if (correlations) *correlations = s->corr_done;
  if (queued) *queued = (int32_t)s->queue.size();
  if (on_device) *on_device = s->admitted;
  return BF_OK;
}

bf_status bf_server_destroy(bf_server* s) {
  if (!s) return BF_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Request* r : s->queue) r->cancel = true;  // queued requests are dropped
  }
  s->cv.notify_one();
  if (s->worker.joinable()) s->worker.join();  // running ticks drain first
  free_server(s);
  return BF_OK;
}

}  // extern "C"
