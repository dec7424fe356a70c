// The search of one series with no allocation: bf_search_segment_noalloc (include/bfly.h).
//
// The workspace of bf_search_segment (batch table, prefix sums, window norms, running
// maxima, spectrum sums; the FFT form's block spectra) lives in a file-scope device array of
// NOALLOC_SCRATCH_BYTES, one per GPU, held until the process ends.  The batch table is
// written into it by a one-work-group kernel that receives the table as its argument, so the
// call needs neither a pinned staging buffer nor a device allocation.  The kernels and their
// results are those of bf_search_segment.
#include "bfly.h"
#include "bfly_internal.h"
#include "bfly_runtime.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace bfly {

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// Copies the table word by word from the kernel argument into device memory.
__global__ __launch_bounds__(64) void k_put_table(OneSeriesTable t, OneSeriesTable* dst) {
  static_assert(sizeof(OneSeriesTable) % 8 == 0, "whole 8-byte words");
  const unsigned long long* s = reinterpret_cast<const unsigned long long*>(&t);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(OneSeriesTable) / 8); i += blockDim.x) d[i] = s[i];
}

// Device address of `scratch` on each device, taken once per device with it current.
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

bf_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return set_error(BF_EINVAL, "device %d: the no-allocation path serves devices 0..%d", dev,
                     NOALLOC_MAX_DEVICES - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      if (e == hipSuccess) e = hipErrorInvalidSymbol;
      return hip_error(e, "hipGetSymbolAddress(scratch)");
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BF_OK;
}

}  // namespace

hipError_t launch_put_table(const OneSeriesTable& t, OneSeriesTable* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_put_table, dim3(1), dim3(64), 0, s, t, dst);
  return hipGetLastError();
}

}  // namespace bfly

using namespace bfly;

extern "C" bf_status bf_search_segment_noalloc(const bf_bank* bank, const float* x, int64_t n,
                                               const bf_search_params* params,
                                               const bf_result* out, bf_stream stream) {
  try {
    if (!bank) return set_error(BF_EINVAL, "bank is NULL");
    if (!out) return set_error(BF_EINVAL, "out is NULL");
    if (n < bank->dev.L)
      return set_error(BF_EINVAL, "series has %lld samples, fewer than L = %d", (long long)n,
                       bank->dev.L);
    const int64_t max_n = ((int64_t)1 << 31) - MAX_N_WG - bank->dev.L_pad - STRIP_SLACK;
    if (n > max_n) return set_error(BF_EINVAL, "series is too long");
    const size_t need = table_bytes(1) + series_ws_bytes(bank->dev, n);
    if (need > NOALLOC_SCRATCH_BYTES)
      return set_error(BF_EINVAL,
                       "a series of %lld samples needs %zu bytes of workspace; the "
                       "no-allocation search has %zu",
                       (long long)n, need, NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    bf_status st = scratch_address(&ws);
    if (st != BF_OK) return st;
    bf_segment s;
    s.x = x;
    s.n = n;
    s.out = *out;
    return run_batch(bank, &s, 1, params, ws, NOALLOC_SCRATCH_BYTES, (hipStream_t)stream,
                     nullptr, 0.0f, TableUpload::Kernel);
  } catch (...) {
    return set_error(BF_ENOMEM, "internal error");
  }
}
