// Two-detector coincidence of kappa-sigma tails (Fig. 6 caption: pseudo-spectra of
// simultaneous tails of two detectors, counted by frequency with pairs within a frequency
// width).  Channel B's tails are bucketed by offset (count, scan, scatter), then every tail
// of A scans the buckets of the offsets within dtau of its own and counts the B tails whose
// start frequencies lie within df of its own.  All results are integer counts:
// deterministic, independent of the order of the tail lists.
#include "bfly_internal.h"

#include <hip/hip_runtime.h>

namespace bfly {

namespace {

// f0 of global f0 index i, as the bank grid computes it (inclusive linspace).
__device__ __forceinline__ double grid_f0(const GridDev& g, int64_t i) {
  return (g.n_f0 > 1 && i == g.n_f0 - 1) ? g.f0_max : (double)i * g.f0_step + g.f0_min;
}

// Entries of a tail list: min(n_tails, capacity).
__device__ __forceinline__ int64_t n_listed(const CoincSide& s) {
  const int64_t n = s.n_tails[0];
  return n < s.capacity ? n : s.capacity;
}

__global__ __launch_bounds__(256) void k_coinc_zero(CoincSide a, CoincSide b, CoincWork w,
                                                    int64_t W, int32_t n_bins) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i <= W; i += stride) w.start[i] = 0u;
  for (int64_t i = t0; i < b.capacity; i += stride) w.flag_b[i] = 0u;
  for (int64_t i = t0; i < n_bins; i += stride) {
    a.counts[i] = 0u;
    b.counts[i] = 0u;
  }
  if (t0 == 0) w.n_pairs[0] = 0ull;
}

// start[tau] = number of B tails at offset tau (shifted by one for the exclusive scan).
__global__ __launch_bounds__(256) void k_coinc_count(CoincSide b, CoincWork w, int64_t W) {
  const int64_t nb = n_listed(b);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nb; j += stride) {
    const int32_t t = b.tau[j];
    if (t >= 0 && t < W) atomicAdd(w.start + t + 1, 1u);
  }
}

// In-place inclusive scan of start[1..W] by one 1024-thread work-group, so that start[t]
// becomes the first slot of offset t's bucket; cursor[t] = start[t].
__global__ __launch_bounds__(1024) void k_coinc_scan(CoincWork w, int64_t W) {
  __shared__ uint32_t part[16];
  __shared__ uint32_t carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0u;
  __syncthreads();
  for (int64_t base = 1; base <= W; base += 1024) {
    const int64_t i = base + tid;
    uint32_t v = i <= W ? w.start[i] : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(v, o, 64);
      if (lane >= o) v += u;
    }
    if (lane == 63) part[wave] = v;
    __syncthreads();
    if (tid == 0) {
      uint32_t r = carry;
      for (int k = 0; k < 16; ++k) {
        const uint32_t t = part[k];
        part[k] = r;
        r += t;
      }
      carry = r;
    }
    __syncthreads();
    v += part[wave];
    if (i <= W) w.start[i] = v;
    __syncthreads();
  }
  for (int64_t t = tid; t < W; t += 1024) w.cursor[t] = w.start[t];
}

__global__ __launch_bounds__(256) void k_coinc_scatter(CoincSide b, CoincWork w, int64_t W) {
  const int64_t nb = n_listed(b);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nb; j += stride) {
    const int32_t t = b.tau[j];
    if (t >= 0 && t < W) w.order[atomicAdd(w.cursor + t, 1u)] = (uint32_t)j;
  }
}

__global__ __launch_bounds__(256) void k_coinc_match(CoincSide a, CoincSide b, CoincWork w,
                                                     GridDev g, int64_t W, int32_t dtau,
                                                     double df, int32_t n_fdot,
                                                     int32_t n_bins) {
  const int64_t na = n_listed(a);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += stride) {
    const int64_t ta = a.tau[i];
    const int64_t fia = (int64_t)a.k[i] / n_fdot;
    const int64_t bin = fia - g.f0_lo;
    if (ta < 0 || ta >= W || a.k[i] < 0 || bin < 0 || bin >= n_bins) continue;  // not ours
    const double fa = grid_f0(g, fia);
    const int64_t t_lo = ta - dtau > 0 ? ta - dtau : 0;
    const int64_t t_hi = ta + dtau < W - 1 ? ta + dtau : W - 1;
    unsigned long long pairs = 0ull;
    for (int64_t t = t_lo; t <= t_hi; ++t) {
      for (uint32_t s = w.start[t]; s < w.start[t + 1]; ++s) {
        const uint32_t j = w.order[s];
        const int64_t fib = (int64_t)b.k[j] / n_fdot;
        if (b.k[j] < 0 || fib - g.f0_lo < 0 || fib - g.f0_lo >= n_bins) continue;
        const double fb = grid_f0(g, fib);
        if (fabs(fa - fb) <= df) {
          ++pairs;
          w.flag_b[j] = 1u;
        }
      }
    }
    if (pairs) {
      atomicAdd(a.counts + bin, 1u);
      atomicAdd(w.n_pairs, pairs);
    }
  }
}

__global__ __launch_bounds__(256) void k_coinc_count_b(CoincSide b, CoincWork w, GridDev g,
                                                       int32_t n_fdot) {
  const int64_t nb = n_listed(b);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // only tails that passed the bin check of k_coinc_match are flagged
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nb; j += stride)
    if (w.flag_b[j]) atomicAdd(b.counts + ((int64_t)b.k[j] / n_fdot - g.f0_lo), 1u);
}

}  // namespace

hipError_t launch_coincidence(const CoincSide& a, const CoincSide& b, const CoincWork& w,
                              const GridDev& g, int32_t n_bins, int32_t n_fdot, int64_t W,
                              int32_t dtau, double df, hipStream_t s) {
  const unsigned grid = 1024;
  hipLaunchKernelGGL(k_coinc_zero, dim3(grid), dim3(256), 0, s, a, b, w, W, n_bins);
  hipLaunchKernelGGL(k_coinc_count, dim3(grid), dim3(256), 0, s, b, w, W);
  hipLaunchKernelGGL(k_coinc_scan, dim3(1), dim3(1024), 0, s, w, W);
  hipLaunchKernelGGL(k_coinc_scatter, dim3(grid), dim3(256), 0, s, b, w, W);
  hipLaunchKernelGGL(k_coinc_match, dim3(grid), dim3(256), 0, s, a, b, w, g, W, dtau, df,
                     n_fdot, n_bins);
  hipLaunchKernelGGL(k_coinc_count_b, dim3(grid), dim3(256), 0, s, b, w, g, n_fdot);
  return hipGetLastError();
}

}  // namespace bfly
