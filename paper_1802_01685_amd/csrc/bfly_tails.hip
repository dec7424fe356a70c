// Single-pass kappa-sigma tail search (Sec. 2.2 and the Fig. 5 caption: sigma is predicted by
// Parseval's theorem, and only correlations above kappa sigma leave the GPU).
//
// sigma_k^2 = (1/n_ok) sum_tau rho_k(tau)^2 is complete only after every offset, so an exact
// tail extraction needs sigma before the pass that forms rho.  The predictor here takes the
// paper's route in the lag domain: with z the series normalised window by window (centred
// and scaled by 1/sqrt(E) of the window around each sample), sum_tau (h . z_tau)^2 equals
// sum_l R_h(l) R_z(l) over the lags |l| < L, R the autocorrelations, which by Parseval is
// sum_f |H(f)|^2 Q(f) / N with Q the cosine transform of R_z.  The search pass then keeps
// every (tau, k) with |rho| above kappa * margin * sigma_pred as a candidate (the FFT form:
// every (block, k) pair holding one) while it sums the exact rho^2; afterwards the exact
// thresholds kappa * sigma_k select the tails among the candidates (the FFT form transforms
// the listed pairs again).  That is exact whenever no exact threshold lies below its
// predicted one and the candidates fit: k_tails_check verifies both per series and flags a
// series for which either fails, and the ordinary tails pass then runs for it.  Either way
// the tails, sigma and counts are those of the two-pass search, bit for bit.
#include "bfly_internal.h"

#include <hip/hip_runtime.h>

namespace bfly {

namespace {

// z[j] = (x[j] - mean of the window around j) / sqrt(E of that window), the window around j
// being tau = clamp(j - L/2, 0, W - 1); 0 where that window is degenerate or x[j] is not
// finite.
__global__ __launch_bounds__(256) void k_zloc(const BatchHdr* __restrict__ hdr, int L) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  if (!sg.zloc) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < sg.n; j += stride) {
    int64_t tau = j - L / 2;
    tau = tau < 0 ? 0 : (tau >= sg.W ? sg.W - 1 : tau);
    const double s = sg.inv_norm[tau];
    float z = 0.0f;
    const float v = sg.x[j];
    if (s > 0.0 && isfinite(v)) {
      // the window mean of x from the prefix sums (the level cancels)
      const double s1 = (sg.pre[4 * (tau + L)] - sg.pre[4 * tau]) +
                        (sg.pre[4 * (tau + L) + 1] - sg.pre[4 * tau + 1]);
      z = (float)(((double)v - s1 / (double)L) * s);
    }
    sg.zloc[j] = z;
  }
}

// Lag sums over one chunk of the series: block (lag block, chunk, series), 64 lags x 4
// phases per block; acf_part[chunk][l] = sum over j in the chunk of z[j] z[j + l], in
// float64, the four phases added in a fixed order (deterministic).
constexpr int ACF_TILE = 1024;
__global__ __launch_bounds__(256) void k_acf(const BatchHdr* __restrict__ hdr, int L) {
  if ((int)blockIdx.z >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.z];
  if (!sg.zloc) return;
  __shared__ float zj[ACF_TILE];
  __shared__ float zt[ACF_TILE + 64];
  __shared__ double part[4][64];
  const int t = threadIdx.x, lane = t & 63, ph = t >> 6;
  const int l = (int)blockIdx.x * 64 + lane;   // this thread's lag
  const int64_t n = sg.n;
  const int64_t per = (n + ACF_CHUNKS - 1) / ACF_CHUNKS;
  const int64_t j_lo = (int64_t)blockIdx.y * per;
  const int64_t j_hi = j_lo + per < n ? j_lo + per : n;
  const int l0 = (int)blockIdx.x * 64;
  double acc = 0.0;
  for (int64_t j0 = j_lo; j0 < j_hi; j0 += ACF_TILE) {
    __syncthreads();
    // zj[i] = z[j0 + i] within the chunk, zt[i] = z[j0 + l0 + i] (0 past the series end)
    for (int i = t; i < ACF_TILE + 64; i += 256) {
      const int64_t jj = j0 + l0 + i;
      zt[i] = jj < n ? sg.zloc[jj] : 0.0f;
    }
    for (int i = t; i < ACF_TILE; i += 256) {
      const int64_t jj = j0 + i;
      zj[i] = jj < j_hi ? sg.zloc[jj] : 0.0f;
    }
    __syncthreads();
    // zt is 0 past the series end, so products beyond it add nothing
    for (int i = ph; i < ACF_TILE; i += 4) acc = fma((double)zj[i], (double)zt[i + lane], acc);
  }
  part[ph][lane] = acc;
  __syncthreads();
  if (ph == 0 && l < L)
    sg.acf_part[(int64_t)blockIdx.y * L + l] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// acf[l] = sum of the chunks' lag sums in chunk order; acf[L] = non-degenerate offsets.
__global__ __launch_bounds__(256) void k_acf_sum(const BatchHdr* __restrict__ hdr, int L) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  if (!sg.zloc) return;
  const int l = (int)blockIdx.x * 256 + threadIdx.x;
  if (l < L) {
    double a = 0.0;
    for (int c = 0; c < ACF_CHUNKS; ++c) a += sg.acf_part[(int64_t)c * L + l];
    sg.acf[l] = a;
  }
  if (blockIdx.x == 0) {
    __shared__ unsigned int cnt;
    if (threadIdx.x == 0) cnt = 0u;
    __syncthreads();
    unsigned int mine = 0u;
    for (int64_t tau = threadIdx.x; tau < sg.W; tau += 256) mine += sg.inv_norm[tau] > 0.0 ? 1u : 0u;
    atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) sg.acf[L] = (double)cnt;
  }
}

// Q(f) = R(0) + 2 sum_{l=1}^{L-1} R(l) cos(2 pi f l / N), f = 0 .. N/2.
__global__ __launch_bounds__(256) void k_qspec(const BatchHdr* __restrict__ hdr, int L, int N) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  if (!sg.zloc) return;
  __shared__ float ct[8192];
  for (int i = threadIdx.x; i < N; i += 256) {
    double sn, cs;
    sincospi(2.0 * (double)i / (double)N, &sn, &cs);
    ct[i] = (float)cs;
  }
  __syncthreads();
  const int f = (int)blockIdx.x * 256 + threadIdx.x;
  if (f > N / 2) return;
  const int lmax = L < N ? L : N;
  double q = sg.acf[0];
  int idx = 0;
  for (int l = 1; l < lmax; ++l) {
    idx += f;
    if (idx >= N) idx -= N;
    q = fma(2.0 * sg.acf[l], (double)ct[idx], q);
  }
  sg.qspec[f] = (float)q;
}

// Per series: redo = 1 if any exact threshold lies below its predicted lower threshold, or
// the candidates of a shard did not fit.
__global__ __launch_bounds__(256) void k_tails_check(const BatchHdr* __restrict__ hdr, BankDev b) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  if (!sg.redo) return;
  bool bad = false;
  const int64_t per = sg.cand_cap / CAND_SHARDS;
  if (blockIdx.x == 0 && threadIdx.x < CAND_SHARDS && (int64_t)sg.n_cand[threadIdx.x] > per)
    bad = true;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < b.K; k += stride)
    if (!(sg.thr[k] >= sg.thr_lo[k])) bad = true;
  if (bad) atomicOr(sg.redo, 1u);
}

// Per series not flagged: every candidate above its exact threshold is a tail.
__global__ __launch_bounds__(256) void k_tails_keep(const BatchHdr* __restrict__ hdr, BankDev b) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  if (!sg.redo || sg.redo[0] != 0u) return;
  const int64_t per = sg.cand_cap / CAND_SHARDS;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per * CAND_SHARDS;
       i += stride) {
    if ((unsigned long long)(i % per) >= sg.n_cand[i / per]) continue;
    const int32_t kl = sg.c_k[i];
    const float rf = sg.c_rho[i];
    if (fabsf(rf) > sg.thr[kl]) {
      const unsigned long long slot = atomicAdd(sg.n_tails, 1ull);
      if ((int64_t)slot < sg.tail_cap) {
        sg.t_tau[slot] = sg.c_tau[i];
        sg.t_k[slot] = (int32_t)(b.k_offset + kl);
        sg.t_rho[slot] = rf;
      }
      atomicAdd(sg.t_bins + kl / b.n_fdot, 1u);
    }
  }
}

}  // namespace

int pred_points(const BankDev& b) {
  if (b.precision == P_FFT) return 2 * b.fft_m;
  int n = 1024;
  while (n < 2 * b.L - 1 && n < 8192) n *= 2;
  return n;
}

hipError_t launch_acf(const BatchHdr* hdr, int32_t seg_slots, int L, hipStream_t s) {
  hipLaunchKernelGGL(k_zloc, dim3(256, (unsigned)seg_slots), dim3(256), 0, s, hdr, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_acf, dim3((unsigned)((L + 63) / 64), ACF_CHUNKS, (unsigned)seg_slots),
                     dim3(256), 0, s, hdr, L);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_acf_sum, dim3((unsigned)((L + 255) / 256), (unsigned)seg_slots),
                     dim3(256), 0, s, hdr, L);
  return hipGetLastError();
}

hipError_t launch_qspec(const BatchHdr* hdr, int32_t seg_slots, int L, int pred_n,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_qspec, dim3((unsigned)((pred_n / 2 + 1 + 255) / 256), (unsigned)seg_slots),
                     dim3(256), 0, s, hdr, L, pred_n);
  return hipGetLastError();
}

hipError_t launch_tails_check(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                              hipStream_t s) {
  const int64_t xb = (b.K + 255) / 256;
  hipLaunchKernelGGL(k_tails_check, dim3((unsigned)(xb < 1024 ? (xb > 0 ? xb : 1) : 1024), (unsigned)seg_slots),
                     dim3(256), 0, s, hdr, b);
  return hipGetLastError();
}

hipError_t launch_tails_keep(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_tails_keep, dim3(256, (unsigned)seg_slots), dim3(256), 0, s, hdr, b);
  return hipGetLastError();
}

}  // namespace bfly
