// FFT-correlation form of the search (Sec. 2.2 and the Fig. 5 caption: the paper computes
// the matched-filter correlations with FFTs on the GPU).
//
// Overlap-save with real FFTs of length N = 2M (a power of two >= 2L): block b of a series
// covers x[tau_b, tau_b + N) with tau_b = b (N - L + 1); the circular cross-correlation of a
// zero-padded template with the block equals the direct correlation d(tau_b + t, k) for
// t = 0 .. N - L.  Template spectra H_k (N/2 + 1 bins, float32) are made once at bank
// creation; each search transforms its data blocks once (X_b) and, per (block, template),
// forms C = conj(H_k) X_b, runs one inverse real FFT and reduces the N - L + 1 valid outputs
// straight from registers into the same butterfly output, spectrogram and spectrum as the
// direct contraction (same packed keys, same fixed-point sums, same finalisation).
//
// A real FFT of length N runs as a complex FFT of length M on z[n] = x[2n] + i x[2n+1]
// (even/odd split and the usual post-processing twiddles).  The complex FFT is a Stockham
// autosort FFT in LDS (M = 512 .. 4096): one work-group of M/8 threads per transform, radix-8
// passes after a first pass of radix 2, 4 or 8; each thread holds its butterflies in
// registers.  After the last inverse pass the thread keeps its 16 outputs in registers, at
// fixed positions for every template, so the running maxima never leave registers.
#include "bfly_internal.h"

#include <hip/hip_runtime.h>

#include <cstdlib>

namespace bfly {

namespace {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Complex product with fused multiply-adds: each component rounds once after one product.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// exp(+-2 pi i f) for a fraction f in [0, 1) given exactly (a dyadic rational).
template <bool INV>
__device__ __forceinline__ float2 cis_rev(float f) {
  float s, c;
  sincospif(2.0f * f, &s, &c);
  return make_float2(c, INV ? s : -s);
}

// cos and sin of 2 pi q / 16, q = 0..7.
__device__ constexpr float C16[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f,
                                     0.38268343236508978f, 0.0f, -0.38268343236508978f,
                                     -0.70710678118654752f, -0.92387953251128674f};
__device__ constexpr float S16[8] = {0.0f, 0.38268343236508978f, 0.70710678118654752f,
                                     0.92387953251128674f, 1.0f, 0.92387953251128674f,
                                     0.70710678118654752f, 0.38268343236508978f};

constexpr int bitrev(int i, int R) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// b * exp(-+2 pi i q / 16) for a compile-time q in 0..7: a quarter turn is a swap and a sign,
// an eighth turn two products by sqrt(1/2), the rest one complex product.
template <int Q, bool INV>
__device__ __forceinline__ float2 twiddle16(float2 b) {
  constexpr float R2 = 0.70710678118654752f;
  if constexpr (Q == 0) {
    return b;
  } else if constexpr (Q == 4) {
    return INV ? make_float2(-b.y, b.x) : make_float2(b.y, -b.x);
  } else if constexpr (Q == 2) {
    return INV ? make_float2((b.x - b.y) * R2, (b.x + b.y) * R2)
               : make_float2((b.x + b.y) * R2, (b.y - b.x) * R2);
  } else if constexpr (Q == 6) {
    return INV ? make_float2(-(b.x + b.y) * R2, (b.x - b.y) * R2)
               : make_float2((b.y - b.x) * R2, -(b.x + b.y) * R2);
  } else {
    return cmul(b, make_float2(C16[Q], INV ? S16[Q] : -S16[Q]));
  }
}

// twiddle16 for a q that is a constant after unrolling.
template <bool INV>
__device__ __forceinline__ float2 twiddle16_q(float2 b, int q) {
  switch (q) {
    case 0: return twiddle16<0, INV>(b);
    case 1: return twiddle16<1, INV>(b);
    case 2: return twiddle16<2, INV>(b);
    case 3: return twiddle16<3, INV>(b);
    case 4: return twiddle16<4, INV>(b);
    case 5: return twiddle16<5, INV>(b);
    case 6: return twiddle16<6, INV>(b);
    default: return twiddle16<7, INV>(b);
  }
}

// One radix-2 stage of span S (s in the DIT recursion) over t[], groups of S from offset G.
template <int R, int S, int G, int K, bool INV>
__device__ __forceinline__ void dft_bfly(float2 (&t)[R]) {
  if constexpr (K < S / 2) {
    const float2 a = t[G + K];
    const float2 b = twiddle16<K * (16 / S), INV>(t[G + K + S / 2]);
    t[G + K] = cadd(a, b);
    t[G + K + S / 2] = csub(a, b);
    dft_bfly<R, S, G, K + 1, INV>(t);
  }
}
template <int R, int S, int G, bool INV>
__device__ __forceinline__ void dft_stage(float2 (&t)[R]) {
  if constexpr (G < R) {
    dft_bfly<R, S, G, 0, INV>(t);
    dft_stage<R, S, G + S, INV>(t);
  }
}
template <int R, int S, bool INV>
__device__ __forceinline__ void dft_stages(float2 (&t)[R]) {
  if constexpr (S <= R) {
    dft_stage<R, S, 0, INV>(t);
    dft_stages<R, 2 * S, INV>(t);
  }
}

// In-register DFT of size R (2, 4, 8 or 16), natural order in and out: radix-2
// decimation in time after a bit-reversal permutation.
template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  float2 t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[bitrev(i, R)] = v[i];
  dft_stages<R, 2, INV>(t);
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = t[i];
}

// FFT plan for M points: T = M / 8 threads per work-group, P passes; the first pass has
// radix R0 = M / 8^(P-1) (Ns = 1, T or more butterflies per thread, no twiddles), every
// further pass is radix 8 with one butterfly per thread; the last pass leaves thread j with
// points j + T r, r < 8.  (512: 8 8 8; 1024: 2 8 8 8; 2048: 4 8 8 8; 4096: 8 8 8 8.)
template <int M> struct Plan {
  static constexpr int T = M / 8;
  static constexpr int P = M <= 512 ? 3 : 4;
  static constexpr int R0 = P == 3 ? M / 64 : M / 512;
};

// LDS index of FFT point i: one pad slot after every 8 points, so that the strided writes
// of the passes fall on distinct banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 3); }
template <int M> struct Padded { static constexpr int n = M + M / 8; };

// The twiddle base of a pass for butterfly j: exp(-+2 pi i (j mod Ns) / (Ns R)).
template <bool INV>
__device__ __forceinline__ float2 pass_twiddle(int j, int Ns, int R) {
  return cis_rev<INV>((float)(j & (Ns - 1)) / (float)(Ns * R));
}

// One Stockham pass of radix R over M points in LDS, sub-transform size Ns before the pass:
// butterfly j (< M/R) reads point j + r M/R, twiddles input r by w1^r (w1 = pass_twiddle of
// j), transforms, and writes point (j - j mod Ns) R + j mod Ns + r Ns.  Thread t runs
// butterflies t, t + T, ...  With KEEP the outputs stay in v and are not written back.
template <int M, int R, bool INV, bool KEEP>
__device__ __forceinline__ void fft_pass(float2* buf, int Ns, float2 w1,
                                         float2 (&v)[M / R / Plan<M>::T][R]) {
  constexpr int T = Plan<M>::T;
  constexpr int NB = M / R;
  constexpr int BPT = NB / T;
  static_assert(BPT >= 1 && NB % T == 0, "whole butterflies per thread");
#pragma unroll
  for (int t = 0; t < BPT; ++t) {
    const int j = threadIdx.x + t * T;
#pragma unroll
    for (int r = 0; r < R; ++r) v[t][r] = buf[pad(j + r * NB)];
    if (Ns > 1) {
      // w1^r as a running product (few live registers; at most R - 2 roundings)
      float2 w = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        v[t][r] = cmul(v[t][r], w);
        if (r + 1 < R) w = cmul(w, w1);
      }
    }
    dft<R, INV>(v[t]);
  }
  __syncthreads();
  if (!KEEP) {
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int j = threadIdx.x + t * T;
      const int jm = j & (Ns - 1);
      const int base = (j - jm) * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pad(base + r * Ns)] = v[t][r];
    }
    __syncthreads();
  }
}

// The thread's twiddle bases of passes 2..P.
template <int M, bool INV>
struct PassTw {
  float2 w[3];
  __device__ __forceinline__ void init() {
    int Ns = Plan<M>::R0;
#pragma unroll
    for (int p = 0; p < Plan<M>::P - 1; ++p) {
      w[p] = pass_twiddle<INV>(threadIdx.x, Ns, 8);
      Ns *= 8;
    }
  }
};

// Complex FFT of M points in buf (padded, natural order in).  All passes write buf when
// not KEEP; with KEEP the last pass leaves thread j with points j + T r in out[r].
template <int M, bool INV, bool KEEP>
__device__ __forceinline__ void fft_run(float2* buf, const PassTw<M, INV>& tw,
                                        float2 (&out)[8]) {
  constexpr int R0 = Plan<M>::R0;
  float2 v0[M / R0 / Plan<M>::T][R0];
  fft_pass<M, R0, INV, false>(buf, 1, make_float2(1.0f, 0.0f), v0);
  float2 v[1][8];
  int Ns = R0;
#pragma unroll
  for (int p = 0; p < Plan<M>::P - 2; ++p) {
    fft_pass<M, 8, INV, false>(buf, Ns, tw.w[p], v);
    Ns *= 8;
  }
  fft_pass<M, 8, INV, KEEP>(buf, Ns, tw.w[Plan<M>::P - 2], v);
#pragma unroll
  for (int r = 0; r < 8; ++r) out[r] = v[0][r];
}

// Forward real FFT of N = 2M real samples staged as z[n] = (x[2n], x[2n+1]) in buf:
// writes X[k], k = 0..M, to dst (global).
template <int M>
__device__ __forceinline__ void rfft_post(float2* buf, float2* __restrict__ dst) {
  float2 out[8];
  PassTw<M, false> tw;
  tw.init();
  fft_run<M, false, false>(buf, tw, out);
  for (int k = threadIdx.x; k <= M; k += Plan<M>::T) {
    const float2 zk = buf[pad(k & (M - 1))];
    const float2 zc = cconj(buf[pad((M - k) & (M - 1))]);
    const float2 e = cscale(cadd(zk, zc), 0.5f);
    const float2 d = cscale(csub(zk, zc), 0.5f);
    const float2 o = make_float2(d.y, -d.x);                     // d / i
    const float2 w = cis_rev<false>((float)k / (float)(2 * M));   // exp(-2 pi i k / N)
    dst[k] = cadd(e, cmul(w, o));
  }
}

// Sum of a 64-bit integer over the 64 lanes of a wave, in every lane.  Within each row of 16
// lanes by DPP (swap neighbours, swap pairs, mirror each half row, mirror the row), which
// leaves every lane of a row holding the row's sum; the four rows are then added from one
// lane each.  No LDS round trips (a shuffle chain takes six dependent ones).  Integer sums
// do not depend on the order, so the result equals any other reduction's.
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xF, 0xF, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long lane_u64(unsigned long long v, int lane) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  v += dpp_u64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_u64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_u64<0x141>(v);   // row_half_mirror
  v += dpp_u64<0x140>(v);   // row_mirror
  return (lane_u64(v, 15) + lane_u64(v, 31)) + (lane_u64(v, 47) + lane_u64(v, 63));
}

// The sum of a float over the wave in a fixed order (pairs, quads, half rows, rows, then the
// four rows), the same in every lane: a + b = b + a exactly, so the partners of each step
// hold equal values.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_sum_f32(float v) {
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  v += dpp_f32<0x141>(v);
  v += dpp_f32<0x140>(v);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 15));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 31));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 47));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  return (r0 + r1) + (r2 + r3);
}

// One template sample in float64, with the same formula as the direct bank:
// cos(2 pi frac(f0 t + fdot t^2 / 2)), t = n / fs.
__device__ __forceinline__ double template_sample(double fs, double f0, double fdot, int n) {
  const double t = (double)n / fs;
  double phi = f0 * t + 0.5 * fdot * (t * t);
  phi = phi - floor(phi);
  return cos(2.0 * 3.141592653589793 * phi);
}

// Sum over the work-group's threads (NW waves of 64).
template <int NW>
__device__ __forceinline__ double block_sum_d(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += red[w];
  return t;
}

// Bank spectra: one work-group per template builds the zero-mean unit-norm template in
// float64, rounds it to float32 and stores its real-FFT spectrum (row stride M + 2).
template <int M>
__global__ __launch_bounds__(Plan<M>::T) void k_fft_bank(GridDev g, BankDev b,
                                                          float2* spectra, unsigned int* bad) {
  constexpr int T = Plan<M>::T;
  __shared__ float2 buf[Padded<M>::n];
  __shared__ double red[T / 64];
  const int64_t k = blockIdx.x;
  const bool real = k < b.K;
  double f0 = 0.0, fdot = 0.0, mu = 0.0, nrm = 1.0;
  if (real) {
    const int64_t il = k / g.n_fdot;
    const int j = (int)(k % g.n_fdot);
    const int64_t ig = g.f0_lo + il;
    f0 = (g.n_f0 > 1 && ig == g.n_f0 - 1) ? g.f0_max : (double)ig * g.f0_step + g.f0_min;
    fdot = (g.n_fdot > 1 && j == g.n_fdot - 1) ? g.fdot_max
                                               : (double)j * g.fdot_step + g.fdot_min;
    double s1 = 0.0;
    for (int n = threadIdx.x; n < b.L; n += T) s1 += template_sample(g.fs, f0, fdot, n);
    mu = block_sum_d<T / 64>(s1, red) / (double)b.L;
    double s2 = 0.0;
    for (int n = threadIdx.x; n < b.L; n += T) {
      const double v = template_sample(g.fs, f0, fdot, n) - mu;
      s2 += v * v;
    }
    s2 = block_sum_d<T / 64>(s2, red);
    nrm = sqrt(s2);
    if (!(s2 > 1e-18 * (double)b.L)) {
      if (threadIdx.x == 0) atomicAdd(bad, 1u);
      nrm = 1.0;
    }
  }
  for (int n = threadIdx.x; n < M; n += T) {
    float2 z = make_float2(0.0f, 0.0f);
    if (real && 2 * n < b.L) z.x = (float)((template_sample(g.fs, f0, fdot, 2 * n) - mu) / nrm);
    if (real && 2 * n + 1 < b.L)
      z.y = (float)((template_sample(g.fs, f0, fdot, 2 * n + 1) - mu) / nrm);
    buf[pad(n)] = z;
  }
  __syncthreads();
  rfft_post<M>(buf, spectra + k * (int64_t)(M + 2));
}

// ---- single-pass tail search: predicted lower thresholds ---------------------------------
// thr_lo[k] = kappa * margin * sqrt(P_k / (n_ok N)), P_k = sum over f in [0, N) of
// |H_k(f)|^2 Q(f) (Q from k_qspec, real and even: the bins 1 .. N/2 - 1 count twice), or +inf
// past the bank's templates and for a series without a non-degenerate offset.

__device__ __forceinline__ void pred_store(const SegDesc& sg, int64_t k, const BankDev& b,
                                           double P, int N, float kappa, float margin) {
  const double nok = sg.acf[b.L];
  float v = __builtin_inff();
  if (k < b.K && nok > 0.0) v = (float)((double)kappa * (double)margin * sqrt(P / (nok * (double)N)));
  sg.thr_lo[k] = v;
}

// The FFT form: the spectra are the bank's (N = 2M); one wave per template, NS series per
// sweep of its spectrum.  Every load of a sweep is unconditional (a series without Q reads
// the bank's first row instead, and its sum is dropped), so a lane issues its PRED_U bins'
// loads of the spectrum and of every Q before it waits for any.
template <int NS>
__global__ __launch_bounds__(256) void k_pred_bank(const BatchHdr* __restrict__ hdr, BankDev b,
                                                   float kappa, float margin) {
  typedef const __attribute__((address_space(1))) float* gfloat;
  constexpr int PRED_U = 5;
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= b.K_pad) return;
  const int M = b.fft_m, N = 2 * b.fft_m;
  const float2* hk = (const float2*)b.data + k * (int64_t)(M + 2);
  const SegDesc* segs = hdr_segs(hdr);
  const int n_segs = hdr->n_segs;
  for (int s0 = 0; s0 < n_segs; s0 += NS) {
    gfloat qs[NS];
    bool use[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const float* q = s0 + i < n_segs ? segs[s0 + i].qspec : nullptr;
      use[i] = q && segs[s0 + i].thr_lo;
      qs[i] = (gfloat)(q ? q : (const float*)b.data);
    }
    double P[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) P[i] = 0.0;
    for (int f0 = lane; f0 <= M; f0 += 64 * PRED_U) {
      float2 h[PRED_U];
      float qv[PRED_U][NS];
#pragma unroll
      for (int u = 0; u < PRED_U; ++u) {
        const int f = f0 + 64 * u;
        // bins past M read bin M and get weight 0 below; the spectra hold K_pad rows (the
        // sums of rows past K are dropped)
        const int fc = f <= M ? f : M;
        h[u] = hk[fc];
#pragma unroll
        for (int i = 0; i < NS; ++i) qv[u][i] = qs[i][fc];
      }
#pragma unroll
      for (int u = 0; u < PRED_U; ++u) {
        const int f = f0 + 64 * u;
        const double w = f > M ? 0.0 : (f == 0 || f == M) ? 1.0 : 2.0;
        const double h2 = w * ((double)h[u].x * h[u].x + (double)h[u].y * h[u].y);
#pragma unroll
        for (int i = 0; i < NS; ++i) P[i] += h2 * (double)qv[u][i];
      }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      double v = P[i];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0 && use[i]) pred_store(segs[s0 + i], k, b, v, N, kappa, margin);
    }
  }
}

constexpr int PRED_SERIES = 8;   // series per sweep of a template's spectrum

// The direct forms: one work-group per template builds it as the FFT bank does (float64,
// rounded to float32), transforms it on N = 2M points, and sums |H|^2 Q for every series.
template <int M>
__global__ __launch_bounds__(Plan<M>::T) void k_pred_gen(const BatchHdr* __restrict__ hdr,
                                                         GridDev g, BankDev b, float kappa,
                                                         float margin) {
  constexpr int T = Plan<M>::T;
  __shared__ float2 buf[Padded<M>::n];
  __shared__ double red[T / 64];
  const int64_t k = blockIdx.x;
  const bool real = k < b.K;
  double f0 = 0.0, fdot = 0.0, mu = 0.0, nrm = 1.0;
  if (real) {
    const int64_t il = k / g.n_fdot;
    const int j = (int)(k % g.n_fdot);
    const int64_t ig = g.f0_lo + il;
    f0 = (g.n_f0 > 1 && ig == g.n_f0 - 1) ? g.f0_max : (double)ig * g.f0_step + g.f0_min;
    fdot = (g.n_fdot > 1 && j == g.n_fdot - 1) ? g.fdot_max
                                               : (double)j * g.fdot_step + g.fdot_min;
    double s1 = 0.0;
    for (int n = threadIdx.x; n < b.L; n += T) s1 += template_sample(g.fs, f0, fdot, n);
    mu = block_sum_d<T / 64>(s1, red) / (double)b.L;
    double s2 = 0.0;
    for (int n = threadIdx.x; n < b.L; n += T) {
      const double v = template_sample(g.fs, f0, fdot, n) - mu;
      s2 += v * v;
    }
    s2 = block_sum_d<T / 64>(s2, red);
    nrm = s2 > 0.0 ? sqrt(s2) : 1.0;
  }
  // taps past 2M alias onto the transform (only when L > 2M; a prediction, checked later)
  for (int n = threadIdx.x; n < M; n += T) {
    float2 z = make_float2(0.0f, 0.0f);
    for (int q = 2 * n; q < b.L && real; q += 2 * M) {
      z.x += (float)((template_sample(g.fs, f0, fdot, q) - mu) / nrm);
      if (q + 1 < b.L) z.y += (float)((template_sample(g.fs, f0, fdot, q + 1) - mu) / nrm);
    }
    buf[pad(n)] = z;
  }
  __syncthreads();
  float2 out[8];
  PassTw<M, false> tw;
  tw.init();
  fft_run<M, false, false>(buf, tw, out);
  const SegDesc* segs = hdr_segs(hdr);
  for (int s0 = 0; s0 < hdr->n_segs; s0 += PRED_SERIES) {
    double P[PRED_SERIES];
#pragma unroll
    for (int i = 0; i < PRED_SERIES; ++i) P[i] = 0.0;
    for (int kk = threadIdx.x; kk <= M; kk += T) {
      // X[kk] from the complex transform (the post-processing of rfft_post)
      const float2 zk = buf[pad(kk & (M - 1))];
      const float2 zc = cconj(buf[pad((M - kk) & (M - 1))]);
      const float2 e = cscale(cadd(zk, zc), 0.5f);
      const float2 d = cscale(csub(zk, zc), 0.5f);
      const float2 o = make_float2(d.y, -d.x);
      const float2 w = cis_rev<false>((float)kk / (float)(2 * M));
      const float2 X = cadd(e, cmul(w, o));
      const double wt = (kk == 0 || kk == M) ? 1.0 : 2.0;
      const double h2 = wt * ((double)X.x * X.x + (double)X.y * X.y);
#pragma unroll
      for (int i = 0; i < PRED_SERIES; ++i)
        if (s0 + i < hdr->n_segs && segs[s0 + i].qspec) P[i] += h2 * (double)segs[s0 + i].qspec[kk];
    }
#pragma unroll
    for (int i = 0; i < PRED_SERIES; ++i) {
      const double v = block_sum_d<T / 64>(P[i], red);
      if (threadIdx.x == 0 && s0 + i < hdr->n_segs && segs[s0 + i].thr_lo)
        pred_store(segs[s0 + i], k, b, v, 2 * M, kappa, margin);
    }
  }
}

// Data spectra: one work-group per (series, block) tile, persistent over the batch's tiles.
template <int M>
__global__ __launch_bounds__(Plan<M>::T) void k_fft_data(const BatchHdr* __restrict__ hdr,
                                                          BankDev b) {
  constexpr int T = Plan<M>::T;
  __shared__ float2 buf[Padded<M>::n];
  const SegDesc* segs = hdr_segs(hdr);
  const int64_t n_tiles = hdr->total_tiles;
  const int valid = 2 * M - b.L + 1;
  for (int64_t tt = blockIdx.x; tt < n_tiles; tt += gridDim.x) {
    int lo = 0, hi = hdr->n_segs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].tile0 <= tt) lo = mid; else hi = mid - 1;
    }
    const SegDesc& sg = segs[lo];
    const int64_t tau0 = (tt - sg.tile0) * valid;
    // x - c0 (see series_offset); padding past the end and non-finite samples stage as 0, so
    // a constant level does not enter the block's norm and with it the transform's rounding
    const float c0 = series_offset(sg);
    auto xs = [&](int64_t gi) -> float {
      if (gi >= sg.n) return 0.0f;
      const float v = sg.x[gi];
      return isfinite(v) ? v - c0 : 0.0f;
    };
    for (int n = threadIdx.x; n < M; n += T) {
      const int64_t i0 = tau0 + 2 * n;
      buf[pad(n)] = make_float2(xs(i0), xs(i0 + 1));
    }
    __syncthreads();
    rfft_post<M>(buf, sg.xspec + (tt - sg.tile0) * (int64_t)(M + 2));
    __syncthreads();
  }
}

// Position within the block of a thread's real output o: point j + T r of the inverse
// transform holds outputs 2 (j + T r) (real part) and 2 (j + T r) + 1 (imaginary part),
// o = 2 r + part.
template <int M>
__device__ __forceinline__ int out_pos(int o) {
  return 2 * ((int)threadIdx.x + Plan<M>::T * (o >> 1)) + (o & 1);
}

// Spectrogram / spectrum flush of one f0 bin for this thread's 16 outputs (bit o of vmask:
// output o is a valid offset of the series).
template <int M>
__device__ __forceinline__ void fft_flush(const SegDesc& sg, const SearchDev& p, int bin,
                                          const float (&binmax)[16], int tau_base,
                                          unsigned vmask, float scale) {
  unsigned long long fix = 0ull;
#pragma unroll
  for (int o = 0; o < 16; ++o) {
    if (vmask & (1u << o)) {
      const int tau = tau_base + out_pos<M>(o);
      const double inv = sg.inv_norm[tau];
      if (inv > 0.0) {
        const float s = (float)((double)(binmax[o] * scale) * inv);
        if (sg.spec) {
          const int row = p.t_block == 1 ? tau : tau / p.t_block;
          const int64_t at = (int64_t)bin * sg.spec_rows + row;
          if (p.t_block == 1)
            sg.spec[at] = s;
          else
            atomicMax((unsigned int*)sg.spec + at, __float_as_uint(s));
        }
        fix += (unsigned long long)__double2ll_rn((double)s * SPEC_FIX_SCALE);
      }
    }
  }
  fix = wave_sum_u64(fix);
  if ((threadIdx.x & 63) == 0 && fix != 0ull) atomicAdd(sg.spec_acc + bin, fix);
}

// The search: work item = (series, block, range of whole f0 bins), numbered range-fastest;
// persistent over the batch's items.  Per template of the range: C = conj(H_k) X_b, the
// inverse real FFT, and the running reductions of the thread's 16 outputs.  The next
// template's spectrum is loaded into registers while the current one is transformed.
// OCC: waves per SIMD the register allocation targets (2: no spills in the template loop;
// 4: two work-groups per CU at M = 4096, some spills).
// MODE (MainMode): the search; the pass that sums rho^2 per template (fixed point, one
// atomic per wave and template); the pass that appends every valid (tau, k) with
// |rho| > kappa sigma_k and counts it per bin.  rho = f32(d / sqrt(E)) as in the direct
// forms' tail passes.
template <int M, int OCC, int MODE>
__global__ __launch_bounds__(Plan<M>::T, OCC) void k_fft_main(const BatchHdr* __restrict__ hdr,
                                                            BankDev b, SearchDev p) {
  constexpr int T = Plan<M>::T;
  constexpr int NP = (M / 2 + T) / T;   // spectrum pairs per thread (M / 2 + 1 pairs)
  static_assert(T * 16 == 2 * M, "pairs are T apart: twiddles step by 1/16 of a turn");
  __shared__ float2 xs[M + 2];
  __shared__ float2 buf[Padded<M>::n];
  const SegDesc* segs = hdr_segs(hdr);
  const float2* spectra = (const float2*)b.data;
  const int n_ranges = hdr->n_ranges;
  const int64_t n_items = hdr->n_items;
  const int valid = 2 * M - b.L + 1;
  const int tid = threadIdx.x;
  // 1/M of the inverse transform, times the 1/2 of the even/odd split (applied to the
  // outputs: both are powers of two, so moving them changes no rounding)
  const float scale = 0.5f / (float)M;
  const int nfd = b.n_fdot;

  // per-thread constants: the post-processing twiddle exp(+2 pi i p / N) of pair
  // p = tid + q T is wb * exp(2 pi i q / 16); the inverse passes' twiddle bases
  const float2 wb = cis_rev<true>((float)tid / (float)(2 * M));
  PassTw<M, true> tw;
  tw.init();

  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int rg = (int)(item % n_ranges);
    const int64_t tt = item / n_ranges;
    int lo = 0, hi = hdr->n_segs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].tile0 <= tt) lo = mid; else hi = mid - 1;
    }
    const SegDesc& sg = segs[lo];
    if (MODE == MODE_TAILS && sg.redo && sg.redo[0] == 0u) continue;   // see k_fft4k
    const int64_t blk = tt - sg.tile0;
    const int tau_base = (int)(blk * valid);     // series are shorter than 2^31 samples
    const int b_lo = (int)((int64_t)rg * b.n_bins / n_ranges);
    const int b_hi = (int)((int64_t)(rg + 1) * b.n_bins / n_ranges);
    const float2* xsrc = sg.xspec + blk * (int64_t)(M + 2);
    for (int k = tid; k <= M; k += T) xs[k] = xsrc[k];
    unsigned vmask = 0u;
#pragma unroll
    for (int o = 0; o < 16; ++o)
      if (out_pos<M>(o) < valid && (int64_t)tau_base + out_pos<M>(o) < sg.W) vmask |= 1u << o;

    float best[16], binmax[16];
    int bestk[16];
    float inv[16];     // sigma and tails passes: 1/sqrt(E) of the outputs (0 if not valid)
#pragma unroll
    for (int o = 0; o < 16; ++o) {
      if constexpr (MODE == MODE_SEARCH) {
        best[o] = -1.0f;
        bestk[o] = -1;
        binmax[o] = 0.0f;
      } else {
        inv[o] = (vmask & (1u << o)) ? (float)sg.inv_norm[tau_base + out_pos<M>(o)] : 0.0f;
      }
    }
    const int k_lo = b_lo * nfd, k_hi = b_hi * nfd;
    // spectrum pairs (p, M - p) of the current template, loaded ahead
    float2 h1[NP], h2[NP];
    {
      const float2* hk = spectra + (int64_t)k_lo * (M + 2);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int pp = tid + q * T;
        if (pp <= M / 2) {
          h1[q] = hk[pp];
          h2[q] = hk[M - pp];
        }
      }
    }
    __syncthreads();   // xs filled
    int bin = b_lo, left = nfd;
    for (int k = k_lo; k < k_hi; ++k) {
      // Y[p] and Y[M - p] from C = conj(H) X at bins p and M - p
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int pp = tid + q * T;
        if (pp <= M / 2) {
          const int p2 = M - pp;
          const float2 c1 = cmul(cconj(h1[q]), xs[pp]);
          const float2 c2 = cmul(cconj(h2[q]), xs[p2]);
          // twice E and O (the 1/2 is in `scale`)
          const float2 e = cadd(c1, cconj(c2));
          const float2 d = csub(c1, cconj(c2));
          const float2 w = q == 0 ? wb : cmul(wb, make_float2(C16[q], S16[q]));
          const float2 o = cmul(d, w);
          buf[pad(pp)] = make_float2(e.x - o.y, e.y + o.x);                 // E + iO
          if (pp != 0 && pp != M / 2) buf[pad(p2)] = make_float2(e.x + o.y, o.x - e.y);  // E* + iO*
        }
      }
      if (k + 1 < k_hi) {
        const float2* hk = spectra + (int64_t)(k + 1) * (M + 2);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int pp = tid + q * T;
          if (pp <= M / 2) {
            h1[q] = hk[pp];
            h2[q] = hk[M - pp];
          }
        }
      }
      __syncthreads();
      float2 y[8];
      fft_run<M, true, true>(buf, tw, y);
      if constexpr (MODE == MODE_SIGMA) {
        float q = 0.0f;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const float r0 = (float)((double)(y[r].x * scale) * (double)inv[2 * r]);
          const float r1 = (float)((double)(y[r].y * scale) * (double)inv[2 * r + 1]);
          q = fmaf(r0, r0, q);
          q = fmaf(r1, r1, q);
        }
        unsigned long long f = (unsigned long long)__double2ll_rn((double)q * SIGMA_FIX_SCALE);
        f = wave_sum_u64(f);
        if ((tid & 63) == 0 && f != 0ull) atomicAdd(sg.sig_acc + k, f);
        continue;
      }
      if constexpr (MODE == MODE_TAILS) {
        const float thr = sg.thr[k];
#pragma unroll
        for (int o = 0; o < 16; ++o) {
          const float v = (o & 1) ? y[o >> 1].y : y[o >> 1].x;
          const float rf = (float)((double)(v * scale) * (double)inv[o]);
          if (fabsf(rf) > thr) {
            const unsigned long long slot = atomicAdd(sg.n_tails, 1ull);
            if ((int64_t)slot < sg.tail_cap) {
              sg.t_tau[slot] = tau_base + out_pos<M>(o);
              sg.t_k[slot] = (int32_t)(b.k_offset + k);
              sg.t_rho[slot] = rf;
            }
            atomicAdd(sg.t_bins + k / nfd, 1u);
          }
        }
        continue;
      }
      // running maxima over the templates, lowest k on ties (k increases, strict >)
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const float a0 = fabsf(y[r].x), a1 = fabsf(y[r].y);
        const bool g0 = a0 > best[2 * r], g1 = a1 > best[2 * r + 1];
        best[2 * r] = g0 ? a0 : best[2 * r];
        bestk[2 * r] = g0 ? k : bestk[2 * r];
        best[2 * r + 1] = g1 ? a1 : best[2 * r + 1];
        bestk[2 * r + 1] = g1 ? k : bestk[2 * r + 1];
        binmax[2 * r] = fmaxf(binmax[2 * r], a0);
        binmax[2 * r + 1] = fmaxf(binmax[2 * r + 1], a1);
      }
      if (--left == 0) {
        fft_flush<M>(sg, p, bin, binmax, tau_base, vmask, scale);
#pragma unroll
        for (int o = 0; o < 16; ++o) binmax[o] = 0.0f;
        ++bin;
        left = nfd;
      }
    }
    // per-offset maxima: one packed atomic per valid output (value first, then lower k)
#pragma unroll
    for (int o = 0; o < 16; ++o) {
      const int tau = tau_base + out_pos<M>(o);
      if (MODE == MODE_SEARCH && (vmask & (1u << o)) && bestk[o] >= 0) {
        const unsigned int kg = (unsigned int)(b.k_offset + bestk[o]);
        const unsigned long long key =
            ((unsigned long long)__float_as_uint(best[o] * scale) << 32) |
            (0xFFFFFFFFull - kg);
        atomicMax(sg.mkey + tau, key);
      }
    }
    __syncthreads();   // xs is refilled by the next item
  }
}

// ---------------------------------------------------------------------------------------
// The search kernel at M = 4096 (real FFTs of N = 8192 points; the length the planner picks
// for templates of roughly 1,500 to 4,096 taps).  One transform per work-group of 256
// threads (one wave per SIMD), 16 points per thread, two work-groups per CU:
// * The thread owns inverse-FFT butterflies j0 = t and j1 = 512 - t of the first radix-8
//   pass, whose points j + 512 r are closed under the mirror p -> M - p of the real-FFT
//   post-processing.  It keeps the data spectrum X_b at those points in registers for the
//   whole work item, loads H_k at the same points (the next template's while the current
//   one is transformed), and forms Y = E + iO and the first pass's radix-8 DFTs in registers:
//   the spectrum product never goes through LDS.  (Thread 0's butterflies, 0 and 256, are
//   each their own mirror; lanes 0..3 of wave 0 form butterfly 256's four pairs and hand the
//   values to thread 0 through LDS.)
// * Passes 2..4 run two radix-8 butterflies per thread with their twiddle powers held in
//   registers, ping-ponging between two LDS buffers: three barriers per template.
// * The last pass leaves the thread 16 complex outputs = 32 real outputs at offsets
//   2t + 512 s + part (s < 16); only the first SMAX slots can hold valid offsets
//   (SMAX >= (2M - L + 1) / 512).  Per output the thread keeps the running maximum over the
//   current f0 bin and the template reaching it; at the end of a bin it writes the
//   spectrogram row, adds to the spectrum sums and merges (bin maximum, template) into the
//   per-offset packed maxima with one atomic max each.  That is the same merge as the other
//   forms (value first, then the lower template), so the results do not depend on how the
//   bank is split into bins and ranges.
// The sigma and tails modes are those of k_fft_main.  The single-pass mode also forms rho in
// the same sweep as the maxima: per template each wave sums rho^2 over its lanes' outputs
// (float32 in a fixed order, then fixed point), marks the sum (bit 63) when one of its
// correlations is above the template's kept bound, and stores it to its own row of the
// series' partial sums; the bin's argmax is kept as 16-bit template offsets, two to a
// register, to stay within 256 registers.
namespace fft4k {
constexpr int M = 4096;
constexpr int PADN = M + M / 8;   // the largest stage layout (SH = 3)
// stage layouts: first pass -> second (S1), second -> third (S2), third -> fourth (S3).
// Measured on the light-curve share: (5, 3, 0) 229-230 ms per search, (4, 3, 0) 230-231,
// (3, 3, 0) 235, (3, 3, 3) 233-235.
constexpr int S1 = 5, S2 = 3, S3 = 0;
constexpr unsigned ROW_BYTES = (M + 2) * 8;   // one spectrum row (bins 0..M, padded)
}  // namespace fft4k

// A buffer resource on one spectrum row: the loads below address it with a 32-bit per-lane
// byte offset and a uniform (SGPR) byte offset, so a row needs no per-lane 64-bit address
// arithmetic; reads past the row return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float2* row) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(row), (short)0,
                                           (int)fft4k::ROW_BYTES, 0x00020000);
}
__device__ __forceinline__ float2 row_load(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                           unsigned soff) {
  const float re = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  const float im =
      __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff + 4u, soff, 0));
  return make_float2(re, im);
}

// The spectrum product and the inverse real-FFT post-processing of one mirror pair
// (a, M - a): from C1 = conj(H[a]) X[a] and C2 = conj(H[M - a]) X[M - a], with
// w = exp(+2 pi i a / N), Y[a] = E + iO and Y[M - a] = E* + iO* (both twice their value;
// the 1/2 is in the output scale).
__device__ __forceinline__ void mirror_pair(float2 ha, float2 xa, float2 hb, float2 xb,
                                            float2 w, float2& ya, float2& yb) {
  const float2 c1 = cmul(cconj(ha), xa);
  const float2 c2 = cmul(cconj(hb), xb);
  const float2 e = cadd(c1, cconj(c2));
  const float2 d = csub(c1, cconj(c2));
  const float2 o = cmul(d, w);
  ya = make_float2(e.x - o.y, e.y + o.x);
  yb = make_float2(e.x + o.y, o.x - e.y);
}

// LDS layouts of the M = 4096 transform: element i of a stage's buffer sits at
// i + (i >> SH) (one pad slot per 2^SH elements; SH = 0: no padding).  Each stage's layout
// suits its writer and its reader: the first pass writes 8 consecutive points per thread
// (lanes 8 elements apart), the second writes runs of 8 points 64 apart, the third
// contiguous runs; every pass reads contiguous runs.  Padding every 8 spreads the first two
// write patterns over all banks but makes each 32-lane read of a contiguous run wrap onto
// banks it already used; contiguous writes and reads need no padding at all.
template <int SH>
__device__ __forceinline__ int padk(int i) { return SH ? i + (i >> SH) : i; }

// One radix-8 Stockham pass of two butterflies (t and t + 256) from `src` (layout SP) to
// `dst` (layout DP) with sub-transform size NS before the pass; input r of butterfly t is
// twiddled by wa[r - 1] and of butterfly t + 256 by wb[r - 1].  KEEP leaves the outputs in
// y0, y1 instead of writing them.
template <int NS, bool KEEP, int SP, int DP>
__device__ __forceinline__ void pass8x2(const float2* __restrict__ src, float2* __restrict__ dst,
                                        const float2 (&wa)[7], const float2 (&wb)[7],
                                        float2 (&y0)[8], float2 (&y1)[8]) {
  const int t = threadIdx.x;
  // 512 r and 256 are multiples of 2^SP: padk(t + 512 r) = padk(t) + padk(512 r), and
  // padk(t + 256 + 512 r) = padk(t) + padk(256) + padk(512 r)
  constexpr int R1 = SP ? 512 + (512 >> SP) : 512;
  constexpr int HALF = SP ? 256 + (256 >> SP) : 256;
  const float2* rd = src + padk<SP>(t);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    y0[r] = rd[R1 * r];
    y1[r] = rd[HALF + R1 * r];
  }
#pragma unroll
  for (int r = 1; r < 8; ++r) {
    y0[r] = cmul(y0[r], wa[r - 1]);
    y1[r] = cmul(y1[r], wb[r - 1]);
  }
  dft<8, true>(y0);
  dft<8, true>(y1);
  if constexpr (!KEEP) {
    // output r of butterfly j goes to point o + r NS, o = (j - j mod NS) 8 + j mod NS; NS is a
    // multiple of 2^DP, so padk(o + r NS) = padk(o) + r padk(NS)
    static_assert(DP == 0 || NS % (1 << DP) == 0, "stride must keep the pad phase");
    constexpr int RS = DP ? NS + (NS >> DP) : NS;
    const int m0 = t & (NS - 1), m1 = (t + 256) & (NS - 1);
    float2* w0 = dst + padk<DP>((t - m0) * 8 + m0);
    float2* w1 = dst + padk<DP>((t + 256 - m1) * 8 + m1);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      w0[r * RS] = y0[r];
      w1[r * RS] = y1[r];
    }
  }
}

// A store through a global (not generic) pointer: a generic store also counts on the LDS
// counter, so the LDS reads issued after it would wait for the store to reach memory.
template <typename T>
__device__ __forceinline__ void global_store(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// Running maximum with its argument kept in one 16-bit half of a register: where |v| > m,
// m = |v| and half HI of arg = the low half of rel (the other half is kept).  Three
// instructions: the compare, the select of m, and a select whose sub-dword operands and
// destination (SDWA) replace only the chosen half.  A comparison with a NaN is false, as in
// the plain C form (a = |v|; if (a > m) { m = a; arg.half = rel; }).
template <int HI>
__device__ __forceinline__ void max_arg16(float v, float& m, unsigned& arg, unsigned rel) {
  if constexpr (HI)
    asm("v_cmp_gt_f32_e64 vcc, |%2|, %0\n\t"
        "v_cndmask_b32_e64 %0, %0, |%2|, vcc\n\t"
        "v_cndmask_b32_sdwa %1, %1, %3, vcc dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE "
        "src0_sel:WORD_1 src1_sel:WORD_0"
        : "+v"(m), "+v"(arg) : "v"(v), "v"(rel) : "vcc");
  else
    asm("v_cmp_gt_f32_e64 vcc, |%2|, %0\n\t"
        "v_cndmask_b32_e64 %0, %0, |%2|, vcc\n\t"
        "v_cndmask_b32_sdwa %1, %1, %3, vcc dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE "
        "src0_sel:WORD_0 src1_sel:WORD_0"
        : "+v"(m), "+v"(arg) : "v"(v), "v"(rel) : "vcc");
}

// The lane's index in its wave, formed where it is used: the volatile keeps the compiler
// from hoisting it out of a loop, where it (or an address made from it) would hold a
// register across the whole loop or be spilled and reloaded.
__device__ __forceinline__ int lane_here() {
  int l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0" : "=v"(l));
  return l;
}

template <int SMAX, int MODE>
__global__ __launch_bounds__(256, 2) void k_fft4k(const BatchHdr* __restrict__ hdr, BankDev b,
                                                  SearchDev p) {
  using namespace fft4k;
  static_assert(SMAX >= 1 && SMAX <= 16, "output slots");
  constexpr int NO = 2 * SMAX;          // real outputs per thread that can be valid
  __shared__ float2 lds[2 * PADN];
  __shared__ float2 hand[8];            // butterfly 256's first-pass inputs for thread 0
  __shared__ float2 hand_x[8];          // X_b at the helpers' pairs
  // twiddle powers of passes 2 and 3, w^r = exp(2 pi i (j mod NS) r / (8 NS)) for
  // j mod NS = m: entry [(r - 1) NS + m] (lanes read consecutive entries)
  __shared__ float2 tab2[7 * 8];
  __shared__ float2 tab3[7 * 64];
  const SegDesc* segs = hdr_segs(hdr);
  const float2* spectra = (const float2*)b.data;
  const int n_ranges = hdr->n_ranges;
  const int64_t n_items = hdr->n_items;
  const int valid = 2 * M - b.L + 1;
  const int t = threadIdx.x;
  const float scale = 0.5f / (float)M;
  const int nfd = b.n_fdot;

  // first-pass butterflies j0 = t and j1 = 512 - t (thread 0: 0, and 256 handed over);
  // pair r = (a_r, M - a_r) with a_r = t + 512 r; its post-processing twiddle
  // LEAN forms the pair twiddles and pass 4's twiddle powers per template instead of keeping
  // them in registers (for builds short of registers; off in every mode compiled now).
  constexpr bool LEAN = false;
  const float2 wt = cis_rev<true>((float)t / (float)(2 * M));   // wpair[r] = wt exp(2 pi i r/16)
  float2 wpair[LEAN ? 1 : 8];
  if constexpr (!LEAN) {
#pragma unroll
    for (int r = 0; r < 8; ++r) wpair[r] = cis_rev<true>((float)(t + 512 * r) / (float)(2 * M));
  }
  // lanes 0..3 of wave 0: pair (256 + 512 t, M - 256 - 512 t) of butterfly 256
  const bool helper = t < 4;
  const int ha_idx = 256 + 512 * (t & 3);
  const float2 whelp = cis_rev<true>((float)ha_idx / (float)(2 * M));
  const int j1w = t == 0 ? 256 : 512 - t;   // butterfly written from v1
  // twiddle powers: passes 2 (NS = 8) and 3 (NS = 64) from the LDS tables, pass 4 (NS = 512,
  // butterflies t and t + 256) in registers
  for (int i = t; i < 7 * 64; i += 256) {
    const int r = i / 64 + 1, m = i % 64;
    tab3[i] = cis_rev<true>((float)((m * r) & 511) / 512.0f);
    if (i < 7 * 8) {
      const int r2 = i / 8 + 1, m2 = i % 8;
      tab2[i] = cis_rev<true>((float)((m2 * r2) & 63) / 64.0f);
    }
  }
  float2 tw4a[LEAN ? 1 : 7], tw4b[LEAN ? 1 : 7];
  if constexpr (LEAN) {
    tw4a[0] = cis_rev<true>((float)t / 4096.0f);
    tw4b[0] = cis_rev<true>((float)(t + 256) / 4096.0f);
  } else {
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      tw4a[r - 1] = cis_rev<true>((float)((t * r) & 4095) / 4096.0f);
      tw4b[r - 1] = cis_rev<true>((float)(((t + 256) * r) & 4095) / 4096.0f);
    }
  }
  __syncthreads();

  // Pass 1 of a template writes bufp, pass 2 reads it and writes bufq, pass 3 writes bufp
  // back, pass 4 reads it; then the two swap.  The pass-1 buffer was last read in a pass 3,
  // before that template's third barrier, so the swapping runs on across work items (a
  // reset per item would let an item's first pass-1 writes meet the previous item's last
  // pass-4 reads when an item has an odd number of templates).  The buffers follow the
  // parity of a uniform template count, so no buffer pointer is carried in a VGPR.
  unsigned it = 0;
  const int64_t total_tiles = hdr->total_tiles;
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    // Work-group i runs on XCD i mod 8 and each XCD takes its work-groups in order of i / 8.
    // With 8m ranges, XCD x sweeps its ranges x, x + 8, ... one after another, blocks
    // fastest, so the work-groups resident on an XCD sweep one range's spectra in step and
    // share them through its L2; with other counts, range fastest.
    int rg;
    int64_t tt;
    if (n_ranges % 8 == 0) {
      const int64_t j = item / 8;
      rg = (int)(item % 8) + 8 * (int)(j / total_tiles);
      tt = j % total_tiles;
    } else {
      rg = (int)(item % n_ranges);
      tt = item / n_ranges;
    }
    int lo = 0, hi = hdr->n_segs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].tile0 <= tt) lo = mid; else hi = mid - 1;
    }
    const SegDesc& sg = segs[lo];
    // after a single-pass search the tails pass runs only for series whose prediction failed
    if (MODE == MODE_TAILS && sg.redo && sg.redo[0] == 0u) continue;
    const int64_t blk = tt - sg.tile0;
    const int tau_base = (int)(blk * valid);     // series are shorter than 2^31 samples
    const int b_lo = (int)((int64_t)rg * b.n_bins / n_ranges);
    const int b_hi = (int)((int64_t)(rg + 1) * b.n_bins / n_ranges);
    const float2* xsrc = sg.xspec + blk * (int64_t)(M + 2);
    // bins a_r = t + 512 r at byte 8t + 4096 r; bins M - a_r at 8 (512 - t) + 4096 (7 - r)
    const unsigned va = 8u * (unsigned)t, vb = 8u * (512u - (unsigned)t);
    float2 xa[8], xb[8];
    {
      const __amdgpu_buffer_rsrc_t xr = row_rsrc(xsrc);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        xa[r] = row_load(xr, va, 4096u * r);
        xb[r] = row_load(xr, vb, 4096u * (7 - r));
      }
    }
    // X at the helpers' pairs, kept in LDS (read by the helper lanes only)
    if (helper) {
      hand_x[2 * t] = xsrc[ha_idx];
      hand_x[2 * t + 1] = xsrc[M - ha_idx];
    }
    // output o = 2 s + part sits at block position 2t + 512 s + part; it is a valid offset of
    // the series below this bound
    const int pos_end = (int)min((int64_t)valid, sg.W - (int64_t)tau_base);
    // The single pass keeps the bin's argmax as 1 + (k - the bin's first template), two
    // outputs to a register (0: none yet), to stay within 256 registers with sinv below.
    constexpr bool PACK = MODE == MODE_ONEPASS;
    float binmax[NO];
    int binarg[PACK ? 1 : NO];
    unsigned barg2[PACK ? (NO + 1) / 2 : 1];
    // sigma, tails and single-pass modes: scale / sqrt(E) with 1/sqrt(E) rounded to float
    // (0 if invalid); scale is a power of two, so y sinv = (y scale) (1/sqrt(E))_f32 exactly
    float sinv[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      if constexpr (MODE == MODE_SEARCH || MODE == MODE_ONEPASS) {
        binmax[o] = -1.0f;
        if constexpr (PACK) {
          if ((o & 1) == 0) barg2[o >> 1] = 0u;
        } else {
          binarg[o] = -1;
        }
      }
      if constexpr (MODE != MODE_SEARCH) {
        const int pos = 2 * t + 512 * (o >> 1) + (o & 1);
        sinv[o] = pos < pos_end ? scale * (float)sg.inv_norm[tau_base + pos] : 0.0f;
      }
    }
    const int k_lo = b_lo * nfd, k_hi = b_hi * nfd;
    float2 ha[8], hb[8], hha = make_float2(0.0f, 0.0f), hhb = hha;
    auto load_h = [&](int k) {
      const float2* hk = spectra + (int64_t)k * (M + 2);
      const __amdgpu_buffer_rsrc_t hr = row_rsrc(hk);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        ha[r] = row_load(hr, va, 4096u * r);
        hb[r] = row_load(hr, vb, 4096u * (7 - r));
      }
      // every lane loads the helpers' pair (only lanes 0..3 of wave 0 use it): a load under
      // a lane condition would make the prefetch wait at the join
      hha = row_load(hr, 8u * (unsigned)ha_idx, 0u);
      hhb = row_load(hr, 8u * (unsigned)(M - ha_idx), 0u);
    };
    load_h(k_lo);
    // sigma and single-pass modes: this block's four rows of per-wave rho^2 sums, read once
    // per work item (no scalar load in flight during the template loop: one returns out of
    // order, which makes every LDS wait of a pass wait for all of its reads)
    [[maybe_unused]] unsigned long long* sig_row = nullptr;
    if constexpr (MODE == MODE_SIGMA || MODE == MODE_ONEPASS)
      if (sg.sig_part)
        sig_row = sg.sig_part + (blk * 4 + __builtin_amdgcn_readfirstlane(t >> 6)) * b.K_pad;
    // the single pass's kept bounds: a vector load one template ahead, on the same counter
    // as the spectrum prefetch (a scalar load would be waited for with the LDS reads)
    [[maybe_unused]] __amdgpu_buffer_rsrc_t thr_r;
    [[maybe_unused]] float tlo_next = 0.0f;
    if constexpr (MODE == MODE_ONEPASS) {
      const int64_t bytes = (int64_t)(k_hi - k_lo) * 4;
      thr_r = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(sg.thr_lo + k_lo), (short)0,
                                                (int)(bytes < 0x7FFFFFF0 ? bytes : 0x7FFFFFF0),
                                                0x00020000);
      tlo_next = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(thr_r, 0u, 0u, 0));
    }
    int bin = b_lo, left = nfd;
    for (int k = k_lo; k < k_hi; ++k, ++it) {
      float2* const bufp = lds + (it & 1u) * PADN;
      float2* const bufq = lds + ((it + 1u) & 1u) * PADN;
      [[maybe_unused]] const float tlo = tlo_next;
      // ---- spectrum product, post-processing and the first radix-8 pass, in registers
      float2 v0[8], v1[8];
#pragma unroll
      for (int r = 0; r < 8; ++r)
        mirror_pair(ha[r], xa[r], hb[r], xb[r],
                    LEAN ? twiddle16_q<true>(wt, r) : wpair[LEAN ? 0 : r], v0[r], v1[7 - r]);
      if (helper) {
        // the helpers are lanes 0..3 of wave 0, so t is their lane index
        const int h = lane_here();
        float2 ya, yb;
        mirror_pair(hha, hand_x[2 * h], hhb, hand_x[2 * h + 1], whelp, ya, yb);
        hand[h] = ya;
        hand[7 - h] = yb;
      }
      if constexpr (MODE == MODE_ONEPASS)
        tlo_next = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                 thr_r, 0u, 4u * (unsigned)(min(k + 1, k_hi - 1) - k_lo), 0));
      load_h(min(k + 1, k_hi - 1));   // unconditional (the last one repeats a row)
      if (t == 0) {
        // the helpers are lanes of this wave: their LDS writes precede these reads
#pragma unroll
        for (int r = 0; r < 8; ++r) v1[r] = hand[r];
      }
      dft<8, true>(v0);
      dft<8, true>(v1);
      // point 8 j + r of the first pass's output at padk<S1>(8 j + r) = padk<S1>(8 j) + r
      float2* w0 = bufp + padk<S1>(8 * t);
      float2* w1 = bufp + padk<S1>(8 * j1w);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        w0[r] = v0[r];
        w1[r] = v1[r];
      }
      __syncthreads();
      float2 y0[8], y1[8];
      {
        float2 w[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) w[r] = tab2[8 * r + (t & 7)];
        pass8x2<8, false, S1, S2>(bufp, bufq, w, w, y0, y1);
      }
      __syncthreads();
      {
        float2 w[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) w[r] = tab3[64 * r + (t & 63)];
        pass8x2<64, false, S2, S3>(bufq, bufp, w, w, y0, y1);
      }
      __syncthreads();
      if constexpr (LEAN) {
        // pass 4's twiddle powers as running products of the bases
        float2 wa[7], wb[7];
        wa[0] = tw4a[0];
        wb[0] = tw4b[0];
#pragma unroll
        for (int r = 1; r < 7; ++r) {
          wa[r] = cmul(wa[r - 1], tw4a[0]);
          wb[r] = cmul(wb[r - 1], tw4b[0]);
        }
        pass8x2<512, true, S3, 0>(bufp, bufq, wa, wb, y0, y1);
      } else {
        pass8x2<512, true, S3, 0>(bufp, bufq, tw4a, tw4b, y0, y1);
      }
      // output slot o = 2 s + part: s even -> y0[s / 2], s odd -> y1[s / 2]
      auto outv = [&](int o) -> float {
        const int s = o >> 1;
        const float2 c = (s & 1) ? y1[s >> 1] : y0[s >> 1];
        return (o & 1) ? c.y : c.x;
      };
      // rho = f32(d / sqrt(E)): y sinv is exact in float64 (a product of two floats), so one
      // float32 multiply rounds it exactly as the float64 route would
      if constexpr (MODE == MODE_SIGMA || MODE == MODE_ONEPASS) {
        float q = 0.0f;
        float mr = 0.0f;   // the largest |rho| of the lane (single pass)
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          const float v = outv(o);
          const float rr = v * sinv[o];
          q = fmaf(rr, rr, q);
          if constexpr (MODE == MODE_ONEPASS) {
            mr = fmaxf(mr, fabsf(rr));
            // the running maximum of the search (below), in the same sweep; the low (even o)
            // or high (odd o) half of the register takes rel1 where |v| is a new maximum
            const unsigned rel1 = (unsigned)(k - bin * nfd + 1);
            if (o & 1)
              max_arg16<1>(v, binmax[o], barg2[o >> 1], rel1);
            else
              max_arg16<0>(v, binmax[o], barg2[o >> 1], rel1);
          }
        }
        // the wave's float sum in a fixed order, then fixed point (order-independent across
        // waves, blocks and the atomic route)
        unsigned long long f =
            (unsigned long long)__double2ll_rn((double)wave_sum_f32(q) * SIGMA_FIX_SCALE);
        // single pass: bit 63 of the wave's sum (free: the sums stay below 2^63) flags a
        // correlation above the kept bound in this wave
        if constexpr (MODE == MODE_ONEPASS)
          if (__any(mr > tlo)) f |= SIG_FLAG;
        // each wave stores its own sum (no cross-wave step, so no wave waits for another)
        if ((t & 63) == 0) {
          if (sig_row)
            global_store(sig_row + k, f);
          else if (f != 0ull)
            atomicAdd(sg.sig_acc + k, f);
        }
        if constexpr (MODE == MODE_SIGMA) continue;
      }
      if constexpr (MODE == MODE_TAILS) {
        const float thr = sg.thr[k];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          const float rf = outv(o) * sinv[o];
          if (fabsf(rf) > thr) {
            const unsigned long long slot = atomicAdd(sg.n_tails, 1ull);
            if ((int64_t)slot < sg.tail_cap) {
              sg.t_tau[slot] = tau_base + 2 * t + 512 * (o >> 1) + (o & 1);
              sg.t_k[slot] = (int32_t)(b.k_offset + k);
              sg.t_rho[slot] = rf;
            }
            atomicAdd(sg.t_bins + k / nfd, 1u);
          }
        }
        continue;
      }
      // running maximum over the bin's templates, lowest k on ties (k increases, strict >)
      if constexpr (MODE == MODE_SEARCH) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          const float a = fabsf(outv(o));
          const bool g = a > binmax[o];
          binarg[o] = g ? k : binarg[o];
          binmax[o] = g ? a : binmax[o];
        }
      }
      if (--left == 0) {
        // end of bin: spectrogram row, spectrum sum, packed per-offset maxima
        unsigned long long fix = 0ull;
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          const int pos = 2 * t + 512 * (o >> 1) + (o & 1);
          int ba;
          if constexpr (PACK) {
            const unsigned r1 = (barg2[o >> 1] >> (16 * (o & 1))) & 0xFFFFu;
            ba = r1 ? bin * nfd + (int)r1 - 1 : -1;
          } else {
            ba = binarg[o];
          }
          if (pos < pos_end && ba >= 0) {
            const int tau = tau_base + pos;
            const float v = binmax[o] * scale;
            const double iv = sg.inv_norm[tau];
            if (iv > 0.0) {
              const float s = (float)((double)v * iv);
              if (sg.spec) {
                const int row = p.t_block == 1 ? tau : tau / p.t_block;
                const int64_t at = (int64_t)bin * sg.spec_rows + row;
                if (p.t_block == 1)
                  sg.spec[at] = s;
                else
                  atomicMax((unsigned int*)sg.spec + at, __float_as_uint(s));
              }
              fix += (unsigned long long)__double2ll_rn((double)s * SPEC_FIX_SCALE);
            }
            const unsigned int kg = (unsigned int)(b.k_offset + ba);
            atomicMax(sg.mkey + tau,
                      ((unsigned long long)__float_as_uint(v) << 32) | (0xFFFFFFFFull - kg));
          }
          binmax[o] = -1.0f;
          if constexpr (PACK) {
            if (o & 1) barg2[o >> 1] = 0u;   // after both outputs of the register
          } else {
            binarg[o] = -1;
          }
        }
        fix = wave_sum_u64(fix);
        if ((t & 63) == 0 && fix != 0ull) atomicAdd(sg.spec_acc + bin, fix);
        ++bin;
        left = nfd;
      }
    }
  }
}

// The tails of the (block, template) pairs the single pass of k_fft4k listed, for every
// series whose check passed (redo = 0; a flagged series gets the full tails pass instead).
// Per pair the transform of k_fft4k with the same operations in the same order, so rho is
// the same bit for bit, then the compare against kappa sigma_k.  Work unit = (series, shard
// of the pair list); a work-group takes a shard's pairs one after another.  Two work-groups
// per CU: within 256 registers only the block change (a few times per shard) reloads spilled
// values.
template <int SMAX>
__global__ __launch_bounds__(256, 2) void k_fft4k_pairs(const BatchHdr* __restrict__ hdr,
                                                        BankDev b) {
  using namespace fft4k;
  constexpr int NO = 2 * SMAX;
  __shared__ float2 lds[2 * PADN];
  __shared__ float2 hand[8];
  __shared__ float2 hand_x[8];
  __shared__ float2 tab2[7 * 8];
  __shared__ float2 tab3[7 * 64];
  const SegDesc* segs = hdr_segs(hdr);
  const float2* spectra = (const float2*)b.data;
  const int valid = 2 * M - b.L + 1;
  const int t = threadIdx.x;
  const float scale = 0.5f / (float)M;
  const int nfd = b.n_fdot;
  float2 wpair[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) wpair[r] = cis_rev<true>((float)(t + 512 * r) / (float)(2 * M));
  const bool helper = t < 4;
  const int ha_idx = 256 + 512 * (t & 3);
  const float2 whelp = cis_rev<true>((float)ha_idx / (float)(2 * M));
  const int j1w = t == 0 ? 256 : 512 - t;
  for (int i = t; i < 7 * 64; i += 256) {
    const int r = i / 64 + 1, m = i % 64;
    tab3[i] = cis_rev<true>((float)((m * r) & 511) / 512.0f);
    if (i < 7 * 8) {
      const int r2 = i / 8 + 1, m2 = i % 8;
      tab2[i] = cis_rev<true>((float)((m2 * r2) & 63) / 64.0f);
    }
  }
  float2 tw4a[7], tw4b[7];
#pragma unroll
  for (int r = 1; r < 8; ++r) {
    tw4a[r - 1] = cis_rev<true>((float)((t * r) & 4095) / 4096.0f);
    tw4b[r - 1] = cis_rev<true>((float)(((t + 256) * r) & 4095) / 4096.0f);
  }
  __syncthreads();

  const unsigned va = 8u * (unsigned)t, vb = 8u * (512u - (unsigned)t);
  unsigned it = 0;   // pairs so far: the LDS buffers alternate as in k_fft4k
  const int n_units = hdr->n_segs * CAND_SHARDS;
  for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
    const SegDesc& sg = segs[unit / CAND_SHARDS];
    if (!sg.redo || sg.redo[0] != 0u || !sg.c_tau) continue;
    const int shard = unit % CAND_SHARDS;
    const int64_t per = sg.cand_cap / CAND_SHARDS;
    const int64_t n = min((int64_t)sg.n_cand[shard], per);
    if (n <= 0) continue;
    // A shard's pairs come in runs of one block (a work-group appends the pairs of its
    // current block), so the block's spectrum and scales are reloaded only when the block
    // changes; the next pair's template spectrum is loaded while the current one transforms.
    const int64_t e0 = shard * per;
    int64_t blk_n = sg.c_tau[e0];
    int k_n = sg.c_k[e0];
    float2 ha[8], hb[8], hha, hhb;
    auto load_h = [&](int k) {
      const __amdgpu_buffer_rsrc_t hr = row_rsrc(spectra + (int64_t)k * (M + 2));
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        ha[r] = row_load(hr, va, 4096u * r);
        hb[r] = row_load(hr, vb, 4096u * (7 - r));
      }
      hha = row_load(hr, 8u * (unsigned)ha_idx, 0u);
      hhb = row_load(hr, 8u * (unsigned)(M - ha_idx), 0u);
    };
    load_h(k_n);
    int64_t cur_blk = -1;
    int tau_base = 0;
    float2 xa[8], xb[8];
    float sinv[NO];
    for (int64_t j = 0; j < n; ++j, ++it) {
      const int64_t blk = blk_n;
      const int k = k_n;
      if (blk != cur_blk) {
        cur_blk = blk;
        tau_base = (int)(blk * valid);
        const float2* xsrc = sg.xspec + blk * (int64_t)(M + 2);
        const __amdgpu_buffer_rsrc_t xr = row_rsrc(xsrc);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          xa[r] = row_load(xr, va, 4096u * r);
          xb[r] = row_load(xr, vb, 4096u * (7 - r));
        }
        if (helper) {
          hand_x[2 * t] = xsrc[ha_idx];
          hand_x[2 * t + 1] = xsrc[M - ha_idx];
        }
        // the scales k_fft4k forms: scale / sqrt(E) with 1/sqrt(E) rounded to float
        const int pos_end = (int)min((int64_t)valid, sg.W - (int64_t)tau_base);
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          const int pos = 2 * t + 512 * (o >> 1) + (o & 1);
          sinv[o] = pos < pos_end ? scale * (float)sg.inv_norm[tau_base + pos] : 0.0f;
        }
      }
      float2* const bufp = lds + (it & 1u) * PADN;
      float2* const bufq = lds + ((it + 1u) & 1u) * PADN;
      float2 v0[8], v1[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) mirror_pair(ha[r], xa[r], hb[r], xb[r], wpair[r], v0[r], v1[7 - r]);
      if (helper) {
        float2 ya, yb;
        mirror_pair(hha, hand_x[2 * t], hhb, hand_x[2 * t + 1], whelp, ya, yb);
        hand[t] = ya;
        hand[7 - t] = yb;
      }
      if (j + 1 < n) {
        blk_n = sg.c_tau[e0 + j + 1];
        k_n = sg.c_k[e0 + j + 1];
      }
      load_h(k_n);   // unconditional (the last one repeats a row)
      if (t == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) v1[r] = hand[r];
      }
      dft<8, true>(v0);
      dft<8, true>(v1);
      {
        float2* w0 = bufp + padk<S1>(8 * t);
        float2* w1 = bufp + padk<S1>(8 * j1w);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          w0[r] = v0[r];
          w1[r] = v1[r];
        }
      }
      __syncthreads();
      float2 y0[8], y1[8];
      {
        float2 w[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) w[r] = tab2[8 * r + (t & 7)];
        pass8x2<8, false, S1, S2>(bufp, bufq, w, w, y0, y1);
      }
      __syncthreads();
      {
        float2 w[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) w[r] = tab3[64 * r + (t & 63)];
        pass8x2<64, false, S2, S3>(bufq, bufp, w, w, y0, y1);
      }
      __syncthreads();
      pass8x2<512, true, S3, 0>(bufp, bufq, tw4a, tw4b, y0, y1);
      const float thr = sg.thr[k];
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        const int s = o >> 1;
        const float2 c = (s & 1) ? y1[s >> 1] : y0[s >> 1];
        const float rf = ((o & 1) ? c.y : c.x) * sinv[o];
        if (fabsf(rf) > thr) {
          const unsigned long long slot = atomicAdd(sg.n_tails, 1ull);
          if ((int64_t)slot < sg.tail_cap) {
            sg.t_tau[slot] = tau_base + 2 * t + 512 * s + (o & 1);
            sg.t_k[slot] = (int32_t)(b.k_offset + k);
            sg.t_rho[slot] = rf;
          }
          atomicAdd(sg.t_bins + k / nfd, 1u);
        }
      }
    }
  }
}

// Output slots of the M = 4096 kernel for valid = 2M - L + 1 offsets per block.
inline int fft4k_slots(const BankDev& b) {
  const int need = (2 * 4096 - b.L + 1 + 511) / 512;
  return need <= 9 ? 9 : need <= 13 ? 13 : 16;
}

// BF_FFT_V1=1 runs the M = 4096 searches on k_fft_main instead (a comparison knob; the
// results agree to the float32 bound, not bit for bit).
bool fft4k_enabled() {
  static const bool on = [] {
    const char* e = getenv("BF_FFT_V1");
    return !(e && e[0] == '1');
  }();
  return on;
}

}  // namespace

bool fft_onepass_available(const BankDev& b) {
  return b.fft_m == 4096 && fft4k_enabled() && b.n_fdot < 65535;
}

namespace {

// The single pass's list of (block, template) pairs holding a correlation above the kept
// bound: the pairs with the flag bit in any of their four wave sums.  Shard s takes the
// 64-template groups g with g mod 256 = s, block by block, so a shard's pairs come in runs
// of one block (k_fft4k_pairs reloads a block's spectrum only when the block changes), the
// shards share the flagged templates evenly wherever they cluster, and the list is the same
// on every run.  A shard's count may exceed its capacity (k_tails_check then flags the
// series).  One work-group per (shard, series).
__global__ __launch_bounds__(256) void k_fft_pair_list(const BatchHdr* __restrict__ hdr,
                                                       BankDev b) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  if (!sg.redo || !sg.sig_part || !sg.n_cand || !sg.c_tau) return;
  __shared__ unsigned int cnt[4];
  const int shard = (int)blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t per = sg.cand_cap / CAND_SHARDS;
  const int64_t n_groups = b.K_pad / 64;
  int64_t n = 0;
  for (int64_t blk = 0; blk < sg.n_tiles; ++blk) {
    const unsigned long long* rows = sg.sig_part + blk * 4 * b.K_pad;
    for (int64_t g0 = shard; g0 < n_groups; g0 += 4 * CAND_SHARDS) {
      const int64_t g = g0 + (int64_t)w * CAND_SHARDS;
      const int64_t k = g * 64 + lane;
      bool fl = false;
      // the pass writes the sums of the bank's templates only (k < K); the padding rows'
      // words are whatever the workspace held
      if (g < n_groups && k < b.K)
        fl = ((rows[k] | rows[b.K_pad + k] | rows[2 * b.K_pad + k] | rows[3 * b.K_pad + k]) &
              SIG_FLAG) != 0ull;
      const unsigned long long bal = __ballot(fl);
      if (lane == 0) cnt[w] = (unsigned int)__popcll(bal);
      __syncthreads();
      int64_t at = n;
      for (int i = 0; i < w; ++i) at += cnt[i];
      at += __popcll(bal & ((1ull << lane) - 1ull));
      if (fl && at < per) {
        sg.c_tau[shard * per + at] = (int32_t)blk;
        sg.c_k[shard * per + at] = (int32_t)k;
      }
      n += (int64_t)cnt[0] + cnt[1] + cnt[2] + cnt[3];
      __syncthreads();
    }
  }
  if (t == 0) sg.n_cand[shard] = (unsigned long long)n;
}

}  // namespace

hipError_t launch_fft_pair_list(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_fft_pair_list, dim3(CAND_SHARDS, (unsigned)seg_slots), dim3(256), 0, s,
                     hdr, b);
  return hipGetLastError();
}

hipError_t launch_fft_pairs(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                            hipStream_t s) {
  const unsigned grid = (unsigned)std::min<int64_t>((int64_t)seg_slots * CAND_SHARDS, 512);
  switch (fft4k_slots(b)) {
    case 9:
      hipLaunchKernelGGL(k_fft4k_pairs<9>, dim3(grid), dim3(256), 0, s, hdr, b);
      break;
    case 13:
      hipLaunchKernelGGL(k_fft4k_pairs<13>, dim3(grid), dim3(256), 0, s, hdr, b);
      break;
    default:
      hipLaunchKernelGGL(k_fft4k_pairs<16>, dim3(grid), dim3(256), 0, s, hdr, b);
      break;
  }
  return hipGetLastError();
}

namespace {

template <int MODE>
hipError_t launch_fft4k(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                        const SearchDev& p, hipStream_t s) {
  switch (fft4k_slots(b)) {
    case 9:
      hipLaunchKernelGGL((k_fft4k<9, MODE>), dim3((unsigned)blocks), dim3(256), 0, s, hdr, b, p);
      break;
    case 13:
      hipLaunchKernelGGL((k_fft4k<13, MODE>), dim3((unsigned)blocks), dim3(256), 0, s, hdr, b, p);
      break;
    default:
      hipLaunchKernelGGL((k_fft4k<16, MODE>), dim3((unsigned)blocks), dim3(256), 0, s, hdr, b, p);
      break;
  }
  return hipGetLastError();
}

// Register target of the search kernel: BF_FFT_OCC=4 selects the 4-waves-per-SIMD build
// (a tuning knob; results do not depend on it), else 2.
int fft_occupancy() {
  static const int occ = [] {
    const char* e = getenv("BF_FFT_OCC");
    return (e && e[0] == '4') ? 4 : 2;
  }();
  return occ;
}

template <int M>
hipError_t launch_fft_bank_t(const GridDev& g, const BankDev& b, void* dst, unsigned* bad,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_fft_bank<M>, dim3((unsigned)b.K_pad), dim3(Plan<M>::T), 0, s, g, b,
                     (float2*)dst, bad);
  return hipGetLastError();
}

template <int M>
hipError_t launch_fft_search_t(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                               const SearchDev& p, hipStream_t s) {
  hipLaunchKernelGGL(k_fft_data<M>, dim3((unsigned)blocks), dim3(Plan<M>::T), 0, s, hdr, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (M == 4096 && fft4k_enabled()) {
    if (p.mode == MODE_ONEPASS) return launch_fft4k<MODE_ONEPASS>(hdr, blocks, b, p, s);
    return launch_fft4k<MODE_SEARCH>(hdr, blocks, b, p, s);
  }
  if (p.mode != MODE_SEARCH) return hipErrorInvalidValue;
  if (fft_occupancy() == 4)
    hipLaunchKernelGGL((k_fft_main<M, 4, MODE_SEARCH>), dim3((unsigned)blocks),
                       dim3(Plan<M>::T), 0, s, hdr, b, p);
  else
    hipLaunchKernelGGL((k_fft_main<M, 2, MODE_SEARCH>), dim3((unsigned)blocks),
                       dim3(Plan<M>::T), 0, s, hdr, b, p);
  return hipGetLastError();
}

// The sigma or tails pass (p.mode) over the data spectra the search left in the workspace.
template <int M>
hipError_t launch_fft_pass_t(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                             const SearchDev& p, hipStream_t s) {
  if (M == 4096 && fft4k_enabled()) {
    if (p.mode == MODE_SIGMA) return launch_fft4k<MODE_SIGMA>(hdr, blocks, b, p, s);
    if (p.mode == MODE_TAILS) return launch_fft4k<MODE_TAILS>(hdr, blocks, b, p, s);
    return hipErrorInvalidValue;
  }
  if (p.mode == MODE_SIGMA)
    hipLaunchKernelGGL((k_fft_main<M, 2, MODE_SIGMA>), dim3((unsigned)blocks),
                       dim3(Plan<M>::T), 0, s, hdr, b, p);
  else if (p.mode == MODE_TAILS)
    hipLaunchKernelGGL((k_fft_main<M, 2, MODE_TAILS>), dim3((unsigned)blocks),
                       dim3(Plan<M>::T), 0, s, hdr, b, p);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

#define BFLY_FFT_DISPATCH(FN, ...)                      \
  do {                                                  \
    switch (b.fft_m) {                                  \
      case 512: return FN<512>(__VA_ARGS__);            \
      case 1024: return FN<1024>(__VA_ARGS__);          \
      case 2048: return FN<2048>(__VA_ARGS__);          \
      case 4096: return FN<4096>(__VA_ARGS__);          \
      default: return hipErrorInvalidValue;             \
    }                                                   \
  } while (0)

hipError_t launch_fft_bank(const GridDev& g, const BankDev& b, void* dst, hipStream_t s) {
  unsigned int* bad = (unsigned int*)((char*)dst + bank_data_bytes(b));
  hipError_t e = hipMemsetAsync(bad, 0, 256, s);
  if (e != hipSuccess) return e;
  BFLY_FFT_DISPATCH(launch_fft_bank_t, g, b, dst, bad, s);
}

hipError_t launch_fft_search(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                             const SearchDev& p, hipStream_t s) {
  if (blocks < 1) return hipSuccess;
  BFLY_FFT_DISPATCH(launch_fft_search_t, hdr, blocks, b, p, s);
}

hipError_t launch_fft_pass(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                           const SearchDev& p, hipStream_t s) {
  if (blocks < 1) return hipSuccess;
  BFLY_FFT_DISPATCH(launch_fft_pass_t, hdr, blocks, b, p, s);
}

int contraction_wgs_per_cu(const BankDev& b) {
  if (b.precision != P_FFT) return 1;
  if (b.fft_m == 4096 && fft4k_enabled()) return 2;        // k_fft4k: 2 x 4 waves
  const int waves = 4 * fft_occupancy();                    // k_fft_main: waves per CU
  const int wg_waves = std::max(1, b.fft_m / 512);          // M / 8 threads per work-group
  return std::max(1, waves / std::max(1, wg_waves));
}

hipError_t launch_pred(const BatchHdr* hdr, int32_t seg_slots, const GridDev& g,
                       const BankDev& b, float kappa, float margin, hipStream_t s) {
  if (b.precision == P_FFT) {
    const dim3 grid((unsigned)((b.K_pad + 3) / 4));
    if (seg_slots <= 1)
      hipLaunchKernelGGL(k_pred_bank<1>, grid, dim3(256), 0, s, hdr, b, kappa, margin);
    else if (seg_slots <= 2)
      hipLaunchKernelGGL(k_pred_bank<2>, grid, dim3(256), 0, s, hdr, b, kappa, margin);
    else if (seg_slots <= 4)
      hipLaunchKernelGGL(k_pred_bank<4>, grid, dim3(256), 0, s, hdr, b, kappa, margin);
    else
      hipLaunchKernelGGL(k_pred_bank<8>, grid, dim3(256), 0, s, hdr, b, kappa, margin);
    return hipGetLastError();
  }
  const unsigned blocks = (unsigned)b.K_pad;
  switch (pred_points(b) / 2) {
    case 512:
      hipLaunchKernelGGL(k_pred_gen<512>, dim3(blocks), dim3(Plan<512>::T), 0, s, hdr, g, b, kappa, margin);
      break;
    case 1024:
      hipLaunchKernelGGL(k_pred_gen<1024>, dim3(blocks), dim3(Plan<1024>::T), 0, s, hdr, g, b, kappa, margin);
      break;
    case 2048:
      hipLaunchKernelGGL(k_pred_gen<2048>, dim3(blocks), dim3(Plan<2048>::T), 0, s, hdr, g, b, kappa, margin);
      break;
    default:
      hipLaunchKernelGGL(k_pred_gen<4096>, dim3(blocks), dim3(Plan<4096>::T), 0, s, hdr, g, b, kappa, margin);
      break;
  }
  return hipGetLastError();
}

}  // namespace bfly
