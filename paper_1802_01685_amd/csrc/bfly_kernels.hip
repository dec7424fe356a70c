// HIP kernels of the butterfly-filtering search, written for gfx950 (MI355X).
//
//   k_bank_gen   float64 chirp templates -> quantised bank in the MFMA operand layout
//   k_zero       clears the running maxima, spectrogram, spectrum sums and histograms
//   k_prefix     float64 (double-double) prefix sums of x and x^2, non-finite counts
//   k_norms      per-window energies from the prefix sums -> 1/sqrt(E), degenerate flags
//   k_main       the template x window contraction on MFMA with the reductions fused in
//   k_finalize   butterfly output, histogram of maxima, spectrum
//
// Matched filtering of a series against a bank of chirps (Sec. 2.1) is, for every offset
// tau and template k, d(tau,k) = sum_n h_k[n] x[tau+n]: a GEMM with M = templates,
// N = offsets, K = taps, whose N x K operand is the Hankel matrix X[n][tau] = x[tau+n].
// k_main keeps a strip of the series in LDS and builds every Hankel operand fragment from
// it, streams the templates from HBM in a layout that lets each lane load its MFMA operand
// with 16-byte loads, and never stores d: the per-offset maximum/argmax (the butterfly
// output, Fig. 2) and the per-f0-bin maximum (the chirp spectrogram, Sec. 2.1) are reduced
// in registers as each template tile completes.
#include "bfly_internal.h"

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bfly {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------------------
// Small numeric helpers.
// ---------------------------------------------------------------------------------------

// float -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// double rounded to bf16 precision (8 significant bits), nearest even, kept as a double.
__device__ __forceinline__ double round_bf16_d(double h) {
  unsigned long long u = (unsigned long long)__double_as_longlong(h);
  u = u + ((1ull << 44) - 1ull) + ((u >> 45) & 1ull);
  u &= ~((1ull << 45) - 1ull);
  return __longlong_as_double((long long)u);
}

struct dd {
  double hi, lo;
};

// Double-double sum (Knuth two-sum of the leading parts, then renormalised).
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  double s = a.hi + b.hi;
  double bb = s - a.hi;
  double e = (a.hi - (s - bb)) + (b.hi - bb);
  e += a.lo + b.lo;
  double hi = s + e;
  double lo = e - (hi - s);
  return {hi, lo};
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}

// OCP e2m3 (fp6): sign, 2 exponent bits (bias 1), 3 mantissa bits; max 7.5, subnormal step
// 1/8.  Round to nearest even of |v| <= 7.5: below 1 the code is rint(8 |v|) (8 is the first
// normal, 1.0); from 1 on, exponent e = floor(log2 |v|) and mantissa rint(8 (|v| 2^-e - 1)),
// a mantissa of 8 carrying into the exponent field.  Every step but rint is exact.
__device__ __forceinline__ uint32_t enc_e2m3(float v) {
  const float a = fabsf(v);
  uint32_t code;
  if (a < 1.0f) {
    code = (uint32_t)rintf(a * 8.0f);
  } else {
    const int e = (int)((__float_as_uint(a) >> 23) & 0xFF) - 127;   // 0, 1 or 2
    code = (uint32_t)((e + 1) << 3) + (uint32_t)rintf((ldexpf(a, -e) - 1.0f) * 8.0f);
  }
  return code | (v < 0.0f ? 0x20u : 0u);
}
__device__ __forceinline__ double dec_e2m3(uint32_t c) {
  const int e = (int)((c >> 3) & 3), m = (int)(c & 7);
  const double a = e == 0 ? m / 8.0 : (1.0 + m / 8.0) * ldexp(1.0, e - 1);
  return (c & 0x20u) ? -a : a;
}

// One chirp sample: cos(2 pi frac(f0 t + fdot t^2 / 2)), t = n / fs.
__device__ __forceinline__ double chirp_sample(double fs, double f0, double fdot, int n) {
  double t = (double)n / fs;
  double phi = f0 * t + 0.5 * fdot * (t * t);
  phi = phi - floor(phi);
  return cos(2.0 * 3.141592653589793 * phi);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------------------
// Bank generation: one wave per template, float64 throughout, then quantisation.
//
// FP32 layout, per 32-template block b and 16-tap chunk c: 64 lanes x 8 floats, lane
//   l = h*32 + m holding taps 16c + 2s + h (s = 0..7) of template 32b + m -- the A operand
//   of eight successive v_mfma_f32_32x32x2_f32 steps.
// BF16X3 layout, per (b, c): plane (hi, lo) x 64 lanes x 8 bf16, lane l = h*32 + m holding
//   taps 16c + 8h + i (i = 0..7) of template 32b + m -- the A operand of one
//   v_mfma_f32_32x32x16_bf16 step.
// F16X2 layout: as BF16X3, with fp16 hi and lo of h * 2^10.
// FP8 layout, per (b, 64-tap chunk c): 64 lanes x 32 e4m3 codes, lane l = h*32 + m holding
//   taps 64c + 32h + i (i = 0..31) of template 32b + m -- the A operand of one
//   v_mfma_scale_f32_32x32x64_f8f6f4; template k is stored as h_k * 2^e_k with e_k the
//   largest exponent keeping max |h_k| * 2^e_k <= 448, and e_k is kept in texp[k].  The
//   rounded template no longer sums to zero; that sum (in template units) is kept in
//   tsum[k] so the contraction can remove the window mean's share of it.
// F16F8 layout, per (b, 32-tap chunk c): four planes of 64 lanes x 16 bytes.  Planes 0 and 1
//   are fp16 of h * 2^10, lane h*32 + m holding taps 32c + 16q + 8h + i (i < 8) of template
//   32b + m -- the A operands of two v_mfma_f32_32x32x16_f16 steps.  Planes 2 and 3 hold the
//   A operand of one v_mfma_scale_f32_32x32x64_f8f6f4 over the same 32 taps: lane m carries
//   the e4m3 codes of the residual r = h - fp16(h * 2^10) * 2^-10 scaled by 2^(e_k + 11),
//   lane 32 + m those of h scaled by 2^e_k (codes i < 16 in plane 2, the rest in plane 3).
//   texp[k] = e_k as for FP8; tsum[k] is the sum of fp16(h * 2^10) * 2^-10 plus the rounded
//   residual, the template that multiplies the data's fp16 part.
// F16F6 layout, per (b, 32-tap chunk c): as F16F8 with 3584 bytes: the fp16 planes 0 and 1,
//   then each lane's 32 e2m3 codes packed 6 bits apart (code i at bit 6i of 192 bits), bits
//   0..127 in plane 2 (64 x 16 bytes) and bits 128..191 in plane 3 (64 x 8 bytes).  Lane m
//   carries the residual scaled by 2^(e_k + 11), lane 32 + m the template scaled by 2^e_k,
//   with max |h| * 2^e_k <= 7.5.
// Padding templates (k >= K) and padding taps (n >= L) are zero.  The word after the bank
// counts templates whose centred norm vanished (they cannot be normalised).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bank_gen(GridDev g, BankDev b, void* dst,
                                                  int32_t* texp, unsigned int* bad) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + wave;
  if (k >= b.K_pad) return;
  const bool real = k < b.K;
  double f0 = 0.0, fdot = 0.0;
  if (real) {
    const int64_t il = k / g.n_fdot;
    const int j = (int)(k % g.n_fdot);
    const int64_t ig = g.f0_lo + il;
    f0 = (g.n_f0 > 1 && ig == g.n_f0 - 1) ? g.f0_max : (double)ig * g.f0_step + g.f0_min;
    fdot = (g.n_fdot > 1 && j == g.n_fdot - 1) ? g.fdot_max
                                               : (double)j * g.fdot_step + g.fdot_min;
  }
  double mu = 0.0, nrm = 1.0;
  if (real) {
    double s1 = 0.0;
    for (int n = lane; n < b.L; n += 64) s1 += chirp_sample(g.fs, f0, fdot, n);
    mu = wave_sum_d(s1) / (double)b.L;
    double s2 = 0.0;
    for (int n = lane; n < b.L; n += 64) {
      const double v = chirp_sample(g.fs, f0, fdot, n) - mu;
      s2 += v * v;
    }
    s2 = wave_sum_d(s2);
    nrm = sqrt(s2);
    if (!(s2 > 1e-18 * (double)b.L)) {
      if (lane == 0) atomicAdd(bad, 1u);
      nrm = 1.0;
    }
  }
  const int64_t blk = k >> 5;
  const int m = (int)(k & 31);
  int e8 = 0;
  double qsum = 0.0;   // FP8: sum of the stored codes, in units of 2^-e8
  if (has_side_tables(b.precision)) {
    double mx = 0.0;
    if (real)
      for (int n = lane; n < b.L; n += 64)
        mx = fmax(mx, fabs((chirp_sample(g.fs, f0, fdot, n) - mu) / nrm));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    const double lim = b.precision == P_F16F6 ? 7.5 : 448.0;   // largest code value
    e8 = mx > 0.0 ? (int)floor(log2(lim / mx)) : 0;
    if (lane == 0) texp[k] = e8;
  }
  if (b.precision == P_F16F6) {
    // one 32-tap chunk per lane at a time: the lane packs its two 192-bit code strings
    for (int c = lane; c < b.n_chunks; c += 64) {
      uint32_t wl[6] = {0u, 0u, 0u, 0u, 0u, 0u}, wh[6] = {0u, 0u, 0u, 0u, 0u, 0u};
      char* cbase = (char*)dst + ((int64_t)blk * b.n_chunks + c) * 3584;
      for (int r = 0; r < 32; ++r) {
        const int n = 32 * c + r;
        const double h = (real && n < b.L) ? (chirp_sample(g.fs, f0, fdot, n) - mu) / nrm : 0.0;
        const _Float16 t16 = (_Float16)ldexp(h, F16_TEMPLATE_EXP);
        const double rr = h - ldexp((double)t16, -F16_TEMPLATE_EXP);
        const uint32_t cl = enc_e2m3((float)ldexp(rr, e8 + F6_LO_SHIFT));
        const uint32_t ch = enc_e2m3((float)ldexp(h, e8));
        qsum += ldexp((double)t16, e8 - F16_TEMPLATE_EXP) + ldexp(dec_e2m3(cl), -F6_LO_SHIFT);
        const int q = r >> 4, hh = (r >> 3) & 1, i = r & 7;
        *(_Float16*)(cbase + q * 1024 + (hh * 32 + m) * 16 + i * 2) = t16;
        const int bit = 6 * r, w = bit >> 5, o = bit & 31;
        wl[w] |= cl << o;
        wh[w] |= ch << o;
        if (o > 26) {
          wl[w + 1] |= cl >> (32 - o);
          wh[w + 1] |= ch >> (32 - o);
        }
      }
      *(uint4*)(cbase + 2048 + m * 16) = make_uint4(wl[0], wl[1], wl[2], wl[3]);
      *(uint4*)(cbase + 2048 + (32 + m) * 16) = make_uint4(wh[0], wh[1], wh[2], wh[3]);
      *(uint2*)(cbase + 3072 + m * 8) = make_uint2(wl[4], wl[5]);
      *(uint2*)(cbase + 3072 + (32 + m) * 8) = make_uint2(wh[4], wh[5]);
    }
  }
  for (int n = lane; n < b.L_pad && b.precision != P_F16F6; n += 64) {
    const double h = (real && n < b.L) ? (chirp_sample(g.fs, f0, fdot, n) - mu) / nrm : 0.0;
    if (b.precision == P_FP32) {
      const int c = n >> 4, r = n & 15;
      const int ln = (r & 1) * 32 + m, s = r >> 1;
      float* out = (float*)dst;
      out[(((int64_t)blk * b.n_chunks + c) * 64 + ln) * 8 + s] = (float)h;
    } else if (b.precision == P_BF16X3) {
      const int c = n >> 4, r = n & 15;
      const int ln = (r >> 3) * 32 + m, i = r & 7;
      const double hi = round_bf16_d(h);
      const double lo = round_bf16_d(h - hi);
      uint16_t* out = (uint16_t*)dst;
      const int64_t base = ((int64_t)blk * b.n_chunks + c) * 2;
      out[((base + 0) * 64 + ln) * 8 + i] = (uint16_t)(__float_as_uint((float)hi) >> 16);
      out[((base + 1) * 64 + ln) * 8 + i] = (uint16_t)(__float_as_uint((float)lo) >> 16);
    } else if (b.precision == P_F16X2) {
      // same layout as BF16X3; fp16 hi + lo of h * 2^10 (keeps lo clear of subnormals)
      const int c = n >> 4, r = n & 15;
      const int ln = (r >> 3) * 32 + m, i = r & 7;
      const double hs = ldexp(h, F16_TEMPLATE_EXP);
      const _Float16 hi = (_Float16)hs;
      const _Float16 lo = (_Float16)(hs - (double)hi);
      _Float16* out = (_Float16*)dst;
      const int64_t base = ((int64_t)blk * b.n_chunks + c) * 2;
      out[((base + 0) * 64 + ln) * 8 + i] = hi;
      out[((base + 1) * 64 + ln) * 8 + i] = lo;
    } else if (b.precision == P_F16F8) {
      const int c = n >> 5, r = n & 31;
      const _Float16 t16 = (_Float16)ldexp(h, F16_TEMPLATE_EXP);
      const double rr = h - ldexp((double)t16, -F16_TEMPLATE_EXP);
      // |rr| <= 2^-11 |h| (fp16 rounding), so both codes stay within 448
      const float vl = (float)ldexp(rr, e8 + F8_LO_SHIFT);
      const float vh = (float)ldexp(h, e8);
      const int cl = __builtin_amdgcn_cvt_pk_fp8_f32(vl, 0.0f, 0, false) & 0xFF;
      const int ch = __builtin_amdgcn_cvt_pk_fp8_f32(vh, 0.0f, 0, false) & 0xFF;
      qsum += ldexp((double)t16, e8 - F16_TEMPLATE_EXP) +
              ldexp((double)__builtin_amdgcn_cvt_f32_fp8(cl, 0), -F8_LO_SHIFT);
      char* cbase = (char*)dst + ((int64_t)blk * b.n_chunks + c) * 4096;
      const int q = r >> 4, hh = (r >> 3) & 1, i = r & 7;
      *(_Float16*)(cbase + q * 1024 + (hh * 32 + m) * 16 + i * 2) = t16;
      cbase[(2 + q) * 1024 + m * 16 + (r & 15)] = (char)cl;
      cbase[(2 + q) * 1024 + (32 + m) * 16 + (r & 15)] = (char)ch;
    } else {
      const int c = n >> 6, r = n & 63;
      const int ln = (r >> 5) * 32 + m, i = r & 31;
      const float v = (float)ldexp(h, e8);   // |v| <= 448 by the choice of e8
      const int code = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xFF;
      qsum += (double)__builtin_amdgcn_cvt_f32_fp8(code, 0);
      uint8_t* out = (uint8_t*)dst;
      out[(((int64_t)blk * b.n_chunks + c) * 64 + ln) * 32 + i] = (uint8_t)code;
    }
  }
  if (has_side_tables(b.precision)) {
    qsum = wave_sum_d(qsum);
    if (lane == 0) ((float*)(texp + b.K_pad))[k] = (float)ldexp(qsum, -e8);
  }
}

hipError_t launch_bank_gen(const GridDev& g, const BankDev& b, void* dst, hipStream_t s) {
  int32_t* texp = (int32_t*)((char*)dst + bank_data_bytes(b));
  unsigned int* bad = (unsigned int*)((char*)dst + bank_data_bytes(b) + bank_exp_bytes(b));
  hipError_t e = hipMemsetAsync(bad, 0, 256, s);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)((b.K_pad + 3) / 4);
  hipLaunchKernelGGL(k_bank_gen, dim3(grid), dim3(256), 0, s, g, b, dst, texp, bad);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Clearing: running maxima, spectrogram, spectrum sums, histogram, degenerate count.
// grid = (X, n_segs); each series clears its own buffers with a grid-stride loop.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero(const BatchHdr* __restrict__ hdr, BankDev b,
                                              SearchDev p) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < sg.W; i += stride) sg.mkey[i] = 0ull;
  if (sg.spec) {
    const int64_t ns = sg.spec_rows * b.n_bins;
    for (int64_t i = t0; i < ns; i += stride) sg.spec[i] = 0.0f;
  }
  for (int64_t i = t0; i < b.n_bins; i += stride) sg.spec_acc[i] = 0ull;
  if (sg.hist)
    for (int64_t i = t0; i < p.hist_bins; i += stride) sg.hist[i] = 0u;
  if (sg.n_degenerate && t0 == 0) sg.n_degenerate[0] = 0;
  if (sg.sig_acc) {
    for (int64_t i = t0; i < b.K_pad; i += stride) sg.sig_acc[i] = 0ull;
    for (int64_t i = t0; i < b.n_bins; i += stride) sg.t_bins[i] = 0u;
    if (t0 == 0) {
      sg.n_ok[0] = 0ull;
      sg.n_tails[0] = 0ull;
      if (sg.redo) sg.redo[0] = 0u;
    }
    if (sg.n_cand)
      for (int64_t i = t0; i < CAND_SHARDS; i += stride) sg.n_cand[i] = 0ull;
  }
}

hipError_t launch_zero(const BatchHdr* hdr, int32_t seg_slots, int32_t x_blocks,
                       const BankDev& b, const SearchDev& p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3((unsigned)x_blocks, (unsigned)seg_slots), dim3(256), 0, s,
                     hdr, b, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Prefix sums: one 1024-thread work-group per series scans x in tiles of 1024 x PRE_E
// samples, carrying double-double sums of x and x^2 (non-finite samples count as 0 and are
// counted separately).  pre[i] holds the sums over x[0..i).  Each thread sums its PRE_E
// consecutive samples, the threads' totals are scanned across the wave by shuffles and
// across the 16 waves by thread 0, and each thread then runs through its samples again
// (from cache) from the sum of everything before them, writing each prefix.
// ---------------------------------------------------------------------------------------
constexpr int PRE_E = 16;

__global__ __launch_bounds__(1024) void k_prefix(const BatchHdr* __restrict__ hdr) {
  if ((int)blockIdx.x >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.x];
  __shared__ dd w1[16], w2[16];
  __shared__ int wc[16];
  __shared__ dd c1s, c2s;
  __shared__ int ccs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    c1s = {0.0, 0.0};
    c2s = {0.0, 0.0};
    ccs = 0;
    sg.pre[0] = 0.0;
    sg.pre[1] = 0.0;
    sg.pre[2] = 0.0;
    sg.pre[3] = 0.0;
    sg.cnt[0] = 0;
  }
  __syncthreads();
  for (int64_t base = 0; base < sg.n; base += 1024 * PRE_E) {
    const int64_t i0 = base + (int64_t)tid * PRE_E;
    // this thread's totals over its PRE_E samples
    dd s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
    int c = 0;
#pragma unroll
    for (int e = 0; e < PRE_E; ++e) {
      const int64_t i = i0 + e;
      const float v = i < sg.n ? sg.x[i] : 0.0f;
      const bool fin = isfinite(v);
      const double a = fin ? (double)v : 0.0;
      s1 = dd_add(s1, {a, 0.0});
      s2 = dd_add(s2, {a * a, 0.0});  // a*a is exact for a float a
      c += (i < sg.n && !fin) ? 1 : 0;
    }
    // inclusive scan of the thread totals across the wave
    dd t1 = s1, t2 = s2;
    int tc = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const dd u1 = {__shfl_up(t1.hi, off, 64), __shfl_up(t1.lo, off, 64)};
      const dd u2 = {__shfl_up(t2.hi, off, 64), __shfl_up(t2.lo, off, 64)};
      const int uc = __shfl_up(tc, off, 64);
      if (lane >= off) {
        t1 = dd_add(u1, t1);
        t2 = dd_add(u2, t2);
        tc += uc;
      }
    }
    // exclusive: the inclusive scan of the previous lane (0 on lane 0)
    dd x1 = {__shfl_up(t1.hi, 1, 64), __shfl_up(t1.lo, 1, 64)};
    dd x2 = {__shfl_up(t2.hi, 1, 64), __shfl_up(t2.lo, 1, 64)};
    int xc = __shfl_up(tc, 1, 64);
    if (lane == 0) {
      x1 = {0.0, 0.0};
      x2 = {0.0, 0.0};
      xc = 0;
    }
    if (lane == 63) {
      w1[wave] = t1;
      w2[wave] = t2;
      wc[wave] = tc;
    }
    __syncthreads();
    if (tid == 0) {
      dd r1 = c1s, r2 = c2s;
      int rc = ccs;
      for (int w = 0; w < 16; ++w) {
        const dd a1 = w1[w], a2 = w2[w];
        const int ac = wc[w];
        w1[w] = r1;
        w2[w] = r2;
        wc[w] = rc;
        r1 = dd_add(r1, a1);
        r2 = dd_add(r2, a2);
        rc += ac;
      }
      c1s = r1;
      c2s = r2;
      ccs = rc;
    }
    __syncthreads();
    // everything before this thread's first sample: the carry and earlier waves (from
    // LDS), then the earlier threads of this wave
    dd q1 = dd_add(w1[wave], x1);
    dd q2 = dd_add(w2[wave], x2);
    int qc = wc[wave] + xc;
#pragma unroll
    for (int e = 0; e < PRE_E; ++e) {
      const int64_t i = i0 + e;
      if (i < sg.n) {
        const float v = sg.x[i];
        const bool fin = isfinite(v);
        const double a = fin ? (double)v : 0.0;
        q1 = dd_add(q1, {a, 0.0});
        q2 = dd_add(q2, {a * a, 0.0});
        qc += fin ? 0 : 1;
        double* o = sg.pre + (i + 1) * 4;
        o[0] = q1.hi;
        o[1] = q1.lo;
        o[2] = q2.hi;
        o[3] = q2.lo;
        sg.cnt[i + 1] = qc;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_prefix(const BatchHdr* hdr, int32_t seg_slots, hipStream_t s) {
  hipLaunchKernelGGL(k_prefix, dim3((unsigned)seg_slots), dim3(1024), 0, s, hdr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Window energies.  With D1 = sum x and D2 = sum x^2 over the window (double-double
// differences of the prefix sums), the centred energy is E = (L*D2 - D1^2) / L, formed in
// double-double so that windows with a large mean keep their small variance.  Raw: E = D2.
// Degenerate (inv_norm = 0): a non-finite sample, R = D2 = 0, or E <= 1e-12 R.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_norms(const BatchHdr* __restrict__ hdr, int L,
                                               int norm) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t tau = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; tau < sg.W;
       tau += stride) {
    const double* a = sg.pre + tau * 4;
    const double* z = sg.pre + (tau + L) * 4;
    const dd d1 = dd_add({z[0], z[1]}, dd_neg({a[0], a[1]}));
    const dd d2 = dd_add({z[2], z[3]}, dd_neg({a[2], a[3]}));
    const int nc = sg.cnt[tau + L] - sg.cnt[tau];
    const double R = d2.hi + d2.lo;
    double E;
    if (norm == 0) {
      const double Ld = (double)L;
      dd p1 = two_prod(Ld, d2.hi);
      p1 = dd_add(p1, {Ld * d2.lo, 0.0});
      dd p2 = two_prod(d1.hi, d1.hi);
      p2 = dd_add(p2, {2.0 * d1.hi * d1.lo, 0.0});
      const dd e = dd_add(p1, dd_neg(p2));
      E = (e.hi + e.lo) / Ld;
    } else {
      E = R;
    }
    const bool degenerate = (nc > 0) || !(R > 0.0) || !(E > 1e-12 * R) || !isfinite(E);
    sg.inv_norm[tau] = degenerate ? 0.0 : 1.0 / sqrt(E);
  }
}

// ---------------------------------------------------------------------------------------
// The contraction with the fused reductions.
//
// Work item = (series, offset tile of n_wg = 128*NB offsets, bin range).  The planner uses a
// multiple of 8 ranges and the items are numbered so that each XCD's work-groups sweep only
// their own ranges, one at a time, in step, and share each through that XCD's L2.  A work-group fills an LDS strip with x[tau0 .. tau0 + n_wg + L_pad) (zero
// past the end; non-finite samples as 0 -- their windows are degenerate and discarded),
// then each wave sweeps the item's template tiles: for each tile, a full K-loop over the
// taps into MB x NB accumulators of 32 x 32, then the epilogue.
//
// MFMA fragments (64 lanes, lane = h*32 + n):
//   FP32  v_mfma_f32_32x32x2_f32: A lane holds h_k[kk + h] of template row n,
//         B lane holds x[tau + kk + h] of offset column n.
//   BF16  v_mfma_f32_32x32x16_bf16: A lane holds taps kk + 8h + i (i < 8), B lane holds
//         x[tau + kk + 8h + i].  The strip is kept as four copies shifted by 0..3 samples,
//         interleaved per 4-sample cell, so every lane's 8 consecutive samples are two
//         8-byte-aligned LDS reads whatever tau is.  hi*hi + hi*lo + lo*hi are accumulated.
//   F16F8 per 32-tap chunk: two v_mfma_f32_32x32x16_f16 steps as above (fp16 strip, one
//         plane, four shifted copies) and one v_mfma_scale_f32_32x32x64_f8f6f4 whose K axis
//         holds the two residual products over the same 32 taps: lanes h = 0 pair the
//         template residual with the fp16 data, lanes h = 1 the template with the data
//         residual.  Each of the two e4m3 strip planes keeps eight shifted copies.
//   Output lane holds column n, rows 8g + 4h + i4 (g, i4 < 4) in accumulator 4g + i4.
// ---------------------------------------------------------------------------------------
size_t main_lds_bytes(int precision, int L_pad, int n_wg) {
  const size_t S = (size_t)n_wg + (size_t)L_pad + STRIP_SLACK;
  // F16F8, F16F6: fp16 plane + two code planes, then the item's 1/sqrt(E) (double) and window
  // means (float), then the waves' running maxima between tiles (3 words per offset)
  if (is_f16r(precision)) return S * 24 + (size_t)n_wg * 36;
  return precision == P_FP32 ? S * 4 : (precision == P_FP8 || precision == P_F16X2) ? S * 8 : S * 16;
}

struct ItemCtx {
  int64_t tau0;     // first offset of the item
  int64_t W;
  int64_t k_lo, k_hi;  // local template range owned by the item (whole bins)
};

template <int PREC, int MB>
struct AFrag;
template <int MB>
struct AFrag<P_FP32, MB> {
  float4 v[MB][2];    // 8 taps per lane per block per chunk
};
template <int MB>
struct AFrag<P_BF16X3, MB> {
  uint4 v[MB][2];     // [block][plane hi/lo]
};
template <int MB>
struct AFrag<P_F16X2, MB> {
  uint4 v[MB][2];     // [block][plane hi/lo], fp16
};
template <int MB>
struct AFrag<P_FP8, MB> {
  uint4 v[MB][2];     // 32 e4m3 codes per lane per block per chunk
};

template <int PREC, int MB>
__device__ __forceinline__ void load_a(AFrag<PREC, MB>& f, const void* bank, int64_t blk0, int c,
                                       int nchunks, int lane) {
  if constexpr (PREC == P_FP32) {
    const float4* A = (const float4*)bank;
#pragma unroll
    for (int t = 0; t < MB; ++t) {
      const int64_t idx = (((blk0 + t) * nchunks + c) * 64 + lane) * 2;
      f.v[t][0] = A[idx];
      f.v[t][1] = A[idx + 1];
    }
  } else if constexpr (PREC == P_BF16X3 || PREC == P_F16X2) {
    const uint4* A = (const uint4*)bank;
#pragma unroll
    for (int t = 0; t < MB; ++t) {
      const int64_t idx = (((blk0 + t) * nchunks + c) * 2) * 64 + lane;
      f.v[t][0] = A[idx];
      f.v[t][1] = A[idx + 64];
    }
  } else {
    const uint4* A = (const uint4*)bank;
#pragma unroll
    for (int t = 0; t < MB; ++t) {
      const int64_t idx = (((blk0 + t) * nchunks + c) * 64 + lane) * 2;
      f.v[t][0] = A[idx];
      f.v[t][1] = A[idx + 1];
    }
  }
}

__device__ __forceinline__ float f4get(const float4& v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// B operand fragments of one 16-tap chunk, read from the LDS strip.
template <int PREC, int NB>
struct BFrag;
template <int NB>
struct BFrag<P_FP32, NB> {
  float v[8][NB];     // [2-tap step][offset block]
};
template <int NB>
struct BFrag<P_BF16X3, NB> {
  uint4 v[NB][2];     // [offset block][plane hi/lo]
};
template <int NB>
struct BFrag<P_FP8, NB> {
  uint4 v[NB][2];     // [offset block][32 codes]
};
template <int NB>
struct BFrag<P_F16X2, NB> {
  uint4 v[NB][1];     // [offset block][8 fp16 samples]
};

// Strip fragments of chunk c for the offset blocks j in [J0, J1) (all by default).
template <int PREC, int NB, int J0 = 0, int J1 = NB>
__device__ __forceinline__ void load_b(BFrag<PREC, NB>& f, const char* lds, int off_w, int c,
                                       int n, int h, int plane_bytes) {
  if constexpr (PREC == P_FP32) {
    const float* sx = (const float*)lds;
    const int p0 = off_w + n + 16 * c + h;
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int j = J0; j < J1; ++j) f.v[s][j] = sx[p0 + 32 * j + 2 * s];
  } else if constexpr (PREC == P_FP8) {
    // 8 copies shifted by 0..7 samples, interleaved per 8-sample cell (8 bytes each):
    // a lane's 32 consecutive codes are four 8-byte-aligned reads.  Block j and chunk c
    // move the cell by 4j and 8c, i.e. the address by 256j + 512c bytes.
    const int p0 = off_w + n + 32 * h;
    const int base = (p0 >> 3) * 64 + (p0 & 7) * 8 + 512 * c;
#pragma unroll
    for (int j = J0; j < J1; ++j) {
      const int addr = base + 256 * j;
      const uint2 u0 = *(const uint2*)(lds + addr);
      const uint2 u1 = *(const uint2*)(lds + addr + 64);
      const uint2 u2 = *(const uint2*)(lds + addr + 128);
      const uint2 u3 = *(const uint2*)(lds + addr + 192);
      f.v[j][0] = make_uint4(u0.x, u0.y, u1.x, u1.y);
      f.v[j][1] = make_uint4(u2.x, u2.y, u3.x, u3.y);
    }
  } else {
    // Block j and chunk c move the 4-sample cell by 8j and 4c: the address by 256j + 128c.
    // BF16X3 reads the hi and lo planes, F16X2 its single plane.
    constexpr int NPL = PREC == P_F16X2 ? 1 : 2;
    const int p0 = off_w + n + 8 * h;
    const int base = (p0 >> 2) * 32 + (p0 & 3) * 8 + 128 * c;
#pragma unroll
    for (int j = J0; j < J1; ++j) {
      const int addr = base + 256 * j;
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl) {
        const uint2 u0 = *(const uint2*)(lds + pl * plane_bytes + addr);
        const uint2 u1 = *(const uint2*)(lds + pl * plane_bytes + addr + 32);
        f.v[j][pl] = make_uint4(u0.x, u0.y, u1.x, u1.y);
      }
    }
  }
}

// The MFMAs of one 16-tap chunk.
struct U8 {
  uint4 a, b;
};

// MFMAs of one chunk for the offset blocks j in [J0, J1) (all of them by default).
template <int PREC, int MB, int NB, int J0 = 0, int J1 = NB>
__device__ __forceinline__ void mma_chunk(f32x16 (&acc)[MB][NB], const AFrag<PREC, MB>& a,
                                          const BFrag<PREC, NB>& bf, const int (&sa)[MB],
                                          int sb) {
  if constexpr (PREC == P_FP8) {
    // e4m3 x e4m3, with the E8M0 scales 2^-e_k (per template row, per lane) and 2^-e_x
    // (per strip) undoing the power-of-two scaling of both operands.
#pragma unroll
    for (int t = 0; t < MB; ++t) {
      const i32x8 av = __builtin_bit_cast(i32x8, (U8{a.v[t][0], a.v[t][1]}));
#pragma unroll
      for (int j = J0; j < J1; ++j) {
        const i32x8 bv = __builtin_bit_cast(i32x8, (U8{bf.v[j][0], bf.v[j][1]}));
        acc[t][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[t][j], 0, 0, 0,
                                                                    sa[t], 0, sb);
      }
    }
  } else if constexpr (PREC == P_F16X2) {
    // h_hi*x, then h_lo*x: consecutive MFMAs write different accumulators.
#pragma unroll
    for (int term = 0; term < 2; ++term) {
#pragma unroll
      for (int t = 0; t < MB; ++t) {
        const f16x8 av = __builtin_bit_cast(f16x8, a.v[t][term]);
#pragma unroll
        for (int j = J0; j < J1; ++j) {
          const f16x8 bv = __builtin_bit_cast(f16x8, bf.v[j][0]);
          acc[t][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, acc[t][j], 0, 0, 0);
        }
      }
    }
  } else if constexpr (PREC == P_FP32) {
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int t = 0; t < MB; ++t) {
        const float av = f4get(a.v[t][s >> 2], s & 3);
#pragma unroll
        for (int j = J0; j < J1; ++j)
          acc[t][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bf.v[s][j], acc[t][j], 0, 0, 0);
      }
  } else {
    // hi*hi, then hi*lo, then lo*hi: consecutive MFMAs write different accumulators.
#pragma unroll
    for (int term = 0; term < 3; ++term) {
      const int pa = term == 2 ? 1 : 0, pb = term == 1 ? 1 : 0;
#pragma unroll
      for (int t = 0; t < MB; ++t) {
        const bf16x8 av = __builtin_bit_cast(bf16x8, a.v[t][pa]);
#pragma unroll
        for (int j = J0; j < J1; ++j) {
          const bf16x8 b = __builtin_bit_cast(bf16x8, bf.v[j][pb]);
          acc[t][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b, acc[t][j], 0, 0, 0);
        }
      }
    }
  }
}

// F16F8 / F16F6 template fragments of chunk c: the fp16 planes (code = false) or the residual
// step's code planes (code = true; F16F6 keeps bits 128..191 in the low half of v[t][1]).
template <int PREC>
__device__ __forceinline__ uint4 f16r_load_plane(const void* bank, int64_t blk, int c,
                                                 int nchunks, int lane, int q) {
  if constexpr (PREC == P_F16F8) {
    return ((const uint4*)bank)[((blk * nchunks + c) * 4 + q) * 64 + lane];
  } else {
    const char* base = (const char*)bank + (blk * nchunks + c) * 3584;
    if (q < 3) return *(const uint4*)(base + q * 1024 + lane * 16);
    const uint2 u = *(const uint2*)(base + 3072 + lane * 8);
    return make_uint4(u.x, u.y, 0u, 0u);
  }
}

template <int PREC, int MB>
__device__ __forceinline__ void f16f8_load_a(uint4 (&v)[MB][2], const void* bank, int64_t blk0,
                                             int c, int nchunks, int lane, int q0) {
#pragma unroll
  for (int t = 0; t < MB; ++t) {
    v[t][0] = f16r_load_plane<PREC>(bank, blk0 + t, c, nchunks, lane, q0);
    v[t][1] = f16r_load_plane<PREC>(bank, blk0 + t, c, nchunks, lane, q0 + 1);
  }
}

// Strip fragments of an offset-block pair (blocks 2p, 2p + 1) for chunk c.  fp16 plane at
// lds[0] (8 samples from x[tau + 32c + 16s + 8h], two 8-byte reads of the 4-copy layout, per
// 16-tap step s); e4m3 planes after it (32 codes from x[tau + 32c], lanes h = 0 from the plane
// of the fp16 samples, h = 1 from that of the residuals; four reads of the 8-copy layout).
struct F16F8Pair {
  uint4 h[2][2];   // [block of the pair][16-tap step]
  uint4 e[2][2];   // [block of the pair][16 codes]
};

__device__ __forceinline__ void f16f8_load_pair(F16F8Pair& f, const char* lds, int off_w, int c,
                                                int p, int n, int h, int plane_bytes) {
  const int b16 = 8 * (off_w + n + 8 * h + 32 * c) + 512 * p;
  const int b8 = plane_bytes * (1 + h) + 8 * (off_w + n + 32 * c) + 512 * p;
#pragma unroll
  for (int jj = 0; jj < 2; ++jj)
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int addr = b16 + 256 * jj + 128 * st;
      const uint2 u0 = *(const uint2*)(lds + addr);
      const uint2 u1 = *(const uint2*)(lds + addr + 32);
      f.h[jj][st] = make_uint4(u0.x, u0.y, u1.x, u1.y);
    }
#pragma unroll
  for (int jj = 0; jj < 2; ++jj) {
    const int addr = b8 + 256 * jj;
    const uint2 u0 = *(const uint2*)(lds + addr);
    const uint2 u1 = *(const uint2*)(lds + addr + 64);
    const uint2 u2 = *(const uint2*)(lds + addr + 128);
    const uint2 u3 = *(const uint2*)(lds + addr + 192);
    f.e[jj][0] = make_uint4(u0.x, u0.y, u1.x, u1.y);
    f.e[jj][1] = make_uint4(u2.x, u2.y, u3.x, u3.y);
  }
}

// e2m3 strip operand: the four 8-byte cells hold 48 code bits each; packed 6 bits apart.
__device__ __forceinline__ i32x8 f6_pack(const uint4& c01, const uint4& c23) {
  i32x8 v;
  v[0] = (int)c01.x;
  v[1] = (int)(c01.y | (c01.z << 16));
  v[2] = (int)((c01.z >> 16) | (c01.w << 16));
  v[3] = (int)c23.x;
  v[4] = (int)(c23.y | (c23.z << 16));
  v[5] = (int)((c23.z >> 16) | (c23.w << 16));
  v[6] = 0;
  v[7] = 0;
  return v;
}

// The MFMAs of one chunk on the pair P: the fp16 steps, then the residual step (e4m3 or
// e2m3 codes) scaled by 2^(sa - 127) * 2^(sb - 127).  Four MFMAs separate any two that share
// an accumulator.
template <int PREC, int MB, int NB, int P>
__device__ __forceinline__ void f16f8_mma_pair(f32x16 (&acc)[MB][NB], const uint4 (&ha)[MB][2],
                                               const uint4 (&ea)[MB][2], const F16F8Pair& f,
                                               const int (&sa)[MB], int sb) {
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int t = 0; t < MB; ++t) {
      const f16x8 av = __builtin_bit_cast(f16x8, ha[t][st]);
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
        acc[t][2 * P + jj] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
            av, __builtin_bit_cast(f16x8, f.h[jj][st]), acc[t][2 * P + jj], 0, 0, 0);
    }
  constexpr int FMT = PREC == P_F16F8 ? 0 : 2;   // e4m3 : e2m3
  i32x8 bv[2];
#pragma unroll
  for (int jj = 0; jj < 2; ++jj)
    bv[jj] = PREC == P_F16F8 ? __builtin_bit_cast(i32x8, (U8{f.e[jj][0], f.e[jj][1]}))
                             : f6_pack(f.e[jj][0], f.e[jj][1]);
#pragma unroll
  for (int t = 0; t < MB; ++t) {
    const i32x8 av = __builtin_bit_cast(i32x8, (U8{ea[t][0], ea[t][1]}));
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
      acc[t][2 * P + jj] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
          av, bv[jj], acc[t][2 * P + jj], FMT, FMT, 0, sa[t], 0, sb);
  }
}

// One chunk c of the K-loop: NB / 2 pair steps.  Step P issues its MFMAs on slot P & 1 while
// the next pair's strip fragments (chunk c's pair P + 1, or pair 0 of chunk cn) load into the
// other slot; steps 0 and 1 also load the next chunk's template fragments (chunk cn, into
// hn / en).  Strip reads have one step and template reads at least NB / 2 - 1 steps to
// arrive in.
template <int PREC, int MB, int NB, int P>
__device__ __forceinline__ void f16f8_steps(f32x16 (&acc)[MB][NB], const uint4 (&ha)[MB][2],
                                            const uint4 (&ea)[MB][2], uint4 (&hn)[MB][2],
                                            uint4 (&en)[MB][2], F16F8Pair (&slot)[2],
                                            const char* lds, const void* bank, int64_t blk0,
                                            int c, int cn, int nc, int off_w, int n, int h,
                                            int lane, int plane_bytes, const int (&sa)[MB],
                                            int sb) {
  if constexpr (P < NB / 2) {
    constexpr int NP = NB / 2;
    constexpr int NVM = P < 2 ? 2 * MB : 0;     // template loads of this step
    static_assert(NP >= 2, "two steps carry the template loads");
    if constexpr (P + 1 < NP)
      f16f8_load_pair(slot[(P + 1) & 1], lds, off_w, c, P + 1, n, h, plane_bytes);
    else
      f16f8_load_pair(slot[(P + 1) & 1], lds, off_w, cn, 0, n, h, plane_bytes);
#pragma unroll
    for (int i = 0; i < NVM; ++i) {
      const int q = P * 2 * MB + i;             // 0 .. 4 MB - 1
      const int t = (q >> 1) % MB, half = q & 1;
      const bool is_e = q >= 2 * MB;
      const uint4 v = f16r_load_plane<PREC>(bank, blk0 + t, cn, nc, lane, (is_e ? 2 : 0) + half);
      if (is_e) en[t][half] = v; else hn[t][half] = v;
    }
    f16f8_mma_pair<PREC, MB, NB, P>(acc, ha, ea, slot[P & 1], sa, sb);
    constexpr int NMF = 6 * MB;                 // MFMAs per step
    _Pragma("unroll") for (int i_ = 0; i_ < NVM; ++i_) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
    _Pragma("unroll") for (int i_ = 0; i_ < 8; ++i_) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    if constexpr (NMF > NVM + 8) __builtin_amdgcn_sched_group_barrier(0x008, NMF - NVM - 8, 0);
    __builtin_amdgcn_sched_barrier(0);
    f16f8_steps<PREC, MB, NB, P + 1>(acc, ha, ea, hn, en, slot, lds, bank, blk0, c, cn, nc,
                                     off_w, n, h, lane, plane_bytes, sa, sb);
  }
}

// Spectrogram / spectrum flush of the current bin for this wave's NB x 32 offsets.
template <int NB>
__device__ __forceinline__ void flush_bin(const SegDesc& sg, const BankDev& b,
                                          const SearchDev& p, int bin, const float (&binmax)[NB],
                                          const double (&inv)[NB], int64_t tau_w0, int n,
                                          int h, int lane, float dscale) {
  unsigned long long fix = 0ull;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const float v = fmaxf(binmax[j], __shfl_xor(binmax[j], 32, 64));
    const int64_t tau = tau_w0 + 32 * j + n;
    if (h == 0 && tau < sg.W && inv[j] > 0.0) {
      const float s = (float)((double)v * (double)dscale * inv[j]);
      if (sg.spec) {
        // bin-major rows: the 32 lanes of a flush write 32 consecutive offsets of one row
        const int64_t at = (int64_t)bin * sg.spec_rows + tau / p.t_block;
        if (p.t_block == 1)
          sg.spec[at] = s;                 // each (bin, offset) is owned by one lane
        else
          atomicMax((unsigned int*)sg.spec + at, __float_as_uint(s));  // s >= 0: bits order
      }
      fix += (unsigned long long)__double2ll_rn((double)s * SPEC_FIX_SCALE);
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned lo = __shfl_xor((unsigned)(fix & 0xFFFFFFFFull), o, 64);
    const unsigned hi = __shfl_xor((unsigned)(fix >> 32), o, 64);
    fix += ((unsigned long long)hi << 32) | lo;
  }
  if (lane == 0 && fix != 0ull) atomicAdd(sg.spec_acc + bin, fix);
}

template <bool B>
struct BoolC {
  static constexpr bool value = B;
};

// One work item: strip fill, template sweep, flushes.  PIPE selects the K-loop schedule,
// MODE the pass (MainMode).
constexpr int N_XCD = 8;   // XCDs of the MI355X; work-groups are dealt to them round robin

template <int PREC, int MB, int NB, int PIPE, int MODE>
__device__ __forceinline__ void main_item(const BatchHdr* __restrict__ hdr, int64_t item,
                                          const BankDev& b, const SearchDev& p, char* lds) {
  const SegDesc* segs = hdr_segs(hdr);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = lane & 31, h = lane >> 5;
  const int64_t total_tiles = hdr->total_tiles;
  const int n_ranges = hdr->n_ranges;

  // ---- which item ----
  // Work-group i runs on XCD i mod 8 and each XCD takes its work-groups in order of i / 8.
  // With 8m ranges, XCD x sweeps its ranges x, x + 8, ..., x + 8(m - 1) one after another,
  // offset tiles fastest: the work-groups resident on an XCD at any time sweep one range in
  // step and share it through that XCD's L2 (with m = 1 this is range-fastest numbering).
  // Fewer than 8 ranges (fewer than 8 bins): range fastest.
  int r;
  int64_t tt;
  if (n_ranges % N_XCD == 0) {
    const int64_t j = item / N_XCD;
    r = (int)(item % N_XCD) + N_XCD * (int)(j / total_tiles);
    tt = j % total_tiles;
  } else {
    r = (int)(item % n_ranges);
    tt = item / n_ranges;
  }
  int lo = 0, hi = hdr->n_segs - 1;
  while (lo < hi) {  // last series with tile0 <= tt
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].tile0 <= tt) lo = mid; else hi = mid - 1;
  }
  const SegDesc& sg = segs[lo];
  // after a single-pass search the tails pass runs only for series whose prediction failed
  if (MODE == MODE_TAILS && sg.redo && sg.redo[0] == 0u) return;
  const int64_t tau0 = (tt - sg.tile0) * (32 * NB * WG_WAVES);
  const int b_lo = (int)((int64_t)r * b.n_bins / n_ranges);
  const int b_hi = (int)((int64_t)(r + 1) * b.n_bins / n_ranges);
  const int64_t k_lo = (int64_t)b_lo * b.n_fdot;
  const int64_t k_hi = (int64_t)b_hi * b.n_fdot;
  const int64_t tile_lo = k_lo / (32 * MB);
  const int64_t tile_hi = (k_hi + (32 * MB) - 1) / (32 * MB);

  // ---- strip fill ----
  // Every form stages x - c, c the level from series_offset (the rounded series mean): the
  // correlation does not depend on c, and the rounding then acts on the fluctuations, not on a
  // constant level.
  // Padding past the series end and non-finite samples stage as 0 in this shifted frame: they
  // reach only masked offsets, and a -c there would set the strip scale instead of the data.
  const float c0 = series_offset(sg);
  auto xs = [&](int64_t gi) -> float {
    if (gi >= sg.n) return 0.0f;
    const float v = sg.x[gi];
    return isfinite(v) ? v - c0 : 0.0f;
  };
  const int S = (32 * NB * WG_WAVES) + b.L_pad + STRIP_SLACK;  // multiple of 8
  int sb = 127;          // FP8, F16F8, F16F6: E8M0 scale of the strip's codes (per lane)
  float dscale = 1.0f;   // F16X2, F16F8, F16F6: 2^-(10 + e_x), undoing both power-of-two scales
  if constexpr (PREC == P_FP32) {
    float* sx = (float*)lds;
    for (int i = tid; i < S; i += WG_THREADS) {
      sx[i] = xs(tau0 + i);
    }
  } else if constexpr (PREC == P_FP8 || PREC == P_F16X2 || is_f16r(PREC)) {
    // strip scale 2^e_x: the largest power of two keeping max |x| over the strip <= LIM
    // (448 for e4m3, 2^14 for fp16, 7.5 * 2^11 when the fp16 samples become e2m3 codes)
    constexpr float LIM = PREC == P_FP8 ? 448.0f : PREC == P_F16F6 ? F6_STRIP_LIM : 16384.0f;
    __shared__ float wmax[WG_WAVES];
    float mx = 0.0f;
    for (int i = tid; i < S; i += WG_THREADS) {
      mx = fmaxf(mx, fabsf(xs(tau0 + i)));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) wmax[wave] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    int ex = mx > 0.0f ? (int)floorf(log2f(LIM / mx)) : 0;
    ex = ex < -100 ? -100 : (ex > 100 ? 100 : ex);
    while (ex > -100 && ldexpf(mx, ex) > LIM) --ex;   // guard log2f rounding
    if constexpr (PREC == P_FP8) {
      sb = 127 - ex;
      // cell (q, c): codes of x[tau0 + 8q + c + e] * 2^e_x, e = 0..7
      for (int t = tid; t < S; t += WG_THREADS) {
        const int q = t >> 3, c = t & 7;
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          v[e] = ldexpf(xs(tau0 + 8 * q + c + e), ex);
        }
        int w0 = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
        w0 = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w0, true);
        int w1 = __builtin_amdgcn_cvt_pk_fp8_f32(v[4], v[5], 0, false);
        w1 = __builtin_amdgcn_cvt_pk_fp8_f32(v[6], v[7], w1, true);
        *(uint2*)(lds + t * 8) = make_uint2((unsigned)w0, (unsigned)w1);
      }
    } else if constexpr (is_f16r(PREC)) {
      dscale = ldexpf(1.0f, -(F16_TEMPLATE_EXP + ex));
      // F16F6: each lane half scales its own operands (h = 0 the fp16 samples, h = 1 the
      // data residual); the F16F6 template scale adds 2^-10 on both halves.
      sb = PREC == P_F16F8 ? 127 + F8_XHI_SHIFT
                           : 127 + F16_TEMPLATE_EXP + (h == 0 ? F6_XHI_SHIFT : 0);
      // cell t of the fp16 plane: fp16 of y = x[tau0 + t + e] * 2^e_x, e = 0..3; cell t of the
      // two code planes: codes of fp16(y) * 2^-6 and of (y - fp16(y)) * 2^5 (e4m3), or of
      // fp16(y) * 2^-11 and y - fp16(y) (e2m3, 48 bits in 8 bytes), e = 0..7.  |y| <= 2^14
      // (F16F6: 15360) and |y - fp16(y)| <= 4 keep the codes within 448 (7.5).
      const int plane_bytes = S * 8;
      for (int t = tid; t < S; t += WG_THREADS) {
        float yh[8], yl[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float y = ldexpf(xs(tau0 + t + e), ex);
          yh[e] = (float)(_Float16)y;
          yl[e] = y - yh[e];
        }
        _Float16 hv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) hv[e] = (_Float16)yh[e];
        *(uint2*)(lds + t * 8) = __builtin_bit_cast(uint2, hv);
        int w[4];
        if constexpr (PREC == P_F16F8) {
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            int u = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(yh[4 * e], -F8_XHI_SHIFT),
                                                    ldexpf(yh[4 * e + 1], -F8_XHI_SHIFT), 0, false);
            w[e] = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(yh[4 * e + 2], -F8_XHI_SHIFT),
                                                   ldexpf(yh[4 * e + 3], -F8_XHI_SHIFT), u, true);
            u = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(yl[4 * e], F8_XLO_EXP),
                                                ldexpf(yl[4 * e + 1], F8_XLO_EXP), 0, false);
            w[2 + e] = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(yl[4 * e + 2], F8_XLO_EXP),
                                                       ldexpf(yl[4 * e + 3], F8_XLO_EXP), u, true);
          }
        } else {
          uint64_t ph = 0, pl = 0;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            ph |= (uint64_t)enc_e2m3(ldexpf(yh[e], -F6_XHI_SHIFT)) << (6 * e);
            pl |= (uint64_t)enc_e2m3(yl[e]) << (6 * e);
          }
          w[0] = (int)(uint32_t)ph;
          w[1] = (int)(uint32_t)(ph >> 32);
          w[2] = (int)(uint32_t)pl;
          w[3] = (int)(uint32_t)(pl >> 32);
        }
        *(uint2*)(lds + plane_bytes + t * 8) = make_uint2((unsigned)w[0], (unsigned)w[1]);
        *(uint2*)(lds + 2 * plane_bytes + t * 8) = make_uint2((unsigned)w[2], (unsigned)w[3]);
      }
      // per-offset epilogue operands, kept in LDS rather than in registers across the K-loop:
      // 1/sqrt(E) and the window mean in accumulator units
      const int n_wg = 32 * NB * WG_WAVES;
      double* inv_l = (double*)(lds + 3 * plane_bytes);
      float* mu_l = (float*)(inv_l + n_wg);
      for (int i = tid; i < n_wg; i += WG_THREADS) {
        const int64_t tau = tau0 + i;
        double iv = 0.0;
        float m = 0.0f;
        if (tau < sg.W) {
          iv = sg.inv_norm[tau];
          const double* a = sg.pre + tau * 4;
          const double* z = sg.pre + (tau + b.L) * 4;
          m = (float)(((z[0] - a[0]) + (z[1] - a[1])) / (double)b.L - (double)c0) / dscale;
        }
        inv_l[i] = iv;
        mu_l[i] = m;
      }
    } else {
      dscale = ldexpf(1.0f, -(F16_TEMPLATE_EXP + ex));
      // cell (q, c): fp16 of x[tau0 + 4q + c + e] * 2^e_x, e = 0..3 (one plane)
      for (int t = tid; t < S; t += WG_THREADS) {
        const int q = t >> 2, c = t & 3;
        _Float16 hv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          hv[e] = (_Float16)ldexpf(xs(tau0 + 4 * q + c + e), ex);
        }
        *(uint2*)(lds + t * 8) = __builtin_bit_cast(uint2, hv);
      }
    }
  } else {
    // cell (q, c) of plane pl: samples x[tau0 + 4q + c + e], e = 0..3, as bf16 hi / lo.
    const int plane_bytes = S * 8;
    for (int t = tid; t < S; t += WG_THREADS) {
      const int q = t >> 2, c = t & 3;
      uint32_t hw[2] = {0u, 0u}, lw[2] = {0u, 0u};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float v = xs(tau0 + 4 * q + c + e);
        const uint32_t hb = bf16_bits(v);
        const float hv = __uint_as_float(hb << 16);
        const uint32_t lb = bf16_bits(v - hv);
        hw[e >> 1] |= hb << (16 * (e & 1));
        lw[e >> 1] |= lb << (16 * (e & 1));
      }
      *(uint2*)(lds + t * 8) = make_uint2(hw[0], hw[1]);
      *(uint2*)(lds + plane_bytes + t * 8) = make_uint2(lw[0], lw[1]);
    }
  }
  __syncthreads();

  const int64_t tau_w0 = tau0 + (int64_t)wave * (32 * NB);
  const int off_w = wave * (32 * NB);
  const int plane_bytes = S * 8;

  double inv[NB];
  float mu[NB];   // FP8, F16F8: window means, for the template-sum correction
  // F16F8 reads both from LDS after each tile's K-loop (its K-loop needs the registers); the
  // empty asm keeps the reads inside the tile loop.
  auto load_stats = [&]() {
    int base = off_w + n;
    asm volatile("" : "+v"(base));
    const double* inv_l = (const double*)(lds + 3 * plane_bytes);
#pragma unroll
    for (int j = 0; j < NB; ++j) inv[j] = inv_l[base + 32 * j];
  };
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int64_t tau = tau_w0 + 32 * j + n;
    inv[j] = 0.0;
    mu[j] = 0.0f;
    if constexpr (!is_f16r(PREC)) inv[j] = tau < sg.W ? sg.inv_norm[tau] : 0.0;
    if constexpr (PREC == P_FP8) {
      if (tau < sg.W) {
        const double* a = sg.pre + tau * 4;
        const double* z = sg.pre + (tau + b.L) * 4;
        mu[j] = (float)(((z[0] - a[0]) + (z[1] - a[1])) / (double)b.L - (double)c0);
      }
    }
  }
  float best[NB], binmax[NB];
  int bestk[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    best[j] = -1.0f;
    bestk[j] = -1;
    binmax[j] = 0.0f;
  }
  // F16F8, F16F6: their K-loop needs every register, so between tiles the running maxima
  // wait in LDS (per wave [best | bestk | binmax][NB][64 lanes], after the window means)
  // instead of in scratch.  The address is hidden from the compiler so that it reloads them
  // after each K-loop rather than keeping them live across it.
  const int st_addr = 3 * plane_bytes + 32 * NB * WG_WAVES * 12 + (wave * 3 * NB * 64 + lane) * 4;
  auto park = [&]() {
    if constexpr (is_f16r(PREC)) {
      int a = st_addr;
      asm volatile("" : "+v"(a));
      float* st = (float*)(lds + a);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        st[64 * j] = best[j];
        st[64 * (NB + j)] = __int_as_float(bestk[j]);
        st[64 * (2 * NB + j)] = binmax[j];
      }
    }
  };
  auto unpark = [&]() {
    if constexpr (is_f16r(PREC)) {
      int a = st_addr;
      asm volatile("" : "+v"(a));
      const float* st = (const float*)(lds + a);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        best[j] = st[64 * j];
        bestk[j] = __float_as_int(st[64 * (NB + j)]);
        binmax[j] = st[64 * (2 * NB + j)];
      }
    }
  };
  park();
  int cur_bin = -1;
  const int nfd = b.n_fdot;

  for (int64_t kt = tile_lo; kt < tile_hi; ++kt) {
    f32x16 acc[MB][NB];
#pragma unroll
    for (int t = 0; t < MB; ++t)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[t][j] = (f32x16){};

    const int64_t blk0 = kt * MB;
    int sa[MB];
#pragma unroll
    for (int t = 0; t < MB; ++t)
      sa[t] = PREC == P_FP8     ? 127 - b.texp[(blk0 + t) * 32 + n]
              : PREC == P_F16F8 ? 127 - b.texp[(blk0 + t) * 32 + n] -
                                      (F8_LO_SHIFT - F16_TEMPLATE_EXP)
              : PREC == P_F16F6 ? 127 - b.texp[(blk0 + t) * 32 + n] - (h == 0 ? F6_LO_SHIFT : 0)
                                : 127;
    // Software pipeline over chunk pairs (n_chunks is even): while the MFMAs of chunk c
    // run, the template fragments of chunk c+1 and the strip fragments of chunk c+1 are in
    // flight.  Scheduling barriers keep the compiler from sinking the loads next to their
    // uses.  The prefetches past the last chunk re-read a valid chunk and are unused.
    const int nc = b.n_chunks;
    __builtin_amdgcn_s_waitcnt(0);   // drain the previous tile's atomics before the pipeline
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (is_f16r(PREC)) {
      // Pair-streaming schedule (f16f8_steps): per chunk, NB / 2 steps over offset-block
      // pairs; template fragments double-buffered across chunks, strip fragments across steps.
      static_assert(F8_XLO_EXP == F8_LO_SHIFT - F8_XHI_SHIFT, "residual scales must agree");
      static_assert(NB % 2 == 0 && 6 * MB >= 2 * MB + 8, "pair-step shape");
      uint4 h0[MB][2], e0[MB][2], h1[MB][2], e1[MB][2];
      F16F8Pair slot[2];
      f16f8_load_a<PREC, MB>(h0, b.data, blk0, 0, nc, lane, 0);
      f16f8_load_a<PREC, MB>(e0, b.data, blk0, 0, nc, lane, 2);
      f16f8_load_pair(slot[0], lds, off_w, 0, 0, n, h, plane_bytes);
      __builtin_amdgcn_sched_barrier(0);
      for (int c = 0; c < nc; c += 2) {
        const int c2 = c + 2 < nc ? c + 2 : nc - 1;
        f16f8_steps<PREC, MB, NB, 0>(acc, h0, e0, h1, e1, slot, lds, b.data, blk0, c, c + 1,
                                     nc, off_w, n, h, lane, plane_bytes, sa, sb);
        f16f8_steps<PREC, MB, NB, 0>(acc, h1, e1, h0, e0, slot, lds, b.data, blk0, c + 1, c2,
                                     nc, off_w, n, h, lane, plane_bytes, sa, sb);
      }
    } else if constexpr (PIPE == 1) {
      // Interleaved schedule.  The strip fragments live in two halves (offset blocks
      // [0, H) and [H, NB)); region (c, h) issues the MFMAs of half h of chunk c and, between
      // them, the LDS reads of the other half for the next region (half 1 of chunk c, or half
      // 0 of chunk c + 1) and, in half 0, the template fragments of chunk c + 1.  A region's
      // loads never write registers its own MFMAs read.
      constexpr int H = NB / 2;
      BFrag<PREC, NB> bb;
      AFrag<PREC, MB> a0, a1;
      load_a<PREC, MB>(a0, b.data, blk0, 0, nc, lane);
      load_b<PREC, NB, 0, H>(bb, lds, off_w, 0, n, h, plane_bytes);
      __builtin_amdgcn_sched_barrier(0);
      constexpr int NMF =
          (PREC == P_BF16X3 ? 3 : PREC == P_F16X2 ? 2 : PREC == P_FP32 ? 8 : 1) * MB * H;
      constexpr int NDS = (PREC == P_F16X2 ? 1 : PREC == P_FP32 ? 8 : 2) * H;  // LDS reads
      constexpr int NVM = 2 * MB;                                                        // loads
#define BFLY_INTERLEAVE(WITH_VMEM)                                                    \
      do {                                                                            \
        _Pragma("unroll") for (int i_ = 0; i_ < NDS; ++i_) {                          \
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                          \
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                          \
        }                                                                             \
        if (WITH_VMEM) {                                                              \
          _Pragma("unroll") for (int i_ = 0; i_ < NVM; ++i_) {                        \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                        \
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                        \
          }                                                                           \
        }                                                                             \
        __builtin_amdgcn_sched_group_barrier(0x008, NMF, 0);                          \
        __builtin_amdgcn_sched_barrier(0);                                            \
      } while (0)
      for (int c = 0; c < nc; c += 2) {
        const int c2 = c + 2 < nc ? c + 2 : nc - 1;
        mma_chunk<PREC, MB, NB, 0, H>(acc, a0, bb, sa, sb);
        load_b<PREC, NB, H, NB>(bb, lds, off_w, c, n, h, plane_bytes);
        load_a<PREC, MB>(a1, b.data, blk0, c + 1, nc, lane);
        BFLY_INTERLEAVE(true);
        mma_chunk<PREC, MB, NB, H, NB>(acc, a0, bb, sa, sb);
        load_b<PREC, NB, 0, H>(bb, lds, off_w, c + 1, n, h, plane_bytes);
        BFLY_INTERLEAVE(false);
        mma_chunk<PREC, MB, NB, 0, H>(acc, a1, bb, sa, sb);
        load_b<PREC, NB, H, NB>(bb, lds, off_w, c + 1, n, h, plane_bytes);
        load_a<PREC, MB>(a0, b.data, blk0, c2, nc, lane);
        BFLY_INTERLEAVE(true);
        mma_chunk<PREC, MB, NB, H, NB>(acc, a1, bb, sa, sb);
        load_b<PREC, NB, 0, H>(bb, lds, off_w, c2, n, h, plane_bytes);
        BFLY_INTERLEAVE(false);
      }
#undef BFLY_INTERLEAVE
    } else if constexpr (NB <= 4) {
      // Two strip-fragment buffers: chunk c+1's fragments load while chunk c's MFMAs run.
      BFrag<PREC, NB> b0, b1;
      AFrag<PREC, MB> a0, a1;
      load_a<PREC, MB>(a0, b.data, blk0, 0, nc, lane);
      __builtin_amdgcn_sched_barrier(0);
      load_b<PREC, NB>(b0, lds, off_w, 0, n, h, plane_bytes);
      __builtin_amdgcn_sched_barrier(0);
      for (int c = 0; c < nc; c += 2) {
        load_a<PREC, MB>(a1, b.data, blk0, c + 1, nc, lane);
        __builtin_amdgcn_sched_barrier(0);
        load_b<PREC, NB>(b1, lds, off_w, c + 1, n, h, plane_bytes);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<PREC, MB, NB>(acc, a0, b0, sa, sb);
        __builtin_amdgcn_sched_barrier(0);
        const int c2 = c + 2 < nc ? c + 2 : nc - 1;
        load_a<PREC, MB>(a0, b.data, blk0, c2, nc, lane);
        __builtin_amdgcn_sched_barrier(0);
        load_b<PREC, NB>(b0, lds, off_w, c2, n, h, plane_bytes);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<PREC, MB, NB>(acc, a1, b1, sa, sb);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      // One strip-fragment buffer in two halves: as soon as the MFMAs of one half of the
      // offset blocks are issued, that half reloads for the next chunk, while the other
      // half's MFMAs run.
      constexpr int H = NB / 2;
      BFrag<PREC, NB> bb;
      AFrag<PREC, MB> a0, a1;
      load_a<PREC, MB>(a0, b.data, blk0, 0, nc, lane);
      __builtin_amdgcn_sched_barrier(0);
      load_b<PREC, NB, 0, NB>(bb, lds, off_w, 0, n, h, plane_bytes);
      __builtin_amdgcn_sched_barrier(0);
      for (int c = 0; c < nc; c += 2) {
        load_a<PREC, MB>(a1, b.data, blk0, c + 1, nc, lane);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<PREC, MB, NB, 0, H>(acc, a0, bb, sa, sb);
        __builtin_amdgcn_sched_barrier(0);
        load_b<PREC, NB, 0, H>(bb, lds, off_w, c + 1, n, h, plane_bytes);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<PREC, MB, NB, H, NB>(acc, a0, bb, sa, sb);
        __builtin_amdgcn_sched_barrier(0);
        load_b<PREC, NB, H, NB>(bb, lds, off_w, c + 1, n, h, plane_bytes);
        __builtin_amdgcn_sched_barrier(0);
        const int c2 = c + 2 < nc ? c + 2 : nc - 1;
        load_a<PREC, MB>(a0, b.data, blk0, c2, nc, lane);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<PREC, MB, NB, 0, H>(acc, a1, bb, sa, sb);
        __builtin_amdgcn_sched_barrier(0);
        load_b<PREC, NB, 0, H>(bb, lds, off_w, c2, n, h, plane_bytes);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<PREC, MB, NB, H, NB>(acc, a1, bb, sa, sb);
        __builtin_amdgcn_sched_barrier(0);
        load_b<PREC, NB, H, NB>(bb, lds, off_w, c2, n, h, plane_bytes);
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    // The rounded templates of the FP8, F16F8 and F16F6 forms carry a small sum s_k, which
    // would pick up s_k times the window mean; d - mu * s_k is the contraction of the rounded
    // template with the centred window.  The correction is the rank-1 product of the template
    // sums and the negated window means: one v_mfma_f32_32x32x2_f32 per accumulator block,
    // with the sums and means in K slot 0 (lanes h = 0) and zeros in slot 1.
    if constexpr (PREC == P_FP8 || is_f16r(PREC)) {
      float as[MB], bm[NB];
#pragma unroll
      for (int t = 0; t < MB; ++t) as[t] = h == 0 ? b.tsum[(blk0 + t) * 32 + n] : 0.0f;
      if constexpr (is_f16r(PREC)) {
        int base = off_w + n;
        asm volatile("" : "+v"(base));   // read inside the tile loop, not kept across it
        const float* mu_l = (const float*)((const double*)(lds + 3 * plane_bytes) +
                                           32 * NB * WG_WAVES);
#pragma unroll
        for (int j = 0; j < NB; ++j) bm[j] = h == 0 ? -mu_l[base + 32 * j] : 0.0f;
      } else {
#pragma unroll
        for (int j = 0; j < NB; ++j) bm[j] = h == 0 ? -mu[j] : 0.0f;
      }
#pragma unroll
      for (int t = 0; t < MB; ++t)
#pragma unroll
        for (int j = 0; j < NB; ++j)
          acc[t][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(as[t], bm[j], acc[t][j], 0, 0, 0);
    }
    if constexpr (is_f16r(PREC)) load_stats();

    // ---- epilogue: lane rows are 32t + 8g + 4h + i4 of the tile ----
    const int64_t kbase = kt * (32 * MB);
    const int r_lo = (int)((k_lo > kbase ? k_lo : kbase) - kbase);        // rows owned
    const int r_hi = (int)((k_hi < kbase + (32 * MB) ? k_hi : kbase + (32 * MB)) - kbase);
    // rho of the tail modes: (d dscale) (1/sqrt(E) rounded to float32) in float32.  dscale
    // is a power of two, so d dscale is exact and the product of two floats is exact in
    // float64: this is that product rounded once.
    float invf[NB];
    if constexpr (MODE != MODE_SEARCH) {
#pragma unroll
      for (int j = 0; j < NB; ++j) invf[j] = (float)inv[j];
    }
    if constexpr (MODE == MODE_TAILS) {
      // every owned (tau, k) with |rho| > kappa * sigma_k is appended to the series' list
      // and counted in its bin (rows as in the search epilogue: c + 4h, the ownership test
      // on the immediate c)
      const float* th = sg.thr + kbase + 4 * h;
      const int qh = r_lo - 4 * h;
      const unsigned span = (unsigned)(r_hi - r_lo);
#pragma unroll
      for (int t = 0; t < MB; ++t)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const float4 t4 = *(const float4*)(th + 32 * t + 8 * g);
          const float tv[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int c = 32 * t + 8 * g + i;
              const float rf = (acc[t][j][4 * g + i] * dscale) * invf[j];
              if (fabsf(rf) > tv[i] && (unsigned)(c - qh) < span) {
                const int64_t kl = kbase + c + 4 * h;
                const unsigned long long slot = atomicAdd(sg.n_tails, 1ull);
                if ((int64_t)slot < sg.tail_cap) {
                  sg.t_tau[slot] = (int32_t)(tau_w0 + 32 * j + n);
                  sg.t_k[slot] = (int32_t)(b.k_offset + kl);
                  sg.t_rho[slot] = rf;
                }
                atomicAdd(sg.t_bins + kl / nfd, 1u);
              }
            }
        }
      continue;
    }
    unpark();
    // Per bin the tile touches (one, unless it straddles a bin edge), over the owned rows
    // [q_lo, q_hi) in that bin: per offset column, the maximum of the lane's rows, then the
    // lowest row that reaches it, one column at a time so few accumulators are live in VGPRs.
    // Rows ascend with the bins, so the running (best, bestk) keeps the lowest row on ties.
    const int bA = (int)((kbase + r_lo) / nfd), bB = (int)((kbase + r_hi - 1) / nfd);
    // Row of accumulator v of block t: c + 4h with c = 32t + 8(v >> 2) + (v & 3); the search
    // runs on the lane-independent c (immediates, so no per-lane row table is kept live
    // across the K-loop) and adds 4h once.
    auto reduce = [&](auto full, int q_lo, int q_hi) {
      constexpr bool FULL = decltype(full)::value;
      const unsigned span = (unsigned)(q_hi - q_lo);
      const int qh = q_lo - 4 * h;   // row - q_lo = c - qh
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        float mx = -1.0f;
#pragma unroll
        for (int t = 0; t < MB; ++t)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int c = 32 * t + 8 * (v >> 2) + (v & 3);
            const float a = fabsf(acc[t][j][v]);
            if constexpr (FULL) mx = fmaxf(mx, a);
            else mx = (unsigned)(c - qh) < span ? fmaxf(mx, a) : mx;
          }
        int row = 0;
#pragma unroll
        for (int t = MB - 1; t >= 0; --t)
#pragma unroll
          for (int v = 15; v >= 0; --v) {
            const int c = 32 * t + 8 * (v >> 2) + (v & 3);
            const bool hit = fabsf(acc[t][j][v]) == mx && (FULL || (unsigned)(c - qh) < span);
            row = hit ? c : row;
          }
        row += 4 * h;
        const bool gt = mx > best[j];   // false when no row is owned (mx = -1)
        best[j] = gt ? mx : best[j];
        bestk[j] = gt ? (int)kbase + row : bestk[j];
        binmax[j] = fmaxf(binmax[j], mx);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    for (int bn = bA; bn <= bB; ++bn) {
      if (bn != cur_bin) {
        if (cur_bin >= 0) flush_bin<NB>(sg, b, p, cur_bin, binmax, inv, tau_w0, n, h, lane, dscale);
        cur_bin = bn;
#pragma unroll
        for (int j = 0; j < NB; ++j) binmax[j] = 0.0f;
      }
      const int64_t e_lo = (int64_t)bn * nfd - kbase, e_hi = (int64_t)(bn + 1) * nfd - kbase;
      const int q_lo = (int)(e_lo > r_lo ? e_lo : r_lo);
      const int q_hi = (int)(e_hi < r_hi ? e_hi : r_hi);
      if (q_lo == 0 && q_hi == 32 * MB) reduce(BoolC<true>{}, 0, 32 * MB);
      else reduce(BoolC<false>{}, q_lo, q_hi);
    }
    if constexpr (MODE == MODE_SIGMA) {
      // Sum of rho^2 over this wave's offsets for each owned row: per lane over its NB
      // columns, then across the 32 lanes of each half by a transposing butterfly (after
      // the step of width w a lane keeps the half of its partial sums selected by lane
      // bit w), so lane n of a half ends with the sum for slot n = 16t + 4g + i4.  The sums
      // are added to the per-template fixed-point totals, exact and order-independent.
      static_assert(MB == 2, "the sigma pass is compiled for two template blocks");
      // single-pass tail search: every owned (tau, k) with |rho| above the predicted lower
      // threshold is kept as a candidate (rows and ownership as in the tails pass).  One
      // sweep sums rho^2 and flags a lane holding any candidate (a row it does not own
      // compares against +inf); the rare flagged lanes append theirs in a second sweep.
      const bool cand = sg.c_tau != nullptr;
      const float* th = sg.thr_lo + kbase + 4 * h;
      const int qh = r_lo - 4 * h;
      const unsigned span = (unsigned)(r_hi - r_lo);
      float q[32];
#pragma unroll
      for (int v = 0; v < 32; ++v) q[v] = 0.0f;
      bool any = false;
#pragma unroll
      for (int t = 0; t < MB; ++t)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          float tv[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
          if (cand) {
            const float4 t4 = *(const float4*)(th + 32 * t + 8 * g);
            tv[0] = t4.x; tv[1] = t4.y; tv[2] = t4.z; tv[3] = t4.w;
#pragma unroll
            for (int i = 0; i < 4; ++i)
              tv[i] = (unsigned)(32 * t + 8 * g + i - qh) < span ? tv[i] : INFINITY;
          }
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float rf = (acc[t][j][4 * g + i] * dscale) * invf[j];
              q[16 * t + 4 * g + i] = fmaf(rf, rf, q[16 * t + 4 * g + i]);
              any = any || fabsf(rf) > tv[i];
            }
        }
      if (any) {
#pragma unroll
        for (int t = 0; t < MB; ++t)
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const float4 t4 = *(const float4*)(th + 32 * t + 8 * g);
            const float tv[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int c = 32 * t + 8 * g + i;
                const float rf = (acc[t][j][4 * g + i] * dscale) * invf[j];
                if (fabsf(rf) > tv[i] && (unsigned)(c - qh) < span) {
                  const int shard = (int)(blockIdx.x & (CAND_SHARDS - 1));
                  const int64_t per = sg.cand_cap / CAND_SHARDS;
                  const unsigned long long slot = atomicAdd(sg.n_cand + shard, 1ull);
                  if ((int64_t)slot < per) {
                    const int64_t at = shard * per + (int64_t)slot;
                    sg.c_tau[at] = (int32_t)(tau_w0 + 32 * j + n);
                    sg.c_k[at] = (int32_t)(kbase + c + 4 * h);
                    sg.c_rho[at] = rf;
                  }
                }
              }
          }
      }
#pragma unroll
      for (int w = 16; w >= 1; w >>= 1) {
        const bool up = (n & w) != 0;
#pragma unroll
        for (int i = 0; i < w; ++i) {
          const float keep = up ? q[w + i] : q[i];
          const float give = up ? q[i] : q[w + i];
          q[i] = keep + __shfl_xor(give, w, 64);
        }
      }
      const int row = 32 * (n >> 4) + 8 * ((n & 15) >> 2) + 4 * h + (n & 3);
      if (row >= r_lo && row < r_hi) {
        const unsigned long long f =
            (unsigned long long)__double2ll_rn((double)q[0] * SIGMA_FIX_SCALE);
        if (f) atomicAdd(sg.sig_acc + kbase + row, f);
      }
    }
    park();
  }
  unpark();
  if (cur_bin >= 0) flush_bin<NB>(sg, b, p, cur_bin, binmax, inv, tau_w0, n, h, lane, dscale);

  // ---- per-offset maxima: combine the two row halves, then one atomic per offset ----
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const float ov = __shfl_xor(best[j], 32, 64);
    const int ok = __shfl_xor(bestk[j], 32, 64);
    if (ov > best[j] || (ov == best[j] && ok >= 0 && (bestk[j] < 0 || ok < bestk[j]))) {
      best[j] = ov;
      bestk[j] = ok;
    }
    const int64_t tau = tau_w0 + 32 * j + n;
    if (h == 0 && tau < sg.W && bestk[j] >= 0) {
      const unsigned int kg = (unsigned int)(b.k_offset + bestk[j]);
      const unsigned long long key =
          ((unsigned long long)__float_as_uint(best[j] * dscale) << 32) | (0xFFFFFFFFull - kg);
      atomicMax(sg.mkey + tau, key);
    }
  }
}

// Each work-group runs items blockIdx.x, blockIdx.x + gridDim.x, ...: one item per
// work-group for a plain batch launch, a persistent loop for captured launches whose grid
// is fixed while the batch changes.
template <int PREC, int MB, int NB, int PIPE, int MODE>
__global__ __launch_bounds__(WG_THREADS, 1) void k_main(const BatchHdr* __restrict__ hdr,
                                                        BankDev b, SearchDev p) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int64_t n_items = hdr->n_items;
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    main_item<PREC, MB, NB, PIPE, MODE>(hdr, item, b, p, lds);
    __syncthreads();   // the next item refills the strip
  }
}

template <int PREC, int MB, int NB, int PIPE, int MODE>
static hipError_t prepare_main_t(const BankDev& b) {
  const size_t lds = main_lds_bytes(PREC, b.L_pad, 32 * NB * WG_WAVES);
  return hipFuncSetAttribute((const void*)k_main<PREC, MB, NB, PIPE, MODE>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int PREC, int MB, int NB, int PIPE, int MODE>
static hipError_t launch_main_t(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                                const SearchDev& p, hipStream_t s) {
  const size_t lds = main_lds_bytes(PREC, b.L_pad, 32 * NB * WG_WAVES);
  hipLaunchKernelGGL((k_main<PREC, MB, NB, PIPE, MODE>), dim3((unsigned)blocks), dim3(WG_THREADS), lds, s,
                     hdr, b, p);
  return hipGetLastError();
}

// The compiled kernel variants: (template blocks, offset blocks per wave, K-loop schedule)
// for the search; the two passes of the tail search exist for each precision's default
// shape only (2 x 8 interleaved for the split forms, 2 x 8 pair streaming for F16F8 and
// F16F6, 2 x 4 otherwise).
#define BFLY_DISPATCH(FN, ...)                                                         \
  do {                                                                                 \
    const int v_ = p.pipe * 256 + p.tm * 16 + p.tn;                                    \
    if (p.mode != MODE_SEARCH) {                                                       \
      const bool m1_ = p.mode == MODE_SIGMA;                                           \
      if (b.precision == P_FP32 && v_ == 0x024)                                        \
        return m1_ ? FN<P_FP32, 2, 4, 0, MODE_SIGMA>(__VA_ARGS__)                      \
                   : FN<P_FP32, 2, 4, 0, MODE_TAILS>(__VA_ARGS__);                     \
      if (b.precision == P_BF16X3 && v_ == 0x128)                                      \
        return m1_ ? FN<P_BF16X3, 2, 8, 1, MODE_SIGMA>(__VA_ARGS__)                    \
                   : FN<P_BF16X3, 2, 8, 1, MODE_TAILS>(__VA_ARGS__);                   \
      if (b.precision == P_F16X2 && v_ == 0x128)                                       \
        return m1_ ? FN<P_F16X2, 2, 8, 1, MODE_SIGMA>(__VA_ARGS__)                     \
                   : FN<P_F16X2, 2, 8, 1, MODE_TAILS>(__VA_ARGS__);                    \
      if (b.precision == P_FP8 && v_ == 0x024)                                         \
        return m1_ ? FN<P_FP8, 2, 4, 0, MODE_SIGMA>(__VA_ARGS__)                       \
                   : FN<P_FP8, 2, 4, 0, MODE_TAILS>(__VA_ARGS__);                      \
      if (b.precision == P_F16F8 && v_ == 0x228)                                       \
        return m1_ ? FN<P_F16F8, 2, 8, 2, MODE_SIGMA>(__VA_ARGS__)                     \
                   : FN<P_F16F8, 2, 8, 2, MODE_TAILS>(__VA_ARGS__);                    \
      if (b.precision == P_F16F6 && v_ == 0x228)                                       \
        return m1_ ? FN<P_F16F6, 2, 8, 2, MODE_SIGMA>(__VA_ARGS__)                     \
                   : FN<P_F16F6, 2, 8, 2, MODE_TAILS>(__VA_ARGS__);                    \
      return hipErrorInvalidValue;                                                     \
    }                                                                                  \
    if (b.precision == P_FP32) {                                                       \
      if (v_ == 0x024) return FN<P_FP32, 2, 4, 0, MODE_SEARCH>(__VA_ARGS__);           \
      if (v_ == 0x018) return FN<P_FP32, 1, 8, 0, MODE_SEARCH>(__VA_ARGS__);           \
    } else if (b.precision == P_BF16X3) {                                              \
      if (v_ == 0x024) return FN<P_BF16X3, 2, 4, 0, MODE_SEARCH>(__VA_ARGS__);         \
      if (v_ == 0x018) return FN<P_BF16X3, 1, 8, 0, MODE_SEARCH>(__VA_ARGS__);         \
      if (v_ == 0x028) return FN<P_BF16X3, 2, 8, 0, MODE_SEARCH>(__VA_ARGS__);         \
      if (v_ == 0x124) return FN<P_BF16X3, 2, 4, 1, MODE_SEARCH>(__VA_ARGS__);         \
      if (v_ == 0x128) return FN<P_BF16X3, 2, 8, 1, MODE_SEARCH>(__VA_ARGS__);         \
    } else if (b.precision == P_F16X2) {                                               \
      if (v_ == 0x024) return FN<P_F16X2, 2, 4, 0, MODE_SEARCH>(__VA_ARGS__);          \
      if (v_ == 0x028) return FN<P_F16X2, 2, 8, 0, MODE_SEARCH>(__VA_ARGS__);          \
      if (v_ == 0x128) return FN<P_F16X2, 2, 8, 1, MODE_SEARCH>(__VA_ARGS__);          \
    } else if (b.precision == P_FP8) {                                                 \
      if (v_ == 0x024) return FN<P_FP8, 2, 4, 0, MODE_SEARCH>(__VA_ARGS__);            \
      if (v_ == 0x018) return FN<P_FP8, 1, 8, 0, MODE_SEARCH>(__VA_ARGS__);            \
      if (v_ == 0x128) return FN<P_FP8, 2, 8, 1, MODE_SEARCH>(__VA_ARGS__);            \
    } else if (b.precision == P_F16F8) {                                               \
      if (v_ == 0x228) return FN<P_F16F8, 2, 8, 2, MODE_SEARCH>(__VA_ARGS__);          \
    } else if (b.precision == P_F16F6) {                                               \
      if (v_ == 0x228) return FN<P_F16F6, 2, 8, 2, MODE_SEARCH>(__VA_ARGS__);          \
    }                                                                                  \
    return hipErrorInvalidValue;                                                       \
  } while (0)

bool main_variant_exists(int precision, int tm, int tn, int pipe, int mode) {
  const int v = pipe * 256 + tm * 16 + tn;
  if (is_f16r(precision)) return v == 0x228;
  if (mode != MODE_SEARCH)
    return v == ((precision == P_BF16X3 || precision == P_F16X2) ? 0x128 : 0x024);
  if (precision == P_BF16X3)
    return v == 0x024 || v == 0x018 || v == 0x028 || v == 0x124 || v == 0x128;
  if (precision == P_FP8) return v == 0x024 || v == 0x018 || v == 0x128;
  if (precision == P_F16X2) return v == 0x024 || v == 0x028 || v == 0x128;
  return v == 0x024 || v == 0x018;
}

// Sets the kernel's dynamic-LDS limit; call before launching (and before capturing).
hipError_t prepare_main(const BankDev& b, const SearchDev& p) {
  BFLY_DISPATCH(prepare_main_t, b);
}

hipError_t launch_main(const BatchHdr* hdr, int64_t blocks, const BankDev& b,
                       const SearchDev& p, hipStream_t s) {
  if (blocks < 1) return hipSuccess;
  BFLY_DISPATCH(launch_main_t, hdr, blocks, b, p, s);
}

// ---------------------------------------------------------------------------------------
// Finalise: m = f32(|d|max * inv_norm) in float64, argmax from the packed key, histogram of
// m over non-degenerate windows (LDS-privatised), degenerate count, spectrum = fixed-point
// sum / (2^32 W).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(const BatchHdr* __restrict__ hdr, BankDev b,
                                                  SearchDev p) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  __shared__ unsigned int hl[MAX_HIST_BINS];
  __shared__ unsigned int ndeg, nok;
  const int tid = threadIdx.x;
  for (int i = tid; i < p.hist_bins; i += 256) hl[i] = 0u;
  if (tid == 0) ndeg = nok = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned int my_deg = 0u, my_ok = 0u;
  const double span = p.hist_hi - p.hist_lo;
  for (int64_t tau = (int64_t)blockIdx.x * blockDim.x + tid; tau < sg.W; tau += stride) {
    const double inv = sg.inv_norm[tau];
    if (inv > 0.0) {
      const unsigned long long key = sg.mkey[tau];
      const float d = __uint_as_float((unsigned int)(key >> 32));
      const float m = (float)((double)d * inv);
      const int a = (int)(0xFFFFFFFFull - (key & 0xFFFFFFFFull));
      if (sg.max_abs) sg.max_abs[tau] = m;
      if (sg.argmax) sg.argmax[tau] = a;
      double q = floor(((double)m - p.hist_lo) / span * (double)p.hist_bins);
      q = q > 0.0 ? q : 0.0;  // also maps NaN to bin 0
      q = q > (double)(p.hist_bins - 1) ? (double)(p.hist_bins - 1) : q;
      atomicAdd(&hl[(int)q], 1u);
      ++my_ok;
    } else {
      if (sg.max_abs) sg.max_abs[tau] = 0.0f;
      if (sg.argmax) sg.argmax[tau] = -1;
      ++my_deg;
    }
  }
  if (my_deg) atomicAdd(&ndeg, my_deg);
  if (my_ok) atomicAdd(&nok, my_ok);
  __syncthreads();
  if (tid == 0 && sg.n_ok && nok) atomicAdd(sg.n_ok, (unsigned long long)nok);
  if (sg.hist)
    for (int i = tid; i < p.hist_bins; i += 256)
      if (hl[i]) atomicAdd(sg.hist + i, hl[i]);
  if (tid == 0 && sg.n_degenerate && ndeg)
    atomicAdd((unsigned long long*)sg.n_degenerate, (unsigned long long)ndeg);
  if (blockIdx.x == 0 && sg.spectrum)
    for (int i = tid; i < b.n_bins; i += 256)
      sg.spectrum[i] = (double)sg.spec_acc[i] / SPEC_FIX_SCALE / (double)sg.W;
}

hipError_t launch_finalize(const BatchHdr* hdr, int32_t seg_slots, int32_t x_blocks,
                           const BankDev& b, const SearchDev& p, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)x_blocks, (unsigned)seg_slots), dim3(256), 0, s,
                     hdr, b, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// sigma_k = sqrt(sum_tau rho_k^2 / n_ok) from the fixed-point sums of the sigma pass, and the
// tail threshold kappa * sigma_k (float32, as the tails pass compares float32 rho); +inf for
// padding templates and for a series without a non-degenerate offset.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sigma(const BatchHdr* __restrict__ hdr, BankDev b,
                                               SearchDev p) {
  if ((int)blockIdx.y >= hdr->n_segs) return;
  const SegDesc& sg = hdr_segs(hdr)[blockIdx.y];
  const double nok = (double)sg.n_ok[0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < b.K_pad; k += stride) {
    float thr = __builtin_inff();
    if (k < b.K) {
      unsigned long long acc = 0ull;
      if (sg.sig_part)   // FFT form: per block and wave, with the single pass's flag bit
        for (int64_t r = 0; r < 4 * sg.n_tiles; ++r) acc += sg.sig_part[r * b.K_pad + k] & ~SIG_FLAG;
      else
        acc = sg.sig_acc[k];
      const double sd = nok > 0.0 ? sqrt((double)acc / SIGMA_FIX_SCALE / nok) : 0.0;
      if (sg.sigma) sg.sigma[k] = (float)sd;
      if (nok > 0.0) thr = (float)((double)p.kappa * sd);
    }
    sg.thr[k] = thr;
  }
}

hipError_t launch_sigma(const BatchHdr* hdr, int32_t seg_slots, const BankDev& b,
                        const SearchDev& p, hipStream_t s) {
  const int64_t xb = (b.K_pad + 255) / 256;
  hipLaunchKernelGGL(k_sigma, dim3((unsigned)(xb < 1024 ? xb : 1024), (unsigned)seg_slots),
                     dim3(256), 0, s, hdr, b, p);
  return hipGetLastError();
}

hipError_t launch_norms(const BatchHdr* hdr, int32_t seg_slots, int32_t x_blocks, int L,
                        int norm, hipStream_t s) {
  hipLaunchKernelGGL(k_norms, dim3((unsigned)x_blocks, (unsigned)seg_slots), dim3(256), 0, s,
                     hdr, L, norm);
  return hipGetLastError();
}

}  // namespace bfly
