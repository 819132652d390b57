// Kernels of the DM-time power tiles of the learned DM proposal (incoherent
// dedispersion of power beams).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddx {

// ---------------------------------------------------------------------------
// Power per sample summed over antennas, p[c][n] = sum_p |x_{c,p}[n]|^2, for a
// whole stream [C][M][n] (IN = 0: int8 pairs, 1: float pairs).  For int8 every
// partial sum is an integer below 2^24, so it is exact in FP32.
template <int IN>
__global__ void k_beam_power(const void* __restrict__ volts, int64_t n, int32_t n_ant, float* __restrict__ power) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  float acc = 0.f;
  for (int p = 0; p < n_ant; ++p) {
    const int64_t idx = ((int64_t)c * n_ant + p) * n + i;
    float re, im;
    if (IN == 0) {
      const char2 v = reinterpret_cast<const char2*>(volts)[idx];
      re = v.x;
      im = v.y;
    } else {
      const float2 v = reinterpret_cast<const float2*>(volts)[idx];
      re = v.x;
      im = v.y;
    }
    acc += re * re + im * im;
  }
  power[(int64_t)c * n + i] = acc;
}

constexpr int kScanBlock = 1024;  // elements per scan workgroup (256 threads x 4)

// Inclusive scan of each row of `power` ([rows][units], FP32) into FP64
// prefix[row][1 + u]; prefix[row][0] = 0.  Pass 1: scan within blocks of
// kScanBlock and write block totals.
__global__ __launch_bounds__(256) void k_scan_local(const float* __restrict__ power, int64_t units,
                                                    double* __restrict__ prefix, double* __restrict__ totals,
                                                    int32_t nblk) {
  __shared__ double part[256];
  const int row = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
  const int64_t base = (int64_t)b * kScanBlock + 4 * tid;
  const float* src = power + (int64_t)row * units;
  double v[4], s = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[e] = (base + e < units) ? (double)src[base + e] : 0.0;
    s += v[e];
    v[e] = s;
  }
  part[tid] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 256 thread sums (fixed order: deterministic)
  for (int off = 1; off < 256; off <<= 1) {
    const double add = tid >= off ? part[tid - off] : 0.0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  const double before = tid > 0 ? part[tid - 1] : 0.0;
  double* dst = prefix + (int64_t)row * (units + 1);
  if (b == 0 && tid == 0) dst[0] = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (base + e < units) dst[1 + base + e] = before + v[e];
  if (tid == 255) totals[(int64_t)row * nblk + b] = part[255];
}

// Pass 2: add the sum of all earlier block totals of the row (summed serially in
// a fixed order by one thread, so results do not depend on scheduling).
__global__ __launch_bounds__(256) void k_scan_fix(double* __restrict__ prefix, int64_t units,
                                                  const double* __restrict__ totals, int32_t nblk) {
  __shared__ double off;
  const int row = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
  if (b == 0) return;
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < b; ++j) s += totals[(int64_t)row * nblk + j];
    off = s;
  }
  __syncthreads();
  double* dst = prefix + (int64_t)row * (units + 1) + 1;
  for (int e = tid; e < kScanBlock; e += 256) {
    const int64_t u = (int64_t)b * kScanBlock + e;
    if (u < units) dst[u] += off;
  }
}

// Tile T[tile][d][t] = C B * sum_c (S_c[a1] - S_c[a0]) / sum_c (a1 - a0), with
// a0 = clamp(t B + sh[c][d]), a1 = clamp(a0' + B) in fine units (B = bin length in
// fine units, sh = shift rounded to fine units), S the per-channel prefix sums.
// grid: (ceil(n_bins / 256), D, tiles).
__global__ __launch_bounds__(256) void k_tile(const double* __restrict__ prefix, int64_t units, int32_t n_chan,
                                              const int64_t* __restrict__ sh, int32_t n_dm, int32_t bin_units,
                                              int32_t n_bins, float* __restrict__ tile) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int d = blockIdx.y, tl = blockIdx.z;
  if (t >= n_bins) return;
  const double* pre = prefix + (int64_t)tl * n_chan * (units + 1);
  double tot = 0.0;
  int64_t cnt = 0;
  for (int c = 0; c < n_chan; ++c) {
    const int64_t s0 = (int64_t)t * bin_units + sh[(int64_t)c * n_dm + d];
    const int64_t a0 = s0 < 0 ? 0 : (s0 > units ? units : s0);
    const int64_t e0 = s0 + bin_units;
    const int64_t a1 = e0 < 0 ? 0 : (e0 > units ? units : e0);
    tot += pre[(int64_t)c * (units + 1) + a1] - pre[(int64_t)c * (units + 1) + a0];
    cnt += a1 - a0;
  }
  tile[((int64_t)tl * n_dm + d) * n_bins + t] = cnt > 0 ? (float)(tot * ((double)n_chan * bin_units) / (double)cnt) : 0.f;
}

}  // namespace ddx
