// Device kernels of the dedispersion + correlation path (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "fft.hpp"

namespace ddx {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Workgroup-id remap so that consecutive logical ids run on the same XCD: the
// dispatcher deals workgroup ids round-robin over the 8 XCDs, so logical ids
// [x*q + min(x, r) ...) are made to land on XCD x (q = G / 8, r = G % 8).
__device__ __forceinline__ int xcd_remap(int bid, int grid) {
  const int x = bid & 7, i = bid >> 3, q = grid >> 3, r = grid & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// ---------------------------------------------------------------------------
// Sample source: the current chunk [C][M][n] plus the history carried over from
// earlier calls [C][M][hist_cap]; absolute sample index abs.
struct Source {
  const void* chunk;
  const void* hist;
  int64_t chunk_stride;  // samples per (c, p) row of chunk
  int64_t hist_cap;      // samples per (c, p) row of hist
  int64_t hist_start;    // absolute index of hist row element 0 (this channel)
  int64_t chunk_start;   // absolute index of chunk row element 0
  int64_t chunk_len;     // samples present in the chunk rows
  int32_t row;           // c * M + p
};

template <int IN>
__device__ __forceinline__ float2 load_sample(const Source& s, int64_t abs) {
  if (abs < 0) return make_float2(0.f, 0.f);
  const void* base;
  int64_t idx;
  if (abs < s.chunk_start) {
    base = s.hist;
    idx = (int64_t)s.row * s.hist_cap + (abs - s.hist_start);
  } else {
    const int64_t rel = abs - s.chunk_start;
    if (rel >= s.chunk_len) return make_float2(0.f, 0.f);
    base = s.chunk;
    idx = (int64_t)s.row * s.chunk_stride + rel;
  }
  if (IN == 0) {
    const char2 v = reinterpret_cast<const char2*>(base)[idx];
    return make_float2((float)v.x, (float)v.y);
  } else {
    return reinterpret_cast<const float2*>(base)[idx];
  }
}

// ---------------------------------------------------------------------------
// Forward FFT of every overlap-save block of one channel.
// grid: nblk * M workgroups (block fastest); output spec[(p * nblk + blk) * N + k].
struct FwdArgs {
  Source src;
  float2* spec;
  int64_t b0;  // absolute index of the first block
  int32_t nblk, n_ant, valid, lead, chan;
};

template <int LOGN, int IN>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_forward(FwdArgs a) {
  using G = Geo<LOGN>;
  extern __shared__ float lds[];
  const int t = threadIdx.x;
  const int blk = blockIdx.x % a.nblk, p = blockIdx.x / a.nblk;
  Source s = a.src;
  s.row = a.chan * a.n_ant + p;
  const int64_t win0 = (a.b0 + blk) * (int64_t)a.valid - a.lead;
  float2 v[G::P];
  fft_workgroup<LOGN, -1>(v, lds, t, [&](int i) { return load_sample<IN>(s, win0 + i); });
  // output addresses are formed only now (otherwise they are hoisted and held in registers)
  float2* out = a.spec + ((size_t)p * a.nblk + blk) * G::N + opaque_zero(v[0].x);
#pragma unroll
  for (int u = 0; u < G::P / G::RL; ++u)
#pragma unroll
    for (int q = 0; q < G::RL; ++q) out[t + u * G::T + q * (G::N / G::RL)] = v[u * G::RL + out_reg<G::RL>(q)];
}

// ---------------------------------------------------------------------------
// Chirp table H[d][k] = exp(-2 pi i r) / N with r = u - rint(u), u = kdm[d] * g[k]
// in FP64 (g[k] = f_k^2 / (f_c^2 (f_c + f_k)), kdm[d] = K DM_d).
__global__ __launch_bounds__(256) void k_chirp(const double* __restrict__ g, const double* __restrict__ kdm,
                                               float2* __restrict__ h, int n, float inv_n) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int d = blockIdx.y;
  if (k >= n) return;
  const double u = kdm[d] * g[k];
  const float r = (float)(u - rint(u));
  h[(size_t)d * n + k] = make_float2(cos_rev(r) * inv_n, -sin_rev(r) * inv_n);
}

// ---------------------------------------------------------------------------
// Output conversion of the dedispersed voltages.
template <int OUT> struct YType;
template <> struct YType<0> { typedef float2 T; };   // FP32
template <> struct YType<1> { typedef __half2 T; };  // binary16 pair
template <> struct YType<2> { typedef uint16_t T; }; // two E4M3 bytes (re low, im high)

template <int OUT>
__device__ __forceinline__ typename YType<OUT>::T convert_y(float2 v, float scale) {
  if constexpr (OUT == 0) {
    return v;
  } else if constexpr (OUT == 1) {
    const float m = 65504.f;
    const float re = fminf(fmaxf(v.x * scale, -m), m), im = fminf(fmaxf(v.y * scale, -m), m);
    return __halves2half2(__float2half_rn(re), __float2half_rn(im));
  } else {
    const float m = 448.f;
    const float re = fminf(fmaxf(v.x * scale, -m), m), im = fminf(fmaxf(v.y * scale, -m), m);
    // hardware conversion rounds to nearest even; the clamp above makes it saturate
    const int packed = __builtin_amdgcn_cvt_pk_fp8_f32(re, im, 0, false);
    return (uint16_t)(packed & 0xffff);
  }
}

// Chirp multiply, inverse FFT and overlap-save discard for nd DMs of one channel.
// grid: M * nblk * nd workgroups, logical id = (p * nblk + blk) * nd + d (XCD-remapped).
// y[(d * M + p) * y_stride + blk * V + j] = IDFT(X H)[lead + j] for j < V.
struct DedispArgs {
  const float2* spec;
  const float2* chirp;  // [nd][N] (already offset to the first DM of the group)
  void* y;
  int64_t y_stride;
  const float* scale;   // device scalar: correlator-input scale of this channel
  int32_t n_ant, nblk, nd, valid, lead;
};

template <int LOGN, int OUT>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_dedisperse(DedispArgs a) {
  using G = Geo<LOGN>;
  extern __shared__ float lds[];
  const int t = threadIdx.x;
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int d = lin % a.nd;
  const int rest = lin / a.nd;
  const int blk = rest % a.nblk, p = rest / a.nblk;
  const float2* x = a.spec + ((size_t)p * a.nblk + blk) * G::N;
  const float2* h = a.chirp + (size_t)d * G::N;
  float2 v[G::P];
  fft_workgroup<LOGN, +1>(v, lds, t, [&](int i) { return cmul(x[i], h[i]); });
  const float scale = (OUT == 0) ? 1.f : *a.scale;
  typedef typename YType<OUT>::T YT;
  // output addresses are formed only now (otherwise they are hoisted and held in registers)
  YT* y = reinterpret_cast<YT*>(a.y) + ((size_t)d * a.n_ant + p) * a.y_stride + (size_t)blk * a.valid +
          opaque_zero(v[0].x);
#pragma unroll
  for (int u = 0; u < G::P / G::RL; ++u)
#pragma unroll
    for (int q = 0; q < G::RL; ++q) {
      const int n = t + u * G::T + q * (G::N / G::RL);
      if (n >= a.lead && n < a.lead + a.valid) y[n - a.lead] = convert_y<OUT>(v[u * G::RL + out_reg<G::RL>(q)], scale);
    }
}

// ---------------------------------------------------------------------------
// Correlator: per (DM, dump) the Gram matrix of the stacked real rows
// [Re y_0 .. Re y_{M-1}, Im y_0 .. Im y_{M-1}] over the L samples of the dump,
// G = A A^T on FP32 MFMA (16x16x4) over the upper 16x16 tiles, then
//   Re V_ij = G[i][j] + G[M+i][M+j],  Im V_ij = G[j][M+i] - G[i][M+j].
// grid: n_dumps * nd workgroups of 256 threads (4 waves), logical id = m * nd + d.
struct CorrArgs {
  const void* y;
  int64_t y_stride;      // samples per (d, p) row
  float2* ring;
  int64_t rec_elems;     // complex values per dump record
  int64_t ring_dumps;    // ring capacity in dumps
  int64_t dump0;         // absolute dump index of y sample 0
  const int32_t* dm_pos; // [nd] record position (dm_offset[c] + d) of each DM of the group
  const float* scale;    // device scalar s_c (quantised inputs), ignored for FP32
  int32_t n_dumps, nd, n_ant, dump_len, nbl, out_mode;
};

constexpr int kCorrKC = 32;  // samples per LDS chunk

template <int NT>  // 16 NT >= 2 M rows
struct CorrGeo {
  static constexpr int ROWS = 16 * NT;
  static constexpr int RP = ROWS + ((17 - (ROWS % 32)) + 32) % 32;  // >= ROWS, == 17 mod 32
  static constexpr int NTILES = NT * (NT + 1) / 2;
  static constexpr int TPW = (NTILES + 3) / 4;
  static constexpr int GP = ROWS + 1;
};

template <int NT>
__global__ __launch_bounds__(256) void k_correlate_f32(CorrArgs a) {
  using C = CorrGeo<NT>;
  __shared__ float at[kCorrKC * C::RP];
  __shared__ float gram[C::ROWS * C::GP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lin = blockIdx.x;
  const int d = lin % a.nd, m = lin / a.nd;
  const int M = a.n_ant, L = a.dump_len;

  // tiles of this wave
  int ti[C::TPW], tj[C::TPW];
#pragma unroll
  for (int i = 0; i < C::TPW; ++i) {
    int id = wave + 4 * i, I = 0;
    while (id >= NT - I && I < NT) { id -= NT - I; ++I; }
    ti[i] = I;
    tj[i] = I + id;
  }
  floatx4 acc[C::TPW];
#pragma unroll
  for (int i = 0; i < C::TPW; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};

  // zero the padding rows once
  for (int e = tid; e < kCorrKC * (C::ROWS - 2 * M); e += 256) {
    const int n = e / (C::ROWS - 2 * M), r = 2 * M + e % (C::ROWS - 2 * M);
    at[n * C::RP + r] = 0.f;
  }
  const float2* y = reinterpret_cast<const float2*>(a.y) + (size_t)d * M * a.y_stride + (size_t)m * L;
  for (int k0 = 0; k0 < L; k0 += kCorrKC) {
    for (int e = tid; e < M * kCorrKC; e += 256) {
      const int p = e / kCorrKC, n = e % kCorrKC;
      const float2 val = (k0 + n < L) ? y[(size_t)p * a.y_stride + k0 + n] : make_float2(0.f, 0.f);
      at[n * C::RP + p] = val.x;
      at[n * C::RP + M + p] = val.y;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kCorrKC; kk += 4) {
      const int kr = (kk + (lane >> 4)) * C::RP + (lane & 15);
#pragma unroll
      for (int i = 0; i < C::TPW; ++i) {
        if (wave + 4 * i < C::NTILES) {
          const float av = at[kr + ti[i] * 16], bv = at[kr + tj[i] * 16];
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[i], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < C::TPW; ++i) {
    if (wave + 4 * i < C::NTILES) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        gram[(ti[i] * 16 + 4 * (lane >> 4) + r) * C::GP + tj[i] * 16 + (lane & 15)] = acc[i][r];
    }
  }
  __syncthreads();
  const int64_t dump = a.dump0 + m;
  float2* out = a.ring + (dump % a.ring_dumps) * a.rec_elems + (int64_t)a.dm_pos[d] * a.nbl;
  if (a.out_mode == 0) {
    for (int b = tid; b < a.nbl; b += 256) {
      // invert b = i M - i (i - 1) / 2 + (j - i)
      int i = 0, rem = b;
      while (rem >= M - i) { rem -= M - i; ++i; }
      const int j = i + rem;
      const float re = gram[i * C::GP + j] + gram[(M + i) * C::GP + M + j];
      const float im = gram[j * C::GP + M + i] - gram[i * C::GP + M + j];
      out[b] = make_float2(re, im);
    }
  } else {
    for (int b = tid; b < M * M; b += 256) {
      const int i = b / M, j = b % M;
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      const float re = gram[lo * C::GP + hi] + gram[(M + lo) * C::GP + M + hi];
      const float im = gram[hi * C::GP + M + lo] - gram[lo * C::GP + M + hi];
      out[b] = make_float2(re, i <= j ? im : -im);
    }
  }
}

// Zero the record slots of inactive DMs for the dumps of one call.
__global__ void k_zero_dm(float2* ring, int64_t rec_elems, int64_t ring_dumps, int64_t dump0, int32_t n_dumps,
                          const int32_t* dm_pos, int32_t n_pos, int32_t nbl) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)n_dumps * n_pos * nbl;
  if (e >= total) return;
  const int b = (int)(e % nbl);
  const int64_t rest = e / nbl;
  const int k = (int)(rest % n_pos);
  const int64_t m = rest / n_pos;
  ring[((dump0 + m) % ring_dumps) * rec_elems + (int64_t)dm_pos[k] * nbl + b] = make_float2(0.f, 0.f);
}

// Carry the unconsumed input tail of one channel into the next history buffer.
// grid: (ceil(len / 256), M); dst row c*M+p holds samples [start, start + len).
template <int IN>
__global__ void k_history(Source s, void* dst, int64_t start, int64_t len, int32_t n_ant, int32_t chan) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  s.row = chan * n_ant + blockIdx.y;
  const int64_t di = (int64_t)s.row * s.hist_cap + i;
  if (IN == 0) {
    const float2 v = load_sample<0>(s, start + i);
    reinterpret_cast<char2*>(dst)[di] = make_char2((signed char)v.x, (signed char)v.y);
  } else {
    reinterpret_cast<float2*>(dst)[di] = load_sample<1>(s, start + i);
  }
}

}  // namespace ddx
