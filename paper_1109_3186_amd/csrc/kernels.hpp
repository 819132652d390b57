// Device kernels of the dedispersion + correlation path (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <type_traits>

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

// Element at a 32-bit byte offset from a base pointer (lets the compiler use the
// scalar-base + 32-bit vector-offset form of global loads).
template <class T>
__device__ __forceinline__ T at_byte(const T* base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}

// ---------------------------------------------------------------------------
// Work items of one ddx_process_block call.  The host lists them (all channels,
// all active DMs, all blocks the call completes) and copies the lists to the
// device; each launch below walks one list.  Offsets are in elements.
struct FwdItem {        // one overlap-save block of one channel, all M antennas
  int64_t win0;         // absolute sample index of the block window's first sample
  int64_t spec;         // spectrum of antenna 0 (antenna p at + p N)
  int64_t tb;           // two-pass transforms: intermediate rows of antenna 0 (antenna p at + p N)
  int64_t hist_start;   // absolute index of the channel's history element 0
  int32_t chan;
  int32_t logn;         // N = 2^logn
};
struct ChirpItem {      // one (channel, DM) of a wave
  int64_t g;            // the channel's g table
  int64_t out;          // chirp slot
  double kdm;           // K DM
  int32_t n;            // N_c
  int32_t logr;         // N_c = 2^(15 + logr) for two-pass transforms, else 0
  int32_t chan, pad;
};
struct UnitItem {       // one (channel, DM, block), all M antennas
  int64_t spec;         // spectrum of antenna 0 of the block
  int64_t chirp;        // chirp of the DM
  int64_t y;            // output row of antenna 0 (antenna p at + p y_stride)
  int64_t tb;           // two-pass transforms: intermediate rows of antenna 0
  int64_t dump0;        // absolute index of the block's first dump (b V / L)
  int64_t rec;          // offset of the (channel, DM) slot within a dump record
  int32_t chan, valid, lead;
  int32_t n_dumps;      // complete dumps of the block this call
  int32_t fwd;          // the block's forward item in this call's list
  int32_t pad;
};
struct ZeroItem {       // the inactive-DM slots of one (channel, dump) record
  int64_t rec;          // offset of the dump's record in the ring
  int32_t pos;          // first of the channel's inactive slots in the slot table
  int32_t n;            // inactive DMs of the channel
};

// ---------------------------------------------------------------------------
// Forward FFT of the overlap-save blocks of a list of (channel, block) items.
// grid: n_items * M workgroups (antenna fastest).  spec[it.spec + p N + k] = X[k].
struct FwdArgs {
  Source src;
  const FwdItem* items;
  float2* spec;
  float* l1;            // FP32 correlator inputs: per (item, antenna) 8 row sums of |Re X| + |Im X|
  int32_t n_ant;
  int32_t pad;
};

// Sum over a workgroup of one value per thread, in a fixed order (butterfly within
// each wave, then the waves in order); the result is valid in thread 0.  red: NT/64
// floats of LDS that no thread still reads.
template <int NT>
__device__ __forceinline__ float block_sum(float v, float* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if constexpr (NT <= 64) {
    return v;
  } else {
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0)
      for (int i = 0; i < NT / 64; ++i) t += red[i];
    return t;
  }
}

// sum of |Re| + |Im| of a thread's points, in register order
template <int P>
__device__ __forceinline__ float l1_of(const float2* v) {
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < P; ++i) s += fabsf(v[i].x) + fabsf(v[i].y);
  return s;
}

// FFT plan of k_forward (the 1024-thread 32768-point form spills here: the kernel
// holds both input paths).
template <int LOGN>
using FwdPlan = Plan<LOGN>;

template <int IN>
__device__ __forceinline__ float2 sample_at(const void* row, unsigned i) {
  if constexpr (IN == 0) {
    const char2 v = at_byte(reinterpret_cast<const char2*>(row), 2u * i);
    return make_float2((float)v.x, (float)v.y);
  } else {
    return at_byte(reinterpret_cast<const float2*>(row), 8u * i);
  }
}

template <int LOGN, int IN>
__global__ __launch_bounds__(Geo<FwdPlan<LOGN>>::T) void k_forward(FwdArgs a) {
  using PL = FwdPlan<LOGN>;
  using G = Geo<PL>;
  extern __shared__ float lds[];
  const int t = threadIdx.x;
  const int p = blockIdx.x % a.n_ant;
  const FwdItem w = a.items[blockIdx.x / a.n_ant];
  Source s = a.src;
  s.row = w.chan * a.n_ant + p;
  s.hist_start = w.hist_start;
  float2 v[G::P];
  // A window wholly inside this call's chunk (every block but those at a call's
  // start, the stream's start and the flush) reads its row directly with 32-bit
  // offsets; the others go through the history / chunk / zero selection per sample.
  const int64_t rel0 = w.win0 - s.chunk_start;
  if (rel0 >= 0 && rel0 + G::N <= s.chunk_len) {
    const char* row = reinterpret_cast<const char*>(s.chunk) +
                      ((int64_t)s.row * s.chunk_stride + rel0) * (IN == 0 ? 2 : 8);
    fft_workgroup<PL, -1>(v, lds, t, [&](int i) { return sample_at<IN>(row, (unsigned)i); });
  } else {
    fft_workgroup<PL, -1>(v, lds, t, [&](int i) { return load_sample<IN>(s, w.win0 + i); });
  }
  // output addresses are formed only now (otherwise they are hoisted and held in registers)
  float2* out = a.spec + w.spec + (size_t)p * G::N + opaque_zero(v[0].x);
#pragma unroll
  for (int u = 0; u < G::P / G::RL; ++u)
#pragma unroll
    for (int q = 0; q < G::RL; ++q) out[t + u * G::T + q * (G::N / G::RL)] = v[u * G::RL + out_reg<G::RL>(q)];
  if (a.l1) {  // LDS is free after the last exchange
    const float tot = block_sum<G::T>(l1_of<G::P>(v), lds);
    if (t == 0) a.l1[(size_t)blockIdx.x * 8] = tot;  // (item, antenna) = blockIdx.x, row 0 of 8
  }
}

// Bound on the dedispersed voltages of each forward item (FP32 correlator inputs):
// for every DM, |y[n]| <= (1/N) sum_k |X_k H_k| with |H_k| = 1 and |X_k| <=
// |Re X_k| + |Im X_k|, so bound[item] = (max over antennas of that L1 sum) / N
// bounds every |Re y|, |Im y| of the block in input units (the stored values carry
// the channel's scale s on top).  The max does not depend on order; the row sums of
// a two-pass spectrum are added in row order.  grid: n_items workgroups of 256.
__global__ __launch_bounds__(256) void k_item_bound(const FwdItem* __restrict__ items, const float* __restrict__ l1,
                                                    int32_t n_ant, float* __restrict__ bound) {
  __shared__ float red[256];
  const FwdItem w = items[blockIdx.x];
  const int rows = w.logn > 15 ? 1 << (w.logn - 15) : 1;
  float m = 0.f;
  for (int p = threadIdx.x; p < n_ant; p += 256) {
    const float* r = l1 + ((size_t)blockIdx.x * n_ant + p) * 8;
    float s = 0.f;
    for (int k = 0; k < rows; ++k) s += r[k];
    m = fmaxf(m, s);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) bound[blockIdx.x] = red[0] * exp2f(-(float)w.logn);
}

// ---------------------------------------------------------------------------
// Chirp tables of a wave's (channel, DM) pairs: H[k] = s_c exp(-2 pi i r) / N with
// r = u - rint(u), u = kdm * g[k] in FP64 (g[k] = f_k^2 / (f_c^2 (f_c + f_k))).
// Folding the correlator-input scale s_c (a power of two) and 1/N in here makes the
// inverse transforms produce s_c y directly, with the same bits as scaling afterwards.
// Two-pass lengths store bin k1 + R k2 at position k1 2^15 + k2 (the order in
// which their spectra are kept).  grid: (ceil(max N / 256), n_items).
__global__ __launch_bounds__(256) void k_chirp(const ChirpItem* __restrict__ items, const double* __restrict__ g,
                                               const float* __restrict__ scale, float2* __restrict__ h) {
  const ChirpItem w = items[blockIdx.y];
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= w.n) return;
  const int k = w.logr ? ((q >> 15) + (q & 32767) * (1 << w.logr)) : q;
  const double u = w.kdm * g[w.g + k];
  const float r = (float)(u - rint(u));
  const float f = scale[w.chan] * (1.0f / (float)w.n);  // powers of two: exact
  h[w.out + q] = make_float2(cos_rev(r) * f, -sin_rev(r) * f);
}

// ---------------------------------------------------------------------------
// Output conversion of the dedispersed voltages (already s_c y).
template <int OUT> struct YType;
template <> struct YType<0> { typedef float2 T; };   // FP32
template <> struct YType<1> { typedef __half2 T; };  // binary16 pair
template <> struct YType<2> { typedef uint16_t T; }; // two E4M3 bytes (re low, im high)

template <int OUT>
__device__ __forceinline__ typename YType<OUT>::T convert_y(float2 v) {
  if constexpr (OUT == 0) {
    return v;
  } else if constexpr (OUT == 1) {
    const float m = 65504.f;
    const float re = fminf(fmaxf(v.x, -m), m), im = fminf(fmaxf(v.y, -m), m);
    return __halves2half2(__float2half_rn(re), __float2half_rn(im));
  } else {
    const float m = 448.f;
    const float re = fminf(fmaxf(v.x, -m), m), im = fminf(fmaxf(v.y, -m), m);
    // hardware conversion rounds to nearest even; the clamp above makes it saturate.
    // It writes the low 16 bits only; the high half (passed in, unused) is re's bits.
    const int packed = __builtin_amdgcn_cvt_pk_fp8_f32(re, im, __float_as_int(re), false);
    return (uint16_t)(packed & 0xffff);
  }
}

// Order of a wave's workgroups: logical ids (XCD-remapped, so a run of ids shares
// one XCD's L2) take `tile` units fastest (4; a wave of fewer than 8 units is one
// tile, so no workgroup idles), then the rows (antennas, or antenna x k1 rows of a
// two-pass transform), then the next tile of units.  Units run
// DM-fastest within a block, so the workgroups one XCD runs at a time read a few
// spectra and 4 chirps, and the 4 chirps stay in L2 while every antenna passes over
// them.  Measured on the 36-antenna workload: tiles of 2 to 8 units alike, 1 unit
// and whole-wave order 5-15 % slower, and grouping 8-9 antennas to keep their
// spectra for a whole DM group 3 % slower (more HBM reads, not fewer).
constexpr int kUnitTile = 4;

__host__ __device__ __forceinline__ int unit_tile(int n_units) { return n_units < 2 * kUnitTile ? n_units : kUnitTile; }
__host__ __device__ __forceinline__ int order_units(int n_units, int tile) {  // units covered by the grid
  return (n_units + tile - 1) / tile * tile;
}

__device__ __forceinline__ bool unit_row(int lin, int n_units, int n_rows, int tile, int& row, int& u) {
  const int ul = lin % tile;
  lin /= tile;
  row = lin % n_rows;
  u = (lin / n_rows) * tile + ul;
  return u < n_units;
}

// Dedispersed output stores bypass L2 retention (the spectra and chirps are what
// the next workgroups re-read).
template <class T>
__device__ __forceinline__ void store_stream(T* p, T v) {
  if constexpr (sizeof(T) == 8) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(*reinterpret_cast<const f2v*>(&v), reinterpret_cast<f2v*>(p));
  } else if constexpr (sizeof(T) == 4) {
    __builtin_nontemporal_store(*reinterpret_cast<const unsigned int*>(&v), reinterpret_cast<unsigned int*>(p));
  } else {
    __builtin_nontemporal_store(*reinterpret_cast<const unsigned short*>(&v), reinterpret_cast<unsigned short*>(p));
  }
}

// Buffer resource over `bytes` bytes at `base` (raw, stride 0, 32-bit data format).
// A store whose byte offset is at or past `bytes` is dropped by the hardware's range
// check, so a store that is kept only for some lanes needs no branch around it.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t range_rsrc(void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}

template <class T>
__device__ __forceinline__ void store_ranged(__amdgpu_buffer_rsrc_t r, unsigned byte_off, T v) {
  constexpr int aux = 2;  // non-temporal
  if constexpr (sizeof(T) == 8) {
    typedef unsigned int u2v __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(*reinterpret_cast<const u2v*>(&v), r, byte_off, 0, aux);
  } else if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(*reinterpret_cast<const unsigned int*>(&v), r, byte_off, 0, aux);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(*reinterpret_cast<const unsigned short*>(&v), r, byte_off, 0, aux);
  }
}

// FFT plan of k_dedisperse: the 1024-thread form of the 32768-point plan (four
// waves per SIMD instead of two hide more of the loads and exchanges: 2.41 against
// 2.61 ps per transform point for the FP32 output, measured with the second pass's
// twiddles from LDS; E4M3 2293 -> 2077 ms per 36-antenna step).
template <int LOGN, int OUT>
using DedispPlan = typename std::conditional<LOGN == 15, Plan15Wide, Plan<LOGN>>::type;

// Chirp multiply, inverse FFT and overlap-save discard for a wave of units.
// grid: order_units(n_units, tile) x M workgroups (see unit_row).
// y[u.y + p y_stride + j] = IDFT(X H)[lead + j] for j < V.
struct DedispArgs {
  const float2* spec;
  const float2* chirp;
  void* y;
  float2* tb;           // two-pass transforms: intermediate rows
  const UnitItem* units;
  float* power;         // binary16 / E4M3 outputs: per-dump power of the unrounded s_c y
  int64_t y_stride;
  int32_t n_ant, n_units, logr, tile;
  int32_t ant0;         // two-pass transforms: first antenna of the launch's group (n_ant antennas)
  int32_t dump_len;     // L
  int32_t pw_stride;    // power values per antenna row (dumps per block, V_max / L)
  int32_t pad;
};

// Power row of antenna p of a unit: the unit's y rows are [M][y_stride] from u.y,
// and its power rows [M][pw_stride] sit at the same row index.
__device__ __forceinline__ float* power_row(float* power, const UnitItem& u, int64_t y_stride, int pw_stride, int p) {
  return power + (u.y / y_stride + p) * (int64_t)pw_stride;
}

// Per-dump sums of `valid` values s(j), j < valid (valid a multiple of L), into
// out[m] = sum_{j in [m L, (m+1) L)} s(j), in a fixed order (so the result does not
// depend on scheduling): for L >= 64 (and workgroups of whole waves) one wave per
// dump, lane l summing s(m L + l + 64 i) in i order, then a butterfly over the 64
// lanes; otherwise one thread per dump summing in j order.
template <int NT, class S>
__device__ __forceinline__ void dump_sums(S s, int valid, int L, float* out, int t) {
  const int nd = valid / L;
  if (NT >= 64 && L >= 64) {
    const int wave = t >> 6, lane = t & 63;
    for (int m = wave; m < nd; m += (NT >= 64 ? NT / 64 : 1)) {
      float acc = 0.f;
      for (int i = lane; i < L; i += 64) acc += s(m * L + i);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0) out[m] = acc;
    }
  } else {
    for (int m = t; m < nd; m += NT) {
      float acc = 0.f;
      for (int i = 0; i < L; ++i) acc += s(m * L + i);
      out[m] = acc;
    }
  }
}

template <int LOGN, int OUT>
__global__ __launch_bounds__((Geo<DedispPlan<LOGN, OUT>>::T)) void k_dedisperse(DedispArgs a) {
  using G = Geo<DedispPlan<LOGN, OUT>>;
  extern __shared__ float lds[];
  const int t = threadIdx.x;
  int p, ui;
  if (!unit_row(xcd_remap(blockIdx.x, gridDim.x), a.n_units, a.n_ant, a.tile, p, ui)) return;
  const UnitItem w = a.units[ui];
  const float2* x = a.spec + w.spec + (size_t)p * G::N;
  const float2* h = a.chirp + w.chirp;
  float2 v[G::P];
  // 32-bit byte offsets from a uniform base: each load needs one 32-bit add, not a 64-bit address
  fft_workgroup<DedispPlan<LOGN, OUT>, +1>(v, lds, t,
                                           [&](int i) { return cmul(at_byte(x, 8u * (unsigned)i), at_byte(h, 8u * (unsigned)i)); });
  typedef typename YType<OUT>::T YT;
  // output addresses are formed only now (otherwise they are hoisted and held in registers)
  YT* y = reinterpret_cast<YT*>(a.y) + w.y + (size_t)p * a.y_stride;
  const int z = opaque_zero(v[0].x);
  // points outside [lead, lead + V) get the offset V (unsigned wrap included) and are dropped
  const __amdgpu_buffer_rsrc_t yr = range_rsrc(y, (unsigned)w.valid * (unsigned)sizeof(YT));
#pragma unroll
  for (int u = 0; u < G::P / G::RL; ++u)
#pragma unroll
    for (int q = 0; q < G::RL; ++q) {
      const unsigned j = min((unsigned)(t + z + u * G::T + q * (G::N / G::RL) - w.lead), (unsigned)w.valid);
      const float2 o = v[u * G::RL + out_reg<G::RL>(q)];
      store_ranged(yr, j * (unsigned)sizeof(YT), convert_y<OUT>(o));
      // binary16 / E4M3: |s y|^2 of the unrounded point staged by output index in LDS
      // (free since the last exchange; discarded points all land on slot V, never read)
      if constexpr (OUT != 0) lds[j] = fmaf(o.x, o.x, o.y * o.y);
    }
  if constexpr (OUT != 0) {
    // total power of each dump, summed in a fixed order
    __syncthreads();
    dump_sums<G::T>([&](int j) { return lds[j]; }, w.valid, a.dump_len,
                    power_row(a.power, w, a.y_stride, a.pw_stride, p), t);
  }
}

// ---------------------------------------------------------------------------
// Transforms longer than one workgroup's LDS: N = R 2^15 (R = 2, 4, 8).
// Forward, input index n = n1 2^15 + n2 and output index k = k1 + R k2
// (n1, k1 < R; n2, k2 < 2^15):
//   X[k1 + R k2] = sum_{n2} w_{2^15}^{-k2 n2} [ w_N^{-k1 n2} sum_{n1} w_R^{-k1 n1} x[n1 2^15 + n2] ],
// an R-point DFT per n2 with a twiddle (k_forward_big_pre), then a 2^15-point FFT
// per (antenna, k1) row (k_fft_rows).  The spectrum is kept as rows [k1][k2].
// Inverse of Z = X H, output index n = n1 2^15 + n2:
//   y[n1 2^15 + n2] = sum_{k1} w_R^{k1 n1} [ w_N^{k1 n2} sum_{k2} w_{2^15}^{k2 n2} Z[k1 + R k2] ],
// a 2^15-point FFT per row [k1] with a twiddle on its outputs (k_dedisperse_big_a),
// then an R-point DFT per n2 (k_dedisperse_big_b), which writes y in natural order.
constexpr int kBigLog = 15;
constexpr int kBigN = 1 << kBigLog;
using RowPlan = Plan<kBigLog>;

// exp(S 2 pi i num / 2^(15 + logr)) for 0 <= num < 2^(15 + logr), reduced exactly
template <int S>
__device__ __forceinline__ float2 big_twiddle(int num, int logr) {
  float x = (float)num * (1.0f / (float)(kBigN << logr));
  x = (x >= 0.5f) ? x - 1.0f : x;
  return make_float2(cos_rev(x), (float)S * sin_rev(x));
}

template <int R, int IN>
__device__ __forceinline__ void forward_big_pre(const Source& s, int64_t win0, int n2, float2* row0) {
  float2 v[R];
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) v[in_reg<R>(n1)] = load_sample<IN>(s, win0 + (int64_t)n1 * kBigN + n2);
  dft_reg<R, -1>(v);
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1)
    row0[(size_t)k1 * kBigN + n2] = cmul(v[out_reg<R>(k1)], big_twiddle<-1>(k1 * n2, ilog2(R)));
}

// grid: (2^15 / 256, n_items * M).  tb[it.tb + (p R + k1) 2^15 + n2].
template <int IN>
__global__ __launch_bounds__(256) void k_forward_big_pre(FwdArgs a, float2* __restrict__ tb, int logr) {
  const int n2 = blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y % a.n_ant;
  const FwdItem w = a.items[blockIdx.y / a.n_ant];
  Source s = a.src;
  s.row = w.chan * a.n_ant + p;
  s.hist_start = w.hist_start;
  float2* row0 = tb + w.tb + ((size_t)p << (kBigLog + logr));
  if (logr == 1) forward_big_pre<2, IN>(s, w.win0, n2, row0);
  else if (logr == 2) forward_big_pre<4, IN>(s, w.win0, n2, row0);
  else forward_big_pre<8, IN>(s, w.win0, n2, row0);
}

// Forward 2^15-point FFT of n_rows consecutive rows: dst[r 2^15 + k] from src[r 2^15 + n].
// Row r is row k1 = r & (R - 1) of (item, antenna) r >> logr, counted from the launch's
// first item; with l1, the row's sum of |Re X| + |Im X| goes to l1[(r >> logr) 8 + k1].
// grid: n_rows workgroups.
__global__ __launch_bounds__(Geo<RowPlan>::T) void k_fft_rows(const float2* __restrict__ src, float2* __restrict__ dst,
                                                              float* __restrict__ l1, int32_t logr) {
  using G = Geo<RowPlan>;
  extern __shared__ float lds[];
  const int t = threadIdx.x;
  const float2* x = src + (size_t)blockIdx.x * kBigN;
  float2 v[G::P];
  fft_workgroup<RowPlan, -1>(v, lds, t, [&](int i) { return at_byte(x, 8u * (unsigned)i); });
  float2* out = dst + (size_t)blockIdx.x * kBigN + opaque_zero(v[0].x);
#pragma unroll
  for (int u = 0; u < G::P / G::RL; ++u)
#pragma unroll
    for (int q = 0; q < G::RL; ++q) out[t + u * G::T + q * (G::N / G::RL)] = v[u * G::RL + out_reg<G::RL>(q)];
  if (l1) {
    const float tot = block_sum<G::T>(l1_of<G::P>(v), lds);
    if (t == 0) l1[(size_t)(blockIdx.x >> logr) * 8 + (blockIdx.x & ((1 << logr) - 1))] = tot;
  }
}

// Inverse pass A over a wave of units of one length N = 2^(15 + logr), for the
// antennas ant0 .. ant0 + n_ant - 1: row (p, k1) of unit u times the chirp's row k1,
// inverse 2^15-point FFT, times w_N^{k1 n2}.  The intermediate rows are indexed by
// the antenna within the group, so a group's rows reuse the same tb region.
// grid: order_units(n_units, tile) x n_ant R workgroups (see unit_row, rows p R + k1).
__global__ __launch_bounds__(Geo<Plan<kBigLog>>::T) void k_dedisperse_big_a(DedispArgs a) {
  using G = Geo<Plan<kBigLog>>;
  extern __shared__ float lds[];
  const int t = threadIdx.x;
  int row, ui;  // row = p R + k1
  if (!unit_row(xcd_remap(blockIdx.x, gridDim.x), a.n_units, a.n_ant << a.logr, a.tile, row, ui)) return;
  const UnitItem w = a.units[ui];
  const int k1 = row & ((1 << a.logr) - 1);
  const float2* x = a.spec + w.spec + ((size_t)row + ((size_t)a.ant0 << a.logr)) * kBigN;
  const float2* h = a.chirp + w.chirp + (size_t)k1 * kBigN;
  float2 v[G::P];
  fft_workgroup<Plan<kBigLog>, +1>(v, lds, t,
                             [&](int i) { return cmul(at_byte(x, 8u * (unsigned)i), at_byte(h, 8u * (unsigned)i)); });
  float2* out = a.tb + w.tb + (size_t)row * kBigN + opaque_zero(v[0].x);
#pragma unroll
  for (int u = 0; u < G::P / G::RL; ++u)
#pragma unroll
    for (int q = 0; q < G::RL; ++q) {
      const int n2 = t + u * G::T + q * (G::N / G::RL);
      out[n2] = cmul(v[u * G::RL + out_reg<G::RL>(q)], big_twiddle<+1>(k1 * n2, a.logr));
    }
}

template <int R, int OUT>
__device__ __forceinline__ void dedisperse_big_b(float2* t0, int n2, int lead, int valid,
                                                 typename YType<OUT>::T* y) {
  float2 v[R];
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) v[in_reg<R>(k1)] = t0[(size_t)k1 * kBigN + n2];
  dft_reg<R, +1>(v);
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) {
    const int n = n1 * kBigN + n2;
    if (n >= lead && n < lead + valid) store_stream(y + (n - lead), convert_y<OUT>(v[out_reg<R>(n1)]));
  }
  if constexpr (OUT != 0) {
    // |s y[n]|^2 into the slot this thread alone read (row n1, column n2 = index n of
    // the unit's rows in natural order), for k_dump_power_rows
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) {
      const float2 o = v[out_reg<R>(n1)];
      t0[(size_t)n1 * kBigN + n2] = make_float2(fmaf(o.x, o.x, o.y * o.y), 0.f);
    }
  }
}

// Inverse pass B: R-point DFT over k1, overlap-save discard, output conversion.
// grid: (2^15 / 256, n_units * n_ant), blockIdx.y = p * n_units + u, antenna ant0 + p.
template <int OUT>
__global__ __launch_bounds__(256) void k_dedisperse_big_b(DedispArgs a) {
  const int n2 = blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y / a.n_units;
  const UnitItem w = a.units[blockIdx.y % a.n_units];
  float2* t0 = a.tb + w.tb + ((size_t)p << (kBigLog + a.logr));
  typedef typename YType<OUT>::T YT;
  YT* y = reinterpret_cast<YT*>(a.y) + w.y + (size_t)(a.ant0 + p) * a.y_stride;
  if (a.logr == 1) dedisperse_big_b<2, OUT>(t0, n2, w.lead, w.valid, y);
  else if (a.logr == 2) dedisperse_big_b<4, OUT>(t0, n2, w.lead, w.valid, y);
  else dedisperse_big_b<8, OUT>(t0, n2, w.lead, w.valid, y);
}

// Per-dump power of the two-pass outputs (binary16 / E4M3): sums of the |s y[n]|^2
// that k_dedisperse_big_b left at index n of each unit's rows, n = lead + j.
// grid: n_units * n_ant workgroups of 256 (unit fastest), antennas ant0 + p.
__global__ __launch_bounds__(256) void k_dump_power_rows(DedispArgs a) {
  const int u = blockIdx.x % a.n_units, p = blockIdx.x / a.n_units;
  const UnitItem w = a.units[u];
  const float2* t0 = a.tb + w.tb + ((size_t)p << (kBigLog + a.logr)) + w.lead;
  dump_sums<256>([&](int j) { return t0[j].x; }, w.valid, a.dump_len,
                 power_row(a.power, w, a.y_stride, a.pw_stride, a.ant0 + p), threadIdx.x);
}

// ---------------------------------------------------------------------------
constexpr int kCorrKC = 64;  // samples per LDS chunk

template <int NT>  // 16 NT >= 2 M rows
struct CorrGeo {
  static constexpr int ROWS = 16 * NT;
  static constexpr int NTILES = NT * (NT + 1) / 2;
  static constexpr int TPW = (NTILES + 3) / 4;
  static constexpr int GP = ROWS + 1;
};

// Per input format: sample type, MFMA shape and LDS layout of one chunk.  All
// three keep the chunk row-major in LDS, at[row][k], 8 consecutive k per lane.
//   T = 0: FP32 y (times s), split on staging into binary16 hi = rn(y) and
//          lo = rn(y - hi) in two LDS planes; each product is accumulated as
//          hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_f16 (the dropped lo*lo
//          term is below 2^-22 of the product), FP32 accumulation
//   T = 1: FP16 y, v_mfma_f32_16x16x32_f16
//   T = 2: E4M3 y, v_mfma_f32_16x16x32_fp8_fp8
template <int T> struct CorrIn;
template <> struct CorrIn<0> {
  typedef float2 Y;      // one sample
  typedef float4 Pair;   // two samples
  typedef _Float16 E;    // one stored component (per plane)
  static constexpr int KSTEP = 32;
};
template <> struct CorrIn<1> {
  typedef __half2 Y;
  typedef uint2 Pair;
  typedef _Float16 E;
  static constexpr int KSTEP = 32;
};
template <> struct CorrIn<2> {
  typedef uint16_t Y;
  typedef uint32_t Pair;
  typedef uint8_t E;
  static constexpr int KSTEP = 32;
};

template <int T, int NT> struct CorrLds {
  static constexpr int ROWS = 16 * NT;
  // row-major, k pitch padded by 16 bytes; FP32 keeps a second (lo) plane after the first
  static constexpr int KP = kCorrKC + 16 / (int)sizeof(typename CorrIn<T>::E);
  static constexpr int PLANE = ROWS * KP;
  static constexpr int ELEMS = (T == 0 ? 2 : 1) * PLANE;
  __device__ static int at(int row, int k) { return row * KP + k; }
};

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// Correlator: per (DM, dump) the Gram matrix of the stacked real rows
// [Re y_0 .. Re y_{M-1}, Im y_0 .. Im y_{M-1}] over the L samples of the dump
// (the stored voltages are s y, s = the channel's correlator-input scale),
// G = A A^T on MFMA over the upper 16x16 tiles, FP32 accumulation, then
//   Re V_ij = (G[i][j] + G[M+i][M+j]) / s^2,  Im V_ij = (G[j][M+i] - G[i][M+j]) / s^2,
// except that with binary16 / E4M3 inputs V_ii is the dump's power of the unrounded
// voltages (from the dedispersion kernel) / s^2.  Samples are staged through LDS in chunks of kCorrKC with two chunks in flight:
// chunk k + 2's loads are issued while chunk k is staged, before its MFMAs.
// grid: n_units * max_dumps workgroups of 256 threads (4 waves), one per
// (unit, dump); workgroups past a unit's last dump exit at once.
struct CorrArgs {
  const void* y;
  float2* ring;
  const UnitItem* units;
  const float* scale;    // [C] correlator-input scales s_c (all formats)
  const float* power;    // binary16 / E4M3 inputs: per-dump power rows (the autocorrelations)
  const float* bound;    // FP32 inputs: per forward item, a bound on |Re y|, |Im y| (see k_item_bound)
  int64_t y_stride;      // samples per antenna row of y
  int64_t rec_elems;     // complex values per dump record
  int64_t ring_dumps;    // ring capacity in dumps
  int32_t max_dumps;     // dumps per unit covered by the grid
  int32_t n_ant, dump_len, nbl, out_mode;
  int32_t pw_stride;     // power values per antenna row
  int32_t pad;
};

// The (unit, dump) of workgroup `item`; false when the unit has fewer dumps.
struct CorrJob {
  int64_t yoff;      // element offset in y of the dump's first sample, antenna 0
  int64_t prow;      // offset of the dump's power value of antenna 0 (antenna i at + i pw_stride)
  float2* out;       // the (channel, DM) slot of the dump's record
  int32_t chan;
  int32_t dump_off;  // samples from the unit's row start to the dump's first sample
  float g;           // FP32 inputs: power of two putting the unit's largest |s y| at <= 2^15
};
__device__ __forceinline__ bool corr_job(const CorrArgs& a, int item, CorrJob& j) {
  const UnitItem w = a.units[item / a.max_dumps];
  const int m = item % a.max_dumps;
  if (m >= w.n_dumps) return false;
  j.yoff = w.y + (int64_t)m * a.dump_len;
  j.prow = (w.y / a.y_stride) * a.pw_stride + m;
  j.out = a.ring + ((w.dump0 + m) % a.ring_dumps) * a.rec_elems + w.rec;
  j.chan = w.chan;
  j.dump_off = m * a.dump_len;
  // FP32 inputs: a block whose level grew past the first block's scale is split at
  // a smaller power of two, so binary16 hi = rn(g s y) cannot overflow
  j.g = 1.f;
  if (a.bound) {
    const float top = a.bound[w.fwd] * a.scale[w.chan];
    while (top * j.g > 32768.f) j.g *= 0.5f;
  }
  return true;
}

// Byte offset that lies past every correlator load resource (ranges are at most
// 2^31 + 8 bytes) without wrapping when the access size is added.
constexpr unsigned kCorrSkip = 0xC0000000u;

// Samples (k, k + 1) of one antenna row (k even) as one load through a buffer
// resource: the caller passes an offset past the resource's range for a row past M
// or k past the dump, which the hardware's range check turns into zeros.  The
// value is used only when it is staged (a chunk later), so nothing waits for it here.
template <int T>
__device__ __forceinline__ typename CorrIn<T>::Pair load_pair(__amdgpu_buffer_rsrc_t r, unsigned off) {
  typename CorrIn<T>::Pair v;
  if constexpr (T == 0) {
    typedef unsigned int u4v __attribute__((ext_vector_type(4)));
    const u4v u = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    v = make_float4(__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z), __uint_as_float(u.w));
  } else if constexpr (T == 1) {
    typedef unsigned int u2v __attribute__((ext_vector_type(2)));
    const u2v u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    v = make_uint2(u.x, u.y);
  } else {
    v = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  }
  return v;
}

// The pair with its second sample zeroed when `second` is false (k + 1 past the
// dump: the load read one sample beyond it).
template <int T>
__device__ __forceinline__ typename CorrIn<T>::Pair clip_pair(typename CorrIn<T>::Pair v, bool second) {
  if constexpr (T == 0) {
    if (!second) v.z = v.w = 0.f;
  } else if constexpr (T == 1) {
    if (!second) v.y = 0u;
  } else {
    if (!second) v &= 0xffffu;
  }
  return v;
}

// FP32 pairs times the unit's range factor g (a power of two: exact); other formats as stored
template <int T>
__device__ __forceinline__ typename CorrIn<T>::Pair scale_pair(typename CorrIn<T>::Pair v, float g) {
  if constexpr (T == 0) {
    v.x *= g;
    v.y *= g;
    v.z *= g;
    v.w *= g;
  }
  return v;
}

// binary16 hi = rn(x) and lo = rn(x - hi); x - hi is exact in FP32
__device__ __forceinline__ void split16(float x, _Float16& hi, _Float16& lo) {
  hi = (_Float16)x;
  lo = (_Float16)(x - (float)hi);
}

// Stage two consecutive samples (k, k + 1; k even) of one antenna: the Re row gets
// (re0, re1) and the Im row (im0, im1), each written as one packed LDS store (4
// bytes for binary16 values, 2 for E4M3) instead of one store per value.
template <int T, int PLANE>
__device__ __forceinline__ void store_pair(typename CorrIn<T>::E* at, int ia_re, int ia_im, typename CorrIn<T>::Pair v) {
  if constexpr (T == 0) {
    _Float16 h0, l0, h1, l1;
    split16(v.x, h0, l0);
    split16(v.z, h1, l1);
    *reinterpret_cast<half2v*>(&at[ia_re]) = half2v{h0, h1};
    *reinterpret_cast<half2v*>(&at[PLANE + ia_re]) = half2v{l0, l1};
    split16(v.y, h0, l0);
    split16(v.w, h1, l1);
    *reinterpret_cast<half2v*>(&at[ia_im]) = half2v{h0, h1};
    *reinterpret_cast<half2v*>(&at[PLANE + ia_im]) = half2v{l0, l1};
  } else if constexpr (T == 1) {
    // v.x = (re0, im0), v.y = (re1, im1) as binary16 pairs
    *reinterpret_cast<uint32_t*>(&at[ia_re]) = (v.x & 0xffffu) | (v.y << 16);
    *reinterpret_cast<uint32_t*>(&at[ia_im]) = (v.x >> 16) | (v.y & 0xffff0000u);
  } else {
    // v = re0 | im0 << 8 | re1 << 16 | im1 << 24
    *reinterpret_cast<uint16_t*>(&at[ia_re]) = (uint16_t)((v & 0xffu) | ((v >> 8) & 0xff00u));
    *reinterpret_cast<uint16_t*>(&at[ia_im]) = (uint16_t)(((v >> 8) & 0xffu) | ((v >> 16) & 0xff00u));
  }
}

template <int NT, int T>
__global__ __launch_bounds__(256) void k_correlate(CorrArgs a) {
  using C = CorrGeo<NT>;
  using In = CorrIn<T>;
  using Ld = CorrLds<T, NT>;
  typedef typename In::E E;
  typedef typename In::Pair Pair;
  constexpr int PPT = (8 * NT * (kCorrKC / 2) + 255) / 256;  // max sample pairs per thread per chunk (M <= 8 NT)
  // the staged chunks and, after the last MFMA, the Gram matrix share one LDS buffer
  constexpr int AT_BYTES = Ld::ELEMS * (int)sizeof(E), GRAM_BYTES = C::ROWS * C::GP * 4;
  __shared__ __align__(16) char smem[AT_BYTES > GRAM_BYTES ? AT_BYTES : GRAM_BYTES];
  E* at = reinterpret_cast<E*>(smem);
  float* gram = reinterpret_cast<float*>(smem);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  CorrJob w;
  if (!corr_job(a, blockIdx.x, w)) return;
  const int M = a.n_ant, L = a.dump_len;
  const int pairs = M * (kCorrKC / 2);

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

  // padding rows 2M .. ROWS-1 stay zero (both planes for FP32)
  for (int e = tid; e < kCorrKC * (C::ROWS - 2 * M); e += 256) {
    const int k = e / (C::ROWS - 2 * M), r = 2 * M + e % (C::ROWS - 2 * M);
    at[Ld::at(r, k)] = (E)0;
    if constexpr (T == 0) at[Ld::PLANE + Ld::at(r, k)] = (E)0;
  }
  const float s_in = a.scale[w.chan];
  typedef typename In::Y Y;
  const Y* y = reinterpret_cast<const Y*>(a.y) + w.yoff;
  // one pair load per (antenna, sample pair) through a resource over the unit's rows
  // from the chunk's first sample on (see load_pair; the range is at most 2^31 + 8 bytes)
  auto rsrc_at = [&](int k0) {
    const unsigned span = ((unsigned)M * (unsigned)a.y_stride - (unsigned)(w.dump_off + k0) + 1u) * (unsigned)sizeof(Y);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<Y*>(y + k0), (short)0, (int)span, 0x00020000);
  };
  // every call issues its loads (past the last chunk they read zeros through the
  // skip offset), so the count of loads in flight is the same on every path and
  // each staging waits only for its own chunk
  auto load_one = [&](__amdgpu_buffer_rsrc_t r, int k0, int i) {
    const int e = tid + 256 * i;
    const int p = e / (kCorrKC / 2), kl = 2 * (e % (kCorrKC / 2)), k = k0 + kl;
    const unsigned off = (e < pairs && k < L) ? ((unsigned)p * (unsigned)a.y_stride + (unsigned)kl) * (unsigned)sizeof(Y) : kCorrSkip;
    return load_pair<T>(r, off);
  };
  auto stage_one = [&](int i, int k0, const Pair& v) {
    const int e = tid + 256 * i;
    if (e < pairs) {
      const int p = e / (kCorrKC / 2), k = 2 * (e % (kCorrKC / 2));
      store_pair<T, Ld::PLANE>(at, Ld::at(p, k), Ld::at(M + p, k), scale_pair<T>(clip_pair<T>(v, k0 + k + 1 < L), w.g));
    }
  };
  auto mfma_chunk = [&]() {
#pragma unroll
    for (int kk = 0; kk < kCorrKC; kk += In::KSTEP) {
#pragma unroll
      for (int i = 0; i < C::TPW; ++i) {
        if (wave + 4 * i < C::NTILES) {
          const int ra = ti[i] * 16 + (lane & 15), rb = tj[i] * 16 + (lane & 15);
          const int kr = kk + 8 * (lane >> 4);
          if constexpr (T == 0) {
            const half8 ah = *reinterpret_cast<const half8*>(&at[Ld::at(ra, kr)]);
            const half8 bh = *reinterpret_cast<const half8*>(&at[Ld::at(rb, kr)]);
            const half8 al = *reinterpret_cast<const half8*>(&at[Ld::PLANE + Ld::at(ra, kr)]);
            const half8 bl = *reinterpret_cast<const half8*>(&at[Ld::PLANE + Ld::at(rb, kr)]);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, acc[i], 0, 0, 0);
          } else if constexpr (T == 1) {
            const half8 av = *reinterpret_cast<const half8*>(&at[Ld::at(ra, kr)]);
            const half8 bv = *reinterpret_cast<const half8*>(&at[Ld::at(rb, kr)]);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, acc[i], 0, 0, 0);
          } else {
            const long av = *reinterpret_cast<const long*>(&at[Ld::at(ra, kr)]);
            const long bv = *reinterpret_cast<const long*>(&at[Ld::at(rb, kr)]);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc[i], 0, 0, 0);
          }
        }
      }
    }
  };
  // each staged pair's registers are refilled with chunk k+2 at once, so those
  // loads are in flight during the rest of the staging as well as the MFMAs
  auto chunk = [&](Pair* buf, int k0) {
    __syncthreads();  // previous chunk's MFMAs are done with at[]
    const int kn = k0 + 2 * kCorrKC;  // at or past L: the loads read zeros
    const __amdgpu_buffer_rsrc_t r = rsrc_at(kn < L ? kn : 0);
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      stage_one(i, k0, buf[i]);
      buf[i] = load_one(r, kn, i);
    }
    __syncthreads();
    mfma_chunk();
  };
  Pair buf0[PPT], buf1[PPT];
  {
    const __amdgpu_buffer_rsrc_t r0 = rsrc_at(0), r1 = rsrc_at(kCorrKC < L ? kCorrKC : 0);
#pragma unroll
    for (int i = 0; i < PPT; ++i) buf0[i] = load_one(r0, 0, i);
#pragma unroll
    for (int i = 0; i < PPT; ++i) buf1[i] = load_one(r1, kCorrKC, i);
  }
  for (int k0 = 0; k0 < L; k0 += 2 * kCorrKC) {
    chunk(buf0, k0);
    if (k0 + kCorrKC < L) chunk(buf1, k0 + kCorrKC);
  }
  __syncthreads();  // every wave is done with at[] before the Gram matrix overwrites it
#pragma unroll
  for (int i = 0; i < C::TPW; ++i) {
    if (wave + 4 * i < C::NTILES) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        gram[(ti[i] * 16 + 4 * (lane >> 4) + r) * C::GP + tj[i] * 16 + (lane & 15)] = acc[i][r];
    }
  }
  __syncthreads();
  const float inv = 1.f / (s_in * s_in * w.g * w.g);  // powers of two: exact
  float2* out = w.out;
  if (a.out_mode == 0) {
    for (int b = tid; b < a.nbl; b += 256) {
      // invert b = i M - i (i - 1) / 2 + (j - i)
      int i = 0, rem = b;
      while (rem >= M - i) { rem -= M - i; ++i; }
      const int j = i + rem;
      float re = gram[i * C::GP + j] + gram[(M + i) * C::GP + M + j];
      const float im = gram[j * C::GP + M + i] - gram[i * C::GP + M + j];
      if (T != 0 && i == j) re = a.power[w.prow + (int64_t)i * a.pw_stride];  // full-precision autos
      out[b] = make_float2(re * inv, im * inv);
    }
  } else {
    for (int b = tid; b < M * M; b += 256) {
      const int i = b / M, j = b % M;
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      float re = gram[lo * C::GP + hi] + gram[(M + lo) * C::GP + M + hi];
      if (T != 0 && i == j) re = a.power[w.prow + (int64_t)i * a.pw_stride];  // full-precision autos
      const float im = gram[hi * C::GP + M + lo] - gram[lo * C::GP + M + hi];
      out[b] = make_float2(re * inv, (i <= j ? im : -im) * inv);
    }
  }
}

// Correlator for large arrays: the antennas are cut into blocks of BA (64 or 128);
// one workgroup computes, for one (DM, dump), the BA x BA antenna block pair
// (I, J), I <= J, as complex 16 x 16 tiles, each from four real products on MFMA:
//   Re V = Yr_I Yr_J^T + Yi_I Yi_J^T,   Im V = Yi_I Yr_J^T - Yr_I Yi_J^T
// (FP32 form: every product as hi*hi + hi*lo + lo*hi of binary16 halves).  Each
// wave owns RT row tiles of block I against four column tiles of block J (BA = 64:
// 4 waves, RT = 1; BA = 128: 8 waves, RT = 2), so its block-I fragments are read
// once per k-step; in a diagonal pair (I = J) tiles wholly below the diagonal are
// skipped.  Chunks of kCorrKC samples of both blocks are staged through LDS, the
// next chunk's loads in flight during the current chunk's MFMAs.  Writes V_ij for
// i <= j < M only.
// grid: n_units * max_dumps * NB (NB + 1) / 2 workgroups (NB = ceil(M / BA)),
// corr_block_threads(BA) threads, corr_block_lds<T>(BA) bytes of dynamic LDS,
// block pair fastest.
// 128: measured 7 % faster than 64 on the 256-antenna workload (each dump's samples
// are read twice instead of five times; 128-blocks need 512 threads and 147 KB LDS)
constexpr int kBlkAnt = 128;

__host__ __device__ constexpr int corr_block_threads(int ba) { return ba == 128 ? 512 : 256; }
template <int T>
__host__ __device__ constexpr int corr_block_lds(int ba) {
  // rows Re I, Im I, Re J, Im J; k pitch padded by 16 bytes; FP32 keeps a lo plane
  return (T == 0 ? 2 : 1) * 4 * ba * (kCorrKC + 16 / (T == 2 ? 1 : 2)) * (T == 2 ? 1 : 2);
}

template <int T> struct NegFrag;
template <> struct NegFrag<0> {
  __device__ static half8 neg(half8 v) { return -v; }
};
template <> struct NegFrag<1> {
  __device__ static half8 neg(half8 v) { return -v; }
};
template <> struct NegFrag<2> {
  __device__ static long neg(long v) { return v ^ (long)0x8080808080808080LL; }  // flip the 8 sign bits
};

template <int T, int BA>
__global__ __launch_bounds__(corr_block_threads(BA)) void k_correlate_blocks(CorrArgs a) {
  using In = CorrIn<T>;
  typedef typename In::E E;
  typedef typename In::Pair Pair;
  typedef typename std::conditional<T == 2, long, half8>::type Frag;
  constexpr int NTH = corr_block_threads(BA), NW = NTH / 64;
  constexpr int TS = BA / 16;          // tiles per block side
  constexpr int CG = TS / 4;           // column groups of 4 tiles
  constexpr int RT = TS / (NW / CG);   // row tiles per wave
  constexpr int ROWS = 4 * BA;         // Re I, Im I, Re J, Im J
  constexpr int KP = kCorrKC + 16 / (int)sizeof(E);
  constexpr int PLANE = ROWS * KP;
  constexpr int PPT = (2 * BA * (kCorrKC / 2)) / NTH;  // sample pairs per thread per chunk
  static_assert(corr_block_lds<T>(BA) == (T == 0 ? 2 : 1) * PLANE * (int)sizeof(E), "LDS size");
  extern __shared__ __align__(16) char smem_blk[];
  E* at = reinterpret_cast<E*>(smem_blk);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int cg = wave % CG, rg = wave / CG;
  const int M = a.n_ant, L = a.dump_len;
  const int nb = (M + BA - 1) / BA, npair = nb * (nb + 1) / 2;
  int pr = blockIdx.x % npair;
  CorrJob w;
  if (!corr_job(a, blockIdx.x / npair, w)) return;
  int I = 0;
  while (pr >= nb - I) { pr -= nb - I; ++I; }
  const int J = I + pr;
  const float s_in = a.scale[w.chan];

  floatx4 are[RT][4], aim[RT][4];
#pragma unroll
  for (int x = 0; x < RT; ++x)
#pragma unroll
    for (int q = 0; q < 4; ++q) are[x][q] = aim[x][q] = floatx4{0.f, 0.f, 0.f, 0.f};

  const typename In::Y* y = reinterpret_cast<const typename In::Y*>(a.y) + w.yoff;
  // thread e -> (local antenna la in [0, 2 BA): block I then block J; sample pair)
  auto ant_of = [&](int la) { return la < BA ? I * BA + la : J * BA + (la - BA); };
  // resource over the unit's rows from the chunk's first sample to the end of the
  // unit (plus the one-sample overhang of an odd dump's last pair, which is zeroed;
  // the buffer is padded for it).  M y_stride <= 2^28 samples, so the range is at
  // most 2^31 + 8 bytes and the skip offset kCorrSkip lies past it.
  typedef typename In::Y Y;
  auto rsrc_at = [&](int k0) {
    const unsigned span = ((unsigned)M * (unsigned)a.y_stride - (unsigned)(w.dump_off + k0) + 1u) * (unsigned)sizeof(Y);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<Y*>(y + k0), (short)0, (int)span, 0x00020000);
  };
  auto load_one = [&](__amdgpu_buffer_rsrc_t r, int k0, int i) {
    const int e = tid + NTH * i;
    const int la = e / (kCorrKC / 2), kl = 2 * (e % (kCorrKC / 2)), k = k0 + kl;
    const int p = ant_of(la);
    const unsigned off = (p < M && k < L) ? ((unsigned)p * (unsigned)a.y_stride + (unsigned)kl) * (unsigned)sizeof(Y) : kCorrSkip;
    return load_pair<T>(r, off);
  };
  auto row_re = [](int la) { return la < BA ? la : 2 * BA + (la - BA); };
  auto stage_one = [&](int i, int k0, const Pair& v) {
    const int e = tid + NTH * i;
    const int la = e / (kCorrKC / 2), k = 2 * (e % (kCorrKC / 2));
    const int rr = row_re(la), ri = rr + BA;
    store_pair<T, PLANE>(at, rr * KP + k, ri * KP + k, scale_pair<T>(clip_pair<T>(v, k0 + k + 1 < L), w.g));
  };
  auto frag = [&](int plane, int row, int kr) -> Frag {
    return *reinterpret_cast<const Frag*>(&at[plane * PLANE + row * KP + kr]);
  };
  // tile (row tile rt, column tile ct) is needed unless the pair is diagonal and the
  // tile lies wholly below the diagonal (wave-uniform)
  auto needed = [&](int rt, int ct) { return I != J || ct >= rt; };
  Pair buf[PPT];
  {
    const __amdgpu_buffer_rsrc_t r = rsrc_at(0);
#pragma unroll
    for (int i = 0; i < PPT; ++i) buf[i] = load_one(r, 0, i);
  }
  for (int k0 = 0; k0 < L; k0 += kCorrKC) {
    __syncthreads();
    // each staged pair's registers are refilled with the next chunk at once, so
    // those loads are in flight during the rest of the staging and the MFMAs
    const int kn = k0 + kCorrKC;  // at or past L: the loads read zeros (same count on every path)
    const __amdgpu_buffer_rsrc_t r = rsrc_at(kn < L ? kn : 0);
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      stage_one(i, k0, buf[i]);
      buf[i] = load_one(r, kn, i);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kCorrKC; kk += In::KSTEP) {
      const int kr = kk + 8 * (lane >> 4);
      if constexpr (T == 0) {
        Frag rh[RT], rl[RT], ih[RT], il[RT];
#pragma unroll
        for (int x = 0; x < RT; ++x) {
          const int ra = (rg * RT + x) * 16 + (lane & 15);
          rh[x] = frag(0, ra, kr);
          rl[x] = frag(1, ra, kr);
          ih[x] = frag(0, BA + ra, kr);
          il[x] = frag(1, BA + ra, kr);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ct = cg * 4 + q;
          const int rb = 2 * BA + ct * 16 + (lane & 15);
          const Frag jrh = frag(0, rb, kr), jrl = frag(1, rb, kr);
          const Frag jih = frag(0, BA + rb, kr), jil = frag(1, BA + rb, kr);
          // Im V takes -Yr_I Yi_J^T: the column fragment is negated (once per tile column)
          const Frag njih = NegFrag<T>::neg(jih), njil = NegFrag<T>::neg(jil);
#pragma unroll
          for (int x = 0; x < RT; ++x) {
            if (!needed(rg * RT + x, ct)) continue;
            floatx4 r = are[x][q], m = aim[x][q];
            r = __builtin_amdgcn_mfma_f32_16x16x32_f16(rh[x], jrh, r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_16x16x32_f16(rh[x], jrl, r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_16x16x32_f16(rl[x], jrh, r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_16x16x32_f16(ih[x], jih, r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_16x16x32_f16(ih[x], jil, r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_16x16x32_f16(il[x], jih, r, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_16x16x32_f16(ih[x], jrh, m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_16x16x32_f16(ih[x], jrl, m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_16x16x32_f16(il[x], jrh, m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_16x16x32_f16(rh[x], njih, m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_16x16x32_f16(rh[x], njil, m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_16x16x32_f16(rl[x], njih, m, 0, 0, 0);
            are[x][q] = r;
            aim[x][q] = m;
          }
        }
      } else {
        Frag rr[RT], ii[RT];
#pragma unroll
        for (int x = 0; x < RT; ++x) {
          const int ra = (rg * RT + x) * 16 + (lane & 15);
          rr[x] = frag(0, ra, kr);
          ii[x] = frag(0, BA + ra, kr);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ct = cg * 4 + q;
          const int rb = 2 * BA + ct * 16 + (lane & 15);
          const Frag jr = frag(0, rb, kr), ji = frag(0, BA + rb, kr);
          const Frag nji = NegFrag<T>::neg(ji);
#pragma unroll
          for (int x = 0; x < RT; ++x) {
            if (!needed(rg * RT + x, ct)) continue;
            floatx4 r = are[x][q], m = aim[x][q];
            if constexpr (T == 1) {
              r = __builtin_amdgcn_mfma_f32_16x16x32_f16(rr[x], jr, r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_f16(ii[x], ji, r, 0, 0, 0);
              m = __builtin_amdgcn_mfma_f32_16x16x32_f16(ii[x], jr, m, 0, 0, 0);
              m = __builtin_amdgcn_mfma_f32_16x16x32_f16(rr[x], nji, m, 0, 0, 0);
            } else {
              r = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(rr[x], jr, r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ii[x], ji, r, 0, 0, 0);
              m = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ii[x], jr, m, 0, 0, 0);
              m = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(rr[x], nji, m, 0, 0, 0);
            }
            are[x][q] = r;
            aim[x][q] = m;
          }
        }
      }
    }
  }
  const float inv = 1.f / (s_in * s_in * w.g * w.g);
  float2* out = w.out;
#pragma unroll
  for (int x = 0; x < RT; ++x)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * BA + (rg * RT + x) * 16 + 4 * (lane >> 4) + r;
        const int j = J * BA + (cg * 4 + q) * 16 + (lane & 15);
        if (i >= M || j >= M || j < i) continue;
        float re = are[x][q][r] * inv;
        const float im = (i == j) ? 0.f : aim[x][q][r] * inv;  // autos are real
        if (T != 0 && i == j) re = a.power[w.prow + (int64_t)i * a.pw_stride] * inv;  // full-precision autos
        if (a.out_mode == 0) {
          out[(int64_t)i * M - (int64_t)i * (i - 1) / 2 + (j - i)] = make_float2(re, im);
        } else {
          out[(int64_t)i * M + j] = make_float2(re, im);
          if (i != j) out[(int64_t)j * M + i] = make_float2(re, -im);
        }
      }
    }
}

// Correlator-input scale of a channel from its first block window:
// sigma^2 = sum |x|^2 / (2 M n) over samples [0, n) of every antenna (per-component
// variance), s = 2^rint(log2(target / sigma)), 1 if the window is all zero.  Two
// launches per call for every channel whose first block runs: partial sums per
// (channel, antenna), then one sum per channel over antennas in order.  The
// summation order is fixed, so the result does not depend on how the stream was split.
struct ScaleItem {
  int64_t n;           // window length
  int64_t hist_start;  // absolute index of the channel's history element 0
  int32_t chan, pad;
};

// grid: n_items * M workgroups of 256 (antenna fastest); part[item * M + p].
template <int IN>
__global__ __launch_bounds__(256) void k_scale_part(Source s, const ScaleItem* items, int32_t n_ant, double* part) {
  __shared__ double red[256];
  const ScaleItem w = items[blockIdx.x / n_ant];
  const int p = blockIdx.x % n_ant;
  s.row = w.chan * n_ant + p;
  s.hist_start = w.hist_start;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < w.n; i += 256) {
    const float2 v = load_sample<IN>(s, i);
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// grid: n_items workgroups of 64; one thread per item sums its antennas in order.
__global__ __launch_bounds__(64) void k_scale_final(const ScaleItem* items, const double* part, int32_t n_ant,
                                                    float target, float* scale) {
  if (threadIdx.x != 0) return;
  const ScaleItem w = items[blockIdx.x];
  double tot = 0.0;
  for (int p = 0; p < n_ant; ++p) tot += part[(int64_t)blockIdx.x * n_ant + p];
  const double var = tot / (2.0 * n_ant * (double)w.n);
  scale[w.chan] = var > 0 ? (float)exp2(rint(log2((double)target / sqrt(var)))) : 1.f;
}

// Top-k selection of the learned proposal: mask[d] = 1 for the k largest scores
// (ties to the lower index; NaN below every number), or 1 for every d when more
// than k scores exceed `thr` (the fallback); flag[0] = the number above `thr`.
// One workgroup of 1024 threads; scores staged in LDS (n <= 16384).
constexpr int kTopkMax = 16384;
__global__ __launch_bounds__(1024) void k_topk_mask(const float* __restrict__ scores, int32_t n, int32_t k,
                                                    float thr, uint8_t* __restrict__ mask, int32_t* __restrict__ flag) {
  __shared__ float s[kTopkMax];
  __shared__ int above;
  if (threadIdx.x == 0) above = 0;
  for (int d = threadIdx.x; d < n; d += 1024) {
    const float v = scores[d];
    s[d] = v != v ? -INFINITY : v;
  }
  __syncthreads();
  int cnt = 0;
  for (int d = threadIdx.x; d < n; d += 1024) {
    const float v = s[d];
    int rank = 0;  // scores ahead of d: larger, or equal at a lower index
    for (int e = 0; e < n; ++e) {
      const float w = s[e];
      rank += (w > v) || (w == v && e < d);
    }
    mask[d] = rank < k ? 1 : 0;
    cnt += (scores[d] > thr) ? 1 : 0;  // NaN never counts
  }
  atomicAdd(&above, cnt);  // integer sum: the order does not matter
  __syncthreads();
  if (above > k)
    for (int d = threadIdx.x; d < n; d += 1024) mask[d] = 1;
  if (threadIdx.x == 0) flag[0] = above;
}

// Zero the record slots of inactive DMs for the dumps of one call.
// grid: one workgroup of 256 threads per item.
__global__ __launch_bounds__(256) void k_zero_dm(float2* ring, const ZeroItem* items, const int32_t* slots,
                                                 int32_t nbl) {
  const ZeroItem w = items[blockIdx.x];
  const int64_t total = (int64_t)w.n * nbl;
  for (int64_t e = threadIdx.x; e < total; e += 256)
    ring[w.rec + (int64_t)slots[w.pos + e / nbl] * nbl + e % nbl] = make_float2(0.f, 0.f);
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
