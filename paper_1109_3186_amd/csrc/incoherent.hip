// Classical incoherent dedispersion of power beams on gfx950 (Bannister & Cornwell
// 2011, Sec. 2.3.1 and 2.4.1): the power beam (detected power summed over antennas
// and integrated), brute-force dedispersion over the delays of Eq. dmdelay, and the
// tree method for linear sweeps.
//
//   p[c][t]   = sum_a sum_{n in [t n_int, (t + 1) n_int)} |x_{c,a}[n]|^2
//   out[d][t] = sum_c p[c][t + delay[c][d]]                 (brute force, t < n_out)
//   tree: log2 C merging stages; merging two groups of n/2 channels into n, sweep j
//         = sweep floor(j/2) of the first + sweep floor(j/2) of the second advanced
//         by j - floor(j/2) samples, so sweep j delays channel 0 by 0 and the last
//         channel by j (linear dispersion, the assumption of the tree method).
//
// Channel 0 is the least delayed (highest frequency); samples past the end count
// as zero.  The brute force stages each channel's samples for a tile of 32 DMs in
// LDS (one staged sample serves every DM of the tile); the tree is a memory-bound
// stream, its first five stages fused in LDS and the later ones two per pass, each
// pass reading and writing every row once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "ddx.h"

namespace inc {

constexpr int kThreads = 256;
constexpr int kDmTile = 32;         // brute force: DMs per workgroup (and per thread)
constexpr int kChanGroup = 8;       // brute force: channels staged per LDS round
constexpr int kOut = 2;             // brute force: outputs per thread, 256 apart
constexpr int kSpan = 768;          // brute force: staged samples per channel (tile 512 + spread 256)
constexpr int kStage = kSpan / kThreads;   // brute force: staged samples per thread and channel
static_assert(kSpan % kThreads == 0, "the staging covers the span in whole rounds");
constexpr int kFuseLog = 5;         // tree: the first 5 stages (groups of 32 channels) in LDS
constexpr int kFuseRows = 1 << kFuseLog;
constexpr int kTreeTile = 224;      // tree: samples per fused tile (tile + 32 halo = 256 per row)

// grid: (ceil(n_out / 512), ceil(n_dm / kDmTile)); thread = samples t and t + 256
// for the kDmTile DMs of the workgroup.  The workgroup's outputs read, per
// channel, the samples t0 + [min delay, max delay + 511] over its DMs: staged in LDS for
// kChanGroup channels at a time (each staged sample then serves every DM of the
// tile), or read from global memory for a channel whose delays spread over more
// than kSpan - 512 samples across the tile.
__global__ __launch_bounds__(kThreads) void k_brute(const float* __restrict__ p, int32_t C, int64_t n_t,
                                                    const int32_t* __restrict__ delays, int32_t n_dm,
                                                    float* __restrict__ out, int64_t n_out) {
  __shared__ float buf[kChanGroup][kSpan];
  __shared__ int lo_s[kChanGroup], hi_s[kChanGroup];
  __shared__ unsigned dls[kChanGroup][kDmTile];   // the group's delays for the tile's DMs,
                                                  // as offsets from the channel's least delay
  constexpr int TILE = kThreads * kOut;
  const int64_t t0 = (int64_t)blockIdx.x * TILE;
  const int64_t t = t0 + threadIdx.x;     // and t + 256
  const int d0 = blockIdx.y * kDmTile;
  const int nd = min(kDmTile, n_dm - d0);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // a channel is staged iff its delays spread over at most kSpan - TILE samples
  // (lo <= hi, so the unsigned difference is the exact spread, with no overflow)
  auto fits = [](int lo, int hi) { return (unsigned)hi - (unsigned)lo <= (unsigned)(kSpan - TILE); };
  float acc[kOut][kDmTile] = {};
  for (int c0 = 0; c0 < C; c0 += kChanGroup) {
    const int nc = min(kChanGroup, C - c0);
    __syncthreads();
    // the delay range of each channel over the tile's DMs: one wave per channel,
    // lane i holding DM d0 + i, min and max by butterfly
    for (int ci = wv; ci < nc; ci += kThreads / 64) {
      const int32_t* dl = delays + (int64_t)(c0 + ci) * n_dm + d0;
      const int mine = lane < nd ? dl[lane] : 0;
      int lo = lane < nd ? mine : INT32_MAX;
      int hi = lane < nd ? mine : INT32_MIN;
      for (int o = 16; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
      }
      if (lane == 0) {
        lo_s[ci] = lo;
        hi_s[ci] = hi;
      }
      // every lane of the 32 holds the range now; DMs past nd read offset 0.  As
      // unsigned, mine - lo is exact for any int32 delays
      if (lane < kDmTile) dls[ci][lane] = lane < nd ? (unsigned)mine - (unsigned)lo : 0u;
    }
    __syncthreads();
    {
      // every load of the round is issued before the first LDS store, so that
      // the loads' latencies overlap; a channel read from global below stages
      // nothing, and the unused tail of a span is zero-filled.  Per channel a
      // uniform base (sample t0 + lo) and uniform limits on x: the samples
      // x_lo <= x < x_hi exist and belong to the span
      float v[kChanGroup][kStage];
#pragma unroll
      for (int ci = 0; ci < kChanGroup; ++ci) {
        const int lo = __builtin_amdgcn_readfirstlane(lo_s[ci]);   // stale past nc: unused
        const int hi = __builtin_amdgcn_readfirstlane(hi_s[ci]);
        const bool staged = ci < nc && fits(lo, hi);
        const int n = staged ? hi - lo + TILE : 0;
        const int64_t b = t0 + lo;
        const int x_lo = (int)std::min<int64_t>(kSpan, std::max<int64_t>(0, -b));
        const int x_hi = staged ? (int)std::max<int64_t>(0, std::min<int64_t>(n, n_t - b)) : 0;
        const float* src = p + (int64_t)(c0 + ci) * n_t + b;   // read only at x_lo <= x < x_hi
#pragma unroll
        for (int q = 0; q < kStage; ++q) {
          const int x = threadIdx.x + q * kThreads;
          v[ci][q] = (x >= x_lo && x < x_hi) ? src[x] : 0.f;
        }
      }
#pragma unroll
      for (int ci = 0; ci < kChanGroup; ++ci)
#pragma unroll
        for (int q = 0; q < kStage; ++q) buf[ci][threadIdx.x + q * kThreads] = v[ci][q];
    }
    __syncthreads();
    for (int ci = 0; ci < nc; ++ci) {
      const unsigned* off = dls[ci];   // in [0, hi - lo]; 0 past nd (never written out)
      const int lo = lo_s[ci], hi = hi_s[ci];
      if (fits(lo, hi)) {
        // one address per DM serves both outputs (256 samples apart)
        const float* b = buf[ci] + threadIdx.x;
#pragma unroll
        for (int i = 0; i < kDmTile; ++i) {
          const float* bi = b + off[i];
#pragma unroll
          for (int o = 0; o < kOut; ++o) acc[o][i] += bi[o * kThreads];
        }
      } else {
        const float* row = p + (int64_t)(c0 + ci) * n_t;
#pragma unroll
        for (int i = 0; i < kDmTile; ++i) {
          const int d = (int)((unsigned)lo + off[i]);   // the delay itself, exactly
#pragma unroll
          for (int o = 0; o < kOut; ++o) {
            const int64_t s = t + o * kThreads + d;
            acc[o][i] += (s >= 0 && s < n_t) ? row[s] : 0.f;
          }
          // one DM's loads at a time (this rare path keeps few loads in flight)
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }
#pragma unroll
  for (int o = 0; o < kOut; ++o) {
    const int64_t to = t + o * kThreads;
    if (to >= n_out) continue;
#pragma unroll
    for (int i = 0; i < kDmTile; ++i)
      if (i < nd) out[(int64_t)(d0 + i) * n_out + to] = acc[o][i];
  }
}

// The first kFuseLog tree stages of one group of 32 channels over a tile of
// kTreeTile samples, in LDS.  A stage advances the second half by at most n/2
// samples, so the tile reads kTreeTile + 31 samples of each channel (zero past the
// end).  Rows of the group are combined in place, stage by stage.
// grid: (ceil(n_t / kTreeTile), C / 32) x 256.
__global__ __launch_bounds__(kThreads) void k_tree_fused(const float* __restrict__ in, float* __restrict__ out,
                                                         int64_t n_t) {
  constexpr int W = kTreeTile + kFuseRows;        // samples held per row (tile + halo)
  constexpr int PER = kFuseRows * W / kThreads;   // elements per thread
  // one buffer (32 KB, so that four workgroups share a CU): each stage reads its
  // inputs into registers, then writes the stage's rows back after a barrier
  __shared__ float buf[kFuseRows][W];
  const int g = blockIdx.y;
  const int64_t t0 = (int64_t)blockIdx.x * kTreeTile;
  float v[PER];
  // all the tile's loads are issued before the first store (memory-level parallelism)
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * kThreads;
    const int r = e / W, x = e % W;
    const int64_t t = t0 + x;
    v[q] = t < n_t ? in[((int64_t)g * kFuseRows + r) * n_t + t] : 0.f;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * kThreads;
    buf[e / W][e % W] = v[q];
  }
#pragma unroll
  for (int st = 1; st <= kFuseLog; ++st) {
    const int n = 1 << st;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * kThreads;
      const int r = e / W, x = e % W;
      const int j = r % n, base = r - j;
      const int h = j >> 1, s = j - h;
      v[q] = buf[base + h][x] + (x + s < W ? buf[base + n / 2 + h][x + s] : 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * kThreads;
      buf[e / W][e % W] = v[q];
    }
  }
  // the halo columns past x = kTreeTile - 1 are incomplete after the shifts; only
  // the tile itself is written (straight from the registers)
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * kThreads;
    const int r = e / W, x = e % W;
    const int64_t t = t0 + x;
    if (x < kTreeTile && t < n_t) out[((int64_t)g * kFuseRows + r) * n_t + t] = v[q];
  }
}

// One later tree stage: groups of n = 2 half rows; row = g n + j.  Each thread
// makes kStageVec samples 256 apart (the advanced row is read unaligned).
// grid: (ceil(n_t / (256 kStageVec)), C) x 256.
constexpr int kStageVec = 4;
__global__ __launch_bounds__(kThreads) void k_tree_stage(const float* __restrict__ in, float* __restrict__ out,
                                                         int64_t n_t, int32_t n) {
  const int row = blockIdx.y;
  const int j = row % n, base = row - j;
  const int h = j >> 1, s = j - h;
  const float* ra = in + (int64_t)(base + h) * n_t;
  const float* rb = in + (int64_t)(base + n / 2 + h) * n_t;
  float* ro = out + (int64_t)row * n_t;
  const int64_t t0 = (int64_t)blockIdx.x * kThreads * kStageVec + threadIdx.x;
#pragma unroll
  for (int i = 0; i < kStageVec; ++i) {
    const int64_t t = t0 + (int64_t)i * kThreads;  // each load instruction coalesced
    if (t < n_t) ro[t] = ra[t] + (t + s < n_t ? rb[t + s] : 0.f);
  }
}

// Two later tree stages in one pass: groups of n/4 rows -> n/2 -> n.  Output rows
// j = 4k .. 4k + 3 of a group of n all come from the four input rows k of its
// quarters (A, B, C, D); with h = j >> 1, s = j - h and s2 = h - (h >> 1) (k or
// k + 1), row j = [A + B advanced by s2] + [C + D advanced by s2] advanced by s, each
// bracket the intermediate row, summed in the order the two stages would, so the
// result is bit-identical to two single stages.  One thread makes the four output
// rows of kStageVec samples 256 apart: the four input rows are read once from HBM,
// and the loads the four rows share are issued once.  (A generic pass of K stages,
// 2^K shifted reads per output, ran slower for K = 2 and for K = 3.)
// grid: (ceil(n_t / (256 kStageVec)), C / 4) x 256.
__global__ __launch_bounds__(kThreads) void k_tree_stage2(const float* __restrict__ in, float* __restrict__ out,
                                                          int64_t n_t, int32_t n) {
  const int q = blockIdx.y, nq = n / 4;
  const int k = q % nq;
  const int64_t base = (int64_t)(q - k) * 4;   // first row of the group of n
  const float* ra = in + (base + k) * n_t;
  const float* rb = in + (base + nq + k) * n_t;
  const float* rc = in + (base + 2 * nq + k) * n_t;
  const float* rd = in + (base + 3 * nq + k) * n_t;
  float* ro = out + (base + 4 * k) * n_t;
  const int64_t t0 = (int64_t)blockIdx.x * kThreads * kStageVec + threadIdx.x;
  // the value of an input row at sample u, zero past the end
  auto at = [n_t](const float* r, int64_t u) { return u < n_t ? r[u] : 0.f; };
#pragma unroll
  for (int i = 0; i < kStageVec; ++i) {
    const int64_t t = t0 + (int64_t)i * kThreads;
    if (t >= n_t) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * k + e, h = j >> 1, s = j - h, s2 = h - (h >> 1);
      const float first = ra[t] + at(rb, t + s2);
      const float second = t + s < n_t ? rc[t + s] + at(rd, t + s + s2) : 0.f;
      ro[(int64_t)e * n_t + t] = first + second;
    }
  }
}

// p[c][t] = sum over antennas and the n_int samples of interval t of |x|^2.
// grid: (ceil(n_out / 256), C) x 256; thread = one interval.
__global__ __launch_bounds__(kThreads) void k_power_beam(const float2* __restrict__ x, int32_t M, int64_t S,
                                                         int32_t n_int, float* __restrict__ p, int64_t n_out) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n_out) return;
  const int c = blockIdx.y;
  float acc = 0.f;
  for (int a = 0; a < M; ++a) {
    const float2* row = x + ((int64_t)c * M + a) * S + t * n_int;
    for (int n = 0; n < n_int; ++n) {
      const float2 v = row[n];
      acc = fmaf(v.x, v.x, fmaf(v.y, v.y, acc));
    }
  }
  p[(int64_t)c * n_out + t] = acc;
}

}  // namespace inc

extern "C" {

int ddx_incoherent_delays(int32_t n_chan, const double* chan_freq_hz, double t_samp_s, int32_t n_dm,
                          const double* dm, double k_dm, int32_t* delays) {
  if (n_chan < 1 || !chan_freq_hz || !(t_samp_s > 0.0) || n_dm < 1 || !dm || !delays || !(k_dm >= 0.0))
    return DDX_EINVAL;
  double top = chan_freq_hz[0];
  for (int c = 0; c < n_chan; ++c) {
    if (!(chan_freq_hz[c] > 0.0) || !std::isfinite(chan_freq_hz[c])) return DDX_EINVAL;
    top = std::max(top, chan_freq_hz[c]);
  }
  for (int d = 0; d < n_dm; ++d)
    if (!(dm[d] >= 0.0) || !std::isfinite(dm[d])) return DDX_EINVAL;
  for (int c = 0; c < n_chan; ++c)
    for (int d = 0; d < n_dm; ++d) {
      const double sec = k_dm * dm[d] * (1.0 / (chan_freq_hz[c] * chan_freq_hz[c]) - 1.0 / (top * top));
      const double v = std::nearbyint(sec / t_samp_s);
      if (!(v <= (double)INT32_MAX)) return DDX_EUNSUPPORTED;
      delays[(int64_t)c * n_dm + d] = (int32_t)v;
    }
  return DDX_OK;
}

int ddx_incoherent_dedisperse(const float* d_power, int32_t n_chan, int64_t n_t, const int32_t* d_delays,
                              int32_t n_dm, float* d_out, int64_t n_out, void* hip_stream) {
  if (n_chan < 1 || n_t < 0 || n_dm < 1 || n_out < 0 || !d_power || !d_delays || !d_out) return DDX_EINVAL;
  if (n_out == 0) return DDX_OK;
  const int64_t tile = (int64_t)inc::kThreads * inc::kOut;
  const int64_t gx = (n_out + tile - 1) / tile;
  const int64_t gy = (n_dm + inc::kDmTile - 1) / inc::kDmTile;
  if (gx > INT32_MAX || gy > 65535) return DDX_EUNSUPPORTED;
  hipLaunchKernelGGL(inc::k_brute, dim3((unsigned)gx, (unsigned)gy), dim3(inc::kThreads), 0, (hipStream_t)hip_stream,
                     d_power, n_chan, n_t, d_delays, n_dm, d_out, n_out);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

int ddx_tree_dedisperse(const float* d_power, int32_t n_chan, int64_t n_t, float* d_out, float* d_work,
                        void* hip_stream) {
  if (n_chan < 1 || n_chan > 32768 || (n_chan & (n_chan - 1)) || n_t < 0 || !d_power || !d_out) return DDX_EINVAL;
  if (n_t == 0) return DDX_OK;
  const hipStream_t s = (hipStream_t)hip_stream;
  int stages = 0;
  while ((1 << stages) < n_chan) ++stages;
  const int fused = n_chan >= inc::kFuseRows ? inc::kFuseLog : 0;
  const int rest = stages - fused;
  // work is needed whenever a stage does not write out directly
  if ((fused ? rest >= 1 : stages >= 2) && !d_work) return DDX_EINVAL;
  const int64_t gx = (n_t + (int64_t)inc::kThreads * inc::kStageVec - 1) / ((int64_t)inc::kThreads * inc::kStageVec);
  if (gx > INT32_MAX) return DDX_EUNSUPPORTED;
  // the stages after the fused ones run two per pass (the last alone if their count
  // is odd), alternating between out and work and ending in out.  (Three per pass
  // moves a third less but reads seven shifted rows per output: slower.)
  const int passes = (rest + 1) / 2;
  float* first = (passes % 2 == 0) ? d_out : d_work;
  if (n_chan >= inc::kFuseRows) {
    const int64_t tx = (n_t + inc::kTreeTile - 1) / inc::kTreeTile;
    hipLaunchKernelGGL(inc::k_tree_fused, dim3((unsigned)tx, (unsigned)(n_chan / inc::kFuseRows)),
                       dim3(inc::kThreads), 0, s, d_power, first, n_t);
  } else {
    // fewer than 32 channels: every stage on its own, power -> ... -> out
    const float* src = d_power;
    for (int st = 1; st <= stages; ++st) {
      float* dst = ((stages - st) % 2 == 0) ? d_out : d_work;
      hipLaunchKernelGGL(inc::k_tree_stage, dim3((unsigned)gx, (unsigned)n_chan), dim3(inc::kThreads), 0, s, src,
                         dst, n_t, 1 << st);
      src = dst;
    }
    if (stages == 0)
      if (hipMemcpyAsync(d_out, d_power, (size_t)n_t * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return DDX_EDEVICE;
    return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
  }
  const float* src = first;
  for (int st = fused + 1; st <= stages; st += 2) {
    float* dst = (src == d_out) ? d_work : d_out;
    if (st + 1 <= stages)
      hipLaunchKernelGGL(inc::k_tree_stage2, dim3((unsigned)gx, (unsigned)(n_chan / 4)), dim3(inc::kThreads), 0, s,
                         src, dst, n_t, 1 << (st + 1));
    else
      hipLaunchKernelGGL(inc::k_tree_stage, dim3((unsigned)gx, (unsigned)n_chan), dim3(inc::kThreads), 0, s, src, dst,
                         n_t, 1 << st);
    src = dst;
  }
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

}  // extern "C"

// Workspace of ddx_tree_dedisperse_static: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes `scratch` itself (in
// host code it names a host-side stand-in); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device on the first call there.
namespace {
constexpr size_t kStaticWorkFloats = DDX_TREE_STATIC_MAX;
__device__ __align__(256) float scratch[kStaticWorkFloats];
std::mutex g_scratch_mu;
std::vector<float*> g_scratch_ptr;  // per device ordinal, null until looked up

int scratch_address(float** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return DDX_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return DDX_EDEVICE;
    }
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return DDX_OK;
}
}  // namespace

extern "C" {

int ddx_tree_dedisperse_static(const float* d_power, int32_t n_chan, int64_t n_t, float* d_out, void* hip_stream) {
  if (n_chan < 1 || n_t < 0 || !d_power || !d_out) return DDX_EINVAL;
  if ((uint64_t)n_chan * (uint64_t)n_t > kStaticWorkFloats) return DDX_ESIZE;
  if (n_t == 0) return DDX_OK;
  float* work = nullptr;
  const int rc = scratch_address(&work);
  if (rc) return rc;
  // every tree pass writes each workspace row in full before a later pass reads it,
  // so nothing needs clearing between calls
  return ddx_tree_dedisperse(d_power, n_chan, n_t, d_out, work, hip_stream);
}

int ddx_power_beam(const void* d_volts, int32_t n_chan, int32_t n_ant, int64_t n_samp, int32_t n_int, float* d_power,
                   void* hip_stream) {
  if (n_chan < 1 || n_chan > 65535 || n_ant < 1 || n_samp < 0 || n_int < 1 || !d_volts || !d_power)
    return DDX_EINVAL;
  const int64_t n_out = n_samp / n_int;
  if (n_out == 0) return DDX_OK;
  const int64_t gx = (n_out + inc::kThreads - 1) / inc::kThreads;
  if (gx > INT32_MAX) return DDX_EUNSUPPORTED;
  hipLaunchKernelGGL(inc::k_power_beam, dim3((unsigned)gx, (unsigned)n_chan), dim3(inc::kThreads), 0,
                     (hipStream_t)hip_stream, (const float2*)d_volts, n_ant, n_samp, n_int, d_power, n_out);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

}  // extern "C"
