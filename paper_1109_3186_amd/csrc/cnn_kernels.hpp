// Kernels of the DM-proposal network: a small 1-D CNN (forward, backward, Adam).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddx {

// ---------------------------------------------------------------------------
// CNN.  Rows r = tile * D + d; layer-1 input channels are standardised tile rows
// d-1, d, d+1 (edges repeated).  Activations [R][32][L_l], L_1 = L, L_{l+1} = L_l / 2.
constexpr int kCnnK = 9, kCnnPad = 4, kCnnW = 32;

// Mean and standard deviation (population) of each tile, FP64 accumulation.
__global__ __launch_bounds__(1024) void k_tile_stats(const float* __restrict__ tiles, int64_t per_tile,
                                                     float* __restrict__ stats) {
  __shared__ double s1[1024], s2[1024];
  const float* t = tiles + (int64_t)blockIdx.x * per_tile;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < per_tile; i += 1024) {
    const double v = t[i];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = s1[0] / per_tile;
    const double var = s2[0] / per_tile - m * m;
    const double sd = var > 0 ? sqrt(var) : 0.0;
    stats[2 * blockIdx.x] = (float)m;
    stats[2 * blockIdx.x + 1] = sd > 0 ? (float)(1.0 / sd) : 1.f;
  }
}

// Input value of layer 1: channel i (0..2) of row r at time j (zero outside [0, L)).
__device__ __forceinline__ float cnn_in1(const float* tiles, const float* stats, int r, int i, int j, int n_dm, int L) {
  if (j < 0 || j >= L) return 0.f;
  const int tl = r / n_dm, d = r % n_dm;
  int dd = d + i - 1;
  dd = dd < 0 ? 0 : (dd >= n_dm ? n_dm - 1 : dd);
  const float v = tiles[((int64_t)tl * n_dm + dd) * L + j];
  return (v - stats[2 * tl]) * stats[2 * tl + 1];
}

// Forward convolution + bias + ReLU.  out[r][o][t] = relu(b[o] + sum_{i,k} W[o][i][k] in[r][i][S t + k - 4]).
// grid: (ceil(Lout / 64), R); 256 threads: thread = (o group of 8, t in 64).
template <int CIN, int S, bool FIRST>
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ in, const float* __restrict__ stats,
                                                  int32_t n_dm, int32_t lin, const float* __restrict__ w,
                                                  const float* __restrict__ bias, float* __restrict__ out) {
  constexpr int TW = 64, WIN = TW * S + kCnnK;
  __shared__ float xs[CIN][WIN];
  __shared__ float ws[kCnnW][CIN * kCnnK];
  const int r = blockIdx.y, t0 = blockIdx.x * TW, tid = threadIdx.x;
  const int lout = lin / S;
  for (int e = tid; e < kCnnW * CIN * kCnnK; e += 256) ws[e / (CIN * kCnnK)][e % (CIN * kCnnK)] = w[e];
  for (int e = tid; e < CIN * WIN; e += 256) {
    const int i = e / WIN, q = e % WIN, j = t0 * S + q - kCnnPad;
    float v;
    if (FIRST) v = cnn_in1(in, stats, r, i, j, n_dm, lin);
    else v = (j >= 0 && j < lin) ? in[((int64_t)r * CIN + i) * lin + j] : 0.f;
    xs[i][q] = v;
  }
  __syncthreads();
  const int tt = tid & 63, og = tid >> 6;  // 4 groups of 8 output channels
  const int t = t0 + tt;
  if (t >= lout) return;
  float acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = bias[og * 8 + q];
  for (int i = 0; i < CIN; ++i) {
#pragma unroll
    for (int k = 0; k < kCnnK; ++k) {
      const float x = xs[i][tt * S + k];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += ws[og * 8 + q][i * kCnnK + k] * x;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) out[((int64_t)r * kCnnW + og * 8 + q) * lout + t] = fmaxf(acc[q], 0.f);
}

// Global max over time, then the linear score.  One wave per row.
__global__ __launch_bounds__(64) void k_pool_linear(const float* __restrict__ h, int32_t len,
                                                    const float* __restrict__ w5, const float* __restrict__ b5,
                                                    float* __restrict__ g, int32_t* __restrict__ arg,
                                                    float* __restrict__ score) {
  const int r = blockIdx.x, lane = threadIdx.x;
  __shared__ float gs[kCnnW];
  if (lane < kCnnW) {
    const float* row = h + ((int64_t)r * kCnnW + lane) * len;
    float best = row[0];
    int bi = 0;
    for (int t = 1; t < len; ++t)
      if (row[t] > best) { best = row[t]; bi = t; }  // first maximum, as numpy argmax
    g[r * kCnnW + lane] = best;
    arg[r * kCnnW + lane] = bi;
    gs[lane] = best * w5[lane];
  }
  __syncthreads();
  if (lane == 0) {
    float s = b5[0];
    for (int o = 0; o < kCnnW; ++o) s += gs[o];
    score[r] = s;
  }
}

// Logistic loss per row and dL/dscore = (sigmoid(s) - y) / R.
__global__ void k_logistic(const float* __restrict__ score, const float* __restrict__ y, int32_t rows,
                           float* __restrict__ dscore, float* __restrict__ loss_rows) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  const float s = score[r];
  const float sig = 1.f / (1.f + expf(-s));
  dscore[r] = (sig - y[r]) / (float)rows;
  loss_rows[r] = fmaxf(s, 0.f) + log1pf(expf(-fabsf(s))) - y[r] * s;
}

// Backward of pool + linear: gh4[r][o][t] = ds[r] w5[o] at t = arg[r][o], else 0 (written in full).
__global__ void k_pool_bwd(const float* __restrict__ ds, const float* __restrict__ w5, const int32_t* __restrict__ arg,
                           int32_t rows, int32_t len, float* __restrict__ gh) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * kCnnW * len) return;
  const int t = (int)(e % len);
  const int64_t ro = e / len;
  const int o = (int)(ro % kCnnW), r = (int)(ro / kCnnW);
  gh[e] = (arg[r * kCnnW + o] == t) ? ds[r] * w5[o] : 0.f;
}

// Gradient of the ReLU pre-activation: gp = gh * (h > 0), in place.
__global__ void k_relu_bwd(float* __restrict__ gh, const float* __restrict__ h, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n && !(h[e] > 0.f)) gh[e] = 0.f;
}

// Backward data: gin[r][i][j] = sum_{o, k : S t + k - 4 = j} W[o][i][k] gp[r][o][t].
// grid: (ceil(lin / 64), R); thread = (i group of 8, j in 64).
template <int S>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const float* __restrict__ gp, int32_t lout,
                                                       const float* __restrict__ w, int32_t lin,
                                                       float* __restrict__ gin) {
  constexpr int TW = 64, GW = TW / S + kCnnK;  // gp window per j tile
  __shared__ float gs[kCnnW][GW + 1];
  __shared__ float ws[kCnnW][kCnnW * kCnnK];
  const int r = blockIdx.y, j0 = blockIdx.x * TW, tid = threadIdx.x;
  // gp times needed: t = (j + 4 - k) / S for j in [j0, j0 + 64), k in [0, 9):
  // from floor((j0 - 4) / S) to floor((j0 + 67) / S), at most 64 / S + 9 values
  const int num0 = j0 + kCnnPad - (kCnnK - 1);
  const int tbase = num0 >= 0 ? num0 / S : -((-num0 + S - 1) / S);
  for (int e = tid; e < kCnnW * kCnnW * kCnnK; e += 256) ws[e / (kCnnW * kCnnK)][e % (kCnnW * kCnnK)] = w[e];
  for (int e = tid; e < kCnnW * GW; e += 256) {
    const int o = e / GW, q = e % GW, t = tbase + q;
    gs[o][q] = (t >= 0 && t < lout) ? gp[((int64_t)r * kCnnW + o) * lout + t] : 0.f;
  }
  __syncthreads();
  const int jj = tid & 63, ig = tid >> 6;
  const int j = j0 + jj;
  if (j >= lin) return;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < kCnnK; ++k) {
    const int num = j + kCnnPad - k;
    if (num < 0 || num % S != 0) continue;
    const int q = num / S - tbase;
    for (int o = 0; o < kCnnW; ++o) {
      const float gv = gs[o][q];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += ws[o][(ig * 8 + u) * kCnnK + k] * gv;
    }
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) gin[((int64_t)r * kCnnW + ig * 8 + u) * lin + j] = acc[u];
}

// Backward weights, pass 1: partial sums over a chunk of rows.
// part[chunk][o][i][k] = sum_{r in chunk} sum_t gp[r][o][t] in[r][i][S t + k - 4]; partb[chunk][o] = sum gp.
// grid: (n_chunks); 256 threads, thread = (o, i-slice); loops over rows and time.
template <int CIN, int S, bool FIRST>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float* __restrict__ gp, int32_t lout,
                                                    const float* __restrict__ in, const float* __restrict__ stats,
                                                    int32_t n_dm, int32_t lin, int32_t rows, int32_t rows_per_chunk,
                                                    float* __restrict__ part, float* __restrict__ partb) {
  constexpr int NW = kCnnW * CIN * kCnnK;  // weights
  constexpr int TW = 64, WIN = TW * S + kCnnK;
  __shared__ float gs[kCnnW][TW];
  __shared__ float xs[CIN][WIN];
  const int tid = threadIdx.x, ch = blockIdx.x;
  constexpr int PER = (NW + 255) / 256;
  float acc[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) acc[q] = 0.f;
  float accb = 0.f;
  const int r0 = ch * rows_per_chunk, r1 = min(rows, r0 + rows_per_chunk);
  for (int r = r0; r < r1; ++r) {
    for (int t0 = 0; t0 < lout; t0 += TW) {
      __syncthreads();
      for (int e = tid; e < kCnnW * TW; e += 256) {
        const int o = e / TW, tt = e % TW, t = t0 + tt;
        gs[o][tt] = t < lout ? gp[((int64_t)r * kCnnW + o) * lout + t] : 0.f;
      }
      for (int e = tid; e < CIN * WIN; e += 256) {
        const int i = e / WIN, q = e % WIN, j = t0 * S + q - kCnnPad;
        float v;
        if (FIRST) v = cnn_in1(in, stats, r, i, j, n_dm, lin);
        else v = (j >= 0 && j < lin) ? in[((int64_t)r * CIN + i) * lin + j] : 0.f;
        xs[i][q] = v;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int widx = tid + 256 * q;
        if (widx < NW) {
          const int o = widx / (CIN * kCnnK), rem = widx % (CIN * kCnnK), i = rem / kCnnK, k = rem % kCnnK;
          float s = 0.f;
          for (int tt = 0; tt < TW; ++tt) s += gs[o][tt] * xs[i][tt * S + k];
          acc[q] += s;
        }
      }
      if (tid < kCnnW)
        for (int tt = 0; tt < TW; ++tt) accb += gs[tid][tt];
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int widx = tid + 256 * q;
    if (widx < NW) part[(int64_t)ch * NW + widx] = acc[q];
  }
  if (tid < kCnnW) partb[ch * kCnnW + tid] = accb;
}

// Pass 2: sum the chunk partials in order (deterministic). grid: ceil((nw + 32) / 256).
__global__ void k_reduce_chunks(const float* __restrict__ part, const float* __restrict__ partb, int32_t n_chunks,
                                int32_t nw, float* __restrict__ gw, float* __restrict__ gb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < nw) {
    float s = 0.f;
    for (int c = 0; c < n_chunks; ++c) s += part[(int64_t)c * nw + e];
    gw[e] = s;
  } else if (e < nw + kCnnW) {
    const int o = e - nw;
    float s = 0.f;
    for (int c = 0; c < n_chunks; ++c) s += partb[c * kCnnW + o];
    gb[o] = s;
  }
}

// Gradients of the linear layer: gw5[o] = sum_r ds[r] g[r][o], gb5 = sum_r ds[r] (one workgroup).
__global__ __launch_bounds__(256) void k_linear_bwd(const float* __restrict__ ds, const float* __restrict__ g,
                                                    int32_t rows, float* __restrict__ gw5, float* __restrict__ gb5) {
  __shared__ float red[256];
  for (int o = 0; o <= kCnnW; ++o) {
    float s = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) s += (o < kCnnW) ? ds[r] * g[r * kCnnW + o] : ds[r];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (o < kCnnW) gw5[o] = red[0];
      else gb5[0] = red[0];
    }
    __syncthreads();
  }
}

// Adam (Kingma & Ba 2015) with bias correction; t is the 1-based step.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// FP16 matrix-core form of the three convolutions (forward, backward data,
// backward weights): operands rounded to binary16, products accumulated in FP32
// on v_mfma_f32_16x16x32_f16, master weights, biases, the pooling, the loss and
// Adam in FP32.  Every operand tile is multiplied by a power of two before it is
// rounded, so its largest magnitude sits just below 2^14: the whole binary16
// significand is used whatever the level of the activations or gradients (the
// mean-loss gradients are ~1/rows, below binary16's normal range at training
// batch sizes), nothing overflows, and the scale comes off the FP32 result exactly.
//
// v_mfma_f32_16x16x32_f16(a, b, c): lane l holds a = A[l % 16][8 (l / 16) .. + 7]
// and b = B[l % 16][8 (l / 16) .. + 7]; c[q] += sum_k A[4 (l / 16) + q][k] B[l % 16][k].
typedef _Float16 cnn_h8 __attribute__((ext_vector_type(8)));
typedef float cnn_f4 __attribute__((ext_vector_type(4)));

// Power of two s with max_abs * s in [2^13, 2^14) (1 for an all-zero tile).
__device__ __forceinline__ float h16_scale(float max_abs) {
  if (!(max_abs > 0.f) || !(max_abs < INFINITY)) return 1.f;
  int e;
  (void)frexpf(max_abs, &e);  // max_abs = m 2^e, m in [0.5, 1)
  int p = 14 - e;
  p = p > 126 ? 126 : (p < -126 ? -126 : p);
  return ldexpf(1.f, p);
}

// Maxima of two per-thread values over a 256-thread workgroup (ends synchronised).
__device__ __forceinline__ float2 block_max2_256(float a, float b, float* red) {
  for (int o = 32; o > 0; o >>= 1) {
    a = fmaxf(a, __shfl_xor(a, o));
    b = fmaxf(b, __shfl_xor(b, o));
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[4 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  const float2 m = make_float2(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])),
                               fmaxf(fmaxf(red[4], red[5]), fmaxf(red[6], red[7])));
  __syncthreads();
  return m;
}

// Halves of the four layers' weights, each layer scaled by its own power of two
// (scale[l]), in the layouts the matrix cores read (16-byte rows of 8):
//   layer 1:        f1[o][K], K = 9 i + k for K < 27, zero for K = 27..31       (32 x 32)
//   layers 2-4, l:  fwd_l[k][o][i] (forward) and bwd_l[k][i][o] (backward data) (9 x 32 x 32 each)
// at wh + kCnnHalfOff[l] (forward) and wh + kCnnHalfOff[l] + 9216 (backward).
// grid: 4 (one workgroup per layer), 256 threads.
constexpr int kCnnHalfOff[4] = {0, 1024, 1024 + 2 * 9216, 1024 + 4 * 9216};
constexpr int kCnnHalfTotal = 1024 + 6 * 9216;

__global__ __launch_bounds__(256) void k_cnn_weights_h(const float* __restrict__ params, int64_t off_w1,
                                                       int64_t off_w2, int64_t off_w3, int64_t off_w4,
                                                       _Float16* __restrict__ wh, float* __restrict__ scale) {
  __shared__ float red[8];
  const int l = blockIdx.x, tid = threadIdx.x;
  const int64_t offs[4] = {off_w1, off_w2, off_w3, off_w4};
  const float* w = params + offs[l];
  const int n = l == 0 ? kCnnW * 3 * kCnnK : kCnnW * kCnnW * kCnnK;
  float mx = 0.f;
  for (int e = tid; e < n; e += 256) mx = fmaxf(mx, fabsf(w[e]));
  const float s = h16_scale(block_max2_256(mx, 0.f, red).x);
  if (tid == 0) scale[l] = s;
  _Float16* out = wh + kCnnHalfOff[l];
  if (l == 0) {
    for (int e = tid; e < kCnnW * 32; e += 256) {
      const int o = e / 32, K = e % 32;
      out[e] = (_Float16)(K < 3 * kCnnK ? w[o * 3 * kCnnK + K] * s : 0.f);
    }
  } else {
    constexpr int NW = kCnnW * kCnnW * kCnnK;
    for (int e = tid; e < NW; e += 256) {
      const int k = e / (kCnnW * kCnnW), a = (e / kCnnW) % kCnnW, b = e % kCnnW;
      out[e] = (_Float16)(w[(a * kCnnW + b) * kCnnK + k] * s);       // fwd[k][o = a][i = b]
      out[NW + e] = (_Float16)(w[(b * kCnnW + a) * kCnnK + k] * s);  // bwd[k][i = a][o = b]
    }
  }
}

// Forward convolution + bias + ReLU (as k_conv_fwd).  One workgroup: one row r,
// 64 output times, all 32 output channels; wave w owns the 16 times t0 + 16 w ..
// as the column tile of both 16-channel row tiles.  Contraction over (k, i):
// layer 1 one step of 32 (27 used), layers 2-4 nine steps (one per tap k) of the 32
// input channels, read as 16-byte rows of the time-major scaled window.
// grid: (ceil(Lout / 64), R); 256 threads.
template <int CIN, int S, bool FIRST>
__global__ __launch_bounds__(256) void k_conv_fwd_h(const float* __restrict__ in, const float* __restrict__ stats,
                                                    int32_t n_dm, int32_t lin, const _Float16* __restrict__ wl,
                                                    const float* __restrict__ wscale, const float* __restrict__ bias,
                                                    float* __restrict__ out) {
  constexpr int TW = 64, WIN = TW * S + kCnnK, XP = 40;  // 40 halves: 32 channels + pad, 80 bytes
  __shared__ float xs[CIN][WIN];
  __shared__ __attribute__((aligned(16))) _Float16 xh[FIRST ? 1 : WIN][XP];
  __shared__ float red[8];
  const int r = blockIdx.y, t0 = blockIdx.x * TW, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lout = lin / S;
  float mx = 0.f;
  for (int e = tid; e < CIN * WIN; e += 256) {
    const int i = e / WIN, q = e % WIN, j = t0 * S + q - kCnnPad;
    float v;
    if (FIRST) v = cnn_in1(in, stats, r, i, j, n_dm, lin);
    else v = (j >= 0 && j < lin) ? in[((int64_t)r * CIN + i) * lin + j] : 0.f;
    xs[i][q] = v;
    mx = fmaxf(mx, fabsf(v));
  }
  const float sx = h16_scale(block_max2_256(mx, 0.f, red).x);
  const int n = lane & 15, g = lane >> 4, tl = wave * 16 + n;
  cnn_f4 acc[2];
  acc[0] = cnn_f4{0.f, 0.f, 0.f, 0.f};
  acc[1] = acc[0];
  if constexpr (FIRST) {
    cnn_h8 b;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int K = 8 * g + u;
      b[u] = (_Float16)(K < 3 * kCnnK ? xs[K / kCnnK][tl + K % kCnnK] * sx : 0.f);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const cnn_h8 a = *reinterpret_cast<const cnn_h8*>(wl + (mt * 16 + n) * 32 + 8 * g);
      acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[mt], 0, 0, 0);
    }
  } else {
    for (int e = tid; e < CIN * WIN; e += 256) {
      const int q = e / CIN, i = e % CIN;
      xh[q][i] = (_Float16)(xs[i][q] * sx);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCnnK; ++k) {
      const cnn_h8 b = *reinterpret_cast<const cnn_h8*>(&xh[tl * S + k][8 * g]);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const cnn_h8 a = *reinterpret_cast<const cnn_h8*>(wl + ((k * kCnnW) + mt * 16 + n) * kCnnW + 8 * g);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[mt], 0, 0, 0);
      }
    }
  }
  const int t = t0 + tl;
  if (t >= lout) return;
  const float isx = 1.f / sx, isw = 1.f / wscale[0];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = mt * 16 + 4 * g + q;
      out[((int64_t)r * kCnnW + o) * lout + t] = fmaxf(acc[mt][q] * isx * isw + bias[o], 0.f);
    }
  }
}

// Backward data for a stride-2 layer (as k_conv_bwd_data<2>): gin[r][i][j] =
// sum over taps k of j's parity (j + 4 - k even) and o of W[o][i][k] gp[r][o][(j + 4 - k) / 2].
// One workgroup: one row, 64 input times; wave w owns the 16 times of parity w % 2
// j = j0 + 2 (16 (w / 2) + n) + w % 2, as the column tile of both 16-channel row
// tiles of i, contracting over o one tap at a time (5 taps for even j, 4 for odd).
// grid: (ceil(lin / 64), R); 256 threads.
__global__ __launch_bounds__(256) void k_conv_bwd_data_h(const float* __restrict__ gp, int32_t lout,
                                                         const _Float16* __restrict__ wb,
                                                         const float* __restrict__ wscale, int32_t lin,
                                                         float* __restrict__ gin) {
  constexpr int S = 2, TW = 64, GW = TW / S + kCnnK, XP = 40;
  __shared__ float gs[kCnnW][GW + 1];
  __shared__ __attribute__((aligned(16))) _Float16 gh[GW][XP];
  __shared__ float red[8];
  const int r = blockIdx.y, j0 = blockIdx.x * TW, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // gp times t = (j + 4 - k) / 2 for j in [j0, j0 + 64), k in [0, 9): from j0 / 2 - 2 on
  const int tbase = j0 / S - 2;
  float mx = 0.f;
  for (int e = tid; e < kCnnW * GW; e += 256) {
    const int o = e / GW, q = e % GW, t = tbase + q;
    const float v = (t >= 0 && t < lout) ? gp[((int64_t)r * kCnnW + o) * lout + t] : 0.f;
    gs[o][q] = v;
    mx = fmaxf(mx, fabsf(v));
  }
  const float sg = h16_scale(block_max2_256(mx, 0.f, red).x);
  for (int e = tid; e < kCnnW * GW; e += 256) {
    const int q = e / kCnnW, o = e % kCnnW;
    gh[q][o] = (_Float16)(gs[o][q] * sg);
  }
  __syncthreads();
  const int n = lane & 15, g = lane >> 4, par = wave & 1;
  const int j = j0 + 2 * (16 * (wave >> 1) + n) + par;
  cnn_f4 acc[2];
  acc[0] = cnn_f4{0.f, 0.f, 0.f, 0.f};
  acc[1] = acc[0];
  for (int k = par; k < kCnnK; k += 2) {
    const int q = (j + kCnnPad - k) / S - tbase;  // j + 4 - k is even
    const cnn_h8 b = *reinterpret_cast<const cnn_h8*>(&gh[q][8 * g]);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const cnn_h8 a = *reinterpret_cast<const cnn_h8*>(wb + ((k * kCnnW) + mt * 16 + n) * kCnnW + 8 * g);
      acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[mt], 0, 0, 0);
    }
  }
  if (j >= lin) return;
  const float isg = 1.f / sg, isw = 1.f / wscale[0];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = mt * 16 + 4 * g + q;
      gin[((int64_t)r * kCnnW + i) * lin + j] = acc[mt][q] * isg * isw;
    }
  }
}

// Backward weights, pass 1 (as k_conv_bwd_w): part[chunk][o][c], c = 9 i + k, is the
// sum over the chunk's rows and all times of gp[r][o][t] x[r][i][S t + k - 4], as the
// product of the (o x t) gradient tile and the (c x t) window gather, TW times at a
// time; each (row, TW times) tile has its own two scales, taken off its FP32 product
// before it joins the running sum.  Wave w owns the C tiles (o tile m, c tile nt) with
// 2 nt + m = w + 4 u.  partb[chunk][o] = sum of gp in FP32, each thread keeping one
// slice of one channel's times, the slices summed in order at the end.  Time tiles
// (measured, 8-tile training steps): TW = 256 for the first layer (27 columns, 4 C
// tiles: 712 us with TW = 64, 586 us), 128 for the others (530 us with 64, 491 us).
// grid: (n_chunks); 256 threads.
template <int CIN, int S, bool FIRST, int TW>
__global__ __launch_bounds__(256) void k_conv_bwd_w_h(const float* __restrict__ gp, int32_t lout,
                                                      const float* __restrict__ in, const float* __restrict__ stats,
                                                      int32_t n_dm, int32_t lin, int32_t rows, int32_t rows_per_chunk,
                                                      float* __restrict__ part, float* __restrict__ partb) {
  static_assert(TW % 64 == 0, "whole 32-step contraction pairs");
  constexpr int NC = CIN * kCnnK, NT = (NC + 15) / 16, TPW = (2 * NT + 3) / 4;
  constexpr int WIN = TW * S + kCnnK, GP = TW + 8;  // rows of TW + 8 halves: 16-byte multiples
  __shared__ float gs[kCnnW][TW];
  __shared__ float xs[CIN][WIN];
  __shared__ __attribute__((aligned(16))) _Float16 gh[kCnnW][GP];
  __shared__ _Float16 xh[CIN][WIN];
  __shared__ float red[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, ch = blockIdx.x;
  const int n = lane & 15, g = lane >> 4;
  cnn_f4 tot[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) tot[u] = cnn_f4{0.f, 0.f, 0.f, 0.f};
  float accb = 0.f;
  const int r0 = ch * rows_per_chunk, r1 = min(rows, r0 + rows_per_chunk);
  for (int r = r0; r < r1; ++r) {
    for (int t0 = 0; t0 < lout; t0 += TW) {
      __syncthreads();  // the previous tile's reads of gh, xh, gs are done
      float mg = 0.f, mx = 0.f;
      for (int e = tid; e < kCnnW * TW; e += 256) {
        const int o = e / TW, tt = e % TW, t = t0 + tt;
        const float v = t < lout ? gp[((int64_t)r * kCnnW + o) * lout + t] : 0.f;
        gs[o][tt] = v;
        mg = fmaxf(mg, fabsf(v));
      }
      for (int e = tid; e < CIN * WIN; e += 256) {
        const int i = e / WIN, q = e % WIN, j = t0 * S + q - kCnnPad;
        float v;
        if (FIRST) v = cnn_in1(in, stats, r, i, j, n_dm, lin);
        else v = (j >= 0 && j < lin) ? in[((int64_t)r * CIN + i) * lin + j] : 0.f;
        xs[i][q] = v;
        mx = fmaxf(mx, fabsf(v));
      }
      const float2 m = block_max2_256(mg, mx, red);
      const float sg = h16_scale(m.x), sx = h16_scale(m.y);
      for (int e = tid; e < kCnnW * TW; e += 256) gh[e / TW][e % TW] = (_Float16)(gs[e / TW][e % TW] * sg);
      for (int e = tid; e < CIN * WIN; e += 256) xh[e / WIN][e % WIN] = (_Float16)(xs[e / WIN][e % WIN] * sx);
      {  // bias: thread tid keeps the sum of output channel tid / 8's slice tid % 8 of every tile
        const int o = tid >> 3, q0 = (tid & 7) * (TW / 8);
#pragma unroll
        for (int tt = 0; tt < TW / 8; ++tt) accb += gs[o][q0 + tt];
      }
      __syncthreads();
      const float unscale = (1.f / sg) * (1.f / sx);
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int c = wave + 4 * u;
        if (c < 2 * NT) {
          const int mt = c & 1, col = (c >> 1) * 16 + n;
          const int i = col / kCnnK, k = col % kCnnK;
          cnn_f4 acc = cnn_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kk = 0; kk < TW; kk += 32) {
            const cnn_h8 a = *reinterpret_cast<const cnn_h8*>(&gh[mt * 16 + n][kk + 8 * g]);
            cnn_h8 b;
#pragma unroll
            for (int v = 0; v < 8; ++v) b[v] = col < NC ? xh[i][S * (kk + 8 * g + v) + k] : (_Float16)0;
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
          }
          tot[u] += acc * unscale;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int c = wave + 4 * u;
    if (c < 2 * NT) {
      const int mt = c & 1, col = (c >> 1) * 16 + n;
      if (col < NC) {
#pragma unroll
        for (int q = 0; q < 4; ++q) part[(int64_t)ch * kCnnW * NC + (mt * 16 + 4 * g + q) * NC + col] = tot[u][q];
      }
    }
  }
  __shared__ float bsum[256];
  bsum[tid] = accb;
  __syncthreads();
  if (tid < kCnnW) {
    float b = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) b += bsum[8 * tid + q];  // the slices in order
    partb[ch * kCnnW + tid] = b;
  }
}

}  // namespace ddx
