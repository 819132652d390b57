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

}  // namespace ddx
