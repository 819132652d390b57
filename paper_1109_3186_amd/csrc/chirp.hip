// Chirpolator pre-integrator (Bannister & Cornwell 2011, Sec. 3.2 and App. A.3)
// on gfx950: mixing of antenna pairs, block partial DFTs over a window of bins,
// and the block CIC moving sum (Eq. block_cic).
//
//   x_pq[n] = s_p[n] s_q[n]^*                                   (Eq. xpq), p < q
//   V_k[m]  = sum_{n<L} exp(-2 pi i (n + m L) k / N) x_pq[n + m L]   (block partial DFT)
//   S_k[m]  = S_k[m-1] + V_k[m] - V_k[m - N/L]                  (Eq. block_cic)
//
// The twiddle of sample n + m L factors as w_k[n] exp(-2 pi i ((m mod R) L k mod N) / N)
// with R = N / L, so one table W[n][k] (n < L) and one phase table P[m mod R][k],
// both computed in FP64 on the host and stored in FP32, serve every block.  Bins k
// and -k share their products (App. A.3, Eqs. fpos, fneg): with x = a + i b and
// w_k = c - i d, the four sums P = sum a c, Q = sum b d, R = sum a d, T = sum b c give
//   V_k = (P + Q) + i (T - R),   V_-k = (P - Q) + i (R + T),
// one FMA per sum and sample, half the work of two separate complex products.  Per
// block the partial DFTs of all pairs are then a product [pairs x L] x [L x (kmax+1)]
// in 64 x 64 tiles, the mixing fused into the staging of the pair operand.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "ddx.h"

namespace chirp {

constexpr int kTileP = 64;   // pairs per output tile
constexpr int kTileK = 64;   // bins per output tile
constexpr int kChunk = 32;   // samples per LDS chunk

struct PartialArgs {
  const float2* s;        // [M][n] complex samples
  const int2* pq;         // [nbl] (p, q)
  const float2* w;        // [L_pad][K_pad] (c, d) of w_k[n] = c - i d, k = 0..kmax
  const float2* ph;       // [R][K_pad] (c, d) of the block phase of bin k >= 0
  float2* v;              // [nb][nbl][2 kmax + 1] partial DFTs, bin index k + kmax
  int64_t n_samp;         // samples per antenna row of s
  int32_t nbl, kmax, K_pad, L, R, n_ptiles, n_ktiles;
};

// grid: nb * n_ptiles * n_ktiles workgroups of 256 threads (block slowest).
// Thread (tp, tk) = (tid / 16, tid % 16) accumulates pairs 4 tp .. 4 tp + 3 of the
// tile against bins +-(4 tk .. 4 tk + 3) of the tile.
__global__ __launch_bounds__(256) void k_partial(PartialArgs a) {
  __shared__ float2 xs[kChunk][kTileP];
  __shared__ float2 ws[kChunk][kTileK];
  const int tid = threadIdx.x;
  const int kt = blockIdx.x % a.n_ktiles;
  const int pt = (blockIdx.x / a.n_ktiles) % a.n_ptiles;
  const int m = blockIdx.x / (a.n_ktiles * a.n_ptiles);
  const int p0 = pt * kTileP, k0 = kt * kTileK;
  const int tp = tid >> 4, tk = tid & 15;
  const int64_t base = (int64_t)m * a.L;
  float4 acc[4][4];  // (P, Q, R, T) per pair and bin pair
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_float4(0.f, 0.f, 0.f, 0.f);

  for (int n0 = 0; n0 < a.L; n0 += kChunk) {
    __syncthreads();
    // stage x[n][pair] = s_p conj(s_q) (zero past the block or past the last pair)
#pragma unroll
    for (int r = 0; r < (kChunk * kTileP) / 256; ++r) {
      const int e = tid + 256 * r;
      const int n = e / kTileP, pl = e % kTileP;
      const int pair = p0 + pl;
      float2 x = make_float2(0.f, 0.f);
      if (pair < a.nbl && n0 + n < a.L) {
        const int2 pq = a.pq[pair];
        const float2 sp = a.s[(int64_t)pq.x * a.n_samp + base + n0 + n];
        const float2 sq = a.s[(int64_t)pq.y * a.n_samp + base + n0 + n];
        x = make_float2(sp.x * sq.x + sp.y * sq.y, sp.y * sq.x - sp.x * sq.y);
      }
      xs[n][pl] = x;
    }
    // stage w[n][k] (the table is zero past L and past K)
#pragma unroll
    for (int r = 0; r < (kChunk * kTileK) / 256; ++r) {
      const int e = tid + 256 * r;
      const int n = e / kTileK, kl = e % kTileK;
      ws[n][kl] = a.w[(int64_t)(n0 + n) * a.K_pad + k0 + kl];
    }
    __syncthreads();
#pragma unroll 4
    for (int n = 0; n < kChunk; ++n) {
      float2 xv[4], wv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xv[i] = xs[n][4 * tp + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) wv[j] = ws[n][4 * tk + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j].x = fmaf(xv[i].x, wv[j].x, acc[i][j].x);  // P += a c
          acc[i][j].y = fmaf(xv[i].y, wv[j].y, acc[i][j].y);  // Q += b d
          acc[i][j].z = fmaf(xv[i].x, wv[j].y, acc[i][j].z);  // R += a d
          acc[i][j].w = fmaf(xv[i].y, wv[j].x, acc[i][j].w);  // T += b c
        }
    }
  }
  // V_+-k, times the block phase exp(-+ i phi) = c -+ i d, stored at bin index kmax +- k
  const float2* ph = a.ph + (int64_t)(m % a.R) * a.K_pad;
  const int K = 2 * a.kmax + 1;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = k0 + 4 * tk + j;
    if (k > a.kmax) continue;
    const float2 f = ph[k];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int pair = p0 + 4 * tp + i;
      if (pair >= a.nbl) continue;
      const float4 u = acc[i][j];
      const float pr = u.x + u.y, pi = u.w - u.z;  // V_k
      const float nr = u.x - u.y, ni = u.z + u.w;  // V_-k
      float2* row = a.v + ((int64_t)m * a.nbl + pair) * K + a.kmax;
      row[k] = make_float2(pr * f.x + pi * f.y, pi * f.x - pr * f.y);
      if (k > 0) row[-k] = make_float2(nr * f.x - ni * f.y, ni * f.x + nr * f.y);
    }
  }
}

// Eq. block_cic per (pair, bin), FP64 running sum from zero state; writes the full
// windows m >= R - 1 as out[m - R + 1][pair][k].  The blocks are cut into segments
// of seg blocks run in parallel: a segment starts from S[m0 - 1], the sum of the R
// blocks before it, then follows the recursion.
// grid: (ceil(cols / 256), ceil(nb / seg)) x 256.
__global__ __launch_bounds__(256) void k_cic(const float2* __restrict__ v, float2* __restrict__ out, int64_t cols,
                                             int32_t nb, int32_t R, int32_t seg) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  const int m0 = blockIdx.y * seg, m1 = min(nb, m0 + seg);
  double re = 0.0, im = 0.0;
  for (int m = max(0, m0 - R); m < m0; ++m) {
    const float2 add = v[(int64_t)m * cols + c];
    re += add.x;
    im += add.y;
  }
#pragma unroll 8
  for (int m = m0; m < m1; ++m) {
    const float2 add = v[(int64_t)m * cols + c];
    re += add.x;
    im += add.y;
    if (m >= R) {
      const float2 sub = v[(int64_t)(m - R) * cols + c];
      re -= sub.x;
      im -= sub.y;
    }
    if (m >= R - 1) out[(int64_t)(m - R + 1) * cols + c] = make_float2((float)re, (float)im);
  }
}

}  // namespace chirp

struct ddx_chirp {
  int M = 0, N = 0, L = 0, kmax = 0, K = 0, K_pad = 0, L_pad = 0, R = 0, nbl = 0;
  int64_t max_samples = 0, max_blocks = 0;
  float2* w = nullptr;
  float2* ph = nullptr;
  int2* pq = nullptr;
  float2* v = nullptr;
  std::string err;
};

namespace {

int cfail(ddx_chirp* c, int status, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return status;
}

void cfree(ddx_chirp* c) {
  for (void* p : {(void*)c->w, (void*)c->ph, (void*)c->pq, (void*)c->v})
    if (p) (void)hipFree(p);
  c->w = c->ph = c->v = nullptr;
  c->pq = nullptr;
}

}  // namespace

extern "C" {

int ddx_chirp_create(int32_t n_ant, int32_t fft_n, int32_t block_len, int32_t kmax, int64_t max_samples,
                     ddx_chirp** out) {
  if (!out) return DDX_EINVAL;
  *out = nullptr;
  if (n_ant < 2 || n_ant > 1024 || block_len < 1 || fft_n < block_len || fft_n % block_len != 0 || kmax < 0 ||
      2 * kmax + 1 > fft_n || max_samples < fft_n)
    return DDX_EINVAL;
  ddx_chirp* c = new (std::nothrow) ddx_chirp;
  if (!c) return DDX_ENOMEM;
  c->M = n_ant;
  c->N = fft_n;
  c->L = block_len;
  c->kmax = kmax;
  c->K = 2 * kmax + 1;
  c->K_pad = (kmax + 1 + chirp::kTileK - 1) / chirp::kTileK * chirp::kTileK;
  c->L_pad = (c->L + chirp::kChunk - 1) / chirp::kChunk * chirp::kChunk;
  c->R = fft_n / block_len;
  c->nbl = n_ant * (n_ant - 1) / 2;
  c->max_samples = max_samples;
  c->max_blocks = max_samples / block_len;
  // FP64 tables for k = 0..kmax, as (c, d) with exp(-2 pi i u / N) = c - i d:
  // w_k[n] with u = n k mod N, P[r][k] with u = r L k mod N
  std::vector<float2> w((size_t)c->L_pad * c->K_pad, make_float2(0.f, 0.f));
  std::vector<float2> ph((size_t)c->R * c->K_pad, make_float2(0.f, 0.f));
  auto tw = [&](int64_t num) {
    const int64_t r = ((num % c->N) + c->N) % c->N;
    const double ang = 2.0 * M_PI * (double)r / (double)c->N;
    return make_float2((float)std::cos(ang), (float)std::sin(ang));
  };
  for (int n = 0; n < c->L; ++n)
    for (int j = 0; j <= kmax; ++j) w[(size_t)n * c->K_pad + j] = tw((int64_t)n * j);
  for (int r = 0; r < c->R; ++r)
    for (int j = 0; j <= kmax; ++j) ph[(size_t)r * c->K_pad + j] = tw((int64_t)r * c->L * j);
  std::vector<int2> pq;
  for (int p = 0; p < n_ant; ++p)
    for (int q = p + 1; q < n_ant; ++q) pq.push_back(make_int2(p, q));
  const size_t v_bytes = (size_t)c->max_blocks * c->nbl * c->K * sizeof(float2);
  if (hipMalloc((void**)&c->w, w.size() * sizeof(float2)) != hipSuccess ||
      hipMalloc((void**)&c->ph, ph.size() * sizeof(float2)) != hipSuccess ||
      hipMalloc((void**)&c->pq, pq.size() * sizeof(int2)) != hipSuccess ||
      hipMalloc((void**)&c->v, std::max<size_t>(v_bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    cfree(c);
    delete c;
    return DDX_ENOMEM;
  }
  if (hipMemcpy(c->w, w.data(), w.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->ph, ph.data(), ph.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->pq, pq.data(), pq.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    cfree(c);
    delete c;
    return DDX_EDEVICE;
  }
  *out = c;
  return DDX_OK;
}

int ddx_chirp_output_shape(const ddx_chirp* c, int64_t n, int64_t* n_windows, int32_t* n_pairs, int32_t* n_bins) {
  if (!c || !n_windows || !n_pairs || !n_bins || n < 0) return DDX_EINVAL;
  const int64_t nb = n / c->L;
  *n_windows = nb >= c->R ? nb - c->R + 1 : 0;
  *n_pairs = c->nbl;
  *n_bins = c->K;
  return DDX_OK;
}

int ddx_chirp_preintegrate(ddx_chirp* c, const void* d_volts, int64_t n, void* d_out, void* hip_stream) {
  if (!c) return DDX_EINVAL;
  if (n < 0 || n > c->max_samples) return cfail(c, DDX_EINVAL, "n = %lld outside [0, %lld]", (long long)n,
                                                (long long)c->max_samples);
  const int64_t nb = n / c->L;
  if (nb < c->R) return DDX_OK;  // no complete window
  if (!d_volts || !d_out) return cfail(c, DDX_EINVAL, "NULL device buffer");
  hipStream_t s = (hipStream_t)hip_stream;
  chirp::PartialArgs a{};
  a.s = (const float2*)d_volts;
  a.pq = c->pq;
  a.w = c->w;
  a.ph = c->ph;
  a.v = c->v;
  a.n_samp = n;
  a.nbl = c->nbl;
  a.kmax = c->kmax;
  a.K_pad = c->K_pad;
  a.L = c->L;
  a.R = c->R;
  a.n_ptiles = (c->nbl + chirp::kTileP - 1) / chirp::kTileP;
  a.n_ktiles = c->K_pad / chirp::kTileK;
  const int64_t grid = nb * a.n_ptiles * a.n_ktiles;
  if (grid > INT32_MAX) return cfail(c, DDX_EUNSUPPORTED, "too many blocks in one call");
  hipLaunchKernelGGL(chirp::k_partial, dim3((unsigned)grid), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cfail(c, DDX_EDEVICE, "k_partial: %s", hipGetErrorString(e));
  const int64_t cols = (int64_t)c->nbl * c->K;
  // segments of at least 256 blocks (the R-block restart costs R / seg extra reads), at most 65535
  const int64_t seg = std::max<int64_t>(256, (nb + 65534) / 65535);
  hipLaunchKernelGGL(chirp::k_cic, dim3((unsigned)((cols + 255) / 256), (unsigned)((nb + seg - 1) / seg)), dim3(256), 0,
                     s, (const float2*)c->v, (float2*)d_out, cols, (int32_t)nb, (int32_t)c->R, (int32_t)seg);
  e = hipGetLastError();
  if (e != hipSuccess) return cfail(c, DDX_EDEVICE, "k_cic: %s", hipGetErrorString(e));
  return DDX_OK;
}

const char* ddx_chirp_last_error(const ddx_chirp* c) { return c ? c->err.c_str() : "NULL pre-integrator"; }

int ddx_chirp_destroy(ddx_chirp* c) {
  if (!c) return DDX_OK;
  (void)hipDeviceSynchronize();
  cfree(c);
  delete c;
  return DDX_OK;
}

}  // extern "C"
