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
#include <numeric>
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
  const float2* w;        // [L_pad][K_pad] (c, d) of w_k[n] = c - i d, k = klist[j]
  const float2* ph;       // [R][K_pad] (c, d) of the block phase of bin klist[j]
  const int2* cols;       // [n_list] columns of V for +k and -k (-1: none, k = 0)
  const int* klist;       // [n_list] the listed bins k >= 0, ascending
  const int* tile_bins;   // [n_ptiles] largest bin budget of a pair tile
  float2* v;              // [nb][nbl][Kc] partial DFTs (pairs in budget order)
  int64_t n_samp;         // samples per antenna row of s
  int32_t nbl, n_list, Kc, K_pad, L, R, n_ptiles, n_ktiles;
};

// grid: nb * n_ptiles * n_ktiles workgroups of 256 threads (block slowest).
// Thread (tp, tk) = (tid / 16, tid % 16) accumulates pairs 4 tp .. 4 tp + 3 of the
// tile against the listed bins +-klist[4 tk .. 4 tk + 3] of the tile.
__global__ __launch_bounds__(256) void k_partial(PartialArgs a) {
  __shared__ float2 xs[kChunk][kTileP];
  __shared__ float2 ws[kChunk][kTileK];
  const int tid = threadIdx.x;
  const int kt = blockIdx.x % a.n_ktiles;
  const int pt = (blockIdx.x / a.n_ktiles) % a.n_ptiles;
  const int m = blockIdx.x / (a.n_ktiles * a.n_ptiles);
  const int p0 = pt * kTileP, k0 = kt * kTileK;
  // pairs are sorted by bin budget: a tile whose smallest bin exceeds every budget
  // of its pairs has nothing to compute (the CIC writes those bins as zero)
  if (k0 < a.n_list && a.klist[k0] > a.tile_bins[pt]) return;
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
  // V_+-k, times the block phase exp(-+ i phi) = c -+ i d, stored at columns cols[jl]
  const float2* ph = a.ph + (int64_t)(m % a.R) * a.K_pad;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int jl = k0 + 4 * tk + j;
    if (jl >= a.n_list) continue;
    const float2 f = ph[jl];
    const int2 col = a.cols[jl];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int pair = p0 + 4 * tp + i;
      if (pair >= a.nbl) continue;
      const float4 u = acc[i][j];
      const float pr = u.x + u.y, pi = u.w - u.z;  // V_k
      const float nr = u.x - u.y, ni = u.z + u.w;  // V_-k
      float2* row = a.v + ((int64_t)m * a.nbl + pair) * a.Kc;
      row[col.x] = make_float2(pr * f.x + pi * f.y, pi * f.x - pr * f.y);
      if (col.y >= 0) row[col.y] = make_float2(nr * f.x - ni * f.y, ni * f.x + nr * f.y);
    }
  }
}

// Eq. block_cic per (pair, column), FP64 running sum from zero state; writes the full
// windows m >= R - 1 as out[m - R + 1][pair][cmap[column]] (K bins per pair row of
// out, Kc columns per pair row of v).  The blocks are cut into segments
// of seg blocks run in parallel: a segment starts from S[m0 - 1], the sum of the R
// blocks before it, then follows the recursion.
// grid: (ceil(cols / 256), ceil(nb / seg)) x 256.
__global__ __launch_bounds__(256) void k_cic(const float2* __restrict__ v, float2* __restrict__ out,
                                             const int* __restrict__ cmap, const int* __restrict__ perm,
                                             const int* __restrict__ budget, int64_t cols, int32_t Kc, int32_t K,
                                             int32_t nb, int32_t R, int32_t seg) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  const int sp = (int)(c / Kc), bin = cmap[c % Kc];      // pair in budget order, output bin index
  const int64_t oc = (int64_t)perm[sp] * K + bin;       // (pair, bin) of out
  const int64_t orow = (int64_t)(cols / Kc) * K;        // out elements per window
  if (abs(bin - (K - 1) / 2) > budget[sp]) {            // beyond the pair's bin budget: zero
    for (int m = max(R - 1, (int)blockIdx.y * seg); m < min(nb, ((int)blockIdx.y + 1) * seg); ++m)
      out[(int64_t)(m - R + 1) * orow + oc] = make_float2(0.f, 0.f);
    return;
  }
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
    if (m >= R - 1) out[(int64_t)(m - R + 1) * orow + oc] = make_float2((float)re, (float)im);
  }
}

// App. A.3, "Factorizing the DFTs": bin k of the length N0 d window ending with
// block m is the sum of p adjacent windows of bin k / p of length N0 d / p (p a
// common factor of k and d).  With each length's output starting at its first
// complete window, window w of length d reads windows w + (p - 1 - j) Rs, j < p, of
// length d / p (Rs = its N / L).  items: (k, p) of the bins formed this way.
// grid: ceil(windows nbl n_items / 256) x 256.
__global__ __launch_bounds__(256) void k_factor(const float2* __restrict__ src, float2* __restrict__ dst,
                                                const int2* __restrict__ items, const int* __restrict__ budget_canon,
                                                int32_t n_items, int64_t windows, int32_t nbl, int32_t K, int32_t kmax,
                                                int32_t Rs) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= windows * nbl * n_items) return;
  const int it = (int)(t % n_items);
  const int64_t wp = t / n_items;  // w nbl + pair
  const int pair = (int)(wp % nbl);
  const int64_t w = wp / nbl;
  const int2 kp = items[it];
  if (abs(kp.x) > budget_canon[pair]) {  // beyond the pair's bin budget
    dst[(w * nbl + pair) * K + kmax + kp.x] = make_float2(0.f, 0.f);
    return;
  }
  const int ks = kmax + kp.x / kp.y;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < kp.y; ++j) {
    const float2 u = src[((w + (int64_t)(kp.y - 1 - j) * Rs) * nbl + pair) * K + ks];
    re += u.x;
    im += u.y;
  }
  dst[(w * nbl + pair) * K + kmax + kp.x] = make_float2((float)re, (float)im);
}

}  // namespace chirp

namespace {

// One window length N: its tables and the bins computed directly (both signs of
// each listed k >= 0).
struct Stage {
  int N = 0, R = 0, n_list = 0, Kc = 0, K_pad = 0;
  float2* w = nullptr;   // [L_pad][K_pad]
  float2* ph = nullptr;  // [R][K_pad]
  int2* cols = nullptr;  // [n_list]
  int* cmap = nullptr;   // [Kc] output bin index of each column of V
  int* klist = nullptr;  // [n_list] the listed bins k >= 0
};

struct Common {
  int M = 0, L = 0, kmax = 0, K = 0, L_pad = 0, nbl = 0;
  int64_t max_samples = 0, max_blocks = 0;
  int2* pq = nullptr;           // [nbl] pairs in budget order (descending)
  int* perm = nullptr;          // [nbl] budget order -> row-major pair index
  int* budget = nullptr;        // [nbl] bin budget, budget order
  int* budget_canon = nullptr;  // [nbl] bin budget, row-major pair order
  int* tile_bins = nullptr;     // [pair tiles] largest budget of the tile
  float2* v = nullptr;   // [max_blocks][nbl][max Kc]
  std::vector<void*> allocs;
  std::string err;
};

int cfail(std::string* err, int status, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (err) *err = buf;
  return status;
}

template <class T>
int upload(Common& c, T** dst, const std::vector<T>& src) {
  if (hipMalloc((void**)dst, std::max<size_t>(src.size() * sizeof(T), 256)) != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    return DDX_ENOMEM;
  }
  c.allocs.push_back(*dst);
  if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return DDX_EDEVICE;
  }
  return DDX_OK;
}

void release(Common& c) {
  for (void* p : c.allocs) (void)hipFree(p);
  c.allocs.clear();
  c.pq = nullptr;
  c.v = nullptr;
}

// (c, d) with exp(-2 pi i u / N) = c - i d, u = num mod N, in FP64, stored FP32
float2 twiddle_cd(int64_t num, int n) {
  const int64_t r = ((num % n) + n) % n;
  const double ang = 2.0 * M_PI * (double)r / (double)n;
  return make_float2((float)std::cos(ang), (float)std::sin(ang));
}

// A stage of length n for the bins k >= 0 in klist; columns of V: +k then -k
// (k > 0) in list order; cmap maps them to the output bin index kmax + k.
int make_stage(Common& c, int n, const std::vector<int>& klist, Stage& st) {
  st.N = n;
  st.R = n / c.L;
  st.n_list = (int)klist.size();
  st.K_pad = std::max(1, (st.n_list + chirp::kTileK - 1) / chirp::kTileK) * chirp::kTileK;
  std::vector<float2> w((size_t)c.L_pad * st.K_pad, make_float2(0.f, 0.f));
  std::vector<float2> ph((size_t)st.R * st.K_pad, make_float2(0.f, 0.f));
  std::vector<int2> cols;
  std::vector<int> cmap;
  for (int j = 0; j < st.n_list; ++j) {
    const int kk = klist[j];
    for (int t = 0; t < c.L; ++t) w[(size_t)t * st.K_pad + j] = twiddle_cd((int64_t)t * kk, n);
    for (int r = 0; r < st.R; ++r) ph[(size_t)r * st.K_pad + j] = twiddle_cd((int64_t)r * c.L * kk, n);
    int2 col = make_int2((int)cmap.size(), -1);
    cmap.push_back(c.kmax + kk);
    if (kk > 0) {
      col.y = (int)cmap.size();
      cmap.push_back(c.kmax - kk);
    }
    cols.push_back(col);
  }
  st.Kc = (int)cmap.size();
  int rc;
  if ((rc = upload(c, &st.w, w)) || (rc = upload(c, &st.ph, ph)) || (rc = upload(c, &st.cols, cols)) ||
      (rc = upload(c, &st.cmap, cmap)) || (rc = upload(c, &st.klist, klist.empty() ? std::vector<int>{0} : klist)))
    return rc;
  return DDX_OK;
}

int make_common(Common& c, int n_ant, int block_len, int kmax, int64_t max_samples, int max_kc) {
  c.M = n_ant;
  c.L = block_len;
  c.kmax = kmax;
  c.K = 2 * kmax + 1;
  c.L_pad = (block_len + chirp::kChunk - 1) / chirp::kChunk * chirp::kChunk;
  c.nbl = n_ant * (n_ant - 1) / 2;
  c.max_samples = max_samples;
  c.max_blocks = max_samples / block_len;
  std::vector<int2> pq;
  for (int p = 0; p < n_ant; ++p)
    for (int q = p + 1; q < n_ant; ++q) pq.push_back(make_int2(p, q));
  std::vector<int> perm(c.nbl), budget(c.nbl, kmax);
  for (int i = 0; i < c.nbl; ++i) perm[i] = i;
  std::vector<int> tiles((c.nbl + chirp::kTileP - 1) / chirp::kTileP, kmax);
  int rc;
  if ((rc = upload(c, &c.pq, pq)) || (rc = upload(c, &c.perm, perm)) || (rc = upload(c, &c.budget, budget)) ||
      (rc = upload(c, &c.budget_canon, budget)) || (rc = upload(c, &c.tile_bins, tiles)))
    return rc;
  const size_t vb = (size_t)c.max_blocks * c.nbl * max_kc * sizeof(float2);
  if (hipMalloc((void**)&c.v, std::max<size_t>(vb, 256)) != hipSuccess) {
    (void)hipGetLastError();
    c.v = nullptr;
    return DDX_ENOMEM;
  }
  c.allocs.push_back(c.v);
  return DDX_OK;
}

// Partial DFTs and block CIC of one stage over nb blocks into out [nb - R + 1][nbl][K].
int run_stage(Common& c, const Stage& st, const float2* volts, int64_t n, float2* out, hipStream_t s) {
  const int64_t nb = n / c.L;
  chirp::PartialArgs a{};
  a.s = volts;
  a.pq = c.pq;
  a.w = st.w;
  a.ph = st.ph;
  a.cols = st.cols;
  a.klist = st.klist;
  a.tile_bins = c.tile_bins;
  a.v = c.v;
  a.n_samp = n;
  a.nbl = c.nbl;
  a.n_list = st.n_list;
  a.Kc = st.Kc;
  a.K_pad = st.K_pad;
  a.L = c.L;
  a.R = st.R;
  a.n_ptiles = (c.nbl + chirp::kTileP - 1) / chirp::kTileP;
  a.n_ktiles = st.K_pad / chirp::kTileK;
  const int64_t grid = nb * a.n_ptiles * a.n_ktiles;
  if (grid > INT32_MAX) return cfail(&c.err, DDX_EUNSUPPORTED, "too many blocks in one call");
  hipLaunchKernelGGL(chirp::k_partial, dim3((unsigned)grid), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cfail(&c.err, DDX_EDEVICE, "k_partial: %s", hipGetErrorString(e));
  const int64_t cols = (int64_t)c.nbl * st.Kc;
  // segments of at least 256 blocks (the R-block restart costs R / seg extra reads), at most 65535
  const int64_t seg = std::max<int64_t>(256, (nb + 65534) / 65535);
  hipLaunchKernelGGL(chirp::k_cic, dim3((unsigned)((cols + 255) / 256), (unsigned)((nb + seg - 1) / seg)), dim3(256), 0,
                     s, (const float2*)c.v, out, (const int*)st.cmap, (const int*)c.perm, (const int*)c.budget, cols,
                     (int32_t)st.Kc, (int32_t)c.K, (int32_t)nb, (int32_t)st.R, (int32_t)seg);
  e = hipGetLastError();
  if (e != hipSuccess) return cfail(&c.err, DDX_EDEVICE, "k_cic: %s", hipGetErrorString(e));
  return DDX_OK;
}

int smallest_prime_factor(int x) {
  for (int p = 2; p * p <= x; ++p)
    if (x % p == 0) return p;
  return x;
}

// Per-pair bin budgets (NULL: kmax for every pair): pairs sorted by budget,
// descending and stable, for the tile skip of k_partial; synchronous uploads.
int set_budgets(Common& c, const int32_t* host) {
  std::vector<int> budget(c.nbl, c.kmax);
  if (host)
    for (int i = 0; i < c.nbl; ++i) {
      if (host[i] < 0 || host[i] > c.kmax) return cfail(&c.err, DDX_EINVAL, "pair %d: bin budget %d not in [0, %d]", i, host[i], c.kmax);
      budget[i] = host[i];
    }
  std::vector<int> perm(c.nbl);
  for (int i = 0; i < c.nbl; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return budget[x] > budget[y]; });
  std::vector<int2> rowmajor, pq(c.nbl);
  for (int p = 0; p < c.M; ++p)
    for (int q = p + 1; q < c.M; ++q) rowmajor.push_back(make_int2(p, q));
  std::vector<int> bs(c.nbl), tiles((c.nbl + chirp::kTileP - 1) / chirp::kTileP, 0);
  for (int i = 0; i < c.nbl; ++i) {
    pq[i] = rowmajor[perm[i]];
    bs[i] = budget[perm[i]];
    tiles[i / chirp::kTileP] = std::max(tiles[i / chirp::kTileP], bs[i]);
  }
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(c.pq, pq.data(), pq.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.budget, bs.data(), bs.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.budget_canon, budget.data(), budget.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.tile_bins, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return cfail(&c.err, DDX_EDEVICE, "bin budget upload failed");
  }
  return DDX_OK;
}

}  // namespace

struct ddx_chirp {
  Common c;
  Stage st;
};

struct ddx_chirp_bank {
  Common c;
  int n0 = 0, n_len = 0;
  std::vector<Stage> st;                                  // [d - 1]
  std::vector<std::vector<std::pair<int, int2*>>> fac;    // [d - 1]: (p, device items) groups
  std::vector<std::vector<int>> fac_n;                    // [d - 1]: items per group
};

extern "C" {

int ddx_chirp_create(int32_t n_ant, int32_t fft_n, int32_t block_len, int32_t kmax, int64_t max_samples,
                     ddx_chirp** out) {
  if (!out) return DDX_EINVAL;
  *out = nullptr;
  if (n_ant < 2 || n_ant > 1024 || block_len < 1 || fft_n < block_len || fft_n % block_len != 0 || kmax < 0 ||
      2 * kmax + 1 > fft_n || max_samples < fft_n)
    return DDX_EINVAL;
  ddx_chirp* h = new (std::nothrow) ddx_chirp;
  if (!h) return DDX_ENOMEM;
  std::vector<int> klist(kmax + 1);
  for (int j = 0; j <= kmax; ++j) klist[j] = j;
  int rc = make_common(h->c, n_ant, block_len, kmax, max_samples, 2 * kmax + 1);
  if (!rc) rc = make_stage(h->c, fft_n, klist, h->st);
  if (rc) {
    release(h->c);
    delete h;
    return rc;
  }
  *out = h;
  return DDX_OK;
}

int ddx_chirp_output_shape(const ddx_chirp* h, int64_t n, int64_t* n_windows, int32_t* n_pairs, int32_t* n_bins) {
  if (!h || !n_windows || !n_pairs || !n_bins || n < 0) return DDX_EINVAL;
  const int64_t nb = n / h->c.L;
  *n_windows = nb >= h->st.R ? nb - h->st.R + 1 : 0;
  *n_pairs = h->c.nbl;
  *n_bins = h->c.K;
  return DDX_OK;
}

int ddx_chirp_preintegrate(ddx_chirp* h, const void* d_volts, int64_t n, void* d_out, void* hip_stream) {
  if (!h) return DDX_EINVAL;
  if (n < 0 || n > h->c.max_samples)
    return cfail(&h->c.err, DDX_EINVAL, "n = %lld outside [0, %lld]", (long long)n, (long long)h->c.max_samples);
  if (n / h->c.L < h->st.R) return DDX_OK;  // no complete window
  if (!d_volts || !d_out) return cfail(&h->c.err, DDX_EINVAL, "NULL device buffer");
  return run_stage(h->c, h->st, (const float2*)d_volts, n, (float2*)d_out, (hipStream_t)hip_stream);
}

int ddx_chirp_set_pair_bins(ddx_chirp* h, const int32_t* kmax_pair) {
  if (!h) return DDX_EINVAL;
  return set_budgets(h->c, kmax_pair);
}

int ddx_chirp_bank_set_pair_bins(ddx_chirp_bank* b, const int32_t* kmax_pair) {
  if (!b) return DDX_EINVAL;
  return set_budgets(b->c, kmax_pair);
}

const char* ddx_chirp_last_error(const ddx_chirp* h) { return h ? h->c.err.c_str() : "NULL pre-integrator"; }

int ddx_chirp_destroy(ddx_chirp* h) {
  if (!h) return DDX_OK;
  (void)hipDeviceSynchronize();
  release(h->c);
  delete h;
  return DDX_OK;
}

int ddx_chirp_bank_create(int32_t n_ant, int32_t n0, int32_t n_len, int32_t block_len, int32_t kmax,
                          int64_t max_samples, ddx_chirp_bank** out) {
  if (!out) return DDX_EINVAL;
  *out = nullptr;
  if (n_ant < 2 || n_ant > 1024 || block_len < 1 || n0 < block_len || n0 % block_len != 0 || n_len < 1 ||
      n_len > 64 || kmax < 0 || 2 * kmax + 1 > n0 || max_samples < (int64_t)n0 * n_len)
    return DDX_EINVAL;
  ddx_chirp_bank* b = new (std::nothrow) ddx_chirp_bank;
  if (!b) return DDX_ENOMEM;
  b->n0 = n0;
  b->n_len = n_len;
  // direct bins of length d: the k >= 0 with gcd(k, d) = 1; the others from length d / p
  std::vector<std::vector<int>> direct(n_len);
  int max_kc = 1;
  for (int d = 1; d <= n_len; ++d) {
    for (int kk = 0; kk <= kmax; ++kk)
      if (std::gcd(kk, d) == 1) direct[d - 1].push_back(kk);
    int kc = 0;
    for (int kk : direct[d - 1]) kc += kk > 0 ? 2 : 1;
    max_kc = std::max(max_kc, kc);
  }
  int rc = make_common(b->c, n_ant, block_len, kmax, max_samples, max_kc);
  b->st.resize(n_len);
  b->fac.resize(n_len);
  b->fac_n.resize(n_len);
  for (int d = 1; d <= n_len && !rc; ++d) {
    rc = make_stage(b->c, n0 * d, direct[d - 1], b->st[d - 1]);
    std::vector<std::vector<int2>> groups(d + 1);
    for (int kk = -kmax; kk <= kmax; ++kk) {
      const int g = std::gcd(std::abs(kk), d);  // gcd(0, d) = d
      if (g > 1) {
        const int p = smallest_prime_factor(g);
        groups[p].push_back(make_int2(kk, p));
      }
    }
    for (int p = 2; p <= d && !rc; ++p) {
      if (groups[p].empty()) continue;
      int2* dev = nullptr;
      rc = upload(b->c, &dev, groups[p]);
      b->fac[d - 1].push_back({p, dev});
      b->fac_n[d - 1].push_back((int)groups[p].size());
    }
  }
  if (rc) {
    release(b->c);
    delete b;
    return rc;
  }
  *out = b;
  return DDX_OK;
}

int ddx_chirp_bank_layout(const ddx_chirp_bank* b, int64_t n, int64_t* windows, int64_t* offsets, int64_t* total) {
  if (!b || !windows || !offsets || !total || n < 0) return DDX_EINVAL;
  const int64_t nb = n / b->c.L;
  int64_t off = 0;
  for (int d = 1; d <= b->n_len; ++d) {
    const int64_t r = (int64_t)b->n0 * d / b->c.L;
    windows[d - 1] = nb >= r ? nb - r + 1 : 0;
    offsets[d - 1] = off;
    off += windows[d - 1] * b->c.nbl * b->c.K;
  }
  *total = off;
  return DDX_OK;
}

int ddx_chirp_bank_run(ddx_chirp_bank* b, const void* d_volts, int64_t n, void* d_out, void* hip_stream) {
  if (!b) return DDX_EINVAL;
  if (n < 0 || n > b->c.max_samples)
    return cfail(&b->c.err, DDX_EINVAL, "n = %lld outside [0, %lld]", (long long)n, (long long)b->c.max_samples);
  std::vector<int64_t> win(b->n_len), off(b->n_len);
  int64_t total = 0;
  ddx_chirp_bank_layout(b, n, win.data(), off.data(), &total);
  if (total == 0) return DDX_OK;
  if (!d_volts || !d_out) return cfail(&b->c.err, DDX_EINVAL, "NULL device buffer");
  hipStream_t s = (hipStream_t)hip_stream;
  float2* out = (float2*)d_out;
  for (int d = 1; d <= b->n_len; ++d) {
    if (win[d - 1] == 0) continue;
    int rc = run_stage(b->c, b->st[d - 1], (const float2*)d_volts, n, out + off[d - 1], s);
    if (rc) return rc;
    for (size_t g = 0; g < b->fac[d - 1].size(); ++g) {
      const int p = b->fac[d - 1][g].first;
      const int ni = b->fac_n[d - 1][g];
      const int64_t threads = win[d - 1] * b->c.nbl * ni;
      hipLaunchKernelGGL(chirp::k_factor, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                         (const float2*)(out + off[d / p - 1]), out + off[d - 1], (const int2*)b->fac[d - 1][g].second,
                         (const int*)b->c.budget_canon, (int32_t)ni, win[d - 1], (int32_t)b->c.nbl, (int32_t)b->c.K,
                         (int32_t)b->c.kmax,
                         (int32_t)((int64_t)b->n0 * (d / p) / b->c.L));
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return cfail(&b->c.err, DDX_EDEVICE, "k_factor: %s", hipGetErrorString(e));
    }
  }
  return DDX_OK;
}

const char* ddx_chirp_bank_last_error(const ddx_chirp_bank* b) { return b ? b->c.err.c_str() : "NULL bank"; }

int ddx_chirp_bank_destroy(ddx_chirp_bank* b) {
  if (!b) return DDX_OK;
  (void)hipDeviceSynchronize();
  release(b->c);
  delete b;
  return DDX_OK;
}

}  // extern "C"
