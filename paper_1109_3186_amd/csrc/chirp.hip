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
// in 128-pair x 32-bin tiles on the FP32 matrix cores, each pair mixed as it feeds them from
// its tile's antennas staged in LDS.
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

constexpr int kTileP = 128;                // pairs per output tile
constexpr int kTileK = 4096 / kTileP;      // bins per output tile (4 waves of 32 x 32)
constexpr int kChunk = 32;   // samples per LDS chunk

struct PartialArgs {
  const float2* s;        // [M][n] complex samples
  const float2* w;        // [L_pad][K_pad] (c, d) of w_k[n] = c - i d, k = klist[j]
  const float2* ph;       // [R][K_pad] (c, d) of the block phase of bin klist[j]
  const int2* cols;       // [n_list] columns of V for +k and -k (-1: none, k = 0)
  const int2* act;        // [n_act] (pair tile, bin tile) with bins inside the tile's budgets
  const int* tile_ant;    // [n_ptiles][2 kTileP] antennas that a pair tile reads
  const int* tile_nant;   // [n_ptiles] their count
  const int2* loc;        // [nbl] (p, q) as indices into the tile's antenna list
  float2* v;              // [nb][nbl][Kc] partial DFTs (pairs in budget order)
  int64_t n_samp;         // samples per antenna row of s
  int32_t nbl, n_list, Kc, K_pad, L, R, n_act, sa_rows;
};

typedef float v16f __attribute__((ext_vector_type(16)));

// Workgroups are dealt to the eight XCDs in turn (id mod 8).  Numbering the work
// so that each XCD gets a contiguous run of blocks keeps the tiles of one block
// (which read the same antenna samples) on one L2.  The last total mod 8 keep
// their id.
__device__ __forceinline__ int xcd_order(int id, int total) {
  const int whole = total & ~7;
  return id < whole ? (id & 7) * (whole >> 3) + (id >> 3) : id;
}

// grid: nb * n_act workgroups of 256 threads (block slowest, in the order of
// xcd_order), one per block and active (pair tile, bin tile): tiles whose bins all
// lie beyond the bin budgets of their pairs are left out of the grid on the host
// (an early exit in the kernel instead left whole shader engines idle: the skipped
// tiles fell on every other engine).  The product runs on the FP32 matrix cores (v_mfma_f32_32x32x2_f32: twice the
// FP32 rate of unpacked vector FMAs, FP32 products and sums).  The four sums are
// four real products of the tile: P = a c, Q = b d, R = a d, T = b c,
// each [32 pairs x 2 samples] x [2 samples x 32 bins] per instruction.  The staging
// reads the tile's antennas as rows of consecutive samples (coalesced) and mixes
// each pair when it feeds the matrix core, instead of gathering s_p and s_q per
// pair.  Wave w owns pairs 32 (w / WK) .. and listed bins 32 (w % WK) .. of the
// tile (WK = kTileK / 32 waves along the bins; 32-bin tiles let per-pair budgets
// skip bins in finer steps).
// Lane l supplies pair (or bin) l % 32 of sample l / 32 of each sample pair and
// holds, of each 32 x 32 result, bin l % 32 of the pairs 8 (v / 4) + 4 (l / 32)
// + v % 4, v < 16.
__global__ __launch_bounds__(256) void k_partial_mfma(PartialArgs a) {
  // dynamic LDS: the tile's antennas (sa_rows >= their count, at most two per pair),
  // kChunk samples each, padded by one entry so that the lanes' different antennas
  // fall in different banks; then the W rows of the chunk, kChunk x kTileK
  extern __shared__ float2 lds[];
  float2* sa = lds;
  float2* ws = lds + a.sa_rows * (kChunk + 1);
  const int tid = threadIdx.x;
  const int id = xcd_order(blockIdx.x, gridDim.x);
  const int2 tile = a.act[id % a.n_act];
  const int pt = tile.x, kt = tile.y;
  const int m = id / a.n_act;
  const int p0 = pt * kTileP, k0 = kt * kTileK;
  const int wv = tid >> 6, lane = tid & 63;
  constexpr int WK = kTileK / 32;     // waves along the bins
  const int wp = (wv / WK) * 32, wk = (wv % WK) * 32;
  const int r = lane & 31, h = lane >> 5;
  const int64_t base = (int64_t)m * a.L;
  const int na = a.tile_nant[pt];
  const int* ants = a.tile_ant + pt * 2 * kTileP;
  const int my_pair = p0 + wp + r;
  const int2 lc = my_pair < a.nbl ? a.loc[my_pair] : make_int2(0, 0);
  const float live = my_pair < a.nbl ? 1.f : 0.f;
  v16f P = {}, Q = {}, R = {}, T = {};

  for (int n0 = 0; n0 < a.L; n0 += kChunk) {
    __syncthreads();
    // the antennas' samples: rows of kChunk consecutive samples, coalesced
    for (int e = tid; e < na * kChunk; e += 256) {
      const int ai = e / kChunk, n = e % kChunk;
      float2 v = make_float2(0.f, 0.f);
      if (n0 + n < a.L) v = a.s[(int64_t)ants[ai] * a.n_samp + base + n0 + n];
      sa[ai * (kChunk + 1) + n] = v;
    }
#pragma unroll
    for (int q = 0; q < (kChunk * kTileK) / 256; ++q) {
      const int e = tid + 256 * q;
      const int n = e / kTileK, kl = e % kTileK;
      ws[n * kTileK + kl] = a.w[(int64_t)(n0 + n) * a.K_pad + k0 + kl];
    }
    __syncthreads();
#pragma unroll 4
    for (int n = 0; n < kChunk; n += 2) {
      // x = s_p conj(s_q) of the lane's pair and sample, mixed at the operand
      const float2 sp = sa[lc.x * (kChunk + 1) + n + h], sq = sa[lc.y * (kChunk + 1) + n + h];
      const float xr = live * (sp.x * sq.x + sp.y * sq.y), xi = live * (sp.y * sq.x - sp.x * sq.y);
      const float2 wt = ws[(n + h) * kTileK + wk + r];
      P = __builtin_amdgcn_mfma_f32_32x32x2f32(xr, wt.x, P, 0, 0, 0);
      Q = __builtin_amdgcn_mfma_f32_32x32x2f32(xi, wt.y, Q, 0, 0, 0);
      R = __builtin_amdgcn_mfma_f32_32x32x2f32(xr, wt.y, R, 0, 0, 0);
      T = __builtin_amdgcn_mfma_f32_32x32x2f32(xi, wt.x, T, 0, 0, 0);
    }
  }
  const int jl = k0 + wk + r;
  if (jl >= a.n_list) return;
  const float2 f = a.ph[(int64_t)(m % a.R) * a.K_pad + jl];
  const int2 col = a.cols[jl];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int pair = p0 + wp + 8 * (v >> 2) + 4 * h + (v & 3);
    if (pair >= a.nbl) continue;
    const float pr = P[v] + Q[v], pi = T[v] - R[v];  // V_k
    const float nr = P[v] - Q[v], ni = R[v] + T[v];  // V_-k
    float2* row = a.v + ((int64_t)m * a.nbl + pair) * a.Kc;
    row[col.x] = make_float2(pr * f.x + pi * f.y, pi * f.x - pr * f.y);
    if (col.y >= 0) row[col.y] = make_float2(nr * f.x - ni * f.y, ni * f.x + nr * f.y);
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
  std::vector<int> klist;  // [n_list] the listed bins k >= 0 (host)
  int2* act = nullptr;   // [n_act] active (pair tile, bin tile), see set_active
  int n_act = 0;
};

struct Common {
  int M = 0, L = 0, kmax = 0, K = 0, L_pad = 0, nbl = 0;
  int64_t max_samples = 0, max_blocks = 0;
  int* perm = nullptr;          // [nbl] budget order -> row-major pair index
  int* budget = nullptr;        // [nbl] bin budget, budget order
  int* budget_canon = nullptr;  // [nbl] bin budget, row-major pair order
  std::vector<int> tile_bins;   // [pair tiles] largest budget of the tile (host)
  int* tile_ant = nullptr;      // [pair tiles][2 kTileP] antennas read by the tile
  int* tile_nant = nullptr;     // [pair tiles] their count
  int na_max = 1;               // the largest count
  int2* loc = nullptr;          // [nbl] (p, q) as indices into the tile's antennas
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
  c.v = nullptr;
}

// (c, d) with exp(-2 pi i u / N) = c - i d, u = num mod N, in FP64, stored FP32
float2 twiddle_cd(int64_t num, int n) {
  const int64_t r = ((num % n) + n) % n;
  const double ang = 2.0 * M_PI * (double)r / (double)n;
  return make_float2((float)std::cos(ang), (float)std::sin(ang));
}

// The (pair tile, bin tile) pairs of a stage that hold a bin within the largest
// budget of the tile's pairs, bin tile fastest; uploaded to the stage's list
// (allocated once at its largest size).  Synchronous.
int set_active(Common& c, Stage& st) {
  const int n_ptiles = (c.nbl + chirp::kTileP - 1) / chirp::kTileP;
  const int n_ktiles = st.K_pad / chirp::kTileK;
  std::vector<int2> act;
  for (int pt = 0; pt < n_ptiles; ++pt)
    for (int kt = 0; kt < n_ktiles; ++kt) {
      const int k0 = kt * chirp::kTileK;
      if (k0 < st.n_list && st.klist[k0] > c.tile_bins[pt]) continue;
      act.push_back(make_int2(pt, kt));
    }
  if (!st.act) {
    std::vector<int2> all((size_t)n_ptiles * n_ktiles, make_int2(0, 0));
    int rc = upload(c, &st.act, all);
    if (rc) return rc;
  }
  if (hipMemcpy(st.act, act.data(), act.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return cfail(&c.err, DDX_EDEVICE, "tile list upload failed");
  }
  st.n_act = (int)act.size();
  return DDX_OK;
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
      (rc = upload(c, &st.cmap, cmap)))
    return rc;
  st.klist = klist;
  return set_active(c, st);
}

// The distinct antennas of each tile of kTileP consecutive pairs (pair order pq),
// and each pair's (p, q) as indices into its tile's list.
void tile_antennas(const std::vector<int2>& pq, int n_ant, std::vector<int>& ants, std::vector<int>& nant,
                   std::vector<int2>& loc) {
  const int n_tiles = ((int)pq.size() + chirp::kTileP - 1) / chirp::kTileP;
  ants.assign((size_t)n_tiles * 2 * chirp::kTileP, 0);
  nant.assign(n_tiles, 0);
  loc.assign(pq.size(), make_int2(0, 0));
  std::vector<int> slot(n_ant, -1);
  for (int t = 0; t < n_tiles; ++t) {
    std::fill(slot.begin(), slot.end(), -1);
    int cnt = 0;
    for (int i = t * chirp::kTileP; i < std::min((int)pq.size(), (t + 1) * chirp::kTileP); ++i) {
      for (int ant : {pq[i].x, pq[i].y})
        if (slot[ant] < 0) {
          slot[ant] = cnt;
          ants[(size_t)t * 2 * chirp::kTileP + cnt++] = ant;
        }
      loc[i] = make_int2(slot[pq[i].x], slot[pq[i].y]);
    }
    nant[t] = cnt;
  }
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
  c.tile_bins.assign((c.nbl + chirp::kTileP - 1) / chirp::kTileP, kmax);
  std::vector<int> ants, nant;
  std::vector<int2> loc;
  tile_antennas(pq, n_ant, ants, nant, loc);
  c.na_max = std::max(1, *std::max_element(nant.begin(), nant.end()));
  int rc;
  if ((rc = upload(c, &c.perm, perm)) || (rc = upload(c, &c.budget, budget)) ||
      (rc = upload(c, &c.budget_canon, budget)) ||
      (rc = upload(c, &c.tile_ant, ants)) || (rc = upload(c, &c.tile_nant, nant)) || (rc = upload(c, &c.loc, loc)))
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
  a.w = st.w;
  a.ph = st.ph;
  a.cols = st.cols;
  a.act = st.act;
  a.tile_ant = c.tile_ant;
  a.tile_nant = c.tile_nant;
  a.loc = c.loc;
  a.v = c.v;
  a.n_samp = n;
  a.nbl = c.nbl;
  a.n_list = st.n_list;
  a.Kc = st.Kc;
  a.K_pad = st.K_pad;
  a.L = c.L;
  a.R = st.R;
  a.n_act = st.n_act;
  a.sa_rows = c.na_max;
  const int64_t grid = nb * st.n_act;
  if (grid > INT32_MAX) return cfail(&c.err, DDX_EUNSUPPORTED, "too many blocks in one call");
  // no active tile: every listed bin lies beyond every budget, and the CIC writes zeros
  const size_t lds = ((size_t)c.na_max * (chirp::kChunk + 1) + chirp::kChunk * chirp::kTileK) * sizeof(float2);
  if (grid > 0) hipLaunchKernelGGL(chirp::k_partial_mfma, dim3((unsigned)grid), dim3(256), lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cfail(&c.err, DDX_EDEVICE, "k_partial_mfma: %s", hipGetErrorString(e));
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
  std::vector<int> ants, nant;
  std::vector<int2> loc;
  tile_antennas(pq, c.M, ants, nant, loc);
  const int na_max = std::max(1, *std::max_element(nant.begin(), nant.end()));
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(c.tile_ant, ants.data(), ants.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.tile_nant, nant.data(), nant.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.loc, loc.data(), loc.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.budget, bs.data(), bs.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.budget_canon, budget.data(), budget.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return cfail(&c.err, DDX_EDEVICE, "bin budget upload failed");
  }
  c.tile_bins = tiles;
  c.na_max = na_max;
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
  const int rc = set_budgets(h->c, kmax_pair);
  return rc ? rc : set_active(h->c, h->st);
}

int ddx_chirp_bank_set_pair_bins(ddx_chirp_bank* b, const int32_t* kmax_pair) {
  if (!b) return DDX_EINVAL;
  int rc = set_budgets(b->c, kmax_pair);
  for (size_t d = 0; !rc && d < b->st.size(); ++d) rc = set_active(b->c, b->st[d]);
  return rc;
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
