// The Chimageator on a uniform linear array (Bannister & Cornwell 2011, Sec. 4) on
// gfx950: mixing and gridding of redundant spacings, integration over blocks of L
// samples (the pre-integrator), the spatial DFT of each block, and the
// phase-corrected trajectory sums of the post-integrator (Eq. chimg_pth).
//
//   G_l[m]  = w_l / L sum_{p < M - l} sum_{n in block m} s_p[n] s_{p+l}[n]^*,  l = 1 .. M - 1
//             (natural weights w_l = 1 / (M - l), or uniform w_l = 1)
//   Y_k[m]  = sum_l G_l[m] exp(-2 pi i k l / N_s),  k < N_s
//   P[i][m0] = sum_{m=m0}^{m0+T_i-1} conj(Phi(x_m)) Y_{k_m}[m],  k0 = k_end,i ((m - m0) L
//             + (L - 1) / 2) / (T_i L), k_m = rint(k0) mod N_s, x_m = k0 - rint(k0),
//             Phi(x) = exp(pi i M x / N_s)
//
// A block's gridded products are a small correlation (M antennas x L samples), so
// one workgroup makes one block: the block's samples in LDS, each thread a
// (spacing, sample phase) share of the products, then one thread per spatial bin
// with a twiddle table in LDS.  The
// trajectory sums are gathers along a line in (block, bin): one thread per (trial,
// start block), the bin decided in FP64 like the plain definition.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ddx.h"

namespace chimg {

constexpr int kThreads = 256;
constexpr int kMaxAnt = kThreads + 1;     // spacings 1 .. M - 1, at least one thread each
constexpr int kMaxBins = 1024;            // N_s
constexpr int kStage = 5120;              // complex samples staged per round (40 KB)

// grid: nb workgroups of 256 threads, one per block m.
__global__ __launch_bounds__(kThreads) void k_pre(const float2* __restrict__ s, int32_t M, int64_t n, int32_t L,
                                                  int32_t n_s, int32_t natural, float2* __restrict__ y) {
  __shared__ float2 xs[kStage];
  __shared__ float2 g[kMaxAnt];
  __shared__ float2 tw[kMaxBins];
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  for (int r = tid; r < n_s; r += kThreads) {
    float sn, cs;
    sincospif(2.0f * (float)r / (float)n_s, &sn, &cs);   // r / n_s exact for n_s a power of two
    tw[r] = make_float2(cs, -sn);                        // exp(-2 pi i r / N_s)
  }
  // thread (spacing l, phase ph): the samples j = ph, ph + S, ... of every pair at
  // spacing l, S = floor(256 / (M - 1)) phases so that all threads work
  const int S = max(1, kThreads / (M - 1));
  const int l = tid / S + 1, ph = tid % S;
  float2 acc = make_float2(0.f, 0.f);
  const int chunk = max(1, kStage / M);
  for (int n0 = 0; n0 < L; n0 += chunk) {
    const int len = min(chunk, L - n0);
    __syncthreads();
    for (int e = tid; e < M * len; e += kThreads) {
      const int p = e / len, j = e - p * len;
      xs[p * len + j] = s[(int64_t)p * n + (int64_t)m * L + n0 + j];
    }
    __syncthreads();
    if (l < M) {
      for (int p = 0; p + l < M; ++p) {
        const float2* a = xs + p * len;
        const float2* b = xs + (p + l) * len;
        for (int j = ph; j < len; j += S) {   // a b^*
          acc.x = fmaf(a[j].x, b[j].x, fmaf(a[j].y, b[j].y, acc.x));
          acc.y = fmaf(a[j].y, b[j].x, fmaf(-a[j].x, b[j].y, acc.y));
        }
      }
    }
  }
  // the phases of each spacing, summed in a fixed order
  __syncthreads();
  float2* part = xs;   // the staged samples are no longer needed
  if (l < M) part[tid] = acc;
  __syncthreads();
  if (tid < M - 1) {
    float2 v = make_float2(0.f, 0.f);
    for (int q = 0; q < S; ++q) {
      const float2 a = part[tid * S + q];
      v.x += a.x;
      v.y += a.y;
    }
    const float w = (natural ? 1.0f / (float)(M - 1 - tid) : 1.0f) / (float)L;
    g[tid] = make_float2(v.x * w, v.y * w);
  }
  __syncthreads();
  for (int k = tid; k < n_s; k += kThreads) {
    float2 v = make_float2(0.f, 0.f);
    for (int q = 1; q < M; ++q) {
      const float2 a = g[q - 1];
      const float2 t = tw[(int)(((int64_t)k * q) % n_s)];
      v.x = fmaf(a.x, t.x, fmaf(-a.y, t.y, v.x));
      v.y = fmaf(a.x, t.y, fmaf(a.y, t.x, v.y));
    }
    y[(int64_t)k * gridDim.x + m] = v;   // bin-major: a trajectory reads along blocks
  }
}

typedef float v16f __attribute__((ext_vector_type(16)));

// The same pre-integrator for M <= 64 with the pair products on the FP32 matrix
// cores: per block, C = X X^H over its L samples (X the M x L block, rows padded to
// 64), Re C = Xr Xr^T + Xi Xi^T and Im C = Xi Xr^T - Xr Xi^T as
// v_mfma_f32_32x32x2_f32 products (two samples per instruction), wave w making the
// 32 x 32 quadrant (w / 2, w % 2) (the lower-left one is not needed).  C is then
// written to LDS and each spacing's diagonal summed in a fixed order, so results
// do not depend on scheduling.  Lane l supplies antenna l % 32 of the quadrant's
// rows (A) or columns (B) at sample l / 32 of each pair of samples and holds C at
// column l % 32, rows 8 (v / 4) + 4 (l / 32) + v % 4.
// CELLS: the pairs are gridded onto cells given as lists (cell_ptr [n_cells + 1],
// cell_pairs [(a, b)]: the product s_a s_b^*, read from C[a][b] or, for a > b, as
// conj(C[b][a])) with natural weights instead of the line's spacings.  PLANAR: the
// cells sit at grid points uv[c] = (cu, cv) of a plane and the spatial DFT is
// two-dimensional, Y[ku N_s + kv][m] = sum_c g_c exp(-2 pi i (ku cu + kv cv) / N_s).
// grid: nb workgroups of 256 threads.
template <bool CELLS, bool PLANAR = false>
__global__ __launch_bounds__(kThreads) void k_pre_mfma(const float2* __restrict__ s, int32_t M, int64_t n, int32_t L,
                                                       int32_t n_s, int32_t natural, const int32_t* __restrict__ cell_ptr,
                                                       const int2* __restrict__ cell_pairs, int32_t n_cells,
                                                       float2* __restrict__ y, const int2* __restrict__ uv = nullptr) {
  constexpr int R = 64;                 // padded antenna rows
  constexpr int CH = kStage / R;        // samples per staging round (80)
  constexpr int NG = CELLS ? kMaxBins : R;
  __shared__ float2 xs[kStage];         // [R][CH] samples, then C [R][R + 1]
  __shared__ float2 g[NG];
  __shared__ float2 tw[kMaxBins];
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  for (int r = tid; r < n_s; r += kThreads) {
    float sn, cs;
    sincospif(2.0f * (float)r / (float)n_s, &sn, &cs);
    tw[r] = make_float2(cs, -sn);
  }
  const int wv = tid >> 6, lane = tid & 63;
  const int rp = (wv >> 1) * 32, cq = (wv & 1) * 32;
  const int i = lane & 31, h = lane >> 5;
  const bool used = !(rp == 32 && cq == 0);
  v16f re = {}, im = {};
  for (int n0 = 0; n0 < L; n0 += CH) {
    const int len = min(CH, L - n0);
    __syncthreads();
    {
      // all the round's loads are issued before the first LDS store (their
      // latencies overlap)
      static_assert(R * CH % kThreads == 0, "the staging covers the tile in whole rounds");
      constexpr int PER = R * CH / kThreads;
      float2 v[PER];
      const float2* sm = s + (int64_t)m * L + n0;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = tid + u * kThreads;
        const int p = e / CH, j = e - p * CH;
        v[u] = (p < M && j < len) ? sm[(int64_t)p * n + j] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) xs[tid + u * kThreads] = v[u];
    }
    __syncthreads();
    if (used) {
      for (int j = 0; j < len; j += 2) {   // samples past len are staged as zero
        const float2 a = xs[(rp + i) * CH + j + h];
        const float2 b = xs[(cq + i) * CH + j + h];
        re = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_32x32x2f32(-a.x, b.y, im, 0, 0, 0);
      }
    }
  }
  __syncthreads();
  float2* C = xs;                       // [R][R + 1]
  if (used) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = rp + 8 * (v >> 2) + 4 * h + (v & 3);
      C[row * (R + 1) + cq + i] = make_float2(re[v], im[v]);
    }
  }
  __syncthreads();
  int n_g;   // gridded cells 1 .. n_g
  if (CELLS) {
    n_g = n_cells;
    for (int c = tid; c < n_cells; c += kThreads) {
      const int b0 = cell_ptr[c], b1 = cell_ptr[c + 1];
      float2 v = make_float2(0.f, 0.f);
      for (int b = b0; b < b1; ++b) {
        const int2 pq = cell_pairs[b];   // a != b < M by contract; clamped to the tile
        const int lo = min(max(min(pq.x, pq.y), 0), R - 1), hi = min(max(max(pq.x, pq.y), 0), R - 1);
        const float2 cc = C[lo * (R + 1) + hi];   // the upper triangle holds s_lo s_hi^*
        v.x += cc.x;
        v.y += pq.x <= pq.y ? cc.y : -cc.y;
      }
      const float w = b1 > b0 ? 1.0f / ((float)(b1 - b0) * (float)L) : 0.f;
      g[c] = make_float2(v.x * w, v.y * w);
    }
  } else {
    n_g = M - 1;
    if (tid < M - 1) {
      const int l = tid + 1;
      float2 v = make_float2(0.f, 0.f);
      for (int p = 0; p + l < M; ++p) {
        const float2 c = C[p * (R + 1) + p + l];
        v.x += c.x;
        v.y += c.y;
      }
      const float w = (natural ? 1.0f / (float)(M - l) : 1.0f) / (float)L;
      g[tid] = make_float2(v.x * w, v.y * w);
    }
  }
  __syncthreads();
  if constexpr (PLANAR) {
    __shared__ int2 uvs[kMaxBins];
    for (int c = tid; c < n_cells; c += kThreads) uvs[c] = uv[c];
    __syncthreads();
    // n_s a power of two: (ku cu + kv cv) mod N_s by a mask, negative coordinates included
    const int mask = n_s - 1;
    for (int k = tid; k < n_s * n_s; k += kThreads) {
      const int ku = k / n_s, kv = k - ku * n_s;
      float2 v = make_float2(0.f, 0.f);
      for (int c = 0; c < n_cells; ++c) {
        const float2 a = g[c];
        const int2 w = uvs[c];
        const float2 t = tw[(ku * w.x + kv * w.y) & mask];
        v.x = fmaf(a.x, t.x, fmaf(-a.y, t.y, v.x));
        v.y = fmaf(a.x, t.y, fmaf(a.y, t.x, v.y));
      }
      y[(int64_t)k * gridDim.x + m] = v;
    }
  } else {
    for (int k = tid; k < n_s; k += kThreads) {
      float2 v = make_float2(0.f, 0.f);
      for (int q = 1; q <= n_g; ++q) {
        const float2 a = g[q - 1];
        const float2 t = tw[(int)(((int64_t)k * q) % n_s)];
        v.x = fmaf(a.x, t.x, fmaf(-a.y, t.y, v.x));
        v.y = fmaf(a.x, t.y, fmaf(a.y, t.x, v.y));
      }
      y[(int64_t)k * gridDim.x + m] = v;
    }
  }
}

// grid: (ceil(nb / 256), n_trials) x 256; thread = start block m0 of trial i.  The
// bin k_q and phase conj(Phi(x_q)) of step q depend on the trial only: they are
// made once per workgroup in LDS (kSteps at a time), and every thread then reads
// Y[k_q][m0 + q], contiguous across the threads.
constexpr int kSteps = 1024;
__global__ __launch_bounds__(kThreads) void k_traj(const float2* __restrict__ y, int64_t nb, int32_t M,
                                                   int32_t n_s, int32_t L, const double* __restrict__ k_end,
                                                   const int32_t* __restrict__ t_blocks, float2* __restrict__ p) {
  __shared__ int kq[kSteps];
  __shared__ float2 cq[kSteps];
  const int64_t m0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int i = blockIdx.y;
  const int tb = t_blocks[i];
  const double ke = k_end[i];
  const bool live = tb >= 1 && m0 + tb <= nb;
  float2 acc = make_float2(0.f, 0.f);
  for (int q0 = 0; q0 < tb; q0 += kSteps) {
    const int nq = min(kSteps, tb - q0);
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += kThreads) {
      double k0;
      {
#pragma clang fp contract(off)
        // the plain definition's operation order, so that rint(k0) is decided alike
        k0 = ke * ((double)((int64_t)(q0 + q) * L) + (L - 1) / 2.0) / (double)((int64_t)tb * L);
      }
      const double kr = rint(k0);
      const float x = (float)(k0 - kr);
      int64_t kb = (int64_t)kr % n_s;
      if (kb < 0) kb += n_s;
      float sn, cs;
      sincospif(-(float)M * x / (float)n_s, &sn, &cs);    // conj(Phi(x))
      kq[q] = (int)kb;
      cq[q] = make_float2(cs, sn);
    }
    __syncthreads();
    if (live) {
      for (int q = 0; q < nq; ++q) {
        const float2 v = y[(int64_t)kq[q] * nb + m0 + q0 + q];
        const float2 c = cq[q];
        acc.x += v.x * c.x - v.y * c.y;
        acc.y += v.x * c.y + v.y * c.x;
      }
    }
  }
  if (m0 < nb) p[(int64_t)i * nb + m0] = acc;
}

// Trajectories sharing a gradient g (bins per block) lie on one line, so the sums
// for several durations are partial sums of the longest (the paper's optimisation
// of the imaging step): one pass along the line per (gradient, start), the running
// sum written out each time the step count reaches a requested duration.
// lengths: ascending.  grid: (ceil(nb / 256), n_grad) x 256.
__global__ __launch_bounds__(kThreads) void k_grad(const float2* __restrict__ y, int64_t nb, int32_t M, int32_t n_s,
                                                   int32_t L, const double* __restrict__ grad,
                                                   const int32_t* __restrict__ lengths, int32_t n_len,
                                                   float2* __restrict__ p) {
  __shared__ int kq[kSteps];
  __shared__ float2 cq[kSteps];
  const int64_t m0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int i = blockIdx.y;
  const double g = grad[i];
  const int tmax = lengths[n_len - 1];
  float2 acc = make_float2(0.f, 0.f);
  int jn = 0;                  // next duration to write
  int next = lengths[0];       // its step count
  for (int q0 = 0; q0 < tmax; q0 += kSteps) {
    const int nq = min(kSteps, tmax - q0);
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += kThreads) {
      double k0;
      {
#pragma clang fp contract(off)
        k0 = g * ((double)((int64_t)(q0 + q) * L) + (L - 1) / 2.0) / (double)L;
      }
      const double kr = rint(k0);
      const float x = (float)(k0 - kr);
      int64_t kb = (int64_t)kr % n_s;
      if (kb < 0) kb += n_s;
      float sn, cs;
      sincospif(-(float)M * x / (float)n_s, &sn, &cs);    // conj(Phi(x))
      kq[q] = (int)kb;
      cq[q] = make_float2(cs, sn);
    }
    __syncthreads();
    if (m0 < nb) {
      // steps inside the blocks, then none: the remaining durations only get zeros
      const int nin = (int)min((int64_t)nq, max((int64_t)0, nb - m0 - q0));
      for (int q = 0; q < nq; ++q) {
        if (q < nin) {
          const float2 v = y[(int64_t)kq[q] * nb + m0 + q0 + q];
          const float2 c = cq[q];
          acc.x += v.x * c.x - v.y * c.y;
          acc.y += v.x * c.y + v.y * c.x;
        }
        if (q0 + q + 1 == next) {
          const float2 out = m0 + next <= nb ? acc : make_float2(0.f, 0.f);
          for (; jn < n_len && lengths[jn] == next; ++jn) p[((int64_t)i * n_len + jn) * nb + m0] = out;
          next = jn < n_len ? lengths[jn] : INT32_MAX;
        }
      }
    }
  }
}

// App. B's widened and sampled trajectories in one kernel: trial i integrates a_i
// blocks per sample (the integrate-and-dump of Eq. Yk) and, with F >= 1, sums the
// 2F + 1 bins around each step weighted by the spatial tone's matched filter
// conj(Phi(x_t)) S(x_t) / (M - 1), x_t = k0 - (k_j + t), S(x) = sin(pi (M - 1) x /
// N_s) / sin(pi x / N_s); F = 0 is Eq. chimg_pth's phase-only single bin.  Sample j
// stands at the mean of its a L samples: k0 = k_end (j a L + (a L - 1) / 2) / (T L).
// The (step, tap) bins and weights of a trial are made in LDS, kExtEntries at a time.
// grid: (ceil(nb / 256), n_trials) x 256; thread = start block m0.
constexpr int kExtEntries = 4096;
__global__ __launch_bounds__(kThreads) void k_traj_ext(const float2* __restrict__ y, int64_t nb, int32_t M,
                                                       int32_t n_s, int32_t L, const double* __restrict__ k_end,
                                                       const int32_t* __restrict__ t_blocks,
                                                       const int32_t* __restrict__ a_blocks, int32_t F,
                                                       float2* __restrict__ p) {
  __shared__ int kq[kExtEntries];
  __shared__ float2 cq[kExtEntries];
  const int64_t m0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int i = blockIdx.y;
  const int tb = t_blocks[i];
  const int a = a_blocks ? a_blocks[i] : 1;
  const double ke = k_end[i];
  const int taps = 2 * F + 1;
  const int J = (tb >= 1 && a >= 1) ? tb / a : 0;
  const bool live = J >= 1 && m0 + tb <= nb;
  const int per = kExtEntries / taps;
  float2 acc = make_float2(0.f, 0.f);
  for (int j0 = 0; j0 < J; j0 += per) {
    const int nj = min(per, J - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < nj * taps; e += kThreads) {
      const int j = j0 + e / taps, t = e % taps - F;
      double k0;
      {
#pragma clang fp contract(off)
        // the plain definition's operation order, so that rint(k0) is decided alike
        k0 = ke * ((double)((int64_t)j * a * L) + (a * L - 1) / 2.0) / (double)((int64_t)tb * L);
      }
      const double kr = rint(k0);
      const float x = (float)(k0 - (kr + t));
      int64_t kb = ((int64_t)kr + t) % n_s;
      if (kb < 0) kb += n_s;
      float sn, cs;
      sincospif(-(float)M * x / (float)n_s, &sn, &cs);    // conj(Phi(x))
      float amp = 1.f;
      if (F > 0) {
        const float den = sinpif(x / (float)n_s);
        amp = (fabsf(den) < 1e-30f ? (float)(M - 1) : sinpif((float)(M - 1) * x / (float)n_s) / den) /
              (float)(M - 1);
      }
      kq[e] = (int)kb;
      cq[e] = make_float2(cs * amp, sn * amp);
    }
    __syncthreads();
    if (live) {
      for (int jj = 0; jj < nj; ++jj) {
        const int64_t base = m0 + (int64_t)(j0 + jj) * a;
        for (int t = 0; t < taps; ++t) {
          const int e = jj * taps + t;
          const float2* row = y + (int64_t)kq[e] * nb + base;
          float2 s = make_float2(0.f, 0.f);
          for (int r = 0; r < a; ++r) {
            s.x += row[r].x;
            s.y += row[r].y;
          }
          const float2 c = cq[e];
          acc.x += s.x * c.x - s.y * c.y;
          acc.y += s.x * c.y + s.y * c.x;
        }
      }
    }
  }
  if (m0 < nb) p[(int64_t)i * nb + m0] = acc;
}

// Step tables of planar trajectories: for trial i and step q the image bin ku N_s + kv
// (k0 = k_end f per axis, f = (q L + (L - 1) / 2) / (T L), rint in FP64 like the plain
// definition) and the phase correction conj(R(x)) / |R(x)|, R(x) = sum over the
// occupied cells of exp(2 pi i (xu cu + xv cv) / N_s).
// grid: (ceil(max_t / 256), n_trials) x 256.
__global__ __launch_bounds__(kThreads) void k_traj2d_table(const int2* __restrict__ uv, int32_t n_cells,
                                                           int32_t n_s, int32_t L, const double* __restrict__ k_end,
                                                           const int32_t* __restrict__ t_blocks, int32_t max_t,
                                                           int32_t* __restrict__ bins, float2* __restrict__ w) {
  const int q = blockIdx.x * kThreads + threadIdx.x;
  const int i = blockIdx.y;
  const int tb = t_blocks[i];
  if (q >= tb || q >= max_t) return;
  double k0u, k0v;
  {
#pragma clang fp contract(off)
    const double f = ((double)((int64_t)q * L) + (L - 1) / 2.0) / (double)((int64_t)tb * L);
    k0u = k_end[2 * i] * f;
    k0v = k_end[2 * i + 1] * f;
  }
  const double ru = rint(k0u), rv = rint(k0v);
  const float xu = (float)(k0u - ru), xv = (float)(k0v - rv);
  float re = 0.f, im = 0.f;
  for (int c = 0; c < n_cells; ++c) {
    const int2 e = uv[c];
    float sn, cs;
    sincospif(2.0f * (xu * (float)e.x + xv * (float)e.y) / (float)n_s, &sn, &cs);
    re += cs;
    im += sn;
  }
  const float mag = sqrtf(re * re + im * im);
  int64_t bu = (int64_t)ru % n_s, bv = (int64_t)rv % n_s;
  if (bu < 0) bu += n_s;
  if (bv < 0) bv += n_s;
  bins[(int64_t)i * max_t + q] = (int)(bu * n_s + bv);
  w[(int64_t)i * max_t + q] = mag > 0.f ? make_float2(re / mag, -im / mag) : make_float2(0.f, 0.f);
}

// Trajectory sums from step tables: P[i][m0] = sum_{q < T_i} w[i][q] Y[bins[i][q]][m0 + q],
// zero where m0 + T_i > nb.  grid: (ceil(nb / 256), n_trials) x 256.
__global__ __launch_bounds__(kThreads) void k_traj_table(const float2* __restrict__ y, int64_t nb,
                                                         const int32_t* __restrict__ t_blocks, int32_t max_t,
                                                         const int32_t* __restrict__ bins,
                                                         const float2* __restrict__ w, float2* __restrict__ p) {
  __shared__ int kq[kSteps];
  __shared__ float2 cq[kSteps];
  const int64_t m0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int i = blockIdx.y;
  const int tb = min(t_blocks[i], max_t);
  const bool live = tb >= 1 && t_blocks[i] <= max_t && m0 + tb <= nb;
  float2 acc = make_float2(0.f, 0.f);
  for (int q0 = 0; q0 < tb; q0 += kSteps) {
    const int nq = min(kSteps, tb - q0);
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += kThreads) {
      kq[q] = bins[(int64_t)i * max_t + q0 + q];
      cq[q] = w[(int64_t)i * max_t + q0 + q];
    }
    __syncthreads();
    if (live) {
      for (int q = 0; q < nq; ++q) {
        const float2 v = y[(int64_t)kq[q] * nb + m0 + q0 + q];
        const float2 c = cq[q];
        acc.x += v.x * c.x - v.y * c.y;
        acc.y += v.x * c.y + v.y * c.x;
      }
    }
  }
  if (m0 < nb) p[(int64_t)i * nb + m0] = acc;
}

}  // namespace chimg


extern "C" {

int ddx_chimg_preintegrate(const void* d_volts, int32_t n_ant, int64_t n, int32_t block_len, int32_t n_s,
                           int32_t natural_weights, void* d_y, void* hip_stream) {
  if (n_ant < 2 || n_ant > chimg::kMaxAnt || n < 0 || block_len < 1 || n_s < 1 || n_s > chimg::kMaxBins ||
      (n_s & (n_s - 1)) || !d_volts || !d_y)
    return DDX_EINVAL;
  const int64_t nb = n / block_len;
  if (nb == 0) return DDX_OK;
  if (nb > INT32_MAX) return DDX_EUNSUPPORTED;
  // up to 64 antennas: the pair products on the matrix cores; more: on the vector units
  if (n_ant <= 64)
    hipLaunchKernelGGL((chimg::k_pre_mfma<false>), dim3((unsigned)nb), dim3(chimg::kThreads), 0,
                       (hipStream_t)hip_stream, (const float2*)d_volts, n_ant, n, block_len, n_s,
                       natural_weights ? 1 : 0, nullptr, nullptr, 0, (float2*)d_y);
  else
    hipLaunchKernelGGL(chimg::k_pre, dim3((unsigned)nb), dim3(chimg::kThreads), 0, (hipStream_t)hip_stream,
                       (const float2*)d_volts, n_ant, n, block_len, n_s, natural_weights ? 1 : 0, (float2*)d_y);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

int ddx_chimg_cells(int32_t n_ant, const double* positions, double spacing, int32_t n_cells, int32_t* cell_ptr,
                    int32_t* cell_pairs, int32_t* n_pairs) {
  if (n_ant < 2 || n_ant > 64 || !positions || !(spacing > 0.0) || !std::isfinite(spacing) || n_cells < 1 ||
      n_cells > chimg::kMaxBins || !cell_ptr || !cell_pairs || !n_pairs)
    return DDX_EINVAL;
  for (int p = 0; p < n_ant; ++p)
    if (!std::isfinite(positions[p]) || (p > 0 && !(positions[p] > positions[p - 1]))) return DDX_EINVAL;
  // counting pass, then the pairs of each cell in row-major order
  for (int c = 0; c <= n_cells; ++c) cell_ptr[c] = 0;
  for (int p = 0; p < n_ant; ++p)
    for (int q = p + 1; q < n_ant; ++q) {
      const double l = std::nearbyint((positions[q] - positions[p]) / spacing);
      if (l >= 1.0 && l <= (double)n_cells) ++cell_ptr[(int)l];
    }
  for (int c = 0; c < n_cells; ++c) cell_ptr[c + 1] += cell_ptr[c];
  std::vector<int32_t> fill(cell_ptr, cell_ptr + n_cells);
  for (int p = 0; p < n_ant; ++p)
    for (int q = p + 1; q < n_ant; ++q) {
      const double l = std::nearbyint((positions[q] - positions[p]) / spacing);
      if (l >= 1.0 && l <= (double)n_cells) {
        const int b = fill[(int)l - 1]++;
        cell_pairs[2 * b] = p;
        cell_pairs[2 * b + 1] = q;
      }
    }
  *n_pairs = cell_ptr[n_cells];
  return DDX_OK;
}

int ddx_chimg_preintegrate_cells(const void* d_volts, int32_t n_ant, int64_t n, int32_t block_len, int32_t n_s,
                                 int32_t n_cells, const int32_t* d_cell_ptr, const int32_t* d_cell_pairs, void* d_y,
                                 void* hip_stream) {
  if (n_ant < 2 || n_ant > 64 || n < 0 || block_len < 1 || n_s < 1 || n_s > chimg::kMaxBins || (n_s & (n_s - 1)) ||
      n_cells < 1 || n_cells > chimg::kMaxBins || !d_volts || !d_cell_ptr || !d_cell_pairs || !d_y)
    return DDX_EINVAL;
  const int64_t nb = n / block_len;
  if (nb == 0) return DDX_OK;
  if (nb > INT32_MAX) return DDX_EUNSUPPORTED;
  hipLaunchKernelGGL((chimg::k_pre_mfma<true>), dim3((unsigned)nb), dim3(chimg::kThreads), 0, (hipStream_t)hip_stream,
                     (const float2*)d_volts, n_ant, n, block_len, n_s, 1, d_cell_ptr, (const int2*)d_cell_pairs,
                     n_cells, (float2*)d_y);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

int ddx_chimg_trajectories(const void* d_y, int64_t n_blocks, int32_t n_ant, int32_t n_s, int32_t block_len,
                           const double* d_k_end, const int32_t* d_t_blocks, int32_t n_trials, void* d_p,
                           void* hip_stream) {
  if (!d_y || n_blocks < 0 || n_ant < 2 || n_s < 1 || block_len < 1 || !d_k_end || !d_t_blocks || n_trials < 1 ||
      !d_p)
    return DDX_EINVAL;
  if (n_blocks == 0) return DDX_OK;
  const int64_t gx = (n_blocks + chimg::kThreads - 1) / chimg::kThreads;
  if (gx > INT32_MAX || n_trials > 65535) return DDX_EUNSUPPORTED;
  hipLaunchKernelGGL(chimg::k_traj, dim3((unsigned)gx, (unsigned)n_trials), dim3(chimg::kThreads), 0,
                     (hipStream_t)hip_stream, (const float2*)d_y, n_blocks, n_ant, n_s, block_len, d_k_end, d_t_blocks,
                     (float2*)d_p);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

int ddx_chimg_gradient_sums(const void* d_y, int64_t n_blocks, int32_t n_ant, int32_t n_s, int32_t block_len,
                            const double* d_grad, int32_t n_grad, const int32_t* d_lengths, int32_t n_len, void* d_p,
                            void* hip_stream) {
  if (!d_y || n_blocks < 0 || n_ant < 2 || n_s < 1 || block_len < 1 || !d_grad || n_grad < 1 || !d_lengths ||
      n_len < 1 || !d_p)
    return DDX_EINVAL;
  if (n_blocks == 0) return DDX_OK;
  const int64_t gx = (n_blocks + chimg::kThreads - 1) / chimg::kThreads;
  if (gx > INT32_MAX || n_grad > 65535) return DDX_EUNSUPPORTED;
  hipLaunchKernelGGL(chimg::k_grad, dim3((unsigned)gx, (unsigned)n_grad), dim3(chimg::kThreads), 0,
                     (hipStream_t)hip_stream, (const float2*)d_y, n_blocks, n_ant, n_s, block_len, d_grad, d_lengths,
                     n_len, (float2*)d_p);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

int ddx_chimg_sampling_blocks(double k_end, int32_t t_blocks, double kappa_t0) {
  if (t_blocks < 1 || !std::isfinite(k_end) || !(kappa_t0 >= 0.0) || !std::isfinite(kappa_t0)) return DDX_EINVAL;
  const double kappa_t = std::max(1.0, std::fabs(k_end) * kappa_t0);
  return std::max(1, (int)std::floor((double)t_blocks / kappa_t));
}

int ddx_chimg_trajectories_ext(const void* d_y, int64_t n_blocks, int32_t n_ant, int32_t n_s, int32_t block_len,
                               const double* d_k_end, const int32_t* d_t_blocks, const int32_t* d_a_blocks,
                               int32_t half_width, int32_t n_trials, void* d_p, void* hip_stream) {
  if (!d_y || n_blocks < 0 || n_ant < 2 || n_s < 1 || block_len < 1 || !d_k_end || !d_t_blocks || n_trials < 1 ||
      !d_p || half_width < 0 || half_width > 16)
    return DDX_EINVAL;
  if (n_blocks == 0) return DDX_OK;
  const int64_t gx = (n_blocks + chimg::kThreads - 1) / chimg::kThreads;
  if (gx > INT32_MAX || n_trials > 65535) return DDX_EUNSUPPORTED;
  hipLaunchKernelGGL(chimg::k_traj_ext, dim3((unsigned)gx, (unsigned)n_trials), dim3(chimg::kThreads), 0,
                     (hipStream_t)hip_stream, (const float2*)d_y, n_blocks, n_ant, n_s, block_len, d_k_end,
                     d_t_blocks, d_a_blocks, half_width, (float2*)d_p);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

int ddx_chimg_cells_2d(int32_t n_ant, const double* positions, double spacing, int32_t max_cells, int32_t* n_cells,
                       int32_t* cell_ptr, int32_t* cell_pairs, int32_t* cell_uv, int32_t* n_pairs) {
  if (n_ant < 2 || n_ant > 64 || !positions || !(spacing > 0.0) || !std::isfinite(spacing) || max_cells < 1 ||
      !n_cells || !cell_ptr || !cell_pairs || !cell_uv || !n_pairs)
    return DDX_EINVAL;
  for (int e = 0; e < 2 * n_ant; ++e)
    if (!std::isfinite(positions[e])) return DDX_EINVAL;
  // each pair's cell in the half plane cu > 0 or (cu = 0, cv > 0), the pair turned
  // round (a = q, b = p) when its own offset falls in the other half
  struct Entry { int32_t cu, cv, a, b; };
  std::vector<Entry> e;
  for (int p = 0; p < n_ant; ++p)
    for (int q = p + 1; q < n_ant; ++q) {
      const double du = std::nearbyint((positions[2 * q] - positions[2 * p]) / spacing);
      const double dv = std::nearbyint((positions[2 * q + 1] - positions[2 * p + 1]) / spacing);
      if (std::fabs(du) > 1e6 || std::fabs(dv) > 1e6) return DDX_EINVAL;
      int cu = (int)du, cv = (int)dv, a = p, b = q;
      if (cu < 0 || (cu == 0 && cv < 0)) { cu = -cu; cv = -cv; a = q; b = p; }
      if (cu != 0 || cv != 0) e.push_back({cu, cv, a, b});
    }
  // cells in ascending (cu, cv), each cell's pairs in the row-major order of p < q
  std::stable_sort(e.begin(), e.end(), [](const Entry& x, const Entry& y) {
    return x.cu != y.cu ? x.cu < y.cu : x.cv < y.cv;
  });
  int nc = 0;
  for (size_t k = 0; k < e.size(); ++k) {
    if (k == 0 || e[k].cu != e[k - 1].cu || e[k].cv != e[k - 1].cv) {
      if (nc == max_cells) return DDX_ESIZE;
      cell_uv[2 * nc] = e[k].cu;
      cell_uv[2 * nc + 1] = e[k].cv;
      cell_ptr[nc] = (int32_t)k;
      ++nc;
    }
    cell_pairs[2 * k] = e[k].a;
    cell_pairs[2 * k + 1] = e[k].b;
  }
  cell_ptr[nc] = (int32_t)e.size();
  *n_cells = nc;
  *n_pairs = (int32_t)e.size();
  return DDX_OK;
}

int ddx_chimg_preintegrate_2d(const void* d_volts, int32_t n_ant, int64_t n, int32_t block_len, int32_t n_s,
                              int32_t n_cells, const int32_t* d_cell_ptr, const int32_t* d_cell_pairs,
                              const int32_t* d_cell_uv, void* d_y, void* hip_stream) {
  if (n_ant < 2 || n_ant > 64 || n < 0 || block_len < 1 || n_s < 1 || n_s > 256 || (n_s & (n_s - 1)) ||
      n_cells < 1 || n_cells > chimg::kMaxBins || !d_volts || !d_cell_ptr || !d_cell_pairs || !d_cell_uv || !d_y)
    return DDX_EINVAL;
  const int64_t nb = n / block_len;
  if (nb == 0) return DDX_OK;
  if (nb > INT32_MAX) return DDX_EUNSUPPORTED;
  hipLaunchKernelGGL((chimg::k_pre_mfma<true, true>), dim3((unsigned)nb), dim3(chimg::kThreads), 0,
                     (hipStream_t)hip_stream, (const float2*)d_volts, n_ant, n, block_len, n_s, 1, d_cell_ptr,
                     (const int2*)d_cell_pairs, n_cells, (float2*)d_y, (const int2*)d_cell_uv);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

int ddx_chimg_trajectories_2d(const void* d_y, int64_t n_blocks, int32_t n_s, int32_t block_len, int32_t n_cells,
                              const int32_t* d_cell_uv, const double* d_k_end, const int32_t* d_t_blocks,
                              int32_t n_trials, int32_t max_t, int32_t* d_table_bins, void* d_table_w, void* d_p,
                              void* hip_stream) {
  if (!d_y || n_blocks < 0 || n_s < 1 || n_s > 256 || block_len < 1 || n_cells < 1 || !d_cell_uv || !d_k_end ||
      !d_t_blocks || n_trials < 1 || max_t < 1 || !d_table_bins || !d_table_w || !d_p)
    return DDX_EINVAL;
  if (n_blocks == 0) return DDX_OK;
  const int64_t gx = (n_blocks + chimg::kThreads - 1) / chimg::kThreads;
  if (gx > INT32_MAX || n_trials > 65535) return DDX_EUNSUPPORTED;
  const hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(chimg::k_traj2d_table, dim3((unsigned)((max_t + chimg::kThreads - 1) / chimg::kThreads),
                                                 (unsigned)n_trials),
                     dim3(chimg::kThreads), 0, s, (const int2*)d_cell_uv, n_cells, n_s, block_len, d_k_end,
                     d_t_blocks, max_t, d_table_bins, (float2*)d_table_w);
  if (hipGetLastError() != hipSuccess) return DDX_EDEVICE;
  hipLaunchKernelGGL(chimg::k_traj_table, dim3((unsigned)gx, (unsigned)n_trials), dim3(chimg::kThreads), 0, s,
                     (const float2*)d_y, n_blocks, d_t_blocks, max_t, (const int32_t*)d_table_bins,
                     (const float2*)d_table_w, (float2*)d_p);
  return hipGetLastError() == hipSuccess ? DDX_OK : DDX_EDEVICE;
}

}  // extern "C"
