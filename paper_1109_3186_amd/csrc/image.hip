// Chirpolator post-integrator on gfx950: the detection image P(theta) and E(theta)
// = |P|^2 (Bannister & Cornwell 2011, Sec. 3.3, 3.4 and App. A.1) from the
// pre-integrator's DFT bins.
//
//   tau_pq = (u l + v m + w (n - 1)) / c,  (u, v, w) = r_p - r_q          (Eq. tau3D)
//   k0 = fdot tau N / f_s,  k0' = rint(k0)                         (Eqs. f0, f0dash)
//   P_w(l, m) = sum_{p<q} sum_{t=-F}^{F} g_pq,t X_w,pq[k0' + t]
//   g_pq,t = conj(Phi_pq(x)) D_N(x) / N,  x = k0' + t - k0           (Sec. 3.4)
//   Phi_pq(x) = exp(-pi i fdot tau (a_p + a_q)) exp(-pi i x (N - 1) / N)  (Eq. phipq1)
//
// with a_p = -r_p . (l, m, n - 1) / c the arrival delay of antenna p relative to the
// phase centre (for one baseline with p at the centre the constant phase is Eq.
// phipq1's -pi fdot tau^2), X_w[k] = S_w[k] exp(2 pi i w L k / N) the window that
// starts at sample w L re-referenced to its first sample (the pre-integrator's S is
// referenced to sample 0), and bins |k| > kmax contributing nothing.
//
// The weights depend on the direction and the pair only, so they are made once per
// plan (k_weights, FP64, stored FP32 with k0' as an integer), the same for every
// window.  k_image then is a gather-contraction on the FP32 VALU: one thread per
// direction, 32 windows per thread, the pairs' bins staged in LDS.  Only the bins
// that a tile of 256 directions reaches are staged: for neighbouring directions k0'
// of a pair moves over a few bins, so the span per (pair, tile) is computed with
// the weights and the staging shrinks from 2 kmax + 1 bins to that span.
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

namespace img {

constexpr int kPixTile = 256;            // directions per workgroup, one per thread
constexpr int kMaxHalfWidth = 8;         // F <= 8: at most 17 taps
constexpr int kLdsBytes = 64 * 1024;     // largest staging of one pair per workgroup
constexpr int kLdsStage = 28 * 1024;     // staging target: five workgroups per CU
constexpr double kLight = 299792458.0;   // m / s

struct WeightArgs {
  const double* ant;    // [M][3] positions (m)
  const double* lm;     // [n_pix][2] direction cosines
  const int2* pq;       // [nbl] pairs p < q, row-major
  float2* g;            // [nbl][taps][n_pix] weights
  int* j0;              // [nbl][n_pix] bin index of tap -F: k0' - F + kmax
  int2* span;           // [nbl][n_ptiles] (first bin, count) that the tile reads
  double fdot, f_s;
  int32_t n_pix, nbl, n_ptiles, N, kmax, F;
};

// grid: nbl * n_ptiles workgroups of 256 threads, thread = direction of the tile.
__global__ __launch_bounds__(256) void k_weights(WeightArgs a) {
  const int pt = blockIdx.x % a.n_ptiles, b = blockIdx.x / a.n_ptiles;
  const int pix = pt * kPixTile + threadIdx.x;
  const int K = 2 * a.kmax + 1, taps = 2 * a.F + 1;
  __shared__ int lo_s, hi_s;
  if (threadIdx.x == 0) {
    lo_s = K - 1;
    hi_s = 0;
  }
  __syncthreads();
  if (pix < a.n_pix) {
    const int p = a.pq[b].x, q = a.pq[b].y;
    const double l = a.lm[2 * pix], m = a.lm[2 * pix + 1];
    double tau, asum, k0;
    {
#pragma clang fp contract(off)
      // the operation order of the plain definition, so that rint(k0) is decided alike
      const double nm1 = -(l * l + m * m) / (1.0 + sqrt(1.0 - l * l - m * m));
      const double* rp = a.ant + 3 * p;
      const double* rq = a.ant + 3 * q;
      const double u = rp[0] - rq[0], v = rp[1] - rq[1], w = rp[2] - rq[2];
      tau = (u * l + v * m + w * nm1) / kLight;
      const double ap = -(rp[0] * l + rp[1] * m + rp[2] * nm1) / kLight;
      const double aq = -(rq[0] * l + rq[1] * m + rq[2] * nm1) / kLight;
      asum = ap + aq;
      k0 = a.fdot * tau * (double)a.N / a.f_s;
    }
    const double lim = (double)(a.kmax + a.F + 1);
    const double k0r = fmin(fmax(rint(k0), -lim), lim);
    const int jb = (int)k0r - a.F + a.kmax;
    a.j0[(int64_t)b * a.n_pix + pix] = jb;
    // phase of conj(Phi(x)) in half-cycles: fdot tau (a_p + a_q) + x (N - 1) / N
    const double c0 = a.fdot * tau * asum;
    for (int t = 0; t < taps; ++t) {
      const int k = (int)k0r - a.F + t;
      float2 gw = make_float2(0.f, 0.f);
      if (k >= -a.kmax && k <= a.kmax) {
        const double x = (double)k - k0;
        double h = c0 + x * ((double)(a.N - 1) / (double)a.N);
        h -= 2.0 * rint(0.5 * h);
        double sn, cs;
        sincospi(h, &sn, &cs);
        const double amp = x == 0.0 ? 1.0 : sinpi(x) / ((double)a.N * sinpi(x / (double)a.N));
        gw = make_float2((float)(amp * cs), (float)(amp * sn));
      }
      a.g[((int64_t)b * taps + t) * a.n_pix + pix] = gw;
    }
    atomicMin(&lo_s, min(max(jb, 0), K - 1));
    atomicMax(&hi_s, min(max(jb + taps - 1, 0), K - 1));
  }
  __syncthreads();
  if (threadIdx.x == 0) a.span[(int64_t)b * a.n_ptiles + pt] = make_int2(lo_s, max(hi_s - lo_s + 1, 1));
}

struct ImageArgs {
  const float2* s;      // [rows][nbl][K] pre-integrator bins, row r = window first + r
  const float2* g;      // [nbl][taps][n_pix]
  const int* j0;        // [nbl][n_pix]
  const int2* span;     // [nbl][n_ptiles]
  const float2* root;   // [R] exp(2 pi i r / R) as (cos, sin)
  const uint32_t* kmod; // [K] (k mod R) of bin index j, k = j - kmax
  float2* p;            // [n_img][n_pix] or null
  float* e;             // [n_img][n_pix] or null
  int64_t first, n_img, w_step;
  int32_t n_pix, nbl, n_ptiles, K, taps, R, smax, pb;
};

// grid: n_ptiles * ceil(n_img / WT) workgroups of 256 threads (mapped by tile_of);
// Workgroup -> (direction tile, window tile).  Workgroups are dealt to the eight XCDs
// in turn (id mod 8); the remap gives each XCD a contiguous run of the tile order,
// window tile fastest, so the window tiles of one direction tile run on one XCD at
// about the same time and read that tile's weights (the dominant traffic) through
// the same L2.  The last total mod 8 workgroups keep their own index.
__device__ __forceinline__ void tile_of(int id, int n_ptiles, int n_wtiles, int& pt, int& wt) {
  const int whole = (n_ptiles * n_wtiles) & ~7;
  const int v = id < whole ? (id & 7) * (whole >> 3) + (id >> 3) : id;
  pt = v / n_wtiles;
  wt = v - pt * n_wtiles;
}

// one tap: acc[i] += w X[window i] for the WT windows of a staged bin
template <int WT>
__device__ __forceinline__ void mac_tap(float2 (&acc)[WT], float2 w, const float2* bin) {
  const float4* col = reinterpret_cast<const float4*>(bin);
#pragma unroll
  for (int i = 0; i < WT; i += 2) {
    const float4 x = col[i / 2];  // windows i and i + 1
    acc[i].x = fmaf(w.x, x.x, fmaf(-w.y, x.y, acc[i].x));
    acc[i].y = fmaf(w.x, x.y, fmaf(w.y, x.x, acc[i].y));
    acc[i + 1].x = fmaf(w.x, x.z, fmaf(-w.y, x.w, acc[i + 1].x));
    acc[i + 1].y = fmaf(w.x, x.w, fmaf(w.y, x.z, acc[i + 1].y));
  }
}

// dynamic LDS: pb pairs x smax bins x (WT + 2) windows of float2: the windows of a bin
// are adjacent, so a thread reads two windows per 16-byte load at fixed offsets, and
// the 2-entry pad puts neighbouring bins 4 banks apart (no conflicts between the
// bins that the lanes of a wave read).  TAPS > 0: the tap count is fixed and the
// weights of the next pair are loaded while the current one is summed (the weights
// stream from HBM once per window tile); TAPS = 0: any count, loaded at use.
template <int WT, int TAPS>
__global__ __launch_bounds__(256) void k_image(ImageArgs a) {
  extern __shared__ float2 xs[];
  __shared__ uint32_t wmod[WT];
  const int tid = threadIdx.x;
  int pt, wt;
  tile_of(blockIdx.x, a.n_ptiles, (int)((a.n_img + WT - 1) / WT), pt, wt);
  const int64_t img0 = (int64_t)wt * WT;
  const int pix = pt * kPixTile + tid;
  const bool live = pix < a.n_pix;
  if (tid < WT) wmod[tid] = (uint32_t)((a.first + (img0 + tid) * a.w_step) % a.R);
  float2 acc[WT];
#pragma unroll
  for (int i = 0; i < WT; ++i) acc[i] = make_float2(0.f, 0.f);
  const int64_t row = (int64_t)a.nbl * a.K;  // elements per window row of s
  constexpr int NT = TAPS > 0 ? TAPS : 1;
  float2 wn[NT];  // weights and first bin of the next pair (TAPS > 0)
  int jn = 0;
  auto fetch = [&](int b) {
    if (TAPS > 0 && live && b < a.nbl) {
      jn = a.j0[(int64_t)b * a.n_pix + pix];
      const float2* gp = a.g + (int64_t)b * TAPS * a.n_pix + pix;
#pragma unroll
      for (int t = 0; t < NT; ++t) wn[t] = gp[(int64_t)t * a.n_pix];
    }
  };
  fetch(0);

  for (int b0 = 0; b0 < a.nbl; b0 += a.pb) {
    const int nb = min(a.pb, a.nbl - b0);
    __syncthreads();
    // stage X_w[k] = S_w[k] exp(2 pi i (w k mod R) / R) over each pair's span
    for (int sl = 0; sl < nb; ++sl) {
      const int b = b0 + sl;
      const int2 sp = a.span[(int64_t)b * a.n_ptiles + pt];
      float2* dst = xs + (size_t)sl * a.smax * (WT + 2);
      for (int e = tid; e < WT * sp.y; e += kPixTile) {
        const int wl = e / sp.y, jj = e - wl * sp.y;
        const int j = sp.x + jj;
        float2 x = make_float2(0.f, 0.f);
        if (img0 + wl < a.n_img) {
          const float2 v = a.s[(img0 + wl) * a.w_step * row + (int64_t)b * a.K + j];
          const float2 r = a.root[(wmod[wl] * a.kmod[j]) % (uint32_t)a.R];
          x = make_float2(v.x * r.x - v.y * r.y, v.x * r.y + v.y * r.x);
        }
        dst[jj * (WT + 2) + wl] = x;
      }
    }
    __syncthreads();
    if (live) {
      for (int sl = 0; sl < nb; ++sl) {
        const int b = b0 + sl;
        const int lo = a.span[(int64_t)b * a.n_ptiles + pt].x;
        const float2* src = xs + (size_t)sl * a.smax * (WT + 2);
        if constexpr (TAPS > 0) {
          float2 wc[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) wc[t] = wn[t];
          const int jb = jn;
          fetch(b + 1);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const int jj = min(max(jb + t, 0), a.K - 1) - lo;  // inside the span by construction
            mac_tap<WT>(acc, wc[t], src + jj * (WT + 2));
          }
        } else {
          const int jb = a.j0[(int64_t)b * a.n_pix + pix];
          const float2* gp = a.g + (int64_t)b * a.taps * a.n_pix + pix;
          for (int t = 0; t < a.taps; ++t) {
            const int jj = min(max(jb + t, 0), a.K - 1) - lo;
            mac_tap<WT>(acc, gp[(int64_t)t * a.n_pix], src + jj * (WT + 2));
          }
        }
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int i = 0; i < WT; ++i) {
    const int64_t im = img0 + i;
    if (im >= a.n_img) break;
    if (a.p) a.p[im * a.n_pix + pix] = acc[i];
    if (a.e) a.e[im * a.n_pix + pix] = acc[i].x * acc[i].x + acc[i].y * acc[i].y;
  }
}

}  // namespace img

namespace {

int ifail(std::string* err, int status, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (err) *err = buf;
  return status;
}

}  // namespace

struct ddx_image {
  int M = 0, n_pix = 0, nbl = 0, n_ptiles = 0, N = 0, L = 0, R = 0, kmax = 0, K = 0, F = 0, taps = 0;
  int smax = 1;
  float2* g = nullptr;
  int* j0 = nullptr;
  int2* span = nullptr;
  float2* root = nullptr;
  uint32_t* kmod = nullptr;
  std::vector<void*> allocs;
  std::string err;
};

namespace {

template <class T>
int dev_alloc(ddx_image* h, T** dst, size_t count) {
  if (hipMalloc((void**)dst, std::max<size_t>(count * sizeof(T), 256)) != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    return DDX_ENOMEM;
  }
  h->allocs.push_back(*dst);
  return DDX_OK;
}

template <class T>
int dev_upload(ddx_image* h, T** dst, const T* src, size_t count) {
  int rc = dev_alloc(h, dst, count);
  if (rc) return rc;
  if (hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return DDX_EDEVICE;
  }
  return DDX_OK;
}

void image_release(ddx_image* h) {
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
}

// windows per thread (a staged bin row of WT + 2 windows must fit the LDS budget, else 4)
constexpr int kImgWt = 32;

int window_tile(const ddx_image* h) {
  return (int64_t)(kImgWt + 2) * h->smax * (int64_t)sizeof(float2) <= img::kLdsBytes ? kImgWt : 4;
}

}  // namespace

extern "C" {

int ddx_image_create(int32_t n_ant, const double* ant_xyz, int32_t n_pix, const double* pix_lm, double fdot_hz_s,
                     double samp_rate_hz, int32_t fft_n, int32_t block_len, int32_t kmax, int32_t half_width,
                     ddx_image** out) {
  if (!out) return DDX_EINVAL;
  *out = nullptr;
  if (n_ant < 2 || n_ant > 1024 || !ant_xyz || n_pix < 1 || !pix_lm || block_len < 1 || fft_n < block_len ||
      fft_n % block_len != 0 || fft_n / block_len > 65535 || kmax < 0 || kmax > 640 || 2 * kmax + 1 > fft_n ||
      half_width < 0 || half_width > img::kMaxHalfWidth || !std::isfinite(fdot_hz_s) ||
      !(samp_rate_hz > 0.0) || !std::isfinite(samp_rate_hz))
    return DDX_EINVAL;
  for (int i = 0; i < 3 * n_ant; ++i)
    if (!std::isfinite(ant_xyz[i])) return DDX_EINVAL;
  for (int i = 0; i < n_pix; ++i) {
    const double l = pix_lm[2 * i], m = pix_lm[2 * i + 1];
    if (!std::isfinite(l) || !std::isfinite(m) || !(l * l + m * m < 1.0)) return DDX_EINVAL;
  }
  if ((int64_t)n_ant * (n_ant - 1) / 2 * ((n_pix + img::kPixTile - 1) / img::kPixTile) > INT32_MAX)
    return DDX_EUNSUPPORTED;
  ddx_image* h = new (std::nothrow) ddx_image;
  if (!h) return DDX_ENOMEM;
  h->M = n_ant;
  h->n_pix = n_pix;
  h->nbl = n_ant * (n_ant - 1) / 2;
  h->n_ptiles = (n_pix + img::kPixTile - 1) / img::kPixTile;
  h->N = fft_n;
  h->L = block_len;
  h->R = fft_n / block_len;
  h->kmax = kmax;
  h->K = 2 * kmax + 1;
  h->F = half_width;
  h->taps = 2 * half_width + 1;
  std::vector<int2> pq;
  for (int p = 0; p < n_ant; ++p)
    for (int q = p + 1; q < n_ant; ++q) pq.push_back(make_int2(p, q));
  // exp(2 pi i r / R) in FP64, stored FP32; (k mod R) of each bin index
  std::vector<float2> root(h->R);
  for (int r = 0; r < h->R; ++r) {
    const double ang = 2.0 * M_PI * (double)r / (double)h->R;
    root[r] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  std::vector<uint32_t> kmod(h->K);
  for (int j = 0; j < h->K; ++j) kmod[j] = (uint32_t)((((j - kmax) % h->R) + h->R) % h->R);
  double* d_ant = nullptr;
  double* d_lm = nullptr;
  int2* d_pq = nullptr;
  const size_t n_w = (size_t)h->nbl * h->taps * n_pix;
  int rc = dev_upload(h, &d_ant, ant_xyz, (size_t)3 * n_ant);
  if (!rc) rc = dev_upload(h, &d_lm, pix_lm, (size_t)2 * n_pix);
  if (!rc) rc = dev_upload(h, &d_pq, pq.data(), pq.size());
  if (!rc) rc = dev_upload(h, &h->root, root.data(), root.size());
  if (!rc) rc = dev_upload(h, &h->kmod, kmod.data(), kmod.size());
  if (!rc) rc = dev_alloc(h, &h->g, n_w);
  if (!rc) rc = dev_alloc(h, &h->j0, (size_t)h->nbl * n_pix);
  if (!rc) rc = dev_alloc(h, &h->span, (size_t)h->nbl * h->n_ptiles);
  std::vector<int2> span((size_t)h->nbl * h->n_ptiles);
  if (!rc) {
    img::WeightArgs a{d_ant, d_lm, d_pq, h->g, h->j0, h->span, fdot_hz_s, samp_rate_hz,
                      n_pix, h->nbl, h->n_ptiles, fft_n, kmax, half_width};
    hipLaunchKernelGGL(img::k_weights, dim3((unsigned)((int64_t)h->nbl * h->n_ptiles)), dim3(img::kPixTile), 0, 0, a);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(span.data(), h->span, span.size() * sizeof(int2), hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      rc = DDX_EDEVICE;
    }
  }
  if (rc) {
    image_release(h);
    delete h;
    return rc;
  }
  for (const int2& s : span) h->smax = std::max(h->smax, s.y);
  // the geometry inputs are needed only by the weights
  for (void* p : {(void*)d_ant, (void*)d_lm, (void*)d_pq}) {
    (void)hipFree(p);
    h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), p));
  }
  *out = h;
  return DDX_OK;
}

int ddx_image_output_count(const ddx_image* h, int64_t n_rows, int32_t w_step, int64_t* n_images) {
  if (!h || !n_images || n_rows < 0 || w_step < 1) return DDX_EINVAL;
  *n_images = (n_rows + w_step - 1) / w_step;
  return DDX_OK;
}

int ddx_image_run(ddx_image* h, const void* d_bins, int64_t n_rows, int64_t first_window, int32_t w_step,
                  void* d_p, void* d_e, void* hip_stream) {
  if (!h) return DDX_EINVAL;
  if (n_rows < 0 || first_window < 0 || w_step < 1)
    return ifail(&h->err, DDX_EINVAL, "n_rows %lld, first_window %lld, w_step %d", (long long)n_rows,
                 (long long)first_window, (int)w_step);
  if (n_rows == 0) return DDX_OK;
  if (!d_bins || (!d_p && !d_e)) return ifail(&h->err, DDX_EINVAL, "NULL device buffer");
  const int64_t n_img = (n_rows + w_step - 1) / w_step;
  const int wt = window_tile(h);
  const int64_t n_wtiles = (n_img + wt - 1) / wt;
  if (n_wtiles * h->n_ptiles > INT32_MAX) return ifail(&h->err, DDX_EUNSUPPORTED, "too many images in one call");
  const int per_pair = (wt + 2) * h->smax * (int)sizeof(float2);
  const int pb = std::max(1, std::min(h->nbl, std::min(64, img::kLdsStage / per_pair)));
  img::ImageArgs a{(const float2*)d_bins, h->g, h->j0, h->span, h->root, h->kmod, (float2*)d_p, (float*)d_e,
                   first_window, n_img, w_step, h->n_pix, h->nbl, h->n_ptiles, h->K, h->taps, h->R, h->smax, pb};
  const size_t lds = (size_t)pb * per_pair;
  const dim3 grid((unsigned)(n_wtiles * h->n_ptiles));
  const hipStream_t st = (hipStream_t)hip_stream;
  const dim3 blk(img::kPixTile);
  if (wt != kImgWt)
    hipLaunchKernelGGL((img::k_image<4, 0>), grid, blk, lds, st, a);
  else if (h->taps == 1)
    hipLaunchKernelGGL((img::k_image<kImgWt, 1>), grid, blk, lds, st, a);
  else if (h->taps == 3)
    hipLaunchKernelGGL((img::k_image<kImgWt, 3>), grid, blk, lds, st, a);
  else if (h->taps == 5)
    hipLaunchKernelGGL((img::k_image<kImgWt, 5>), grid, blk, lds, st, a);
  else if (h->taps == 7)
    hipLaunchKernelGGL((img::k_image<kImgWt, 7>), grid, blk, lds, st, a);
  else
    hipLaunchKernelGGL((img::k_image<kImgWt, 0>), grid, blk, lds, st, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ifail(&h->err, DDX_EDEVICE, "k_image: %s", hipGetErrorString(e));
  return DDX_OK;
}

const char* ddx_image_last_error(const ddx_image* h) { return h ? h->err.c_str() : "NULL image plan"; }

int ddx_image_destroy(ddx_image* h) {
  if (!h) return DDX_OK;
  (void)hipDeviceSynchronize();
  image_release(h);
  delete h;
  return DDX_OK;
}

}  // extern "C"
