// Host side of the ddx C ABI: plan state, blocking, tables, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ddx.h"
#include "kernels.hpp"
#include "tiles.hpp"

namespace {

constexpr double kDefaultKdm = 4.148808e15;
constexpr int kMaxLogN = 15;
constexpr int kMinLogN = 8;
constexpr int kMaxStackedAnt = 64;  // stacked-row Gram kernel up to 2 M = 128 rows
constexpr int kMaxCorrAnt = 1024;   // antenna-block kernel beyond
// Scale rule targets: E4M3 puts sigma near 32, so even after the power-of-two
// rounding (up to x sqrt 2) about 10 sigma, and the int8 extreme 127 at sigma 16,
// stay below its largest finite value 448; binary16 puts sigma near 4 (far from
// both its subnormal range and its maximum).  Away from those extremes a power-of-
// two scale does not change the relative rounding error of either format.
constexpr float kScaleTargetE4M3 = 32.f;
constexpr float kScaleTargetF16 = 4.f;

struct Chan {
  double fc = 0;
  std::vector<double> dm;       // trial DMs
  std::vector<uint8_t> active;  // per DM
  int fft_len = 0, logn = 0, valid = 0, lead = 0;
  float scale = 1.f;
  // stream state
  int64_t blocks_done = 0;
  int64_t dumps_done = 0;
  int64_t hist_start = 0;  // absolute index of history element 0
};

}  // namespace

struct ddx_plan {
  // descriptor
  int M = 0, C = 0, L = 0, sideband = 1, in_dtype = 0, corr_dtype = 0, out_mode = 0;
  double fs = 0, kdm = kDefaultKdm;
  int64_t max_block = 0;
  size_t max_bytes = 0;
  std::vector<int> fft_req;
  std::vector<float> scale_req;
  bool have_scale = false;
  std::vector<Chan> ch;
  int nbl = 0;
  // derived
  bool ready = false, started = false, flushed = false;
  std::vector<int32_t> lay_fft, lay_valid, lay_lead, lay_ndm;
  std::vector<int64_t> dm_off, lay_shift;
  std::vector<double> lay_dm, lay_delay, lay_fc;
  std::vector<float> lay_scale;
  int64_t rec_elems = 0;
  // stream
  int64_t recv = 0;
  int64_t dumps_fetched = 0;
  // device memory
  size_t dev_bytes = 0;
  std::vector<void*> allocs;
  void* hist[2] = {nullptr, nullptr};
  int hist_cur = 0;
  int64_t hist_cap = 0;
  float2* spec = nullptr;
  size_t spec_elems = 0;
  float2* chirp = nullptr;
  void* ybuf = nullptr;
  int64_t y_stride = 0;
  int dm_group = 8;
  float2* ring = nullptr;
  int64_t ring_dumps = 0;
  double* gtab = nullptr;        // [sum N_c] FP64 g_c[k]
  std::vector<int64_t> gtab_off;
  double* kdm_dev = nullptr;     // [sum D_c] K DM for the active list (compacted per channel)
  int32_t* pos_dev = nullptr;    // [sum D_c] record positions, active first then inactive
  std::vector<int> n_active;
  float* scale_dev = nullptr;    // [C]
  // DM-time tiles: scratch grown on demand
  float* tile_power = nullptr;
  size_t tile_power_cap = 0;
  double* tile_prefix = nullptr;
  size_t tile_prefix_cap = 0;
  double* tile_totals = nullptr;
  size_t tile_totals_cap = 0;
  int64_t* tile_shift = nullptr;
  int tile_shift_fine = 0;
  hipStream_t last_stream = nullptr;
  bool scale_pending = false;    // scale_dev holds rule scales not yet copied to lay_scale
  std::string err;
  // profiling
  bool profiling = false;
  struct Rec { hipEvent_t a, b; int kind; double flops, bytes; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;
  size_t events_used = 0;
};

namespace {

int fail(ddx_plan* p, int code, const char* fmt, ...) {
  if (p) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    p->err = buf;
  }
  return code;
}

#define HIPCHECK(plan, call)                                                                     \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail(plan, DDX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2i(int64_t n) { int l = 0; while ((int64_t(1) << l) < n) ++l; return l; }

int dev_alloc(ddx_plan* p, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (p->max_bytes && p->dev_bytes + bytes > p->max_bytes)
    return fail(p, DDX_ENOMEM, "plan needs %zu device bytes, cap is %zu", p->dev_bytes + bytes, p->max_bytes);
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(p, DDX_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  p->allocs.push_back(*ptr);
  p->dev_bytes += bytes;
  return DDX_OK;
}

void free_device(ddx_plan* p) {
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
  p->dev_bytes = 0;
  p->hist[0] = p->hist[1] = nullptr;
  p->spec = p->chirp = p->ring = nullptr;
  p->ybuf = nullptr;
  p->gtab = p->kdm_dev = nullptr;
  p->pos_dev = nullptr;
  p->scale_dev = nullptr;
  p->tile_power = nullptr;
  p->tile_power_cap = 0;
  p->tile_prefix = nullptr;
  p->tile_prefix_cap = 0;
  p->tile_totals = nullptr;
  p->tile_totals_cap = 0;
  p->tile_shift = nullptr;
  p->tile_shift_fine = 0;
}

size_t in_bytes(int in_dtype) { return in_dtype == DDX_IN_CI8 ? 2 : 8; }
size_t y_bytes(int corr_dtype) { return corr_dtype == DDX_CORR_F32 ? 8 : corr_dtype == DDX_CORR_F16 ? 4 : 2; }

// Overlap-save blocking of one channel (reading stated in ddx.h).
int blocking(ddx_plan* p, Chan& c, int fft_req) {
  double dmax = 0;
  for (double d : c.dm) dmax = std::max(dmax, d);
  const double hi = c.fc + 0.5 * p->fs, lo = c.fc - 0.5 * p->fs;
  const double inv_c = 1.0 / (c.fc * c.fc);
  const double early = p->kdm * dmax * (inv_c - 1.0 / (hi * hi)) * p->fs;
  const double late = p->kdm * dmax * (1.0 / (lo * lo) - inv_c) * p->fs;
  const double amax = std::ceil(std::max(early, late));
  if (!(amax < 1e9)) return fail(p, DDX_EUNSUPPORTED, "dispersion smear %.3g samples too long", amax);
  const int64_t a = (int64_t)amax;
  auto kept = [&](int64_t n) { int64_t r = n - 2 * a; return r < 0 ? int64_t(-1) : p->L * (r / p->L); };
  int64_t n = fft_req;
  if (n == 0) {
    n = 256;
    while (kept(n) < n / 2 && n <= (int64_t(1) << 30)) n *= 2;
  }
  const int64_t v = kept(n);
  if (v < p->L) return fail(p, DDX_EINVAL, "FFT length %lld too short for overlap %lld and dump %d", (long long)n, (long long)(2 * a), p->L);
  if (n > (int64_t(1) << kMaxLogN))
    return fail(p, DDX_EUNSUPPORTED, "FFT length %lld > %d not supported", (long long)n, 1 << kMaxLogN);
  c.fft_len = (int)n;
  c.logn = std::max(ilog2i(n), kMinLogN);
  if ((1 << c.logn) != n) return fail(p, DDX_EUNSUPPORTED, "FFT length %lld < 256", (long long)n);
  c.valid = (int)v;
  c.lead = (int)((n - v) / 2);
  return DDX_OK;
}

// ---- kernel dispatch over template parameters ------------------------------------------

template <int LOGN>
size_t fft_lds_bytes() { return sizeof(float) * ddx::Geo<LOGN>::LDS_FLOATS; }

template <int LOGN>
hipError_t launch_forward_n(int in_dtype, const ddx::FwdArgs& a, hipStream_t s) {
  using G = ddx::Geo<LOGN>;
  dim3 grid(a.nblk * a.n_ant), block(G::T);
  if (in_dtype == DDX_IN_CI8)
    hipLaunchKernelGGL((ddx::k_forward<LOGN, 0>), grid, block, fft_lds_bytes<LOGN>(), s, a);
  else
    hipLaunchKernelGGL((ddx::k_forward<LOGN, 1>), grid, block, fft_lds_bytes<LOGN>(), s, a);
  return hipGetLastError();
}

template <int LOGN>
hipError_t launch_dedisp_n(int corr_dtype, const ddx::DedispArgs& a, hipStream_t s) {
  using G = ddx::Geo<LOGN>;
  dim3 grid(a.n_ant * a.nblk * a.nd), block(G::T);
  if (corr_dtype == DDX_CORR_F32)
    hipLaunchKernelGGL((ddx::k_dedisperse<LOGN, 0>), grid, block, fft_lds_bytes<LOGN>(), s, a);
  else if (corr_dtype == DDX_CORR_F16)
    hipLaunchKernelGGL((ddx::k_dedisperse<LOGN, 1>), grid, block, fft_lds_bytes<LOGN>(), s, a);
  else
    hipLaunchKernelGGL((ddx::k_dedisperse<LOGN, 2>), grid, block, fft_lds_bytes<LOGN>(), s, a);
  return hipGetLastError();
}

hipError_t launch_forward(int logn, int in_dtype, const ddx::FwdArgs& a, hipStream_t s) {
  switch (logn) {
    case 8: return launch_forward_n<8>(in_dtype, a, s);
    case 9: return launch_forward_n<9>(in_dtype, a, s);
    case 10: return launch_forward_n<10>(in_dtype, a, s);
    case 11: return launch_forward_n<11>(in_dtype, a, s);
    case 12: return launch_forward_n<12>(in_dtype, a, s);
    case 13: return launch_forward_n<13>(in_dtype, a, s);
    case 14: return launch_forward_n<14>(in_dtype, a, s);
    case 15: return launch_forward_n<15>(in_dtype, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dedisp(int logn, int corr_dtype, const ddx::DedispArgs& a, hipStream_t s) {
  switch (logn) {
    case 8: return launch_dedisp_n<8>(corr_dtype, a, s);
    case 9: return launch_dedisp_n<9>(corr_dtype, a, s);
    case 10: return launch_dedisp_n<10>(corr_dtype, a, s);
    case 11: return launch_dedisp_n<11>(corr_dtype, a, s);
    case 12: return launch_dedisp_n<12>(corr_dtype, a, s);
    case 13: return launch_dedisp_n<13>(corr_dtype, a, s);
    case 14: return launch_dedisp_n<14>(corr_dtype, a, s);
    case 15: return launch_dedisp_n<15>(corr_dtype, a, s);
  }
  return hipErrorInvalidValue;
}

template <int NT>
hipError_t launch_corr_nt(int corr_dtype, const ddx::CorrArgs& a, hipStream_t s) {
  const dim3 g(a.n_dumps * a.nd), b(256);
  if (corr_dtype == DDX_CORR_F32) hipLaunchKernelGGL((ddx::k_correlate<NT, 0>), g, b, 0, s, a);
  else if (corr_dtype == DDX_CORR_F16) hipLaunchKernelGGL((ddx::k_correlate<NT, 1>), g, b, 0, s, a);
  else hipLaunchKernelGGL((ddx::k_correlate<NT, 2>), g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_corr_blocks(int corr_dtype, const ddx::CorrArgs& a, hipStream_t s) {
  const int nb = (a.n_ant + ddx::kBlkAnt - 1) / ddx::kBlkAnt;
  const dim3 g(a.n_dumps * a.nd * (nb * (nb + 1) / 2)), b(256);
  if (corr_dtype == DDX_CORR_F32) hipLaunchKernelGGL((ddx::k_correlate_blocks<0>), g, b, 0, s, a);
  else if (corr_dtype == DDX_CORR_F16) hipLaunchKernelGGL((ddx::k_correlate_blocks<1>), g, b, 0, s, a);
  else hipLaunchKernelGGL((ddx::k_correlate_blocks<2>), g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_corr(int corr_dtype, const ddx::CorrArgs& a, hipStream_t s) {
  if (a.n_ant > kMaxStackedAnt) return launch_corr_blocks(corr_dtype, a, s);
  const int nt = (2 * a.n_ant + 15) / 16;
  switch (nt) {
    case 1: return launch_corr_nt<1>(corr_dtype, a, s);
    case 2: return launch_corr_nt<2>(corr_dtype, a, s);
    case 3: return launch_corr_nt<3>(corr_dtype, a, s);
    case 4: return launch_corr_nt<4>(corr_dtype, a, s);
    case 5: return launch_corr_nt<5>(corr_dtype, a, s);
    case 6: return launch_corr_nt<6>(corr_dtype, a, s);
    case 7: return launch_corr_nt<7>(corr_dtype, a, s);
    case 8: return launch_corr_nt<8>(corr_dtype, a, s);
  }
  return hipErrorInvalidValue;
}

// ---- profiling ------------------------------------------------------------------------------

hipEvent_t take_event(ddx_plan* p) {
  if (p->events_used == p->event_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->event_pool.push_back(e);
  }
  return p->event_pool[p->events_used++];
}

// Launch f() on stream s, bracketed by events when profiling.
template <class F>
hipError_t timed(ddx_plan* p, hipStream_t s, int kind, double flops, double bytes, F f) {
  if (!p->profiling) return f();
  hipEvent_t a = take_event(p), b = take_event(p);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = f();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  p->recs.push_back({a, b, kind, flops, bytes});
  return e;
}

double fft_flops(int n) { return 5.0 * n * std::log2((double)n); }

// ---- layout tables ------------------------------------------------------------------------

void build_layout(ddx_plan* p) {
  p->lay_fft.assign(p->C, 0);
  p->lay_valid.assign(p->C, 0);
  p->lay_lead.assign(p->C, 0);
  p->lay_ndm.assign(p->C, 0);
  p->lay_scale.assign(p->C, 1.f);
  p->dm_off.assign(p->C + 1, 0);
  p->lay_fc.assign(p->C, 0);
  double ftop = 0;
  for (auto& c : p->ch) ftop = std::max(ftop, c.fc);
  p->lay_dm.clear();
  p->lay_delay.clear();
  p->lay_shift.clear();
  for (int i = 0; i < p->C; ++i) {
    Chan& c = p->ch[i];
    p->lay_fft[i] = c.fft_len;
    p->lay_valid[i] = c.valid;
    p->lay_lead[i] = c.lead;
    p->lay_ndm[i] = (int32_t)c.dm.size();
    p->lay_scale[i] = c.scale;
    p->lay_fc[i] = c.fc;
    p->dm_off[i + 1] = p->dm_off[i] + (int64_t)c.dm.size();
    const double inv = 1.0 / (c.fc * c.fc), invt = 1.0 / (ftop * ftop);
    for (double d : c.dm) {
      p->lay_dm.push_back(d);
      p->lay_delay.push_back(p->kdm * d * inv);
      p->lay_shift.push_back((int64_t)std::nearbyint(p->kdm * d * (inv - invt) * p->fs));
    }
  }
  p->rec_elems = p->dm_off[p->C] * p->nbl;
}

// Upload the active-DM lists (K DM compacted, active first) of every channel.
int upload_active(ddx_plan* p, hipStream_t s) {
  std::vector<double> kdm(p->dm_off[p->C]);
  std::vector<int32_t> pos(p->dm_off[p->C]);
  p->n_active.assign(p->C, 0);
  for (int i = 0; i < p->C; ++i) {
    Chan& c = p->ch[i];
    int64_t o = p->dm_off[i];
    int na = 0;
    for (size_t d = 0; d < c.dm.size(); ++d)
      if (c.active[d]) { kdm[o + na] = p->kdm * c.dm[d]; pos[o + na] = (int32_t)(o + d); ++na; }
    int k = na;
    for (size_t d = 0; d < c.dm.size(); ++d)
      if (!c.active[d]) { kdm[o + k] = p->kdm * c.dm[d]; pos[o + k] = (int32_t)(o + d); ++k; }
    p->n_active[i] = na;
  }
  HIPCHECK(p, hipMemcpyAsync(p->kdm_dev, kdm.data(), kdm.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHECK(p, hipMemcpyAsync(p->pos_dev, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHECK(p, hipStreamSynchronize(s));
  return DDX_OK;
}

int setup_device(ddx_plan* p) {
  free_device(p);
  build_layout(p);
  int rc;
  int maxn = 0, maxv = 0, maxd = 0;
  int64_t maxblk = 0, sum_n = 0;
  for (auto& c : p->ch) {
    maxn = std::max(maxn, c.fft_len);
    maxv = std::max(maxv, c.valid);
    maxd = std::max(maxd, (int)c.dm.size());
    sum_n += c.fft_len;
    // blocks one call can complete: history (< N) plus the chunk, plus one for rounding
    maxblk = std::max(maxblk, (p->max_block + c.fft_len) / c.valid + 2);
  }
  p->hist_cap = maxn;
  const size_t ib = in_bytes(p->in_dtype);
  for (int i = 0; i < 2; ++i)
    if ((rc = dev_alloc(p, &p->hist[i], (size_t)p->C * p->M * p->hist_cap * ib))) return rc;
  int64_t spec_elems = 0;
  for (auto& c : p->ch) spec_elems = std::max(spec_elems, (int64_t)p->M * ((p->max_block + c.fft_len) / c.valid + 2) * c.fft_len);
  p->spec_elems = (size_t)spec_elems;
  if ((rc = dev_alloc(p, (void**)&p->spec, p->spec_elems * sizeof(float2)))) return rc;
  if ((rc = dev_alloc(p, (void**)&p->chirp, (size_t)maxd * maxn * sizeof(float2)))) return rc;
  // dedispersed voltages of one DM group: [dm_group][M][blocks * V]
  p->y_stride = 0;
  for (auto& c : p->ch) p->y_stride = std::max(p->y_stride, ((p->max_block + c.fft_len) / c.valid + 2) * c.valid);
  const size_t per_dm = (size_t)p->M * p->y_stride * y_bytes(p->corr_dtype);
  p->dm_group = (int)std::max<size_t>(1, std::min<size_t>(16, ((size_t)2 << 30) / std::max<size_t>(per_dm, 1)));
  p->dm_group = std::min(p->dm_group, maxd);
  if ((rc = dev_alloc(p, &p->ybuf, per_dm * p->dm_group))) return rc;
  // dump ring: dumps one call can produce plus what a lagging channel holds back
  p->ring_dumps = (p->max_block + p->L - 1) / p->L + (2 * (int64_t)maxn + maxv) / p->L + 4;
  if ((rc = dev_alloc(p, (void**)&p->ring, (size_t)p->ring_dumps * p->rec_elems * sizeof(float2)))) return rc;
  // FP64 tables
  p->gtab_off.assign(p->C + 1, 0);
  std::vector<double> g(sum_n);
  for (int i = 0; i < p->C; ++i) {
    Chan& c = p->ch[i];
    p->gtab_off[i + 1] = p->gtab_off[i] + c.fft_len;
    const int n = c.fft_len;
    for (int k = 0; k < n; ++k) {
      const double f = p->sideband * (double)(k < n / 2 ? k : k - n) * (p->fs / n);
      g[p->gtab_off[i] + k] = (f * f) / (c.fc * c.fc * (c.fc + f));
    }
  }
  if ((rc = dev_alloc(p, (void**)&p->gtab, g.size() * sizeof(double)))) return rc;
  if ((rc = dev_alloc(p, (void**)&p->kdm_dev, p->dm_off[p->C] * sizeof(double)))) return rc;
  if ((rc = dev_alloc(p, (void**)&p->pos_dev, p->dm_off[p->C] * sizeof(int32_t)))) return rc;
  if ((rc = dev_alloc(p, (void**)&p->scale_dev, p->C * sizeof(float)))) return rc;
  HIPCHECK(p, hipMemcpy(p->gtab, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHECK(p, hipMemcpy(p->scale_dev, p->lay_scale.data(), p->C * sizeof(float), hipMemcpyHostToDevice));
  if ((rc = upload_active(p, nullptr))) return rc;
  return DDX_OK;
}

}  // namespace

extern "C" {

const char* ddx_strerror(int s) {
  switch (s) {
    case DDX_OK: return "ok";
    case DDX_EINVAL: return "invalid argument";
    case DDX_ENOMEM: return "out of device memory or over max_device_bytes";
    case DDX_EDEVICE: return "HIP device error";
    case DDX_ESTATE: return "call not allowed in the current plan state";
    case DDX_ESIZE: return "output buffer too small";
    case DDX_EFULL: return "dump ring full: fetch visibilities first";
    case DDX_EUNSUPPORTED: return "not supported by this build";
  }
  return "unknown status";
}

const char* ddx_last_error(const ddx_plan* p) { return p ? p->err.c_str() : "null plan"; }

int ddx_plan_create(const ddx_desc* d, ddx_plan** out) {
  if (!d || !out) return DDX_EINVAL;
  if (d->n_ant < 1 || d->n_chan < 1 || !d->chan_freq_hz || !(d->samp_rate_hz > 0) || !std::isfinite(d->samp_rate_hz))
    return DDX_EINVAL;
  if (d->sideband != 1 && d->sideband != -1) return DDX_EINVAL;
  if (d->in_dtype != DDX_IN_CI8 && d->in_dtype != DDX_IN_CF32) return DDX_EINVAL;
  if (d->corr_dtype < DDX_CORR_F32 || d->corr_dtype > DDX_CORR_E4M3) return DDX_EINVAL;
  if (d->dump_len < 1 || d->max_block_samples < 1) return DDX_EINVAL;
  if (d->out_mode != DDX_OUT_PACKED && d->out_mode != DDX_OUT_FULL) return DDX_EINVAL;
  if (d->k_dm < 0 || !std::isfinite(d->k_dm)) return DDX_EINVAL;
  for (int c = 0; c < d->n_chan; ++c) {
    const double f = d->chan_freq_hz[c];
    if (!std::isfinite(f) || !(f > 0.5 * d->samp_rate_hz)) return DDX_EINVAL;
    if (d->fft_len && d->fft_len[c] != 0 && (!is_pow2(d->fft_len[c]) || d->fft_len[c] < 2)) return DDX_EINVAL;
    if (d->chan_scale && (!(d->chan_scale[c] > 0) || !std::isfinite(d->chan_scale[c]))) return DDX_EINVAL;
  }
  if (d->n_ant > kMaxCorrAnt) return DDX_EUNSUPPORTED;
  ddx_plan* p = new (std::nothrow) ddx_plan;
  if (!p) return DDX_ENOMEM;
  p->M = d->n_ant;
  p->C = d->n_chan;
  p->L = d->dump_len;
  p->fs = d->samp_rate_hz;
  p->sideband = d->sideband;
  p->in_dtype = d->in_dtype;
  p->corr_dtype = d->corr_dtype;
  p->out_mode = d->out_mode;
  p->kdm = d->k_dm == 0 ? kDefaultKdm : d->k_dm;
  p->max_block = d->max_block_samples;
  p->max_bytes = d->max_device_bytes;
  p->nbl = d->out_mode == DDX_OUT_PACKED ? d->n_ant * (d->n_ant + 1) / 2 : d->n_ant * d->n_ant;
  p->ch.resize(p->C);
  p->fft_req.assign(p->C, 0);
  for (int c = 0; c < p->C; ++c) {
    p->ch[c].fc = d->chan_freq_hz[c];
    if (d->fft_len) p->fft_req[c] = d->fft_len[c];
    p->ch[c].scale = d->chan_scale ? d->chan_scale[c] : 1.f;
  }
  p->have_scale = d->chan_scale != nullptr;
  *out = p;
  return DDX_OK;
}

int ddx_set_dm_trials(ddx_plan* p, int32_t chan, const double* dm, int32_t n_dm) {
  if (!p) return DDX_EINVAL;
  if (p->started) return fail(p, DDX_ESTATE, "DM trials are fixed once streaming has started");
  if (chan < -1 || chan >= p->C) return fail(p, DDX_EINVAL, "channel %d out of range", chan);
  if (!dm || n_dm < 1) return fail(p, DDX_EINVAL, "need at least one DM");
  for (int i = 0; i < n_dm; ++i)
    if (!std::isfinite(dm[i]) || dm[i] < 0) return fail(p, DDX_EINVAL, "DM[%d] = %g is not finite and >= 0", i, dm[i]);
  const int c0 = chan < 0 ? 0 : chan, c1 = chan < 0 ? p->C : chan + 1;
  // transactional: a failure leaves every channel as it was
  std::vector<Chan> saved = p->ch;
  for (int c = c0; c < c1; ++c) {
    p->ch[c].dm.assign(dm, dm + n_dm);
    p->ch[c].active.assign(n_dm, 1);
  }
  bool all = true;
  for (int c = 0; c < p->C; ++c) {
    if (p->ch[c].dm.empty()) { all = false; continue; }
    int rc = blocking(p, p->ch[c], p->fft_req[c]);
    if (rc) { p->ch = saved; return rc; }
  }
  if (!all) { p->ready = false; return DDX_OK; }
  int rc = setup_device(p);
  p->ready = rc == DDX_OK;
  return rc;
}

int ddx_set_active_dms(ddx_plan* p, int32_t chan, const uint8_t* mask) {
  if (!p) return DDX_EINVAL;
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials first");
  if (chan < -1 || chan >= p->C) return fail(p, DDX_EINVAL, "channel %d out of range", chan);
  const int c0 = chan < 0 ? 0 : chan, c1 = chan < 0 ? p->C : chan + 1;
  for (int c = c0; c < c1; ++c)
    for (size_t d = 0; d < p->ch[c].dm.size(); ++d) p->ch[c].active[d] = mask ? (mask[d] != 0) : 1;
  if (p->last_stream) HIPCHECK(p, hipStreamSynchronize(p->last_stream));
  return upload_active(p, p->last_stream);
}

int ddx_get_layout(const ddx_plan* pc, ddx_layout* o) {
  if (!pc || !o) return DDX_EINVAL;
  ddx_plan* p = const_cast<ddx_plan*>(pc);
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials for every channel first");
  if (p->scale_pending) {
    HIPCHECK(p, hipStreamSynchronize(p->last_stream));
    HIPCHECK(p, hipMemcpy(p->lay_scale.data(), p->scale_dev, p->C * sizeof(float), hipMemcpyDeviceToHost));
    for (int i = 0; i < p->C; ++i) p->ch[i].scale = p->lay_scale[i];
    p->scale_pending = false;
  }
  std::memset(o, 0, sizeof *o);
  o->n_ant = p->M;
  o->n_chan = p->C;
  o->n_baselines = p->nbl;
  o->dump_len = p->L;
  o->out_mode = p->out_mode;
  o->corr_dtype = p->corr_dtype;
  o->in_dtype = p->in_dtype;
  o->sideband = p->sideband;
  o->samp_rate_hz = p->fs;
  o->k_dm = p->kdm;
  o->chan_freq_hz = p->lay_fc.data();
  o->fft_len = p->lay_fft.data();
  o->valid = p->lay_valid.data();
  o->lead = p->lay_lead.data();
  o->n_dm = p->lay_ndm.data();
  o->dm_offset = p->dm_off.data();
  o->dm = p->lay_dm.data();
  o->delay_s = p->lay_delay.data();
  o->shift = p->lay_shift.data();
  o->scale = p->lay_scale.data();
  o->record_elems = p->rec_elems;
  o->samples_in = p->recv;
  int64_t ready = INT64_MAX;
  for (auto& c : p->ch) ready = std::min(ready, c.dumps_done);
  o->dumps_ready = ready;
  o->dumps_fetched = p->dumps_fetched;
  o->ring_dumps = p->ring_dumps;
  o->device_bytes = p->dev_bytes;
  return DDX_OK;
}

int ddx_process_block(ddx_plan* p, const void* d_volts, int64_t n, int32_t flags, void* hip_stream) {
  if (!p) return DDX_EINVAL;
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials for every channel first");
  if (p->flushed) return fail(p, DDX_ESTATE, "stream already flushed");
  if (n < 0 || n > p->max_block) return fail(p, DDX_EINVAL, "n = %lld outside [0, %lld]", (long long)n, (long long)p->max_block);
  if (n > 0 && !d_volts) return fail(p, DDX_EINVAL, "null input with n > 0");
  if (flags & ~DDX_FLUSH) return fail(p, DDX_EINVAL, "unknown flags 0x%x", flags);
  hipStream_t s = (hipStream_t)hip_stream;
  const bool flush = flags & DDX_FLUSH;
  const int64_t total = p->recv + n;

  // Blocks each channel can run now, and the dumps they complete.
  std::vector<int64_t> b_end(p->C), dumps_new(p->C);
  int64_t fetched_floor = p->dumps_fetched;
  for (int i = 0; i < p->C; ++i) {
    Chan& c = p->ch[i];
    int64_t be;
    if (flush) {
      be = (total + c.valid - 1) / c.valid;
    } else {
      const int64_t lim = total - c.fft_len + c.lead;  // b V <= lim
      be = lim < 0 ? 0 : lim / c.valid + 1;
    }
    be = std::max(be, c.blocks_done);
    b_end[i] = be;
    int64_t out_end = be * (int64_t)c.valid;
    if (flush) out_end = std::min(out_end, total);
    dumps_new[i] = std::max(c.dumps_done, out_end / p->L);
    if (dumps_new[i] - fetched_floor > p->ring_dumps)
      return fail(p, DDX_EFULL, "channel %d would hold %lld unfetched dumps, ring has %lld", i,
                  (long long)(dumps_new[i] - fetched_floor), (long long)p->ring_dumps);
    const int64_t nb = be - c.blocks_done;
    if ((nb * (int64_t)p->M * c.fft_len) > (int64_t)p->spec_elems)
      return fail(p, DDX_EINVAL, "internal: %lld blocks exceed the spectrum buffer", (long long)nb);
  }
  p->started = true;
  p->last_stream = s;

  ddx::Source src{};
  src.chunk = d_volts;
  src.hist = p->hist[p->hist_cur];
  src.chunk_stride = n;
  src.hist_cap = p->hist_cap;
  src.chunk_start = p->recv;
  src.chunk_len = n;

  for (int i = 0; i < p->C; ++i) {
    Chan& c = p->ch[i];
    const int64_t b0 = c.blocks_done, nb = b_end[i] - b0;
    if (nb <= 0) continue;
    src.hist_start = c.hist_start;
    if (b0 == 0 && !p->have_scale) {
      // first block of the channel: fix its correlator-input scale from the block's window
      const float target = p->corr_dtype == DDX_CORR_E4M3 ? kScaleTargetE4M3 : kScaleTargetF16;  // F32 too
      const int64_t nwin = std::min<int64_t>(c.fft_len - c.lead, total);
      HIPCHECK(p, timed(p, s, DDX_K_OTHER, 0.0, (double)nwin * p->M * in_bytes(p->in_dtype), [&] {
        if (p->in_dtype == DDX_IN_CI8)
          hipLaunchKernelGGL(ddx::k_scale<0>, dim3(1), dim3(1024), 0, s, src, i, p->M, nwin, target, p->scale_dev);
        else
          hipLaunchKernelGGL(ddx::k_scale<1>, dim3(1), dim3(1024), 0, s, src, i, p->M, nwin, target, p->scale_dev);
        return hipGetLastError();
      }));
      p->scale_pending = true;
    }
    ddx::FwdArgs fa{};
    fa.src = src;
    fa.spec = p->spec;
    fa.b0 = b0;
    fa.nblk = (int)nb;
    fa.n_ant = p->M;
    fa.valid = c.valid;
    fa.lead = c.lead;
    fa.chan = i;
    HIPCHECK(p, timed(p, s, DDX_K_FORWARD, (double)nb * p->M * fft_flops(c.fft_len),
                      (double)nb * p->M * c.fft_len * (in_bytes(p->in_dtype) + 8.0),
                      [&] { return launch_forward(c.logn, p->in_dtype, fa, s); }));
    const int na = p->n_active[i];
    const int64_t dump0 = b0 * (int64_t)c.valid / p->L;
    const int n_dumps = (int)(dumps_new[i] - dump0);
    if (na > 0) {
      dim3 g((c.fft_len + 255) / 256, na);
      HIPCHECK(p, timed(p, s, DDX_K_CHIRP, 0.0, (double)c.fft_len * (8.0 + 8.0 * na), [&] {
        hipLaunchKernelGGL(ddx::k_chirp, g, dim3(256), 0, s, p->gtab + p->gtab_off[i], p->kdm_dev + p->dm_off[i],
                           p->chirp, c.fft_len, 1.0f / (float)c.fft_len);
        return hipGetLastError();
      }));
    }
    for (int g0 = 0; g0 < na; g0 += p->dm_group) {
      const int nd = std::min(p->dm_group, na - g0);
      ddx::DedispArgs da{};
      da.spec = p->spec;
      da.chirp = p->chirp + (size_t)g0 * c.fft_len;
      da.y = p->ybuf;
      da.y_stride = p->y_stride;
      da.scale = p->scale_dev + i;
      da.n_ant = p->M;
      da.nblk = (int)nb;
      da.nd = nd;
      da.valid = c.valid;
      da.lead = c.lead;
      HIPCHECK(p, timed(p, s, DDX_K_DEDISP, (double)nb * p->M * nd * (fft_flops(c.fft_len) + 6.0 * c.fft_len),
                        8.0 * c.fft_len * ((double)nb * p->M + nd) + (double)nd * p->M * nb * c.valid * y_bytes(p->corr_dtype),
                        [&] { return launch_dedisp(c.logn, p->corr_dtype, da, s); }));
      if (n_dumps > 0) {
        ddx::CorrArgs ca{};
        ca.y = p->ybuf;
        ca.y_stride = p->y_stride;
        ca.ring = p->ring;
        ca.rec_elems = p->rec_elems;
        ca.ring_dumps = p->ring_dumps;
        ca.dump0 = dump0;
        ca.dm_pos = p->pos_dev + p->dm_off[i] + g0;
        ca.scale = p->scale_dev + i;
        ca.n_dumps = n_dumps;
        ca.nd = nd;
        ca.n_ant = p->M;
        ca.dump_len = p->L;
        ca.nbl = p->nbl;
        ca.out_mode = p->out_mode;
        const double nbl_h = p->M * (p->M + 1) / 2.0;
        HIPCHECK(p, timed(p, s, DDX_K_CORR, (double)n_dumps * nd * 8.0 * p->L * nbl_h,
                          (double)n_dumps * nd * ((double)p->L * p->M * y_bytes(p->corr_dtype) + 8.0 * p->nbl),
                          [&] { return launch_corr(p->corr_dtype, ca, s); }));
      }
    }
    const int n_inactive = (int)c.dm.size() - na;
    if (n_inactive > 0 && n_dumps > 0) {
      const int64_t tot = (int64_t)n_dumps * n_inactive * p->nbl;
      HIPCHECK(p, timed(p, s, DDX_K_OTHER, 0.0, 8.0 * tot, [&] {
        hipLaunchKernelGGL(ddx::k_zero_dm, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p->ring, p->rec_elems,
                           p->ring_dumps, dump0, n_dumps, p->pos_dev + p->dm_off[i] + na, n_inactive, p->nbl);
        return hipGetLastError();
      }));
    }
  }

  // Carry the unconsumed tail of every row into the other history buffer.
  if (!flush) {
    void* dst = p->hist[1 - p->hist_cur];
    for (int i = 0; i < p->C; ++i) {
      Chan& c = p->ch[i];
      const int64_t start = std::max<int64_t>(0, b_end[i] * c.valid - c.lead);
      const int64_t len = std::max<int64_t>(0, total - start);
      if (len > p->hist_cap) return fail(p, DDX_EINVAL, "internal: history of %lld samples", (long long)len);
      if (len > 0) {
        ddx::Source hs = src;
        hs.hist_start = c.hist_start;
        dim3 g((unsigned)((len + 255) / 256), p->M);
        HIPCHECK(p, timed(p, s, DDX_K_OTHER, 0.0, 2.0 * len * p->M * in_bytes(p->in_dtype), [&] {
          if (p->in_dtype == DDX_IN_CI8)
            hipLaunchKernelGGL(ddx::k_history<0>, g, dim3(256), 0, s, hs, dst, start, len, p->M, i);
          else
            hipLaunchKernelGGL(ddx::k_history<1>, g, dim3(256), 0, s, hs, dst, start, len, p->M, i);
          return hipGetLastError();
        }));
      }
      c.hist_start = start;
    }
    p->hist_cur = 1 - p->hist_cur;
  }
  for (int i = 0; i < p->C; ++i) {
    p->ch[i].blocks_done = b_end[i];
    p->ch[i].dumps_done = dumps_new[i];
  }
  p->recv = total;
  if (flush) p->flushed = true;
  return DDX_OK;
}

int ddx_fetch_visibilities(ddx_plan* p, void* out, size_t cap, int64_t* first, int64_t* nd, void* hip_stream) {
  if (!p || !first || !nd) return DDX_EINVAL;
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials for every channel first");
  int64_t ready = INT64_MAX;
  for (auto& c : p->ch) ready = std::min(ready, c.dumps_done);
  const int64_t avail = ready - p->dumps_fetched;
  *first = p->dumps_fetched;
  *nd = avail;
  if (avail == 0) return DDX_OK;
  const size_t rec = (size_t)p->rec_elems * sizeof(float2);
  if (cap < rec * (size_t)avail) return fail(p, DDX_ESIZE, "need %zu bytes for %lld dumps", rec * avail, (long long)avail);
  if (!out) return fail(p, DDX_EINVAL, "null output");
  hipStream_t s = (hipStream_t)hip_stream;
  int64_t k = 0;
  while (k < avail) {
    const int64_t slot = (p->dumps_fetched + k) % p->ring_dumps;
    const int64_t cnt = std::min(avail - k, p->ring_dumps - slot);
    HIPCHECK(p, hipMemcpyAsync((char*)out + rec * k, p->ring + slot * p->rec_elems, rec * cnt, hipMemcpyDefault, s));
    k += cnt;
  }
  p->dumps_fetched = ready;
  p->last_stream = s;
  return DDX_OK;
}

}  // extern "C"

namespace {

// Grow a plan-owned scratch buffer (old contents are not kept).
template <class T>
int ensure(ddx_plan* p, T** buf, size_t* cap, size_t elems) {
  if (*cap >= elems) return DDX_OK;
  if (p->last_stream) HIPCHECK(p, hipStreamSynchronize(p->last_stream));
  if (*buf) {
    for (auto it = p->allocs.begin(); it != p->allocs.end(); ++it)
      if (*it == (void*)*buf) { p->allocs.erase(it); break; }
    (void)hipFree(*buf);
    p->dev_bytes -= *cap * sizeof(T);
    *buf = nullptr;
    *cap = 0;
  }
  int rc = dev_alloc(p, (void**)buf, elems * sizeof(T));
  if (rc == DDX_OK) *cap = elems;
  return rc;
}

// Common tail of both tile entry points: per-channel power rows -> prefix sums -> tiles.
int tiles_from_rows(ddx_plan* p, const float* power, int n_tiles, int64_t units, int fine, int bin_len, int n_bins,
                    float* tiles, hipStream_t s) {
  const int C = p->C, D = (int)p->ch[0].dm.size();
  const int64_t rows = (int64_t)n_tiles * C;
  const int nblk = (int)((units + ddx::kScanBlock - 1) / ddx::kScanBlock);
  int rc;
  if ((rc = ensure(p, &p->tile_prefix, &p->tile_prefix_cap, (size_t)rows * (units + 1)))) return rc;
  if ((rc = ensure(p, &p->tile_totals, &p->tile_totals_cap, (size_t)rows * nblk))) return rc;
  if (p->tile_shift_fine != fine) {
    if (!p->tile_shift && (rc = dev_alloc(p, (void**)&p->tile_shift, (size_t)C * D * sizeof(int64_t)))) return rc;
    std::vector<int64_t> sh((size_t)C * D);
    for (int c = 0; c < C; ++c)
      for (int d = 0; d < D; ++d)
        sh[(size_t)c * D + d] = (int64_t)std::nearbyint((double)p->lay_shift[p->dm_off[c] + d] / fine);
    if (p->last_stream) HIPCHECK(p, hipStreamSynchronize(p->last_stream));
    HIPCHECK(p, hipMemcpy(p->tile_shift, sh.data(), sh.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    p->tile_shift_fine = fine;
  }
  const dim3 g(nblk, (unsigned)rows);
  hipLaunchKernelGGL(ddx::k_scan_local, g, dim3(256), 0, s, power, units, p->tile_prefix, p->tile_totals, nblk);
  HIPCHECK(p, hipGetLastError());
  hipLaunchKernelGGL(ddx::k_scan_fix, g, dim3(256), 0, s, p->tile_prefix, units, p->tile_totals, nblk);
  HIPCHECK(p, hipGetLastError());
  hipLaunchKernelGGL(ddx::k_tile, dim3((n_bins + 255) / 256, D, n_tiles), dim3(256), 0, s, p->tile_prefix, units, C,
                     p->tile_shift, D, bin_len / fine, n_bins, tiles);
  HIPCHECK(p, hipGetLastError());
  p->last_stream = s;
  return DDX_OK;
}

int tile_checks(ddx_plan* p, int bin_len, int n_bins, int fine) {
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials for every channel first");
  for (auto& c : p->ch)
    if (c.dm != p->ch[0].dm) return fail(p, DDX_EUNSUPPORTED, "tiles need the same DM trials in every channel");
  if (fine < 1 || bin_len < fine || bin_len % fine != 0 || n_bins < 1)
    return fail(p, DDX_EINVAL, "bin_len must be a positive multiple of the fine bin, n_bins >= 1");
  return DDX_OK;
}

}  // namespace

extern "C" {

int ddx_power_tile(ddx_plan* p, const void* d_volts, int64_t n, int32_t bin_len, int32_t n_bins, float* d_tile,
                   void* hip_stream) {
  if (!p) return DDX_EINVAL;
  int rc = tile_checks(p, bin_len, n_bins, 1);
  if (rc) return rc;
  if (!d_volts || !d_tile || n < 1) return fail(p, DDX_EINVAL, "null buffer or empty stream");
  hipStream_t s = (hipStream_t)hip_stream;
  if ((rc = ensure(p, &p->tile_power, &p->tile_power_cap, (size_t)p->C * n))) return rc;
  const dim3 g((unsigned)((n + 255) / 256), p->C);
  if (p->in_dtype == DDX_IN_CI8)
    hipLaunchKernelGGL(ddx::k_beam_power<0>, g, dim3(256), 0, s, d_volts, n, p->M, p->tile_power);
  else
    hipLaunchKernelGGL(ddx::k_beam_power<1>, g, dim3(256), 0, s, d_volts, n, p->M, p->tile_power);
  HIPCHECK(p, hipGetLastError());
  return tiles_from_rows(p, p->tile_power, 1, n, 1, bin_len, n_bins, d_tile, s);
}

int ddx_power_tile_from_power(ddx_plan* p, const float* d_power, int32_t n_tiles, int64_t units, int32_t fine,
                              int32_t bin_len, int32_t n_bins, float* d_tiles, void* hip_stream) {
  if (!p) return DDX_EINVAL;
  int rc = tile_checks(p, bin_len, n_bins, fine);
  if (rc) return rc;
  if (!d_power || !d_tiles || n_tiles < 1 || units < 1) return fail(p, DDX_EINVAL, "null buffer or empty input");
  return tiles_from_rows(p, d_power, n_tiles, units, fine, bin_len, n_bins, d_tiles, (hipStream_t)hip_stream);
}

int ddx_reset_stream(ddx_plan* p) {
  if (!p) return DDX_EINVAL;
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials for every channel first");
  if (p->started) HIPCHECK(p, hipStreamSynchronize(p->last_stream));
  for (auto& c : p->ch) {
    c.blocks_done = 0;
    c.dumps_done = 0;
    c.hist_start = 0;
  }
  p->recv = 0;
  p->dumps_fetched = 0;
  p->hist_cur = 0;
  p->flushed = false;
  return DDX_OK;
}

int ddx_set_profiling(ddx_plan* p, int32_t on) {
  if (!p) return DDX_EINVAL;
  if (on && p->started) HIPCHECK(p, hipStreamSynchronize(p->last_stream));
  if (on) {
    p->recs.clear();
    p->events_used = 0;
  }
  p->profiling = on != 0;
  return DDX_OK;
}

int ddx_get_profile(ddx_plan* p, ddx_profile* out) {
  if (!p || !out) return DDX_EINVAL;
  std::memset(out, 0, sizeof *out);
  for (auto& r : p->recs) {
    HIPCHECK(p, hipEventSynchronize(r.b));
    float ms = 0.f;
    HIPCHECK(p, hipEventElapsedTime(&ms, r.a, r.b));
    out->launches[r.kind] += 1;
    out->time_ms[r.kind] += ms;
    out->flops[r.kind] += r.flops;
    out->bytes[r.kind] += r.bytes;
  }
  return DDX_OK;
}

int ddx_plan_destroy(ddx_plan* p) {
  if (!p) return DDX_OK;
  if (p->last_stream || p->started) (void)hipStreamSynchronize(p->last_stream);
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  free_device(p);
  delete p;
  return DDX_OK;
}

}  // extern "C"
