// Host side of the ddx C ABI: plan state, blocking, tables, work lists, launches.
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
constexpr int kMaxLogN = 18;        // two-pass transforms above 2^15
// Two-pass inverse: bytes of intermediate rows per antenna group (0: one group of
// all antennas).  Measured on the 256-antenna workload (dedispersion per step):
// one group 29.5 s, 64 MB 28.0 s, 128 MB 26.8 s, 256 MB 28.0 s.
constexpr size_t kTbGroupBytes = (size_t)128 << 20;
constexpr int kMinLogN = 8;
constexpr int kMaxStackedAnt = 64;  // stacked-row Gram kernel up to 2 M = 128 rows
constexpr int kMaxCorrAnt = 1024;   // antenna-block kernel beyond
constexpr int kDefaultDmGroup = 16;
constexpr size_t kAutoYBytes = size_t(2) << 30;  // dedispersed voltages of one wave, automatic schedule
// Automatic blocking (see ddx_set_dm_trials): the DMs of a channel, sorted, are cut
// into classes, each with the overlap-save blocking of its own largest DM, choosing
// the cuts and every class's N to minimise the modelled device time per output
// sample, sum over classes of (n_dm kDedispPs + kForwardPs) N / V (one inverse
// transform per DM, one forward transform, per block and antenna).  Picoseconds
// per transform point of the dedispersion and forward kernels for N = 2^8 .. 2^18
// (FP32 output, complex int8 input, 36 antennas; measured on gfx950 with the
// library's own profiling; 2^8 and 2^9 taken as 2^10).  The descriptor may carry
// another table (the autotuner measures one on the device it runs on).
constexpr double kDedispPs[11] = {2.44, 2.44, 2.44, 2.23, 2.05, 2.04, 2.27, 2.89, 6.18, 6.54, 6.55};
constexpr double kForwardPs[11] = {2.59, 2.59, 2.59, 2.53, 2.77, 3.39, 4.00, 5.63, 7.81, 7.36, 7.48};
// Cuts fall on multiples of this many sorted DMs, so that the DM groups of a block
// keep sharing its spectrum in L2.
constexpr int kClassStep = 16;
// Spectrum buffer: every class keeps the spectra of the blocks one call runs, so
// many classes of many antennas would need hundreds of GB; a call runs its
// classes in batches whose spectra fit this many bytes (or one class, if larger),
// unless the descriptor gives another cap.
constexpr int64_t kSpecBudgetBytes = int64_t(32) << 30;
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
  float scale = 1.f;
  std::vector<int> grp;         // its blocking classes (indices into ddx_plan::grp), by DM
  int cover = 0;                // the class holding its largest DM
  int win = 0;                  // N - lead of that class: the scale rule's window
  // stream state
  bool scaled = false;     // correlator-input scale of this stream computed
  int64_t hist_start = 0;  // absolute index of history element 0
};

// One overlap-save blocking: a class of one channel's DMs.
struct Grp {
  int chan = 0;
  std::vector<int> dms;         // the channel's DM indices in the class, ascending
  int fft_len = 0, logn = 0, valid = 0, lead = 0;
  int64_t gtab = 0;             // offset of the class's FP64 g table
  int32_t slot0 = 0;            // its run of the slot table: active slots, then inactive ones
  int32_t n_active = 0;
  // stream state
  int64_t blocks_done = 0;
  int64_t dumps_done = 0;
};

// Host copies of one call's work lists, packed into one upload.
struct Wave {
  int logn;
  size_t u0, nu;      // units [u0, u0 + nu)
  size_t c0, nc;      // chirp items [c0, c0 + nc)
  int max_dumps;
  int64_t spectra;    // distinct (channel, block) spectra the wave reads
  int64_t y_samples;  // dedispersed samples it writes (all antennas)
  int64_t dumps;      // (unit, dump) pairs it correlates
  double fft_n;       // N of its transforms
  int64_t y_stride;   // elements per antenna row of its dedispersed voltages
};
struct FwdLaunch {
  int logn;
  size_t i0, n;       // forward items [i0, i0 + n)
};

}  // namespace

struct ddx_plan {
  // descriptor
  int M = 0, C = 0, L = 0, sideband = 1, in_dtype = 0, corr_dtype = 0, out_mode = 0;
  double fs = 0, kdm = kDefaultKdm;
  int64_t max_block = 0;
  size_t max_bytes = 0;
  std::vector<int> fft_req;
  bool have_scale = false;
  int wave_req = 0, group_req = 0, compact = 0, max_pairs_req = 0;
  int64_t ring_req = 0;
  int classes_req = 0;
  int64_t spec_budget = 0;  // bytes
  double cost_inv[11] = {}, cost_fwd[11] = {};  // blocking cost model, ps per point, N = 2^8 .. 2^18
  std::vector<Chan> ch;
  std::vector<Grp> grp;
  int nbl = 0;
  // derived
  bool ready = false, started = false, flushed = false;
  std::vector<int32_t> lay_fft, lay_valid, lay_lead, lay_ndm;
  std::vector<int32_t> lay_dm_fft, lay_dm_valid, lay_dm_lead;  // per (channel, DM): its class's blocking
  std::vector<int64_t> dm_off, lay_shift;
  std::vector<double> lay_dm, lay_delay, lay_fc;
  std::vector<float> lay_scale;
  std::vector<int32_t> rec_pos;  // [sum D_c] record slot of (c, d), -1 if not stored
  int64_t rec_pairs = 0, rec_elems = 0, cap_pairs = 0;
  int wave_units = 0, dm_group = 0;
  // per transform length (index log2 N): units a wave may hold, and the row stride
  // of its dedispersed voltages (the length's largest V)
  std::vector<int> wave_cap;
  std::vector<int64_t> wave_ys;
  // stream
  int64_t recv = 0;
  int64_t dumps_fetched = 0;
  // device memory
  size_t dev_bytes = 0;
  std::vector<void*> allocs;
  void* hist[2] = {nullptr, nullptr};
  int hist_cur = 0;
  int64_t hist_cap = 0;
  float2* spec = nullptr;      // spectra of the blocks one batch of classes runs
  size_t spec_elems = 0;
  float2* tb = nullptr;        // intermediate rows of the two-pass transforms
  size_t tb_elems = 0;
  float2* chirp = nullptr;     // [wave_units][max N]
  void* ybuf = nullptr;        // [wave_units][M][y_stride]
  int64_t y_stride = 0;
  float* power = nullptr;      // binary16 / E4M3: [wave_units][M][pw_stride] per-dump power
  float* l1 = nullptr;         // FP32: [forward items][M][8] row sums of |Re X| + |Im X| of one call
  float* bound = nullptr;      // FP32: [forward items] bound on the block's |Re y|, |Im y| (input units)
  uint8_t* sel_dev = nullptr;  // proposal selection: mask [kTopkMax] + flag (device)
  uint8_t* sel_host = nullptr; // pinned host copy
  int pw_stride = 0;
  float2* ring = nullptr;
  int64_t ring_dumps = 0;
  double* gtab = nullptr;      // [sum over classes of N] FP64 g[k]
  std::vector<int32_t> slots;    // [sum D_c] per class: active record slots, then inactive ones
  float* scale_dev = nullptr;    // [C]
  double* scale_part = nullptr;  // [C][M] partial power sums of the scale rule
  char* items_dev = nullptr;     // work lists of one call
  size_t items_cap = 0;
  char* stage[2] = {nullptr, nullptr};  // pinned host staging of the work lists
  hipEvent_t stage_ev[2] = {nullptr, nullptr};
  bool stage_used[2] = {false, false};
  int stage_cur = 0;
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
  for (int i = 0; i < 2; ++i) {
    if (p->stage_ev[i]) {
      (void)hipEventSynchronize(p->stage_ev[i]);
      (void)hipEventDestroy(p->stage_ev[i]);
      p->stage_ev[i] = nullptr;
    }
    if (p->stage[i]) (void)hipHostFree(p->stage[i]);
    if (i == 0 && p->sel_host) (void)hipHostFree(p->sel_host);
    if (i == 0) p->sel_host = nullptr;
    p->stage[i] = nullptr;
    p->stage_used[i] = false;
  }
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
  p->dev_bytes = 0;
  p->hist[0] = p->hist[1] = nullptr;
  p->spec = p->tb = p->chirp = p->ring = nullptr;
  p->spec_elems = p->tb_elems = 0;
  p->ybuf = nullptr;
  p->power = nullptr;
  p->l1 = p->bound = nullptr;
  p->sel_dev = nullptr;
  p->gtab = nullptr;
  p->scale_dev = nullptr;
  p->scale_part = nullptr;
  p->items_dev = nullptr;
  p->items_cap = 0;
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

// Overlap-save blocking (reading stated in ddx.h at ddx_set_dm_trials).
// Half overlap of one DM: the larger intra-channel smear, in samples, rounded up.
double half_overlap(const ddx_plan* p, double fc, double dm) {
  const double hi = fc + 0.5 * p->fs, lo = fc - 0.5 * p->fs;
  const double inv_c = 1.0 / (fc * fc);
  const double early = p->kdm * dm * (inv_c - 1.0 / (hi * hi)) * p->fs;
  const double late = p->kdm * dm * (1.0 / (lo * lo) - inv_c) * p->fs;
  return std::ceil(std::max(early, late));
}

// Outputs kept per block of length n with half overlap a (a multiple of L), -1 if none.
int64_t kept(const ddx_plan* p, int64_t n, int64_t a) {
  const int64_t r = n - 2 * a;
  return r < 0 ? int64_t(-1) : p->L * (r / p->L);
}

// Blocking of class g for half overlap a and FFT length n (0: the smallest power
// of two >= 256 that keeps at least half of each block).
int set_blocking(ddx_plan* p, Grp& g, int64_t a, int64_t n) {
  if (n == 0) {
    n = 256;
    while (kept(p, n, a) < n / 2 && n <= (int64_t(1) << 30)) n *= 2;
  }
  const int64_t v = kept(p, n, a);
  if (v < p->L) return fail(p, DDX_EINVAL, "FFT length %lld too short for overlap %lld and dump %d", (long long)n, (long long)(2 * a), p->L);
  if (n > (int64_t(1) << kMaxLogN))
    return fail(p, DDX_EUNSUPPORTED, "FFT length %lld > %d not supported", (long long)n, 1 << kMaxLogN);
  g.fft_len = (int)n;
  g.logn = std::max(ilog2i(n), kMinLogN);
  if ((1 << g.logn) != n) return fail(p, DDX_EUNSUPPORTED, "FFT length %lld < 256", (long long)n);
  g.valid = (int)v;
  g.lead = (int)((n - v) / 2);
  return DDX_OK;
}

// Split channel ci's DMs into blocking classes (appended to out).  A requested FFT
// length, or one class per channel, keeps every DM in one class with the blocking
// of the largest DM; otherwise the cuts and lengths minimise the cost model above
// by dynamic programming over the sorted DMs.
int plan_channel(ddx_plan* p, int ci, std::vector<Grp>& out) {
  const Chan& c = p->ch[ci];
  const int D = (int)c.dm.size();
  std::vector<int> order(D);
  for (int i = 0; i < D; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return c.dm[x] < c.dm[y]; });
  std::vector<double> a(D);
  for (int k = 0; k < D; ++k) a[k] = half_overlap(p, c.fc, c.dm[order[k]]);
  if (!(a[D - 1] < 1e9)) return fail(p, DDX_EUNSUPPORTED, "dispersion smear %.3g samples too long", a[D - 1]);
  std::vector<int> ends, lens;  // class k covers sorted DMs [ends[k-1], ends[k]) with length lens[k]
  const int fft_req = p->fft_req[ci];
  if (fft_req || p->classes_req == 1) {
    ends.push_back(D);
    lens.push_back(fft_req);
  } else {
    const int step = std::max(kClassStep, (D + 255) / 256);
    std::vector<int> pos;
    for (int k = step; k < D; k += step) pos.push_back(k);
    pos.push_back(D);
    const double inf = HUGE_VAL;
    const size_t np = pos.size();
    std::vector<double> best(np, inf);
    std::vector<int> from(np, -1), blen(np, 0);
    for (size_t jj = 0; jj < np; ++jj) {
      const int j = pos[jj];
      const int64_t aj = (int64_t)a[j - 1];
      for (int ii = -1; ii < (int)jj; ++ii) {
        const double base = ii < 0 ? 0.0 : best[ii];
        if (!(base < inf)) continue;
        const int n = j - (ii < 0 ? 0 : pos[ii]);
        for (int l = kMinLogN; l <= kMaxLogN; ++l) {
          const int64_t N = int64_t(1) << l, v = kept(p, N, aj);
          if (v < p->L) continue;
          const double cost = base + (n * p->cost_inv[l - kMinLogN] + p->cost_fwd[l - kMinLogN]) * (double)N / (double)v;
          if (cost < best[jj]) {
            best[jj] = cost;
            from[jj] = ii;
            blen[jj] = l;
          }
        }
      }
    }
    if (!(best[np - 1] < inf)) {  // no length holds the largest DM's overlap: the rule's own error
      Grp g;
      int rc = set_blocking(p, g, (int64_t)a[D - 1], 0);
      return rc ? rc : fail(p, DDX_EUNSUPPORTED, "no FFT length up to %d holds the overlap", 1 << kMaxLogN);
    }
    for (int jj = (int)np - 1; jj >= 0; jj = from[jj]) {
      ends.push_back(pos[jj]);
      lens.push_back(1 << blen[jj]);
    }
    std::reverse(ends.begin(), ends.end());
    std::reverse(lens.begin(), lens.end());
  }
  for (size_t k = 0; k < ends.size(); ++k) {
    const int i = k ? ends[k - 1] : 0, j = ends[k];
    Grp g;
    g.chan = ci;
    g.dms.assign(order.begin() + i, order.begin() + j);
    std::sort(g.dms.begin(), g.dms.end());
    int rc = set_blocking(p, g, (int64_t)a[j - 1], lens[k]);
    if (rc) return rc;
    out.push_back(std::move(g));
  }
  return DDX_OK;
}

// ---- kernel dispatch over template parameters ------------------------------------------

template <int LOGN>
size_t fft_lds_bytes() {
  static_assert(LOGN != 15 || ddx::Geo<ddx::Plan15Wide>::LDS_TOTAL == ddx::Geo<ddx::Plan<15>>::LDS_TOTAL,
                "both 32768-point plans take the same LDS");
  return sizeof(float) * ddx::Geo<ddx::Plan<LOGN>>::LDS_TOTAL;
}

template <int LOGN>
hipError_t launch_forward_n(int in_dtype, const ddx::FwdArgs& a, int n_items, hipStream_t s) {
  using G = ddx::Geo<ddx::FwdPlan<LOGN>>;
  dim3 grid(n_items * a.n_ant), block(G::T);
  if (in_dtype == DDX_IN_CI8)
    hipLaunchKernelGGL((ddx::k_forward<LOGN, 0>), grid, block, fft_lds_bytes<LOGN>(), s, a);
  else
    hipLaunchKernelGGL((ddx::k_forward<LOGN, 1>), grid, block, fft_lds_bytes<LOGN>(), s, a);
  return hipGetLastError();
}


template <int LOGN>
hipError_t launch_dedisp_n(int corr_dtype, const ddx::DedispArgs& a, hipStream_t s) {
  const dim3 grid(ddx::order_units(a.n_units, a.tile) * a.n_ant);
  auto block = [](auto out) { return dim3(ddx::Geo<ddx::DedispPlan<LOGN, decltype(out)::value>>::T); };
  if (corr_dtype == DDX_CORR_F32)
    hipLaunchKernelGGL((ddx::k_dedisperse<LOGN, 0>), grid, block(std::integral_constant<int, 0>()),
                       fft_lds_bytes<LOGN>(), s, a);
  else if (corr_dtype == DDX_CORR_F16)
    hipLaunchKernelGGL((ddx::k_dedisperse<LOGN, 1>), grid, block(std::integral_constant<int, 1>()),
                       fft_lds_bytes<LOGN>(), s, a);
  else
    hipLaunchKernelGGL((ddx::k_dedisperse<LOGN, 2>), grid, block(std::integral_constant<int, 2>()),
                       fft_lds_bytes<LOGN>(), s, a);
  return hipGetLastError();
}

hipError_t launch_forward(int logn, int in_dtype, const ddx::FwdArgs& a, int n_items, hipStream_t s) {
  switch (logn) {
    case 8: return launch_forward_n<8>(in_dtype, a, n_items, s);
    case 9: return launch_forward_n<9>(in_dtype, a, n_items, s);
    case 10: return launch_forward_n<10>(in_dtype, a, n_items, s);
    case 11: return launch_forward_n<11>(in_dtype, a, n_items, s);
    case 12: return launch_forward_n<12>(in_dtype, a, n_items, s);
    case 13: return launch_forward_n<13>(in_dtype, a, n_items, s);
    case 14: return launch_forward_n<14>(in_dtype, a, n_items, s);
    case 15: return launch_forward_n<15>(in_dtype, a, n_items, s);
  }
  return hipErrorInvalidValue;
}

// Two-pass forward transform of n_items items whose spectra and intermediate
// rows are consecutive from items[0].spec and tb offset 0.
hipError_t launch_forward_big(int logn, int in_dtype, ddx::FwdArgs a, const ddx::FwdItem* first_host, int n_items,
                              float2* tb, hipStream_t s) {
  const int logr = logn - ddx::kBigLog;
  // the pre-pass grid takes one y index per (item, antenna): at most 65535 per launch
  const int per = std::max(1, 65535 / a.n_ant);
  for (int i0 = 0; i0 < n_items; i0 += per) {
    ddx::FwdArgs ai = a;
    ai.items = a.items + i0;  // each item carries its own source window and tb offset
    const dim3 gpre(ddx::kBigN / 256, (unsigned)(std::min(per, n_items - i0) * a.n_ant));
    if (in_dtype == DDX_IN_CI8)
      hipLaunchKernelGGL(ddx::k_forward_big_pre<0>, gpre, dim3(256), 0, s, ai, tb, logr);
    else
      hipLaunchKernelGGL(ddx::k_forward_big_pre<1>, gpre, dim3(256), 0, s, ai, tb, logr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const unsigned rows = (unsigned)((size_t)n_items * a.n_ant << logr);
  hipLaunchKernelGGL(ddx::k_fft_rows, dim3(rows), dim3(ddx::Geo<ddx::RowPlan>::T), fft_lds_bytes<ddx::kBigLog>(), s,
                     (const float2*)tb, a.spec + first_host->spec, a.l1, logr);
  return hipGetLastError();
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
  if (logn <= kMaxLogN) {
    // antennas in groups whose intermediate rows (n_units x group x N complex) fit
    // kTbGroupBytes, so that pass B reads them back from the Infinity Cache
    const size_t per_ant = (size_t)a.n_units * ((size_t)1 << logn) * sizeof(float2);
    const int group = kTbGroupBytes == 0 ? a.n_ant
                                         : (int)std::max<size_t>(1, std::min<size_t>(a.n_ant, kTbGroupBytes / per_ant));
    for (int g0 = 0; g0 < a.n_ant; g0 += group) {
      ddx::DedispArgs ag = a;
      ag.ant0 = g0;
      ag.n_ant = std::min(group, a.n_ant - g0);
      const unsigned ga = (unsigned)((size_t)ddx::order_units(ag.n_units, ag.tile) * ag.n_ant << ag.logr);
      hipLaunchKernelGGL(ddx::k_dedisperse_big_a, dim3(ga), dim3(ddx::Geo<ddx::Plan<ddx::kBigLog>>::T),
                         fft_lds_bytes<ddx::kBigLog>(), s, ag);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      const dim3 gb(ddx::kBigN / 256, ag.n_units * ag.n_ant);
      if (corr_dtype == DDX_CORR_F32) hipLaunchKernelGGL(ddx::k_dedisperse_big_b<0>, gb, dim3(256), 0, s, ag);
      else if (corr_dtype == DDX_CORR_F16) hipLaunchKernelGGL(ddx::k_dedisperse_big_b<1>, gb, dim3(256), 0, s, ag);
      else hipLaunchKernelGGL(ddx::k_dedisperse_big_b<2>, gb, dim3(256), 0, s, ag);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      if (corr_dtype != DDX_CORR_F32) {  // per-dump power, before the next group reuses the rows
        hipLaunchKernelGGL(ddx::k_dump_power_rows, dim3(ag.n_units * ag.n_ant), dim3(256), 0, s, ag);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    return hipSuccess;
  }
  return hipErrorInvalidValue;
}

template <int NT>
hipError_t launch_corr_nt(int corr_dtype, const ddx::CorrArgs& a, int n_units, hipStream_t s) {
  const dim3 g(n_units * a.max_dumps), b(256);
  if (corr_dtype == DDX_CORR_F32) hipLaunchKernelGGL((ddx::k_correlate<NT, 0>), g, b, 0, s, a);
  else if (corr_dtype == DDX_CORR_F16) hipLaunchKernelGGL((ddx::k_correlate<NT, 1>), g, b, 0, s, a);
  else hipLaunchKernelGGL((ddx::k_correlate<NT, 2>), g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_corr_blocks(int corr_dtype, const ddx::CorrArgs& a, int n_units, hipStream_t s) {
  constexpr int BA = ddx::kBlkAnt;
  const int nb = (a.n_ant + BA - 1) / BA;
  const dim3 g(n_units * a.max_dumps * (nb * (nb + 1) / 2)), b(ddx::corr_block_threads(BA));
  if (corr_dtype == DDX_CORR_F32)
    hipLaunchKernelGGL((ddx::k_correlate_blocks<0, BA>), g, b, ddx::corr_block_lds<0>(BA), s, a);
  else if (corr_dtype == DDX_CORR_F16)
    hipLaunchKernelGGL((ddx::k_correlate_blocks<1, BA>), g, b, ddx::corr_block_lds<1>(BA), s, a);
  else
    hipLaunchKernelGGL((ddx::k_correlate_blocks<2, BA>), g, b, ddx::corr_block_lds<2>(BA), s, a);
  return hipGetLastError();
}

hipError_t launch_corr(int corr_dtype, const ddx::CorrArgs& a, int n_units, hipStream_t s) {
  if (a.n_ant > kMaxStackedAnt) return launch_corr_blocks(corr_dtype, a, n_units, s);
  const int nt = (2 * a.n_ant + 15) / 16;
  switch (nt) {
    case 1: return launch_corr_nt<1>(corr_dtype, a, n_units, s);
    case 2: return launch_corr_nt<2>(corr_dtype, a, n_units, s);
    case 3: return launch_corr_nt<3>(corr_dtype, a, n_units, s);
    case 4: return launch_corr_nt<4>(corr_dtype, a, n_units, s);
    case 5: return launch_corr_nt<5>(corr_dtype, a, n_units, s);
    case 6: return launch_corr_nt<6>(corr_dtype, a, n_units, s);
    case 7: return launch_corr_nt<7>(corr_dtype, a, n_units, s);
    case 8: return launch_corr_nt<8>(corr_dtype, a, n_units, s);
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

double fft_flops(double n) { return 5.0 * n * std::log2(n); }

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
    const Grp& cv = p->grp[c.cover];
    p->lay_fft[i] = cv.fft_len;
    p->lay_valid[i] = cv.valid;
    p->lay_lead[i] = cv.lead;
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
  const int64_t total = p->dm_off[p->C];
  p->lay_dm_fft.assign(total, 0);
  p->lay_dm_valid.assign(total, 0);
  p->lay_dm_lead.assign(total, 0);
  for (const Grp& g : p->grp)
    for (int d : g.dms) {
      const int64_t k = p->dm_off[g.chan] + d;
      p->lay_dm_fft[k] = g.fft_len;
      p->lay_dm_valid[k] = g.valid;
      p->lay_dm_lead[k] = g.lead;
    }
}

// Record slots of the active DMs (compact records: active pairs numbered in
// (channel, DM) order; full records: dm_offset[c] + d) and the per-class slot
// table (each class's active slots first, then its inactive ones, which k_zero_dm
// clears).  Host state only: the next ddx_process_block copies what its kernels need.
void update_active(ddx_plan* p) {
  const int64_t total = p->dm_off[p->C];
  p->rec_pos.assign(total, -1);
  int64_t next = 0;
  for (int i = 0; i < p->C; ++i) {
    Chan& c = p->ch[i];
    const int64_t o = p->dm_off[i];
    for (size_t d = 0; d < c.dm.size(); ++d)
      if (c.active[d]) p->rec_pos[o + d] = (int32_t)(p->compact ? next++ : o + (int64_t)d);
      else if (!p->compact) p->rec_pos[o + d] = (int32_t)(o + d);
  }
  std::vector<int32_t>& slots = p->slots;
  slots.assign(total, 0);
  int32_t k = 0;
  for (Grp& g : p->grp) {
    const Chan& c = p->ch[g.chan];
    const int64_t o = p->dm_off[g.chan];
    g.slot0 = k;
    for (int d : g.dms)
      if (c.active[d]) slots[k++] = p->rec_pos[o + d];
    g.n_active = k - g.slot0;
    for (int d : g.dms)
      if (!c.active[d]) slots[k++] = (int32_t)(o + d);
  }
  p->rec_pairs = p->compact ? next : total;
  p->rec_elems = p->rec_pairs * p->nbl;
}

// Largest number of blocks of class g that one call can run: the history (< N)
// plus the chunk, plus one for rounding.
int64_t max_blocks(const ddx_plan* p, const Grp& g) { return (p->max_block + g.fft_len) / g.valid + 2; }

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

int setup_device(ddx_plan* p) {
  free_device(p);
  build_layout(p);
  int rc;
  int maxn = 0, maxv = 0, maxd = 0;
  int64_t sum_n = 0, spec_elems = 0, spec_one = 0, max_units = 0, max_fwd = 0, max_zero = 0, big_rows = 0;
  for (auto& c : p->ch) maxd = std::max(maxd, (int)c.dm.size());
  for (auto& g : p->grp) {
    maxn = std::max(maxn, g.fft_len);
    maxv = std::max(maxv, g.valid);
    sum_n += g.fft_len;
    const int64_t nb = max_blocks(p, g);
    spec_elems += (int64_t)p->M * nb * g.fft_len;
    spec_one = std::max<int64_t>(spec_one, (int64_t)p->M * nb * g.fft_len);
    max_fwd += nb;
    max_units += nb * (int64_t)g.dms.size();
    max_zero += nb * g.valid / p->L + 1;
    if (g.logn > ddx::kBigLog) big_rows = std::max<int64_t>(big_rows, (int64_t)p->M * g.fft_len);
  }
  p->hist_cap = maxn;
  const size_t ib = in_bytes(p->in_dtype);
  for (int i = 0; i < 2; ++i)
    if ((rc = dev_alloc(p, &p->hist[i], (size_t)p->C * p->M * p->hist_cap * ib))) return rc;
  p->spec_elems = (size_t)std::max(spec_one, std::min(spec_elems, p->spec_budget / (int64_t)sizeof(float2)));
  if ((rc = dev_alloc(p, (void**)&p->spec, p->spec_elems * sizeof(float2)))) return rc;
  // schedule: DM group and wave size
  p->y_stride = maxv;
  const size_t per_unit = (size_t)p->M * p->y_stride * y_bytes(p->corr_dtype);
  p->dm_group = p->group_req ? p->group_req : kDefaultDmGroup;
  p->dm_group = std::max(1, std::min(p->dm_group, maxd));
  if (p->wave_req) {
    p->wave_units = p->wave_req;
  } else {
    p->wave_units = (int)std::max<size_t>(1, std::min<size_t>(1024, kAutoYBytes / std::max<size_t>(per_unit, 1)));
  }
  p->wave_units = (int)std::min<int64_t>(p->wave_units, std::max<int64_t>(max_units, 1));
  // + 256 bytes: the correlator's pair loads may read one sample past a unit's rows
  if ((rc = dev_alloc(p, &p->ybuf, per_unit * p->wave_units + 256))) return rc;
  p->pw_stride = maxv / p->L;
  if (p->corr_dtype != DDX_CORR_F32 &&
      (rc = dev_alloc(p, (void**)&p->power, (size_t)p->wave_units * p->M * p->pw_stride * sizeof(float))))
    return rc;


  if ((rc = dev_alloc(p, (void**)&p->chirp, (size_t)p->wave_units * maxn * sizeof(float2)))) return rc;
  // two-pass transforms: intermediate rows of one wave (dedispersion); the forward
  // transform runs its items in chunks of the same size
  p->tb_elems = (size_t)big_rows * p->wave_units;
  // Waves of a shorter length hold more units in the same buffers: as many as the
  // voltages (rows of the length's largest V), the per-dump power, the chirps (N
  // each) and the two-pass rows allow (a requested wave size is kept as given).
  p->wave_cap.assign(kMaxLogN + 1, 0);
  p->wave_ys.assign(kMaxLogN + 1, 0);
  for (auto& g : p->grp) p->wave_ys[g.logn] = std::max<int64_t>(p->wave_ys[g.logn], g.valid);
  for (int l = 0; l <= kMaxLogN; ++l) {
    const int64_t ys = p->wave_ys[l];
    if (!ys) continue;
    int64_t cap = p->wave_units;
    if (!p->wave_req) {
      const int64_t wu = p->wave_units;
      cap = wu * p->y_stride / ys;
      if (p->power) cap = std::min<int64_t>(cap, wu * p->pw_stride / std::max<int64_t>(1, ys / p->L));
      cap = std::min<int64_t>(cap, wu * maxn / (int64_t(1) << l));
      if (l > ddx::kBigLog) cap = std::min<int64_t>(cap, (int64_t)p->tb_elems / ((int64_t)p->M << l));
      cap = std::max<int64_t>(1, std::min<int64_t>(cap, int64_t(1) << 20));
    }
    p->wave_cap[l] = (int)cap;
  }
  if (p->tb_elems && (rc = dev_alloc(p, (void**)&p->tb, p->tb_elems * sizeof(float2)))) return rc;
  // dump ring
  p->cap_pairs = p->compact && p->max_pairs_req ? p->max_pairs_req : p->dm_off[p->C];
  p->ring_dumps = p->ring_req ? p->ring_req
                              : (p->max_block + p->L - 1) / p->L + (2 * (int64_t)maxn + maxv) / p->L + 4;
  if ((rc = dev_alloc(p, (void**)&p->ring, (size_t)p->ring_dumps * p->cap_pairs * p->nbl * sizeof(float2)))) return rc;
  if (p->corr_dtype == DDX_CORR_F32) {
    if ((rc = dev_alloc(p, (void**)&p->l1, (size_t)max_fwd * p->M * 8 * sizeof(float)))) return rc;
    if ((rc = dev_alloc(p, (void**)&p->bound, (size_t)max_fwd * sizeof(float)))) return rc;
  }
  // work lists of one call
  p->items_cap = align_up(max_fwd * sizeof(ddx::FwdItem)) + align_up(max_units * sizeof(ddx::UnitItem)) +
                 align_up(max_units * sizeof(ddx::ChirpItem)) + align_up(max_zero * sizeof(ddx::ZeroItem)) +
                 align_up(p->dm_off[p->C] * sizeof(int32_t)) + p->C * sizeof(ddx::ScaleItem);
  if ((rc = dev_alloc(p, (void**)&p->items_dev, p->items_cap))) return rc;
  for (int i = 0; i < 2; ++i) {
    if (hipHostMalloc((void**)&p->stage[i], p->items_cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p->stage[i] = nullptr;
      return fail(p, DDX_ENOMEM, "pinned staging of %zu bytes", p->items_cap);
    }
    HIPCHECK(p, hipEventCreateWithFlags(&p->stage_ev[i], hipEventDisableTiming));
  }
  // FP64 tables: g[k] of every class (its channel's frequency, its length)
  std::vector<double> g(sum_n);
  int64_t goff = 0;
  for (Grp& gr : p->grp) {
    const double fc = p->ch[gr.chan].fc;
    const int n = gr.fft_len;
    gr.gtab = goff;
    for (int k = 0; k < n; ++k) {
      const double f = p->sideband * (double)(k < n / 2 ? k : k - n) * (p->fs / n);
      g[goff + k] = (f * f) / (fc * fc * (fc + f));
    }
    goff += n;
  }
  if ((rc = dev_alloc(p, (void**)&p->gtab, g.size() * sizeof(double)))) return rc;
  if ((rc = dev_alloc(p, (void**)&p->scale_dev, p->C * sizeof(float)))) return rc;
  if ((rc = dev_alloc(p, (void**)&p->scale_part, (size_t)p->C * p->M * sizeof(double)))) return rc;
  HIPCHECK(p, hipMemcpy(p->gtab, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHECK(p, hipMemcpy(p->scale_dev, p->lay_scale.data(), p->C * sizeof(float), hipMemcpyHostToDevice));
  if (p->compact) {
    int64_t na = 0;
    for (auto& c : p->ch) for (uint8_t a : c.active) na += a;
    if (na > p->cap_pairs)
      for (auto& c : p->ch) std::fill(c.active.begin(), c.active.end(), 0);  // the caller selects a subset
  }
  update_active(p);
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
  if (d->wave_units < 0 || d->dm_group < 0 || d->max_record_pairs < 0 || d->ring_dumps < 0) return DDX_EINVAL;
  if (d->wave_units > 65535) return DDX_EINVAL;  // the chirp launch takes one grid row per (channel, DM) of a wave
  if (d->compact_records != 0 && d->compact_records != 1) return DDX_EINVAL;
  if (d->dm_classes != 0 && d->dm_classes != 1) return DDX_EINVAL;
  if (d->spectrum_bytes < 0) return DDX_EINVAL;
  if (d->cost_ps)
    for (int i = 0; i < 22; ++i)
      if (!(d->cost_ps[i] > 0) || !std::isfinite(d->cost_ps[i])) return DDX_EINVAL;
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
  p->wave_req = d->wave_units;
  p->group_req = d->dm_group;
  p->compact = d->compact_records;
  p->max_pairs_req = d->max_record_pairs;
  p->ring_req = d->ring_dumps;
  p->classes_req = d->dm_classes;
  p->spec_budget = d->spectrum_bytes ? d->spectrum_bytes : kSpecBudgetBytes;
  for (int i = 0; i < 11; ++i) {
    p->cost_inv[i] = d->cost_ps ? d->cost_ps[i] : kDedispPs[i];
    p->cost_fwd[i] = d->cost_ps ? d->cost_ps[11 + i] : kForwardPs[i];
  }
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
  std::vector<Grp> grp;
  for (int c = 0; c < p->C; ++c) {
    if (p->ch[c].dm.empty()) { all = false; continue; }
    int rc = plan_channel(p, c, grp);
    if (rc) { p->ch = saved; return rc; }
  }
  if (!all) { p->ready = false; return DDX_OK; }
  p->grp = std::move(grp);
  for (auto& c : p->ch) c.grp.clear();
  for (int k = 0; k < (int)p->grp.size(); ++k) {
    Chan& c = p->ch[p->grp[k].chan];
    c.grp.push_back(k);
    c.cover = k;  // classes come in DM order: the last holds the largest DM
    c.win = p->grp[k].fft_len - p->grp[k].lead;
  }
  int rc = setup_device(p);
  p->ready = rc == DDX_OK;
  return rc;
}

int ddx_plan_blocking(const ddx_desc* desc, int32_t chan, const double* dm, int32_t n_dm, int32_t* fft_len,
                      int32_t* valid, int32_t* lead) {
  if (!desc || !dm || n_dm < 1 || !fft_len || !valid || !lead) return DDX_EINVAL;
  if (chan < 0 || chan >= desc->n_chan) return DDX_EINVAL;
  for (int i = 0; i < n_dm; ++i)
    if (!std::isfinite(dm[i]) || dm[i] < 0) return DDX_EINVAL;
  ddx_plan* p = nullptr;
  int rc = ddx_plan_create(desc, &p);
  if (rc) return rc;
  p->ch[chan].dm.assign(dm, dm + n_dm);
  std::vector<Grp> grp;
  rc = plan_channel(p, chan, grp);
  if (rc == DDX_OK) {
    for (const Grp& g : grp)
      for (int d : g.dms) {
        fft_len[d] = g.fft_len;
        valid[d] = g.valid;
        lead[d] = g.lead;
      }
    rc = (int)grp.size();
  }
  delete p;
  return rc;
}

int ddx_set_active_dms(ddx_plan* p, int32_t chan, const uint8_t* mask) {
  if (!p) return DDX_EINVAL;
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials first");
  if (chan < -1 || chan >= p->C) return fail(p, DDX_EINVAL, "channel %d out of range", chan);
  const int c0 = chan < 0 ? 0 : chan, c1 = chan < 0 ? p->C : chan + 1;
  if (p->compact) {
    int64_t done = 0;
    for (auto& g : p->grp) done = std::max(done, g.dumps_done);
    if (done > p->dumps_fetched)
      return fail(p, DDX_ESTATE, "compact records: fetch every dump before changing the active DMs");
    int64_t na = 0;
    for (int c = 0; c < p->C; ++c)
      for (size_t d = 0; d < p->ch[c].dm.size(); ++d)
        na += (c >= c0 && c < c1) ? (mask ? mask[d] != 0 : 1) : p->ch[c].active[d];
    if (na > p->cap_pairs)
      return fail(p, DDX_EINVAL, "%lld active (channel, DM) pairs exceed the record capacity %lld", (long long)na,
                  (long long)p->cap_pairs);
  }
  for (int c = c0; c < c1; ++c)
    for (size_t d = 0; d < p->ch[c].dm.size(); ++d) p->ch[c].active[d] = mask ? (mask[d] != 0) : 1;
  update_active(p);
  return DDX_OK;
}

int ddx_select_active_dms(ddx_plan* p, int32_t chan, const float* d_scores, int32_t k, float logit_threshold,
                          uint8_t* d_mask_out, int32_t* fallback, void* hip_stream) {
  if (!p) return DDX_EINVAL;
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials first");
  if (chan < -1 || chan >= p->C) return fail(p, DDX_EINVAL, "channel %d out of range", chan);
  if (!d_scores || k < 1) return fail(p, DDX_EINVAL, "NULL scores or k = %d < 1", k);
  const int c0 = chan < 0 ? 0 : chan, c1 = chan < 0 ? p->C : chan + 1;
  const int n = (int)p->ch[c0].dm.size();
  for (int c = c0; c < c1; ++c)
    if ((int)p->ch[c].dm.size() != n) return fail(p, DDX_EUNSUPPORTED, "channels hold different DM counts");
  if (n > ddx::kTopkMax) return fail(p, DDX_EUNSUPPORTED, "%d DMs exceed %d", n, ddx::kTopkMax);
  hipStream_t s = (hipStream_t)hip_stream;
  if (!p->sel_dev) {
    const size_t bytes = align_up((size_t)ddx::kTopkMax + sizeof(int32_t));
    int rc = dev_alloc(p, (void**)&p->sel_dev, bytes);
    if (rc) return rc;
    if (hipHostMalloc((void**)&p->sel_host, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p->sel_host = nullptr;
      return fail(p, DDX_ENOMEM, "pinned selection buffer");
    }
  }
  // [mask: n bytes][pad to 4][flag]
  int32_t* flag_dev = reinterpret_cast<int32_t*>(p->sel_dev + ddx::kTopkMax);
  hipLaunchKernelGGL(ddx::k_topk_mask, dim3(1), dim3(1024), 0, s, d_scores, n, k, logit_threshold, p->sel_dev,
                     flag_dev);
  HIPCHECK(p, hipGetLastError());
  if (d_mask_out) HIPCHECK(p, hipMemcpyAsync(d_mask_out, p->sel_dev, n, hipMemcpyDeviceToDevice, s));
  HIPCHECK(p, hipMemcpyAsync(p->sel_host, p->sel_dev, ddx::kTopkMax + sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(p, hipStreamSynchronize(s));
  const int32_t above = *reinterpret_cast<const int32_t*>(p->sel_host + ddx::kTopkMax);
  if (fallback) *fallback = above > k ? 1 : 0;
  return ddx_set_active_dms(p, chan, p->sel_host);
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
  o->record_pos = p->rec_pos.data();
  o->record_pairs = p->rec_pairs;
  o->record_elems = p->rec_elems;
  o->samples_in = p->recv;
  int64_t ready = INT64_MAX;
  for (auto& g : p->grp) ready = std::min(ready, g.dumps_done);
  o->dumps_ready = ready;
  o->dumps_fetched = p->dumps_fetched;
  o->ring_dumps = p->ring_dumps;
  o->device_bytes = p->dev_bytes;
  o->wave_units = p->wave_units;
  o->dm_group = p->dm_group;
  o->compact_records = p->compact;
  o->dump_t0_s = 0.5 * (double)(p->L - 1) / p->fs;
  o->dump_period_s = (double)p->L / p->fs;
  o->dm_fft_len = p->lay_dm_fft.data();
  o->dm_valid = p->lay_dm_valid.data();
  o->dm_lead = p->lay_dm_lead.data();
  o->n_classes = (int32_t)p->grp.size();
  return DDX_OK;
}

int ddx_dump_times(const ddx_plan* pc, int32_t chan, int32_t dm_index, int64_t first_dump, int64_t n_dumps,
                   int32_t refer_infinite, double* out) {
  if (!pc) return DDX_EINVAL;
  ddx_plan* p = const_cast<ddx_plan*>(pc);
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials for every channel first");
  if (chan < 0 || chan >= p->C) return fail(p, DDX_EINVAL, "channel %d outside [0, %d)", chan, p->C);
  const int nd = (int)p->ch[chan].dm.size();
  if (dm_index < 0 || dm_index >= nd) return fail(p, DDX_EINVAL, "DM index %d outside [0, %d)", dm_index, nd);
  if (first_dump < 0 || n_dumps < 0) return fail(p, DDX_EINVAL, "negative dump range");
  if (n_dumps > 0 && !out) return fail(p, DDX_EINVAL, "null output");
  const double delay = refer_infinite ? p->lay_delay[p->dm_off[chan] + dm_index] : 0.0;
  for (int64_t i = 0; i < n_dumps; ++i) {
    const double m = (double)(first_dump + i);
    out[i] = (m * p->L + 0.5 * (p->L - 1)) / p->fs - delay;
  }
  return DDX_OK;
}

}  // extern "C"

namespace {

// One call's work lists (see ddx_process_block in ddx.h).
// Classes whose spectra share the spectrum buffer at one time: a call runs its
// batches in turn, each its forward transforms, then its waves.
struct Batch {
  size_t l0, nl;  // forward launches [l0, l0 + nl)
  size_t f0, nf;  // forward items [f0, f0 + nf)
  size_t w0, nw;  // waves [w0, w0 + nw)
};
struct CallLists {
  std::vector<ddx::FwdItem> fwd;
  std::vector<FwdLaunch> fwd_launch;
  std::vector<ddx::UnitItem> units;
  std::vector<ddx::ChirpItem> chirps;
  std::vector<Wave> waves;
  std::vector<Batch> batches;
  std::vector<ddx::ZeroItem> zeros;
  std::vector<ddx::ScaleItem> scales;
};

// Build the lists for blocks [blocks_done, b_end[k]) of every class k; out_end[k] is
// the end of the class's output this call (complete dumps only are correlated).
// Classes run in (transform length, class) order, cut into batches whose spectra
// fit the spectrum buffer.
void build_lists(ddx_plan* p, const std::vector<int64_t>& b_end, const std::vector<int64_t>& out_end, CallLists& w) {
  const int M = p->M;
  const int G = (int)p->grp.size();
  std::vector<int> run;
  for (int k = 0; k < G; ++k)  // classes with no active DM need no transforms
    if (b_end[k] > p->grp[k].blocks_done && p->grp[k].n_active > 0) run.push_back(k);
  std::stable_sort(run.begin(), run.end(), [&](int x, int y) { return p->grp[x].logn < p->grp[y].logn; });
  std::vector<int32_t> slot_of(p->dm_off[p->C], -1);
  std::vector<int64_t> slot_wave(p->dm_off[p->C], -1);
  std::vector<int64_t> spec_wave;
  std::vector<size_t> fwd_first(G, 0);
  size_t r0 = 0;
  while (r0 < run.size()) {
    // the batch: classes run[r0, r1) whose spectra fit the buffer (at least one)
    size_t r1 = r0;
    int64_t need = 0;
    while (r1 < run.size()) {
      const Grp& g = p->grp[run[r1]];
      const int64_t n = (b_end[run[r1]] - g.blocks_done) * (int64_t)M * g.fft_len;
      if (r1 > r0 && need + n > (int64_t)p->spec_elems) break;
      need += n;
      ++r1;
    }
    Batch bt{w.fwd_launch.size(), 0, w.fwd.size(), 0, w.waves.size(), 0};
    // forward items and spectrum offsets (from the buffer's start): length, class,
    // block.  Two-pass lengths run in chunks of `chunk` items whose intermediate
    // rows start at offset 0.
    int64_t off = 0;
    for (size_t r = r0; r < r1;) {
      const int logn = p->grp[run[r]].logn;
      FwdLaunch fl{logn, w.fwd.size(), 0};
      const size_t per = (size_t)M << logn;
      const size_t chunk = logn > ddx::kBigLog ? std::max<size_t>(1, p->tb_elems / per) : 1;
      for (; r < r1 && p->grp[run[r]].logn == logn; ++r) {
        const int k = run[r];
        const Grp& g = p->grp[k];
        fwd_first[k] = w.fwd.size();
        for (int64_t b = g.blocks_done; b < b_end[k]; ++b) {
          ddx::FwdItem it{};
          it.win0 = b * (int64_t)g.valid - g.lead;
          it.spec = off;
          it.tb = logn > ddx::kBigLog ? (int64_t)(((w.fwd.size() - fl.i0) % chunk) * per) : 0;
          it.hist_start = p->ch[g.chan].hist_start;
          it.chan = g.chan;
          it.logn = logn;
          w.fwd.push_back(it);
          off += (int64_t)per;
        }
      }
      fl.n = w.fwd.size() - fl.i0;
      w.fwd_launch.push_back(fl);
    }
    spec_wave.resize(w.fwd.size(), -1);
    // units: length, class, DM group, block, DM; waves of wave_units within a length
    for (size_t r = r0; r < r1;) {
      const int logn = p->grp[run[r]].logn;
      Wave cur{};
      bool open = false;
      auto close = [&]() {
        if (open && cur.nu) w.waves.push_back(cur);
        open = false;
      };
      for (; r < r1 && p->grp[run[r]].logn == logn; ++r) {
        const int k = run[r];
        const Grp& g = p->grp[k];
        const int i = g.chan;
        const Chan& c = p->ch[i];
        // the class's active DMs, in DM index order
        std::vector<int> act;
        for (int d : g.dms)
          if (c.active[d]) act.push_back(d);
        for (size_t g0 = 0; g0 < act.size(); g0 += p->dm_group) {
          const size_t g1 = std::min(act.size(), g0 + p->dm_group);
          for (int64_t b = g.blocks_done; b < b_end[k]; ++b) {
            const int64_t first = b * g.valid / p->L;
            const int64_t last = std::min(b * g.valid + g.valid, out_end[k]) / p->L;
            if (last <= first) continue;
            for (size_t q = g0; q < g1; ++q) {
              const int d = act[q];
              if (!open || cur.nu == (size_t)p->wave_cap[logn]) {
                close();
                cur = Wave{};
                cur.logn = logn;
                cur.u0 = w.units.size();
                cur.c0 = w.chirps.size();
                cur.fft_n = g.fft_len;
                cur.y_stride = p->wave_ys[logn];
                open = true;
              }
              const int64_t wid = (int64_t)w.waves.size();
              const int64_t pair = p->dm_off[i] + d;
              if (slot_wave[pair] != wid) {
                slot_wave[pair] = wid;
                slot_of[pair] = (int32_t)cur.nc;
                ddx::ChirpItem ci{};
                ci.g = g.gtab;
                ci.out = (int64_t)cur.nc * g.fft_len;
                ci.kdm = p->kdm * c.dm[d];
                ci.n = g.fft_len;
                ci.logr = g.logn > ddx::kBigLog ? g.logn - ddx::kBigLog : 0;
                ci.chan = i;
                w.chirps.push_back(ci);
                ++cur.nc;
              }
              const size_t sidx = fwd_first[k] + (size_t)(b - g.blocks_done);
              if (spec_wave[sidx] != wid) { spec_wave[sidx] = wid; ++cur.spectra; }
              ddx::UnitItem u{};
              u.spec = w.fwd[sidx].spec;
              u.chirp = (int64_t)slot_of[pair] * g.fft_len;
              u.y = (int64_t)cur.nu * M * cur.y_stride;
              u.tb = (int64_t)cur.nu * M * g.fft_len;
              u.dump0 = first;
              u.rec = (int64_t)p->rec_pos[pair] * p->nbl;
              u.chan = i;
              u.valid = g.valid;
              u.lead = g.lead;
              u.n_dumps = (int32_t)(last - first);
              u.fwd = (int32_t)sidx;
              w.units.push_back(u);
              ++cur.nu;
              cur.max_dumps = std::max(cur.max_dumps, u.n_dumps);
              cur.y_samples += (int64_t)M * g.valid;
              cur.dumps += u.n_dumps;
            }
          }
        }
      }
      close();
    }
    bt.nl = w.fwd_launch.size() - bt.l0;
    bt.nf = w.fwd.size() - bt.f0;
    bt.nw = w.waves.size() - bt.w0;
    w.batches.push_back(bt);
    r0 = r1;
  }
  // full records: zero the inactive DMs' slots of every dump a class completes
  if (!p->compact) {
    for (int k = 0; k < G; ++k) {
      const Grp& g = p->grp[k];
      const int n_in = (int)g.dms.size() - g.n_active;
      if (n_in <= 0) continue;
      const int64_t m0 = g.blocks_done * g.valid / p->L, m1 = out_end[k] / p->L;
      for (int64_t m = m0; m < m1; ++m) {
        ddx::ZeroItem z{};
        z.rec = (m % p->ring_dumps) * p->rec_elems;
        z.pos = g.slot0 + g.n_active;
        z.n = n_in;
        w.zeros.push_back(z);
      }
    }
  }
}

// Copy the lists into the pinned staging buffer and on to the device (stream
// ordered: the previous call's kernels have read the device copy before this
// copy overwrites it).  Returns the device addresses of the four lists.
int upload_lists(ddx_plan* p, const CallLists& w, hipStream_t s, ddx::FwdItem** fwd, ddx::UnitItem** units,
                 ddx::ChirpItem** chirps, ddx::ZeroItem** zeros, int32_t** slots, ddx::ScaleItem** scales) {
  const size_t o1 = align_up(w.fwd.size() * sizeof(ddx::FwdItem));
  const size_t o2 = o1 + align_up(w.units.size() * sizeof(ddx::UnitItem));
  const size_t o3 = o2 + align_up(w.chirps.size() * sizeof(ddx::ChirpItem));
  const size_t o4 = o3 + align_up(w.zeros.size() * sizeof(ddx::ZeroItem));
  const size_t n_slots = w.zeros.empty() ? 0 : p->slots.size();
  const size_t o5 = o4 + align_up(n_slots * sizeof(int32_t));
  const size_t bytes = o5 + w.scales.size() * sizeof(ddx::ScaleItem);
  if (bytes > p->items_cap) return fail(p, DDX_EINVAL, "internal: work lists of %zu bytes exceed %zu", bytes, p->items_cap);
  const int k = p->stage_cur;
  if (p->stage_used[k]) HIPCHECK(p, hipEventSynchronize(p->stage_ev[k]));
  char* h = p->stage[k];
  if (!w.fwd.empty()) std::memcpy(h, w.fwd.data(), w.fwd.size() * sizeof(ddx::FwdItem));
  if (!w.units.empty()) std::memcpy(h + o1, w.units.data(), w.units.size() * sizeof(ddx::UnitItem));
  if (!w.chirps.empty()) std::memcpy(h + o2, w.chirps.data(), w.chirps.size() * sizeof(ddx::ChirpItem));
  if (!w.zeros.empty()) std::memcpy(h + o3, w.zeros.data(), w.zeros.size() * sizeof(ddx::ZeroItem));
  if (n_slots) std::memcpy(h + o4, p->slots.data(), n_slots * sizeof(int32_t));
  if (!w.scales.empty()) std::memcpy(h + o5, w.scales.data(), w.scales.size() * sizeof(ddx::ScaleItem));
  if (bytes) HIPCHECK(p, hipMemcpyAsync(p->items_dev, h, bytes, hipMemcpyHostToDevice, s));
  HIPCHECK(p, hipEventRecord(p->stage_ev[k], s));
  p->stage_used[k] = true;
  p->stage_cur = 1 - k;
  *fwd = reinterpret_cast<ddx::FwdItem*>(p->items_dev);
  *units = reinterpret_cast<ddx::UnitItem*>(p->items_dev + o1);
  *chirps = reinterpret_cast<ddx::ChirpItem*>(p->items_dev + o2);
  *zeros = reinterpret_cast<ddx::ZeroItem*>(p->items_dev + o3);
  *slots = reinterpret_cast<int32_t*>(p->items_dev + o4);
  *scales = reinterpret_cast<ddx::ScaleItem*>(p->items_dev + o5);
  return DDX_OK;
}

}  // namespace

extern "C" {

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

  // Blocks each class can run now, and the dumps they complete.  A channel's
  // classes start once its scale window [0, win) is in (or at the flush), so the
  // scale rule sees the same samples however the classes are cut.
  const int G = (int)p->grp.size();
  std::vector<int64_t> b_end(G), dumps_new(G), out_end(G);
  const int64_t fetched_floor = p->dumps_fetched;
  for (int k = 0; k < G; ++k) {
    Grp& g = p->grp[k];
    int64_t be;
    if (flush) {
      be = (total + g.valid - 1) / g.valid;
    } else if (total < p->ch[g.chan].win) {
      be = 0;
    } else {
      const int64_t lim = total - g.fft_len + g.lead;  // b V <= lim
      be = lim < 0 ? 0 : lim / g.valid + 1;
    }
    be = std::max(be, g.blocks_done);
    b_end[k] = be;
    out_end[k] = be * (int64_t)g.valid;
    if (flush) out_end[k] = std::min(out_end[k], total);
    dumps_new[k] = std::max(g.dumps_done, out_end[k] / p->L);
    if (dumps_new[k] - fetched_floor > p->ring_dumps)
      return fail(p, DDX_EFULL, "channel %d would hold %lld unfetched dumps, ring has %lld", g.chan,
                  (long long)(dumps_new[k] - fetched_floor), (long long)p->ring_dumps);
    if (be - g.blocks_done > max_blocks(p, g))
      return fail(p, DDX_EINVAL, "internal: %lld blocks exceed the spectrum buffer", (long long)(be - g.blocks_done));
  }
  if (p->started && p->last_stream != s) HIPCHECK(p, hipStreamSynchronize(p->last_stream));
  p->started = true;
  p->last_stream = s;

  CallLists w;
  build_lists(p, b_end, out_end, w);
  // correlator-input scale of each channel whose first blocks run now (window [0, win))
  std::vector<uint8_t> runs(p->C, 0);
  for (int k = 0; k < G; ++k)
    if (b_end[k] > p->grp[k].blocks_done) runs[p->grp[k].chan] = 1;
  if (!p->have_scale)
    for (int i = 0; i < p->C; ++i) {
      Chan& c = p->ch[i];
      if (!runs[i] || c.scaled) continue;
      ddx::ScaleItem si{};
      si.n = std::min<int64_t>(c.win, total);
      si.hist_start = c.hist_start;
      si.chan = i;
      w.scales.push_back(si);
    }
  ddx::FwdItem* fwd_dev;
  ddx::UnitItem* units_dev;
  ddx::ChirpItem* chirps_dev;
  ddx::ZeroItem* zeros_dev;
  int32_t* slots_dev;
  ddx::ScaleItem* scales_dev;
  int rc = upload_lists(p, w, s, &fwd_dev, &units_dev, &chirps_dev, &zeros_dev, &slots_dev, &scales_dev);
  if (rc) return rc;

  ddx::Source src{};
  src.chunk = d_volts;
  src.hist = p->hist[p->hist_cur];
  src.chunk_stride = n;
  src.hist_cap = p->hist_cap;
  src.chunk_start = p->recv;
  src.chunk_len = n;

  if (!w.scales.empty()) {
    const float target = p->corr_dtype == DDX_CORR_E4M3 ? kScaleTargetE4M3 : kScaleTargetF16;  // F32 too
    double bytes = 0;
    for (auto& si : w.scales) bytes += (double)si.n * p->M * in_bytes(p->in_dtype);
    const int ns = (int)w.scales.size();
    HIPCHECK(p, timed(p, s, DDX_K_OTHER, 0.0, bytes, [&] {
      if (p->in_dtype == DDX_IN_CI8)
        hipLaunchKernelGGL(ddx::k_scale_part<0>, dim3(ns * p->M), dim3(256), 0, s, src,
                           (const ddx::ScaleItem*)scales_dev, p->M, p->scale_part);
      else
        hipLaunchKernelGGL(ddx::k_scale_part<1>, dim3(ns * p->M), dim3(256), 0, s, src,
                           (const ddx::ScaleItem*)scales_dev, p->M, p->scale_part);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(ddx::k_scale_final, dim3(ns), dim3(64), 0, s, (const ddx::ScaleItem*)scales_dev,
                         (const double*)p->scale_part, p->M, target, p->scale_dev);
      return hipGetLastError();
    }));
    p->scale_pending = true;
  }

  // batch by batch: forward transforms, one launch per transform length (two-pass
  // lengths in chunks that fit the intermediate buffer), the blocks' bounds, the waves
  ddx::FwdArgs fa{};
  fa.src = src;
  fa.spec = p->spec;
  fa.n_ant = p->M;
  const double nbl_h = p->M * (p->M + 1) / 2.0;
  for (const Batch& bt : w.batches) {
  for (size_t li = bt.l0; li < bt.l0 + bt.nl; ++li) {
    const FwdLaunch& fl = w.fwd_launch[li];
    const double nn = 1 << fl.logn;
    if (fl.logn <= ddx::kBigLog) {
      fa.items = fwd_dev + fl.i0;
      fa.l1 = p->l1 ? p->l1 + fl.i0 * p->M * 8 : nullptr;
      HIPCHECK(p, timed(p, s, DDX_K_FORWARD, (double)fl.n * p->M * fft_flops(nn),
                        (double)fl.n * p->M * nn * (in_bytes(p->in_dtype) + 8.0),
                        [&] { return launch_forward(fl.logn, p->in_dtype, fa, (int)fl.n, s); }));
    } else {
      const size_t per = (size_t)p->M << fl.logn;
      const size_t chunk = std::max<size_t>(1, p->tb_elems / per);
      for (size_t i0 = 0; i0 < fl.n; i0 += chunk) {
        // the chunk's spectra are consecutive and its intermediate rows start at 0
        const size_t cnt = std::min(chunk, fl.n - i0);
        const std::vector<ddx::FwdItem>& fv = w.fwd;
        fa.items = fwd_dev + fl.i0 + i0;
        fa.l1 = p->l1 ? p->l1 + (fl.i0 + i0) * p->M * 8 : nullptr;
        HIPCHECK(p, timed(p, s, DDX_K_FORWARD, (double)cnt * p->M * fft_flops(nn),
                          (double)cnt * p->M * nn * (in_bytes(p->in_dtype) + 8.0),
                          [&] { return launch_forward_big(fl.logn, p->in_dtype, fa, &fv[fl.i0 + i0], (int)cnt, p->tb, s); }));
      }
    }
  }

  if (p->bound && bt.nf) {  // FP32 correlator inputs: each block's bound on |y|
    HIPCHECK(p, timed(p, s, DDX_K_OTHER, 0.0, (double)bt.nf * p->M * 32.0, [&] {
      hipLaunchKernelGGL(ddx::k_item_bound, dim3((unsigned)bt.nf), dim3(256), 0, s,
                         (const ddx::FwdItem*)(fwd_dev + bt.f0), (const float*)(p->l1 + bt.f0 * p->M * 8), p->M,
                         p->bound + bt.f0);
      return hipGetLastError();
    }));
  }

  // waves: chirps, dedispersion, correlation.  (A second stream for the correlator,
  // overlapping it with the next wave's dedispersion, measured no faster: both
  // kernels are limited by the same memory system.)
  for (size_t wi = bt.w0; wi < bt.w0 + bt.nw; ++wi) {
    const Wave& wv = w.waves[wi];
    const double nn = wv.fft_n;
    HIPCHECK(p, timed(p, s, DDX_K_CHIRP, 0.0, (double)wv.nc * nn * 16.0, [&] {
      hipLaunchKernelGGL(ddx::k_chirp, dim3((unsigned)((wv.fft_n + 255) / 256), (unsigned)wv.nc), dim3(256), 0, s,
                         (const ddx::ChirpItem*)(chirps_dev + wv.c0), (const double*)p->gtab,
                         (const float*)p->scale_dev, p->chirp);
      return hipGetLastError();
    }));
    ddx::DedispArgs da{};
    da.spec = p->spec;
    da.chirp = p->chirp;
    da.y = p->ybuf;
    da.tb = p->tb;
    da.units = units_dev + wv.u0;
    da.power = p->power;
    da.dump_len = p->L;
    da.pw_stride = (int32_t)(wv.y_stride / p->L);
    da.y_stride = wv.y_stride;
    da.n_ant = p->M;
    da.n_units = (int)wv.nu;
    da.logr = wv.logn > ddx::kBigLog ? wv.logn - ddx::kBigLog : 0;
    da.tile = ddx::unit_tile(da.n_units);
    HIPCHECK(p, timed(p, s, DDX_K_DEDISP, (double)wv.nu * p->M * (fft_flops(nn) + 6.0 * nn),
                      8.0 * nn * ((double)wv.nu * p->M + wv.nc) + (double)wv.y_samples * y_bytes(p->corr_dtype),
                      [&] { return launch_dedisp(wv.logn, p->corr_dtype, da, s); }));
    ddx::CorrArgs ca{};
    ca.y = p->ybuf;
    ca.ring = p->ring;
    ca.units = units_dev + wv.u0;
    ca.scale = p->scale_dev;
    ca.power = p->power;
    ca.bound = p->bound;
    ca.pw_stride = (int32_t)(wv.y_stride / p->L);
    ca.y_stride = wv.y_stride;
    ca.rec_elems = p->rec_elems;
    ca.ring_dumps = p->ring_dumps;
    ca.max_dumps = wv.max_dumps;
    ca.n_ant = p->M;
    ca.dump_len = p->L;
    ca.nbl = p->nbl;
    ca.out_mode = p->out_mode;
    HIPCHECK(p, timed(p, s, DDX_K_CORR, (double)wv.dumps * 8.0 * p->L * nbl_h,
                      (double)wv.dumps * ((double)p->L * p->M * y_bytes(p->corr_dtype) + 8.0 * p->nbl),
                      [&] { return launch_corr(p->corr_dtype, ca, (int)wv.nu, s); }));
  }
  }
  if (!w.zeros.empty()) {
    HIPCHECK(p, timed(p, s, DDX_K_OTHER, 0.0, 8.0 * (double)w.zeros.size() * w.zeros[0].n * p->nbl, [&] {
      hipLaunchKernelGGL(ddx::k_zero_dm, dim3((unsigned)w.zeros.size()), dim3(256), 0, s, p->ring,
                         (const ddx::ZeroItem*)zeros_dev, (const int32_t*)slots_dev, p->nbl);
      return hipGetLastError();
    }));
  }

  // Carry the unconsumed tail of every row into the other history buffer: from the
  // earliest sample any class of the channel still needs.
  if (!flush) {
    void* dst = p->hist[1 - p->hist_cur];
    std::vector<int64_t> need(p->C, INT64_MAX);
    for (int k = 0; k < G; ++k) {
      const Grp& g = p->grp[k];
      need[g.chan] = std::min(need[g.chan], std::max<int64_t>(0, b_end[k] * g.valid - g.lead));
    }
    for (int i = 0; i < p->C; ++i) {
      Chan& c = p->ch[i];
      const int64_t start = need[i];
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
  for (int k = 0; k < G; ++k) {
    p->grp[k].blocks_done = b_end[k];
    p->grp[k].dumps_done = dumps_new[k];
  }
  for (int i = 0; i < p->C; ++i)
    if (runs[i]) p->ch[i].scaled = true;
  p->recv = total;
  if (flush) p->flushed = true;
  return DDX_OK;
}

int ddx_fetch_visibilities(ddx_plan* p, void* out, size_t cap, int64_t* first, int64_t* nd, void* hip_stream) {
  if (!p || !first || !nd) return DDX_EINVAL;
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials for every channel first");
  int64_t ready = INT64_MAX;
  for (auto& g : p->grp) ready = std::min(ready, g.dumps_done);
  const int64_t avail = ready - p->dumps_fetched;
  *first = p->dumps_fetched;
  *nd = avail;
  if (avail == 0) return DDX_OK;
  const size_t rec = (size_t)p->rec_elems * sizeof(float2);
  if (cap < rec * (size_t)avail) return fail(p, DDX_ESIZE, "need %zu bytes for %lld dumps", rec * avail, (long long)avail);
  if (!out) return fail(p, DDX_EINVAL, "null output");
  hipStream_t s = (hipStream_t)hip_stream;
  int64_t k = 0;
  while (k < avail && rec > 0) {
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
  if ((int)p->ch[0].dm.size() > 65535) return fail(p, DDX_EUNSUPPORTED, "tiles take at most 65535 DM trials");
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
  if ((int64_t)n_tiles * p->C > 65535)  // the scans' grids take one y index per (tile, channel) row
    return fail(p, DDX_EINVAL, "n_tiles x channels must be at most 65535");
  return tiles_from_rows(p, d_power, n_tiles, units, fine, bin_len, n_bins, d_tiles, (hipStream_t)hip_stream);
}

int ddx_reset_stream(ddx_plan* p) {
  if (!p) return DDX_EINVAL;
  if (!p->ready) return fail(p, DDX_ESTATE, "set DM trials for every channel first");
  if (p->started) HIPCHECK(p, hipStreamSynchronize(p->last_stream));
  for (auto& c : p->ch) {
    c.scaled = false;
    c.hist_start = 0;
  }
  for (auto& g : p->grp) {
    g.blocks_done = 0;
    g.dumps_done = 0;
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
