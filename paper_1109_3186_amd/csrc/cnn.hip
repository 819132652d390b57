// Host side of the DM-proposal network (ddx_cnn_* in ddx.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ddx.h"
#include "cnn_kernels.hpp"

namespace {

constexpr int kW = ddx::kCnnW, kK = ddx::kCnnK;
// flat parameter layout: W1 [32][3][9], b1, W2 [32][32][9], b2, W3, b3, W4, b4, w5 [32], b5 [1]
constexpr int64_t kNW1 = kW * 3 * kK, kNW = kW * kW * kK;
constexpr int64_t kOffW[4] = {0, kNW1 + kW, kNW1 + kW + kNW + kW, kNW1 + kW + 2 * (kNW + kW)};
constexpr int64_t kOffB[4] = {kNW1, kNW1 + kW + kNW, kNW1 + kW + 2 * kNW + kW, kNW1 + kW + 3 * kNW + 2 * kW};
constexpr int64_t kOffW5 = kNW1 + kW + 3 * (kNW + kW);
constexpr int64_t kOffB5 = kOffW5 + kW;
constexpr int64_t kNParams = kOffB5 + 1;
constexpr int kChunks = 256;  // row chunks of the weight-gradient reduction
constexpr int64_t kMaxRows = 65535;  // the convolutions' grids take one y index per row

}  // namespace

struct ddx_cnn {
  int n_dm = 0, n_bins = 0, max_tiles = 0;
  int64_t rows_max = 0;
  std::vector<void*> allocs;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  float *stats = nullptr, *h[4] = {nullptr, nullptr, nullptr, nullptr}, *gh[4] = {nullptr, nullptr, nullptr, nullptr};
  float *g = nullptr, *ds = nullptr, *part = nullptr, *partb = nullptr;
  int32_t* arg = nullptr;
  int precision = DDX_CNN_FP32;
  _Float16* wh = nullptr;  // binary16 weights of the FP16 form (k_cnn_weights_h)
  float* wscale = nullptr;  // their per-layer powers of two
  // state of the last forward
  const float* tiles = nullptr;
  float* scores = nullptr;
  int rows = 0;
  bool have_forward = false, have_loss = false;
  int64_t step = 0;
  std::string err;
};

namespace {

int cfail(ddx_cnn* n, int code, const char* fmt, ...) {
  if (n) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    n->err = buf;
  }
  return code;
}

#define CCHECK(n, call)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return cfail(n, DDX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

int calloc_dev(ddx_cnn* n, void** p, size_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 256) != hipSuccess) {
    (void)hipGetLastError();
    return cfail(n, DDX_ENOMEM, "hipMalloc(%zu) failed", bytes);
  }
  n->allocs.push_back(*p);
  return DDX_OK;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

int ddx_cnn_num_params(int64_t* n) {
  if (!n) return DDX_EINVAL;
  *n = kNParams;
  return DDX_OK;
}

int ddx_cnn_create(int32_t n_dm, int32_t n_bins, int32_t max_tiles, ddx_cnn** out) {
  if (!out || n_dm < 1 || max_tiles < 1 || n_bins < 64 || n_bins % 64 != 0) return DDX_EINVAL;
  if ((int64_t)n_dm * max_tiles > kMaxRows) return DDX_EINVAL;  // one grid row per DM row
  ddx_cnn* n = new (std::nothrow) ddx_cnn;
  if (!n) return DDX_ENOMEM;
  n->n_dm = n_dm;
  n->n_bins = n_bins;
  n->max_tiles = max_tiles;
  n->rows_max = (int64_t)n_dm * max_tiles;
  const int64_t R = n->rows_max;
  int rc = 0;
  rc |= calloc_dev(n, (void**)&n->params, kNParams * 4);
  rc |= calloc_dev(n, (void**)&n->grads, kNParams * 4);
  rc |= calloc_dev(n, (void**)&n->m, kNParams * 4);
  rc |= calloc_dev(n, (void**)&n->v, kNParams * 4);
  rc |= calloc_dev(n, (void**)&n->stats, 2 * max_tiles * 4);
  for (int l = 0; l < 4; ++l) {
    const int64_t len = n_bins >> (l == 0 ? 0 : l);
    rc |= calloc_dev(n, (void**)&n->h[l], R * kW * len * 4);
    rc |= calloc_dev(n, (void**)&n->gh[l], R * kW * len * 4);
  }
  rc |= calloc_dev(n, (void**)&n->g, R * kW * 4);
  rc |= calloc_dev(n, (void**)&n->arg, R * kW * 4);
  rc |= calloc_dev(n, (void**)&n->ds, R * 4);
  rc |= calloc_dev(n, (void**)&n->part, (size_t)kChunks * kNW * 4);
  rc |= calloc_dev(n, (void**)&n->partb, (size_t)kChunks * kW * 4);
  rc |= calloc_dev(n, (void**)&n->wh, (size_t)ddx::kCnnHalfTotal * sizeof(_Float16));
  rc |= calloc_dev(n, (void**)&n->wscale, 4 * sizeof(float));
  if (rc) {
    for (void* a : n->allocs) (void)hipFree(a);
    delete n;
    return DDX_ENOMEM;
  }
  if (hipMemset(n->m, 0, kNParams * 4) != hipSuccess || hipMemset(n->v, 0, kNParams * 4) != hipSuccess ||
      hipMemset(n->params, 0, kNParams * 4) != hipSuccess) {
    for (void* a : n->allocs) (void)hipFree(a);
    delete n;
    return DDX_EDEVICE;
  }
  *out = n;
  return DDX_OK;
}

int ddx_cnn_set_weights(ddx_cnn* n, const float* host, int64_t count) {
  if (!n || !host || count != kNParams) return cfail(n, DDX_EINVAL, "need %lld parameters", (long long)kNParams);
  CCHECK(n, hipMemcpy(n->params, host, kNParams * 4, hipMemcpyHostToDevice));
  CCHECK(n, hipMemset(n->m, 0, kNParams * 4));
  CCHECK(n, hipMemset(n->v, 0, kNParams * 4));
  n->step = 0;
  return DDX_OK;
}

int ddx_cnn_get_weights(ddx_cnn* n, float* host, int64_t count) {
  if (!n || !host || count != kNParams) return cfail(n, DDX_EINVAL, "need %lld parameters", (long long)kNParams);
  CCHECK(n, hipDeviceSynchronize());
  CCHECK(n, hipMemcpy(host, n->params, kNParams * 4, hipMemcpyDeviceToHost));
  return DDX_OK;
}

int ddx_cnn_set_precision(ddx_cnn* n, int32_t precision) {
  if (!n) return DDX_EINVAL;
  if (precision != DDX_CNN_FP32 && precision != DDX_CNN_FP16)
    return cfail(n, DDX_EINVAL, "precision must be DDX_CNN_FP32 or DDX_CNN_FP16");
  n->precision = precision;
  n->have_forward = n->have_loss = false;  // a backward pass follows a forward pass of its own precision
  return DDX_OK;
}

int ddx_cnn_get_grads(ddx_cnn* n, float* host, int64_t count) {
  if (!n || !host || count != kNParams) return cfail(n, DDX_EINVAL, "need %lld parameters", (long long)kNParams);
  CCHECK(n, hipDeviceSynchronize());
  CCHECK(n, hipMemcpy(host, n->grads, kNParams * 4, hipMemcpyDeviceToHost));
  return DDX_OK;
}

int ddx_cnn_get_activations(ddx_cnn* n, int32_t layer, float* host, int64_t count) {
  if (!n) return DDX_EINVAL;
  if (!n->have_forward) return cfail(n, DDX_ESTATE, "run ddx_cnn_forward first");
  if (layer < 1 || layer > 4 || !host) return cfail(n, DDX_EINVAL, "layer must be 1..4 and the buffer non-null");
  const int64_t need = (int64_t)n->rows * kW * (n->n_bins >> (layer - 1));
  if (count != need) return cfail(n, DDX_EINVAL, "layer %d holds %lld values", layer, (long long)need);
  CCHECK(n, hipDeviceSynchronize());
  CCHECK(n, hipMemcpy(host, n->h[layer - 1], need * 4, hipMemcpyDeviceToHost));
  return DDX_OK;
}

int ddx_cnn_forward(ddx_cnn* n, const float* tiles, int32_t n_tiles, float* scores, void* stream) {
  if (!n) return DDX_EINVAL;
  if (!tiles || !scores || n_tiles < 1 || n_tiles > n->max_tiles)
    return cfail(n, DDX_EINVAL, "need 1..%d tiles and device buffers", n->max_tiles);
  hipStream_t s = (hipStream_t)stream;
  const int R = n_tiles * n->n_dm, L = n->n_bins;
  hipLaunchKernelGGL(ddx::k_tile_stats, dim3(n_tiles), dim3(1024), 0, s, tiles, (int64_t)n->n_dm * L, n->stats);
  CCHECK(n, hipGetLastError());
  const float* p = n->params;
  const bool h16 = n->precision == DDX_CNN_FP16;
  if (h16) {
    hipLaunchKernelGGL(ddx::k_cnn_weights_h, dim3(4), dim3(256), 0, s, p, kOffW[0], kOffW[1], kOffW[2], kOffW[3],
                       n->wh, n->wscale);
    CCHECK(n, hipGetLastError());
    hipLaunchKernelGGL((ddx::k_conv_fwd_h<3, 1, true>), dim3(L / 64, R), dim3(256), 0, s, tiles, n->stats, n->n_dm,
                       L, n->wh + ddx::kCnnHalfOff[0], n->wscale, p + kOffB[0], n->h[0]);
  } else {
    hipLaunchKernelGGL((ddx::k_conv_fwd<3, 1, true>), dim3(L / 64, R), dim3(256), 0, s, tiles, n->stats, n->n_dm, L,
                       p + kOffW[0], p + kOffB[0], n->h[0]);
  }
  CCHECK(n, hipGetLastError());
  int lin = L;
  for (int l = 1; l < 4; ++l) {
    const int lout = lin / 2;
    if (h16)
      hipLaunchKernelGGL((ddx::k_conv_fwd_h<kW, 2, false>), dim3((lout + 63) / 64, R), dim3(256), 0, s, n->h[l - 1],
                         n->stats, n->n_dm, lin, n->wh + ddx::kCnnHalfOff[l], n->wscale + l, p + kOffB[l], n->h[l]);
    else
      hipLaunchKernelGGL((ddx::k_conv_fwd<kW, 2, false>), dim3((lout + 63) / 64, R), dim3(256), 0, s, n->h[l - 1],
                         n->stats, n->n_dm, lin, p + kOffW[l], p + kOffB[l], n->h[l]);
    CCHECK(n, hipGetLastError());
    lin = lout;
  }
  hipLaunchKernelGGL(ddx::k_pool_linear, dim3(R), dim3(64), 0, s, n->h[3], lin, p + kOffW5, p + kOffB5, n->g, n->arg,
                     scores);
  CCHECK(n, hipGetLastError());
  n->tiles = tiles;
  n->scores = scores;
  n->rows = R;
  n->have_forward = true;
  n->have_loss = false;
  return DDX_OK;
}

int ddx_cnn_loss(ddx_cnn* n, const float* labels, float* loss_rows, void* stream) {
  if (!n) return DDX_EINVAL;
  if (!n->have_forward) return cfail(n, DDX_ESTATE, "run ddx_cnn_forward first");
  if (!labels || !loss_rows) return cfail(n, DDX_EINVAL, "null device buffer");
  hipLaunchKernelGGL(ddx::k_logistic, dim3(blocks(n->rows)), dim3(256), 0, (hipStream_t)stream, n->scores, labels,
                     n->rows, n->ds, loss_rows);
  CCHECK(n, hipGetLastError());
  n->have_loss = true;
  return DDX_OK;
}

int ddx_cnn_backward(ddx_cnn* n, void* stream) {
  if (!n) return DDX_EINVAL;
  if (!n->have_loss) return cfail(n, DDX_ESTATE, "run ddx_cnn_forward and ddx_cnn_loss first");
  hipStream_t s = (hipStream_t)stream;
  const int R = n->rows, L = n->n_bins;
  float* gr = n->grads;
  const float* p = n->params;
  hipLaunchKernelGGL(ddx::k_linear_bwd, dim3(1), dim3(256), 0, s, n->ds, n->g, R, gr + kOffW5, gr + kOffB5);
  CCHECK(n, hipGetLastError());
  int len[4] = {L, L / 2, L / 4, L / 8};
  const int64_t n4 = (int64_t)R * kW * len[3];
  hipLaunchKernelGGL(ddx::k_pool_bwd, dim3(blocks(n4)), dim3(256), 0, s, n->ds, p + kOffW5, n->arg, R, len[3],
                     n->gh[3]);
  CCHECK(n, hipGetLastError());
  const int chunks = kChunks < R ? kChunks : R;
  const int per = (R + chunks - 1) / chunks;
  const bool h16 = n->precision == DDX_CNN_FP16;  // the forward pass of this precision left n->wh, n->wscale
  for (int l = 3; l >= 0; --l) {
    const int64_t nl = (int64_t)R * kW * len[l];
    hipLaunchKernelGGL(ddx::k_relu_bwd, dim3(blocks(nl)), dim3(256), 0, s, n->gh[l], n->h[l], nl);
    CCHECK(n, hipGetLastError());
    const int nw = l == 0 ? (int)kNW1 : (int)kNW;
    if (l == 0) {
      if (h16)
        hipLaunchKernelGGL((ddx::k_conv_bwd_w_h<3, 1, true, 256>), dim3(chunks), dim3(256), 0, s, n->gh[0], len[0],
                           n->tiles, n->stats, n->n_dm, L, R, per, n->part, n->partb);
      else
        hipLaunchKernelGGL((ddx::k_conv_bwd_w<3, 1, true>), dim3(chunks), dim3(256), 0, s, n->gh[0], len[0],
                           n->tiles, n->stats, n->n_dm, L, R, per, n->part, n->partb);
    } else {
      if (h16)
        hipLaunchKernelGGL((ddx::k_conv_bwd_w_h<kW, 2, false, 128>), dim3(chunks), dim3(256), 0, s, n->gh[l], len[l],
                           n->h[l - 1], n->stats, n->n_dm, len[l - 1], R, per, n->part, n->partb);
      else
        hipLaunchKernelGGL((ddx::k_conv_bwd_w<kW, 2, false>), dim3(chunks), dim3(256), 0, s, n->gh[l], len[l],
                           n->h[l - 1], n->stats, n->n_dm, len[l - 1], R, per, n->part, n->partb);
    }
    CCHECK(n, hipGetLastError());
    hipLaunchKernelGGL(ddx::k_reduce_chunks, dim3(blocks(nw + kW)), dim3(256), 0, s, n->part, n->partb, chunks, nw,
                       gr + kOffW[l], gr + kOffB[l]);
    CCHECK(n, hipGetLastError());
    if (l > 0) {
      if (h16)
        hipLaunchKernelGGL(ddx::k_conv_bwd_data_h, dim3((len[l - 1] + 63) / 64, R), dim3(256), 0, s, n->gh[l], len[l],
                           n->wh + ddx::kCnnHalfOff[l] + kNW, n->wscale + l, len[l - 1], n->gh[l - 1]);
      else
        hipLaunchKernelGGL((ddx::k_conv_bwd_data<2>), dim3((len[l - 1] + 63) / 64, R), dim3(256), 0, s, n->gh[l],
                           len[l], p + kOffW[l], len[l - 1], n->gh[l - 1]);
      CCHECK(n, hipGetLastError());
    }
  }
  return DDX_OK;
}

int ddx_cnn_adam(ddx_cnn* n, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!n) return DDX_EINVAL;
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return cfail(n, DDX_EINVAL, "bad Adam hyper-parameters");
  n->step += 1;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)n->step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)n->step));
  hipLaunchKernelGGL(ddx::k_adam, dim3(blocks(kNParams)), dim3(256), 0, (hipStream_t)stream, n->params, n->grads,
                     n->m, n->v, kNParams, lr, beta1, beta2, eps, c1, c2);
  CCHECK(n, hipGetLastError());
  return DDX_OK;
}

int ddx_cnn_destroy(ddx_cnn* n) {
  if (!n) return DDX_OK;
  (void)hipDeviceSynchronize();
  for (void* a : n->allocs) (void)hipFree(a);
  delete n;
  return DDX_OK;
}

const char* ddx_cnn_last_error(const ddx_cnn* n) { return n ? n->err.c_str() : "null network"; }

}  // extern "C"
