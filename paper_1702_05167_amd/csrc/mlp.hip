// Surrogate network of the learned energy grid: FP32 fully connected layers, tanh hidden
// activations, mean-squared-error loss, Adam.  Forward, backward and the optimiser step are
// device kernels; the host only sequences launches.
//
// The contractions are small (4 -> 256 -> 256 -> 2 on a few thousand samples: under 1 GFLOP
// per epoch), so one LDS-tiled FP32 kernel with general strides serves all three products of
// a layer (forward X W^T, input gradient dY W, weight gradient dY^T X) with fused epilogues;
// the run time is set by launch latency, not by arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "hsc_internal.h"
#include "../../include/hsc_mlp.h"

struct hsc_mlp {
  int device = 0;
  std::vector<int> w;                      // layer widths
  std::vector<int64_t> off_w, off_b;       // parameter offsets per layer
  int64_t P = 0;
  float* params = nullptr;                 // [P]
  float* grads = nullptr;                  // [P]
  float* m1 = nullptr;                     // Adam first moment [P]
  float* m2 = nullptr;                     // Adam second moment [P]
  int64_t t = 0;                           // Adam steps taken
  int64_t cap = 0;                         // samples the workspace holds
  float* act = nullptr;                    // hidden activations, layer after layer, [cap * sum hidden]
  float* dbuf[2] = {nullptr, nullptr};     // back-propagated gradients, [cap * max width] each
  float* out = nullptr;                    // network output for the loss, [cap * w_out]
  float* xb = nullptr;                     // gathered batch inputs [cap * w_in]
  float* tb = nullptr;                     // gathered batch targets [cap * w_out]
  float* loss = nullptr;                   // [1] when the caller keeps no loss history
};

namespace hsc {
namespace {

#define MLPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t err_ = (x);                                                          \
    if (err_ != hipSuccess) {                                                       \
      set_error(std::string("HIP error: ") + hipGetErrorString(err_) + " at " #x);  \
      return HSC_E_HIP;                                                             \
    }                                                                               \
  } while (0)

constexpr int TM = 64, TN = 64, TK = 16, NTH = 256;

enum Epi { EPI_PLAIN = 0, EPI_BIAS_TANH = 1, EPI_BIAS = 2, EPI_TANH_BACK = 3 };

// C[m][n] (row stride ldc) = sum_k A(m, k) B(k, n), A(m, k) = A[m*am + k*ak], B(k, n) = B[k*bk + n*bn]
// EPI_BIAS_TANH: tanh(acc + bias[n]); EPI_BIAS: acc + bias[n];
// EPI_TANH_BACK: acc * (1 - H[m][n]^2) with H the tanh output the gradient flows back through.
template <int EPI>
__global__ __launch_bounds__(NTH) void k_sgemm(int M, int N, int K, const float* __restrict__ A, int64_t am,
                                               int64_t ak, const float* __restrict__ B, int64_t bk, int64_t bn,
                                               const float* __restrict__ bias, const float* __restrict__ H,
                                               float* __restrict__ C, int64_t ldc) {
  __shared__ float As[TK][TM + 4];
  __shared__ float Bs[TK][TN + 4];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tr = tid / 16, tc = tid % 16;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += TK) {
    for (int i = 0; i < TM * TK / NTH; ++i) {
      const int e = tid + i * NTH;
      const int mm = e % TM, kk = e / TM;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < K) ? A[m * am + k * ak] : 0.f;
    }
    for (int i = 0; i < TN * TK / NTH; ++i) {
      const int e = tid + i * NTH;
      const int nn = e % TN, kk = e / TN;
      const int n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < N && k < K) ? B[k * bk + n * bn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + tr * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tc * 4 + j;
      if (n >= N) continue;
      float v = acc[i][j];
      if (EPI == EPI_BIAS_TANH) v = tanhf(v + bias[n]);
      if (EPI == EPI_BIAS) v = v + bias[n];
      if (EPI == EPI_TANH_BACK) {
        const float h = H[m * ldc + n];
        v = v * (1.f - h * h);
      }
      C[m * ldc + n] = v;
    }
  }
}

// db[j] = sum over samples of dY[s][j]
__global__ void k_colsum(int n, int M, const float* __restrict__ dY, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  float s = 0.f;
  for (int r = 0; r < n; ++r) s += dY[(int64_t)r * M + j];
  db[j] = s;
}

// d = y - t; dY = 2 d / count; loss = sum d^2 / count (one workgroup, fixed reduction order)
__global__ __launch_bounds__(NTH) void k_mse(int64_t count, const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float part[NTH];
  const float inv = 1.f / (float)count;
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < count; i += NTH) {
    const float d = y[i] - t[i];
    dY[i] = 2.f * d * inv;
    s = fmaf(d, d, s);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = NTH / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = part[0] * inv;
}

// dst row r = src row idx[r]; an index outside [0, n_src) yields a NaN row (the loss turns NaN)
__global__ void k_gather_rows(int64_t rows, int width, const int32_t* __restrict__ idx, int64_t n_src,
                              const float* __restrict__ src, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * width) return;
  const int64_t r = e / width;
  const int c = (int)(e % width);
  const int64_t q = idx[r];
  dst[e] = (q >= 0 && q < n_src) ? src[q * width + c] : __builtin_nanf("");
}

__global__ void k_adam(int64_t P, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
}

template <int EPI>
void sgemm(hipStream_t st, int M, int N, int K, const float* A, int64_t am, int64_t ak, const float* B, int64_t bk,
           int64_t bn, const float* bias, const float* H, float* C, int64_t ldc) {
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  hipLaunchKernelGGL((k_sgemm<EPI>), grid, dim3(NTH), 0, st, M, N, K, A, am, ak, B, bk, bn, bias, H, C, ldc);
}

int64_t hidden_sum(const hsc_mlp* m) {
  int64_t s = 0;
  for (size_t l = 1; l + 1 < m->w.size(); ++l) s += m->w[l];
  return s;
}

hsc_status reserve(hsc_mlp* m, int64_t n) {
  if (n <= m->cap) return HSC_OK;
  int64_t cap = std::max<int64_t>(n, 256);
  int wmax = 0;
  for (int v : m->w) wmax = std::max(wmax, v);
  if (m->cap > 0 && hipDeviceSynchronize() != hipSuccess) {   // earlier launches may still use the old buffers
    (void)hipGetLastError();
    set_error("device synchronisation failed");
    return HSC_E_HIP;
  }
  float* old[6] = {m->act, m->dbuf[0], m->dbuf[1], m->out, m->xb, m->tb};
  for (float* p : old)
    if (p) (void)hipFree(p);
  m->act = m->dbuf[0] = m->dbuf[1] = m->out = m->xb = m->tb = nullptr;
  m->cap = 0;
  const int64_t sizes[6] = {cap * std::max<int64_t>(hidden_sum(m), 1), cap * wmax, cap * wmax,
                            cap * m->w.back(), cap * m->w.front(), cap * m->w.back()};
  float** dst[6] = {&m->act, &m->dbuf[0], &m->dbuf[1], &m->out, &m->xb, &m->tb};
  for (int i = 0; i < 6; ++i) {
    if (hipMalloc(dst[i], sizeof(float) * sizes[i]) != hipSuccess) {
      (void)hipGetLastError();
      set_error("MLP workspace allocation failed");
      return HSC_E_OOM;
    }
  }
  m->cap = cap;
  return HSC_OK;
}

// activation of layer l (l = 1 .. L-2) for the current n
float* act_of(hsc_mlp* m, int l, int64_t n) {
  int64_t o = 0;
  for (int q = 1; q < l; ++q) o += m->w[q];
  return m->act + o * n;
}

// forward pass storing every hidden activation; output to y
void forward(hipStream_t st, hsc_mlp* m, int64_t n, const float* x, float* y) {
  const int L = (int)m->w.size();
  const float* h = x;
  for (int l = 0; l + 1 < L; ++l) {
    const int K = m->w[l], N = m->w[l + 1];
    const float* W = m->params + m->off_w[l];
    const float* b = m->params + m->off_b[l];
    if (l + 2 < L) {
      float* o = act_of(m, l + 1, n);
      sgemm<EPI_BIAS_TANH>(st, (int)n, N, K, h, K, 1, W, 1, K, b, nullptr, o, N);
      h = o;
    } else {
      sgemm<EPI_BIAS>(st, (int)n, N, K, h, K, 1, W, 1, K, b, nullptr, y, N);
    }
  }
}

// gradient of the loss into m->grads, loss value to loss_dst; x, t hold n samples
void loss_and_grads(hipStream_t st, hsc_mlp* m, int64_t n, const float* x, const float* t, float* grads,
                    float* loss_dst) {
  const int L = (int)m->w.size();
  forward(st, m, n, x, m->out);
  float* d = m->dbuf[0];
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(NTH), 0, st, n * m->w.back(), m->out, t, d, loss_dst);
  for (int l = L - 2; l >= 0; --l) {
    const int K = m->w[l], N = m->w[l + 1];
    const float* hin = l == 0 ? x : act_of(m, l, n);
    // dW_l[j][k] = sum_s d[s][j] hin[s][k]
    sgemm<EPI_PLAIN>(st, N, K, (int)n, d, 1, N, hin, K, 1, nullptr, nullptr, grads + m->off_w[l], K);
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, st, (int)n, N, d, grads + m->off_b[l]);
    if (l > 0) {
      // d_prev[s][k] = (sum_j d[s][j] W[j][k]) (1 - hin[s][k]^2)
      float* dn = d == m->dbuf[0] ? m->dbuf[1] : m->dbuf[0];
      sgemm<EPI_TANH_BACK>(st, (int)n, K, N, d, N, 1, m->params + m->off_w[l], K, 1, nullptr, hin, dn, K);
      d = dn;
    }
  }
}

}  // namespace
}  // namespace hsc

using namespace hsc;

extern "C" {

hsc_status hsc_mlp_create(hsc_ctx* ctx, int32_t n_widths, const int32_t* widths, hsc_mlp** out) {
  if (!ctx || !widths || !out || n_widths < 2) { set_error("bad arguments to hsc_mlp_create"); return HSC_E_ARG; }
  *out = nullptr;
  for (int i = 0; i < n_widths; ++i)
    if (widths[i] < 1 || widths[i] > 1024) { set_error("layer width outside [1, 1024]"); return HSC_E_ARG; }
  MLPCHK(hipSetDevice(ctx_device(ctx)));
  hsc_mlp* m = new hsc_mlp();
  m->device = ctx_device(ctx);
  m->w.assign(widths, widths + n_widths);
  for (int l = 0; l + 1 < n_widths; ++l) {
    m->off_w.push_back(m->P);
    m->P += (int64_t)m->w[l + 1] * m->w[l];
    m->off_b.push_back(m->P);
    m->P += m->w[l + 1];
  }
  float** bufs[5] = {&m->params, &m->grads, &m->m1, &m->m2, &m->loss};
  for (int i = 0; i < 5; ++i) {
    const int64_t cnt = i == 4 ? 1 : m->P;
    if (hipMalloc(bufs[i], sizeof(float) * cnt) != hipSuccess ||
        hipMemset(*bufs[i], 0, sizeof(float) * cnt) != hipSuccess) {
      (void)hipGetLastError();
      hsc_mlp_destroy(m);
      set_error("MLP parameter allocation failed");
      return HSC_E_OOM;
    }
  }
  *out = m;
  return HSC_OK;
}

hsc_status hsc_mlp_destroy(hsc_mlp* m) {
  if (!m) return HSC_OK;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  float* all[11] = {m->params, m->grads, m->m1, m->m2, m->loss, m->act, m->dbuf[0], m->dbuf[1], m->out, m->xb, m->tb};
  for (float* p : all)
    if (p) (void)hipFree(p);
  delete m;
  return HSC_OK;
}

hsc_status hsc_mlp_n_params(const hsc_mlp* m, int64_t* out) {
  if (!m || !out) { set_error("bad arguments to hsc_mlp_n_params"); return HSC_E_ARG; }
  *out = m->P;
  return HSC_OK;
}

hsc_status hsc_mlp_set_params(hsc_ctx* ctx, hsc_mlp* m, const float* params) {
  if (!ctx || !m || !params) { set_error("bad arguments to hsc_mlp_set_params"); return HSC_E_ARG; }
  MLPCHK(hipSetDevice(m->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(ctx_stream(ctx));
  MLPCHK(hipMemcpyAsync(m->params, params, sizeof(float) * m->P, hipMemcpyDeviceToDevice, st));
  MLPCHK(hipMemsetAsync(m->m1, 0, sizeof(float) * m->P, st));
  MLPCHK(hipMemsetAsync(m->m2, 0, sizeof(float) * m->P, st));
  m->t = 0;
  return HSC_OK;
}

hsc_status hsc_mlp_get_params(hsc_ctx* ctx, const hsc_mlp* m, float* params) {
  if (!ctx || !m || !params) { set_error("bad arguments to hsc_mlp_get_params"); return HSC_E_ARG; }
  MLPCHK(hipSetDevice(m->device));
  MLPCHK(hipMemcpyAsync(params, m->params, sizeof(float) * m->P, hipMemcpyDeviceToDevice,
                        reinterpret_cast<hipStream_t>(ctx_stream(ctx))));
  return HSC_OK;
}

hsc_status hsc_mlp_forward(hsc_ctx* ctx, hsc_mlp* m, int64_t n, const float* x, float* y) {
  if (!ctx || !m || n < 0 || (n > 0 && (!x || !y)) || n > INT32_MAX) { set_error("bad arguments to hsc_mlp_forward"); return HSC_E_ARG; }
  if (n == 0) return HSC_OK;
  MLPCHK(hipSetDevice(m->device));
  hsc_status rc = reserve(m, n);
  if (rc != HSC_OK) return rc;
  forward(reinterpret_cast<hipStream_t>(ctx_stream(ctx)), m, n, x, y);
  MLPCHK(hipGetLastError());
  return HSC_OK;
}

hsc_status hsc_mlp_grads(hsc_ctx* ctx, hsc_mlp* m, int64_t n, const float* x, const float* t, float* grads,
                         float* loss) {
  if (!ctx || !m || n <= 0 || n > INT32_MAX || !x || !t || !grads || !loss) { set_error("bad arguments to hsc_mlp_grads"); return HSC_E_ARG; }
  MLPCHK(hipSetDevice(m->device));
  hsc_status rc = reserve(m, n);
  if (rc != HSC_OK) return rc;
  loss_and_grads(reinterpret_cast<hipStream_t>(ctx_stream(ctx)), m, n, x, t, grads, loss);
  MLPCHK(hipGetLastError());
  return HSC_OK;
}

hsc_status hsc_mlp_train(hsc_ctx* ctx, hsc_mlp* m, int64_t n, const float* x, const float* t,
                         const hsc_train_opts* o, const int32_t* order, float* loss_hist) {
  if (!ctx || !m || !o || n <= 0 || n > INT32_MAX || !x || !t || o->steps < 0 || o->batch <= 0 ||
      !(o->lr > 0.f) || !(o->beta1 >= 0.f && o->beta1 < 1.f) || !(o->beta2 >= 0.f && o->beta2 < 1.f) ||
      !(o->eps > 0.f)) {
    set_error("bad arguments to hsc_mlp_train");
    return HSC_E_ARG;
  }
  MLPCHK(hipSetDevice(m->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(ctx_stream(ctx));
  const int64_t B = order ? o->batch : n;
  hsc_status rc = reserve(m, B);
  if (rc != HSC_OK) return rc;
  const int wi = m->w.front(), wo = m->w.back();
  for (int s = 0; s < o->steps; ++s) {
    const float* xs = x;
    const float* ts = t;
    if (order) {
      const int32_t* idx = order + (int64_t)s * B;
      hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((B * wi + 255) / 256)), dim3(256), 0, st, B, wi, idx, n, x,
                         m->xb);
      hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((B * wo + 255) / 256)), dim3(256), 0, st, B, wo, idx, n, t,
                         m->tb);
      xs = m->xb;
      ts = m->tb;
    }
    loss_and_grads(st, m, B, xs, ts, m->grads, loss_hist ? loss_hist + s : m->loss);
    m->t += 1;
    const float bc1 = 1.f - std::pow(o->beta1, (float)m->t);
    const float bc2 = 1.f - std::pow(o->beta2, (float)m->t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((m->P + 255) / 256)), dim3(256), 0, st, m->P, m->params, m->grads,
                       m->m1, m->m2, o->lr, o->beta1, o->beta2, o->eps, bc1, bc2);
  }
  MLPCHK(hipGetLastError());
  return HSC_OK;
}

}  // extern "C"
