// FP32 multilayer perceptron of the learned warm start: forward, backward
// (mean-squared-error loss) and Adam, all in HIP kernels.
//
// Network: h_0 = x; h_l = GELU(h_{l-1} W_l^T + b_l) for the hidden layers;
// y = h_L W_out^T + b_out; GELU(z) = z/2 (1 + erf(z/sqrt 2)).  Parameters are
// one flat FP32 vector, layer by layer: weight (out x in, row-major), bias.
#include <hip/hip_runtime.h>

#include <mutex>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/swr.h"

namespace {

constexpr int kT = 64;   // output tile (rows and columns)
constexpr int kK = 16;   // reduction chunk

// C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]) (+ C[m][n] if accumulate), with
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], C row-major, on the
// matrix cores: a 64 x 64 tile per block of four waves, 32 x 32 per wave as
// 2 x 2 products of v_mfma_f32_16x16x4f32 (A fragment: lane l holds
// A[l % 16][l / 16], B fragment B[l / 16][l % 16], the 16 x 16 result
// D[4 (l / 16) + v][l % 16] in its v-th register); the operands staged in
// LDS k-chunk by k-chunk (any strides).
// TILE = 64: 32 x 32 per wave (2 x 2 products); TILE = 32: 16 x 16 per wave,
// for products too small to give the chip enough 64 x 64 tiles.  Each
// output's k order is the same for both.
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int TILE>
__global__ void __launch_bounds__(256) k_sgemm(int M, int N, int K, const float* A, int64_t sam,
                                              int64_t sak, const float* B, int64_t sbk,
                                              int64_t sbn, float* C, int64_t ldc,
                                              const float* bias, int accumulate) {
  constexpr int R = TILE / 32;  // 16 x 16 products per wave and dimension
  __shared__ float As[kK][TILE + 4];
  __shared__ float Bs[kK][TILE + 4];
  const int m0 = blockIdx.y * TILE, n0 = blockIdx.x * TILE;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * (TILE / 2), wn = (w & 1) * (TILE / 2);
  const int fr = lane & 15, fk = lane >> 4;
  f32x4 acc[R][R];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += kK) {
    for (int e = threadIdx.x; e < kK * TILE; e += blockDim.x) {
      const int kk = e / TILE, mm = e % TILE;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < K) ? A[m * sam + k * sak] : 0.0f;
      const int n = n0 + mm;
      Bs[kk][mm] = (n < N && k < K) ? B[k * sbk + n * sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < kK; k4 += 4) {
      float a[R], b[R];
#pragma unroll
      for (int i = 0; i < R; ++i) a[i] = As[k4 + fk][wm + 16 * i + fr];
#pragma unroll
      for (int j = 0; j < R; ++j) b[j] = Bs[k4 + fk][wn + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + 4 * fk + v;
        const int n = n0 + wn + 16 * j + fr;
        if (m >= M || n >= N) continue;
        float x = acc[i][j][v];
        if (bias) x += bias[n];
        if (accumulate) x += C[m * ldc + n];
        C[m * ldc + n] = x;
      }
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ void k_gelu(int64_t n, const float* z, float* h) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) h[e] = gelu(z[e]);
}

__global__ void k_gelu_back(int64_t n, const float* z, float* d) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] *= gelu_grad(z[e]);
}

// dy = 2 (y - t) / n and per-block partial sums of (y - t)^2
__global__ void k_mse(int64_t n, const float* y, const float* t, float* dy, float* partial) {
  __shared__ float red[256];
  float acc = 0.0f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float r = y[e] - t[e];
    dy[e] = 2.0f * r / (float)n;
    acc += r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_final(int nb, const float* partial, int64_t n, float* loss) {
  __shared__ float red[256];
  float acc = 0.0f;
  for (int e = threadIdx.x; e < nb; e += blockDim.x) acc += partial[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / (float)n;
}

// gb[o] = sum_b d[b][o]
__global__ void k_bias_grad(int B, int O, const float* d, float* gb) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= O) return;
  float acc = 0.0f;
  for (int b = 0; b < B; ++b) acc += d[(int64_t)b * O + o];
  gb[o] = acc;
}

__global__ void k_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float mm = b1 * m[e] + (1.0f - b1) * g[e];
  const float vv = b2 * v[e] + (1.0f - b2) * g[e] * g[e];
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

struct Net {
  std::vector<int> dims;
  std::vector<int64_t> woff, boff;
  int64_t n_params = 0;
};

int make_net(const swr_mlp_desc* d, Net* net) {
  if (!d || d->n_in < 1 || d->n_hidden < 1 || d->n_layers < 0 || d->n_out < 1) return SWR_E_ARG;
  net->dims.clear();
  net->dims.push_back(d->n_in);
  for (int l = 0; l < d->n_layers; ++l) net->dims.push_back(d->n_hidden);
  net->dims.push_back(d->n_out);
  int64_t off = 0;
  for (size_t l = 0; l + 1 < net->dims.size(); ++l) {
    net->woff.push_back(off);
    off += (int64_t)net->dims[l + 1] * net->dims[l];
    net->boff.push_back(off);
    off += net->dims[l + 1];
  }
  net->n_params = off;
  return SWR_OK;
}

// workspace: per layer pre-activation z and activation h (batch x width),
// one gradient buffer of the widest layer twice, loss partials
struct Ws {
  std::vector<float*> z, h;
  float* d0;
  float* d1;
  float* partial;
  uint64_t bytes;
};

uint64_t plan_ws(const Net& net, int batch, char* base, Ws* ws) {
  uint64_t off = 0;
  auto take = [&](uint64_t n) {
    off = (off + 255) & ~uint64_t(255);
    float* p = base ? (float*)(base + off) : nullptr;
    off += n * sizeof(float);
    return p;
  };
  int widest = 0;
  for (int w : net.dims) widest = w > widest ? w : widest;
  ws->z.clear();
  ws->h.clear();
  for (size_t l = 1; l < net.dims.size(); ++l) {
    ws->z.push_back(take((uint64_t)batch * net.dims[l]));
    ws->h.push_back(take((uint64_t)batch * net.dims[l]));
  }
  ws->d0 = take((uint64_t)batch * widest);
  ws->d1 = take((uint64_t)batch * widest);
  ws->partial = take(1024);
  ws->bytes = off;
  return off;
}

void gemm(hipStream_t st, int M, int N, int K, const float* A, int64_t sam, int64_t sak,
          const float* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc, const float* bias,
          int accumulate) {
  // 64 x 64 tiles where they give at least 256 blocks, else 32 x 32
  const int64_t big = (int64_t)((N + kT - 1) / kT) * ((M + kT - 1) / kT);
  if (big >= 256) {
    dim3 grid((N + kT - 1) / kT, (M + kT - 1) / kT);
    hipLaunchKernelGGL(k_sgemm<64>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C,
                       ldc, bias, accumulate);
  } else {
    dim3 grid((N + 31) / 32, (M + 31) / 32);
    hipLaunchKernelGGL(k_sgemm<32>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C,
                       ldc, bias, accumulate);
  }
}

// forward pass; the output layer's result is ws.h.back() (= ws.z.back())
void forward(const Net& net, const float* params, const float* x, int batch, const Ws& ws,
             hipStream_t st) {
  const float* h = x;
  const int L = (int)net.dims.size() - 1;
  for (int l = 0; l < L; ++l) {
    const int in = net.dims[l], out = net.dims[l + 1];
    gemm(st, batch, out, in, h, in, 1, params + net.woff[l], 1, in, ws.z[l], out,
         params + net.boff[l], 0);
    const int64_t n = (int64_t)batch * out;
    if (l < L - 1)
      hipLaunchKernelGGL(k_gelu, dim3(nblocks(n)), dim3(256), 0, st, n, ws.z[l], ws.h[l]);
    else
      hipMemcpyAsync(ws.h[l], ws.z[l], n * sizeof(float), hipMemcpyDeviceToDevice, st);
    h = ws.h[l];
  }
}

// Scratch of the allocation-free forward pass (swr_mlp_forward_noalloc):
// the per-layer activations of one batch.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, never its device address: the address is looked up
// once per device (hipGetSymbolAddress, with that device current) and kept.
constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;  // 64 MiB
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch (null on a HIP error).
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

}  // namespace

extern "C" {

int32_t swr_mlp_param_count(const swr_mlp_desc* d, int64_t* count) {
  Net net;
  if (!count || make_net(d, &net) != SWR_OK) return SWR_E_ARG;
  *count = net.n_params;
  return SWR_OK;
}

int32_t swr_mlp_workspace_bytes(const swr_mlp_desc* d, int32_t batch, uint64_t* bytes) {
  Net net;
  if (!bytes || batch < 1 || make_net(d, &net) != SWR_OK) return SWR_E_ARG;
  Ws ws;
  *bytes = plan_ws(net, batch, nullptr, &ws);
  return SWR_OK;
}

int32_t swr_mlp_forward(const swr_mlp_desc* d, const float* params, const float* x, int32_t batch,
                        float* y, void* ws_dev, uint64_t ws_bytes, void* stream) {
  Net net;
  if (!params || !x || !y || !ws_dev || batch < 1 || make_net(d, &net) != SWR_OK) return SWR_E_ARG;
  Ws ws;
  if (plan_ws(net, batch, (char*)ws_dev, &ws) > ws_bytes) return SWR_E_SIZE;
  hipStream_t st = (hipStream_t)stream;
  forward(net, params, x, batch, ws, st);
  if (hipMemcpyAsync(y, ws.h.back(), (size_t)batch * d->n_out * sizeof(float),
                     hipMemcpyDeviceToDevice, st) != hipSuccess)
    return SWR_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SWR_OK : SWR_E_DEVICE;
}

int32_t swr_mlp_forward_noalloc(const swr_mlp_desc* d, const float* params, const float* x,
                                int32_t batch, float* y, void* stream) {
  Net net;
  if (!params || !x || !y || batch < 1 || make_net(d, &net) != SWR_OK) return SWR_E_ARG;
  Ws ws;
  if (plan_ws(net, batch, nullptr, &ws) > kNoAllocScratchBytes) return SWR_E_SIZE;
  void* base = scratch_address();
  if (!base) return SWR_E_DEVICE;
  plan_ws(net, batch, (char*)base, &ws);
  hipStream_t st = (hipStream_t)stream;
  forward(net, params, x, batch, ws, st);
  if (hipMemcpyAsync(y, ws.h.back(), (size_t)batch * d->n_out * sizeof(float),
                     hipMemcpyDeviceToDevice, st) != hipSuccess)
    return SWR_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SWR_OK : SWR_E_DEVICE;
}

int32_t swr_mlp_loss_grad(const swr_mlp_desc* d, const float* params, const float* x,
                          const float* t, int32_t batch, float* loss_dev, float* grad,
                          void* ws_dev, uint64_t ws_bytes, void* stream) {
  Net net;
  if (!params || !x || !t || !loss_dev || !grad || !ws_dev || batch < 1 ||
      make_net(d, &net) != SWR_OK)
    return SWR_E_ARG;
  Ws ws;
  if (plan_ws(net, batch, (char*)ws_dev, &ws) > ws_bytes) return SWR_E_SIZE;
  hipStream_t st = (hipStream_t)stream;
  forward(net, params, x, batch, ws, st);
  const int L = (int)net.dims.size() - 1;
  const int64_t ny = (int64_t)batch * d->n_out;
  const int nb = 256;
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, ny, ws.h.back(), t, ws.d0, ws.partial);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, nb, ws.partial, ny, loss_dev);
  float* dcur = ws.d0;  // gradient w.r.t. the pre-activation of layer l
  float* dnext = ws.d1;
  for (int l = L - 1; l >= 0; --l) {
    const int in = net.dims[l], out = net.dims[l + 1];
    const float* hin = l > 0 ? ws.h[l - 1] : x;
    // dW = dZ^T h_in (out x in), db = sum_b dZ
    gemm(st, out, in, batch, dcur, 1, out, hin, in, 1, grad + net.woff[l], in, nullptr, 0);
    hipLaunchKernelGGL(k_bias_grad, dim3(nblocks(out)), dim3(256), 0, st, batch, out, dcur,
                       grad + net.boff[l]);
    if (l > 0) {
      // dH_in = dZ W (batch x in), then through the GELU of layer l-1
      gemm(st, batch, in, out, dcur, out, 1, params + net.woff[l], in, 1, dnext, in, nullptr, 0);
      const int64_t n = (int64_t)batch * in;
      hipLaunchKernelGGL(k_gelu_back, dim3(nblocks(n)), dim3(256), 0, st, n, ws.z[l - 1], dnext);
      float* tmp = dcur;
      dcur = dnext;
      dnext = tmp;
    }
  }
  return hipGetLastError() == hipSuccess ? SWR_OK : SWR_E_DEVICE;
}

int32_t swr_mlp_adam(int64_t n, float* params, const float* grad, float* m, float* v,
                     int32_t step, float lr, float b1, float b2, float eps, void* stream) {
  if (!params || !grad || !m || !v || n < 1 || step < 1) return SWR_E_ARG;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nblocks(n)), dim3(256), 0, (hipStream_t)stream, n, params, grad,
                     m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? SWR_OK : SWR_E_DEVICE;
}

}  // extern "C"
