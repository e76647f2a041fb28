// Makespan model of the tree / tile-size selector: a 13 -> 64 -> 64 -> 1
// multilayer perceptron with ReLU hidden units, mean-squared-error loss and
// Adam, in FP32 on the GPU.
//
// Parameters (one FP32 array, row-major, y = relu(relu(x W1 + b1) W2 + b2) W3 + b3):
//   W1 [13][64] at 0, b1 [64] at 832, W2 [64][64] at 896, b2 [64] at 4992,
//   W3 [64] at 5056, b3 at 5120; 5121 floats in all.
//
// One wave evaluates one sample with lane j holding hidden unit j of both
// layers; a workgroup of four waves takes samples wave, wave + 4, ... of its
// chunk.  The gradient kernel keeps per-lane partial gradients (column j of
// W2, column j of W1, b1[j], b2[j], W3[j], and b3 on lane 0), adds the four
// waves' partials through LDS and writes one partial gradient per
// workgroup; a second kernel adds the workgroups' partials in a fixed order,
// so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "tiledqr.h"

namespace tqr {

namespace {

constexpr int NIN = 13, NH = 64;
constexpr int OW1 = 0, OB1 = NIN * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
constexpr int NPARAM = OB3 + 1;
constexpr int MLP_WAVES = 4;
constexpr int MLP_CHUNK = 64;  // samples per workgroup in the gradient kernel

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Forward pass of one sample on one wave; returns y on every lane and the
// lane's pre-activations z1, z2 (h = max(z, 0)).  h1s: this wave's 64-float
// LDS scratch.
__device__ __forceinline__ float mlp_sample(const float* __restrict__ P, const float* __restrict__ x, int lane,
                                            float* h1s, float& z1, float& z2) {
  float a = P[OB1 + lane];
#pragma unroll
  for (int i = 0; i < NIN; ++i) a += x[i] * P[OW1 + i * NH + lane];
  z1 = a;
  h1s[lane] = a > 0.f ? a : 0.f;
  __builtin_amdgcn_wave_barrier();
  float b = P[OB2 + lane];
#pragma unroll 8
  for (int k = 0; k < NH; ++k) b += h1s[k] * P[OW2 + k * NH + lane];
  z2 = b;
  const float h2 = b > 0.f ? b : 0.f;
  return wave_sum_f(h2 * P[OW3 + lane]) + P[OB3];
}

__global__ __launch_bounds__(64 * MLP_WAVES) void mlp_forward_kernel(const float* __restrict__ P,
                                                                     const float* __restrict__ X, int64_t n,
                                                                     float* __restrict__ y) {
  __shared__ float h1[MLP_WAVES][NH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t s = static_cast<int64_t>(blockIdx.x) * MLP_WAVES + wave;
  if (s >= n) return;
  float z1, z2;
  const float out = mlp_sample(P, X + s * NIN, lane, h1[wave], z1, z2);
  if (lane == 0) y[s] = out;
}

// Partial loss and gradient of one chunk of samples: loss = sum (y - t)^2 / n,
// written to part[blockIdx.x * (NPARAM + 1) + ...] (gradient, then loss).
__global__ __launch_bounds__(64 * MLP_WAVES) void mlp_grad_kernel(const float* __restrict__ P,
                                                                  const float* __restrict__ X,
                                                                  const float* __restrict__ t, int64_t n,
                                                                  float* __restrict__ part) {
  __shared__ float h1[MLP_WAVES][NH];
  __shared__ float dz2s[MLP_WAVES][NH];
  __shared__ float red[MLP_WAVES][NH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float gW2[NH], gW1[NIN];
#pragma unroll
  for (int k = 0; k < NH; ++k) gW2[k] = 0.f;
#pragma unroll
  for (int i = 0; i < NIN; ++i) gW1[i] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gW3 = 0.f, gb3 = 0.f, loss = 0.f;
  const float inv_n = 1.0f / static_cast<float>(n);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * MLP_CHUNK;
  for (int j = wave; j < MLP_CHUNK; j += MLP_WAVES) {
    const int64_t s = base + j;
    if (s >= n) break;
    const float* x = X + s * NIN;
    float z1, z2;
    const float y = mlp_sample(P, x, lane, h1[wave], z1, z2);
    const float r = y - t[s];
    loss += r * r;
    const float dy = 2.f * inv_n * r;
    const float h2 = z2 > 0.f ? z2 : 0.f;
    gW3 += h2 * dy;
    gb3 += dy;
    const float dz2 = z2 > 0.f ? dy * P[OW3 + lane] : 0.f;
    gb2 += dz2;
#pragma unroll
    for (int k = 0; k < NH; ++k) gW2[k] += h1[wave][k] * dz2;  // dW2[k][lane]
    dz2s[wave][lane] = dz2;
    __builtin_amdgcn_wave_barrier();
    // dh1[lane] = sum_j dz2[j] W2[lane][j]
    float dh1 = 0.f;
#pragma unroll 8
    for (int jj = 0; jj < NH; ++jj) dh1 += dz2s[wave][jj] * P[OW2 + lane * NH + jj];
    const float dz1 = z1 > 0.f ? dh1 : 0.f;
    gb1 += dz1;
#pragma unroll
    for (int i = 0; i < NIN; ++i) gW1[i] += x[i] * dz1;  // dW1[i][lane]
    __builtin_amdgcn_wave_barrier();
  }
  // Add the four waves' partials (fixed order) and write this chunk's part.
  float* out = part + static_cast<int64_t>(blockIdx.x) * (NPARAM + 1);
  auto reduce_store = [&](float v, int idx) {
    red[wave][lane] = v;
    __syncthreads();
    if (wave == 0) {
      float s = 0.f;
#pragma unroll
      for (int w = 0; w < MLP_WAVES; ++w) s += red[w][lane];
      out[idx] = s;
    }
    __syncthreads();
  };
  for (int k = 0; k < NH; ++k) reduce_store(gW2[k], OW2 + k * NH + lane);
  for (int i = 0; i < NIN; ++i) reduce_store(gW1[i], OW1 + i * NH + lane);
  reduce_store(gb1, OB1 + lane);
  reduce_store(gb2, OB2 + lane);
  reduce_store(gW3, OW3 + lane);
  gb3 = wave_sum_f(lane == 0 ? gb3 : 0.f);
  loss = wave_sum_f(lane == 0 ? loss : 0.f);
  red[wave][lane] = 0.f;
  if (lane == 0) {
    red[wave][0] = gb3;
    red[wave][1] = loss;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.f, l = 0.f;
    for (int w = 0; w < MLP_WAVES; ++w) {
      a += red[w][0];
      l += red[w][1];
    }
    out[OB3] = a;
    out[NPARAM] = l * inv_n;
  }
}

// grad[e] (and loss at grad[NPARAM] if wanted) = sum over chunks b of part[b][e].
__global__ __launch_bounds__(256) void mlp_sum_kernel(const float* __restrict__ part, int nchunk,
                                                      float* __restrict__ grad, float* __restrict__ loss) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > NPARAM) return;
  float s = 0.f;
  for (int b = 0; b < nchunk; ++b) s += part[static_cast<int64_t>(b) * (NPARAM + 1) + e];
  if (e < NPARAM)
    grad[e] = s;
  else if (loss)
    *loss = s;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ P, const float* __restrict__ g,
                                                       float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float mh = mi / c1, vh = vi / c2;
  P[e] -= lr * mh / (sqrtf(vh) + eps);
}

// Partial gradients of tiledqr_mlp_loss_grad_noalloc: a fixed array in the
// library's device memory (one copy per GPU, held until the process ends),
// NOALLOC_MAX_CHUNKS chunks of MLP_CHUNK samples, 5.2 MB.
constexpr int NOALLOC_MAX_CHUNKS = 256;
__device__ __align__(256) float scratch[NOALLOC_MAX_CHUNKS * (NPARAM + 1)];

}  // namespace

// Device address of scratch on the current device, looked up once per device
// (host code must not pass the array's name to a kernel: on the host it is a
// stand-in, not a device address).  Null if the lookup failed.
float* noalloc_scratch() {
  constexpr int MAXDEV = 64;
  static std::mutex mu;
  static float* ptr[MAXDEV] = {};
  static bool done[MAXDEV] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXDEV) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!done[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    ptr[dev] = static_cast<float*>(p);
    done[dev] = true;
  }
  return ptr[dev];
}

}  // namespace tqr

extern "C" {

int tiledqr_mlp_nparam(void) { return tqr::NPARAM; }

int tiledqr_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* stream) {
  if (!params || n < 0 || (n > 0 && (!X || !y))) return TQR_EINVAL;
  if (n == 0) return TQR_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t blocks = (n + tqr::MLP_WAVES - 1) / tqr::MLP_WAVES;
  hipLaunchKernelGGL(tqr::mlp_forward_kernel, dim3(static_cast<unsigned>(blocks)), dim3(64 * tqr::MLP_WAVES), 0, s,
                     params, X, n, y);
  return hipGetLastError() == hipSuccess ? TQR_OK : TQR_EHIP;
}

int tiledqr_mlp_loss_grad(const float* params, const float* X, const float* t, int64_t n, float* grad, float* loss,
                          void* stream) {
  if (!params || !X || !t || !grad || n < 1) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nchunk = (n + tqr::MLP_CHUNK - 1) / tqr::MLP_CHUNK;
  if (nchunk > (1 << 24)) return TQR_EINVAL;
  float* part = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&part), nchunk * (tqr::NPARAM + 1) * sizeof(float), s) != hipSuccess)
    return TQR_ENOMEM;
  hipLaunchKernelGGL(tqr::mlp_grad_kernel, dim3(static_cast<unsigned>(nchunk)), dim3(64 * tqr::MLP_WAVES), 0, s,
                     params, X, t, n, part);
  hipLaunchKernelGGL(tqr::mlp_sum_kernel, dim3((tqr::NPARAM + 1 + 255) / 256), dim3(256), 0, s, part,
                     static_cast<int>(nchunk), grad, loss);
  const hipError_t e = hipGetLastError();
  (void)hipFreeAsync(part, s);
  return e == hipSuccess ? TQR_OK : TQR_EHIP;
}

int tiledqr_mlp_loss_grad_noalloc(const float* params, const float* X, const float* t, int64_t n, float* grad,
                                  float* loss, void* stream) {
  if (!params || !X || !t || !grad || n < 1 || n > tiledqr_mlp_noalloc_max_samples()) return TQR_EINVAL;
  float* part = tqr::noalloc_scratch();
  if (!part) return TQR_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nchunk = (n + tqr::MLP_CHUNK - 1) / tqr::MLP_CHUNK;
  // Every chunk's kernel writes all NPARAM + 1 entries of its part, so the
  // array needs no clearing between calls.
  hipLaunchKernelGGL(tqr::mlp_grad_kernel, dim3(static_cast<unsigned>(nchunk)), dim3(64 * tqr::MLP_WAVES), 0, s,
                     params, X, t, n, part);
  hipLaunchKernelGGL(tqr::mlp_sum_kernel, dim3((tqr::NPARAM + 1 + 255) / 256), dim3(256), 0, s, part,
                     static_cast<int>(nchunk), grad, loss);
  return hipGetLastError() == hipSuccess ? TQR_OK : TQR_EHIP;
}

int tiledqr_mlp_noalloc_max_samples(void) { return tqr::NOALLOC_MAX_CHUNKS * tqr::MLP_CHUNK; }

int tiledqr_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t nparam, float lr, float beta1,
                     float beta2, float eps, int32_t step, void* stream) {
  if (!params || !grad || !m || !v || nparam < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // Bias corrections 1 - beta^step, computed on the host in double.
  double p1 = 1.0, p2 = 1.0;
  for (int32_t i = 0; i < step; ++i) {
    p1 *= beta1;
    p2 *= beta2;
  }
  const float c1 = static_cast<float>(1.0 - p1), c2 = static_cast<float>(1.0 - p2);
  hipLaunchKernelGGL(tqr::mlp_adam_kernel, dim3(static_cast<unsigned>((nparam + 255) / 256)), dim3(256), 0, s, params,
                     grad, m, v, nparam, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? TQR_OK : TQR_EHIP;
}

}  // extern "C"
