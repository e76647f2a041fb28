// Least-squares helpers: triangular solve with the tiled R, FP64 residuals
// and column norms for the backward error of the refinement loop.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace tqr {

namespace {

__device__ __forceinline__ const double* rtile(const double* tiles, int p, int nb, int r, int c) {
  return tiles + (static_cast<size_t>(c) * p + r) * static_cast<size_t>(nb) * nb;
}

// Solve R_kk X_k = Y_k in place for the diagonal tile k (one workgroup).
// Column-oriented back substitution: x_c = y_c / R[c][c], then
// y_r -= R[r][c] x_c for r < c, one thread per row.
__global__ __launch_bounds__(256) void trsm_diag_kernel(const double* tiles, int p, int nb, int k, double* Y,
                                                        int64_t ldy, int64_t nrhs) {
  __shared__ double xs[8];
  const double* R = rtile(tiles, p, nb, k, k);
  const int tid = threadIdx.x;
  double* Yk = Y + static_cast<int64_t>(k) * nb;
  for (int64_t c0 = 0; c0 < nrhs; c0 += 8) {
    const int nc = static_cast<int>(nrhs - c0 < 8 ? nrhs - c0 : 8);
    double y[8];
    for (int h = 0; h < 8; ++h) y[h] = (tid < nb && h < nc) ? Yk[(c0 + h) * ldy + tid] : 0.0;
    for (int c = nb - 1; c >= 0; --c) {
      if (tid == c) {
        const double d = R[c * nb + c];
        for (int h = 0; h < nc; ++h) {
          y[h] /= d;
          xs[h] = y[h];
        }
      }
      __syncthreads();
      if (tid < c) {
        const double rc = R[c * nb + tid];
        for (int h = 0; h < nc; ++h) y[h] -= rc * xs[h];
      }
      __syncthreads();
    }
    if (tid < nb)
      for (int h = 0; h < nc; ++h) Yk[(c0 + h) * ldy + tid] = y[h];
  }
}

// Y_i -= R_ik X_k for every tile row i < k.  Grid: (k, nrhs); block: nb rows.
__global__ __launch_bounds__(256) void trsm_update_kernel(const double* tiles, int p, int nb, int k, double* Y,
                                                          int64_t ldy) {
  const int i = blockIdx.x, h = blockIdx.y, row = threadIdx.x;
  if (row >= nb) return;
  const double* R = rtile(tiles, p, nb, i, k);
  const double* xk = Y + h * ldy + static_cast<int64_t>(k) * nb;
  double s = 0.0;
  for (int c = 0; c < nb; ++c) s += R[c * nb + row] * xk[c];
  Y[h * ldy + static_cast<int64_t>(i) * nb + row] -= s;
}

// Rv = B - A X for m x n A; grid (row blocks, column chunks), partial sums
// subtracted with FP64 atomics (Rv must hold B on entry).
constexpr int RES_CHUNK = 256;
__global__ __launch_bounds__(256) void residual_kernel(const double* A, int64_t lda, int64_t m, int64_t n,
                                                       const double* X, int64_t ldx, int64_t nrhs, double* Rv,
                                                       int64_t ldr) {
  const int64_t row = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * RES_CHUNK;
  const int64_t c1 = (c0 + RES_CHUNK < n) ? c0 + RES_CHUNK : n;
  if (row >= m) return;
  for (int64_t h0 = 0; h0 < nrhs; h0 += 4) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t c = c0; c < c1; ++c) {
      const double a = A[c * lda + row];
#pragma unroll
      for (int h = 0; h < 4; ++h)
        if (h0 + h < nrhs) s[h] += a * X[(h0 + h) * ldx + c];
    }
#pragma unroll
    for (int h = 0; h < 4; ++h)
      if (h0 + h < nrhs) atomicAdd(Rv + (h0 + h) * ldr + row, -s[h]);
  }
}

__global__ __launch_bounds__(256) void copy_cols_kernel(const double* S, int64_t lds, double* D, int64_t ldd,
                                                        int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t c = e / rows, r = e - c * rows;
    D[c * ldd + r] = S[c * lds + r];
  }
}

// out[c] += sum of squares of column c (out zeroed by the caller).
__global__ __launch_bounds__(256) void colnorms2_kernel(const double* M, int64_t ld, int64_t rows, int64_t cols,
                                                        double* out) {
  __shared__ double red[4];
  const int64_t c = blockIdx.y;
  double s = 0.0;
  for (int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; r < rows;
       r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double v = M[c * ld + r];
    s += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out + c, red[0] + red[1] + red[2] + red[3]);
  (void)cols;
}

__global__ __launch_bounds__(256) void axpy_cols_kernel(double* X, int64_t ldx, const double* D, int64_t ldd,
                                                        int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t c = e / rows, r = e - c * rows;
    X[c * ldx + r] += D[c * ldd + r];
  }
}

int grid_of(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 4096) g = 4096;
  return g < 1 ? 1 : static_cast<int>(g);
}

}  // namespace

hipError_t launch_trsm_upper(const double* tiles, int p, int q, int nb, double* Y, int64_t ldy, int64_t nrhs,
                             hipStream_t s) {
  for (int k = q - 1; k >= 0; --k) {
    hipLaunchKernelGGL(trsm_diag_kernel, dim3(1), dim3(256), 0, s, tiles, p, nb, k, Y, ldy, nrhs);
    if (k > 0) hipLaunchKernelGGL(trsm_update_kernel, dim3(k, static_cast<unsigned>(nrhs)), dim3(nb), 0, s, tiles, p,
                                  nb, k, Y, ldy);
  }
  return hipGetLastError();
}

hipError_t launch_residual(const double* A, int64_t lda, int64_t m, int64_t n, const double* X, int64_t ldx,
                           const double* B, int64_t ldb, int64_t nrhs, double* Rv, int64_t ldr, hipStream_t s) {
  hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_of(m * nrhs)), dim3(256), 0, s, B, ldb, Rv, ldr, m, nrhs);
  const dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>((n + RES_CHUNK - 1) / RES_CHUNK));
  hipLaunchKernelGGL(residual_kernel, grid, dim3(256), 0, s, A, lda, m, n, X, ldx, nrhs, Rv, ldr);
  return hipGetLastError();
}

hipError_t launch_colnorms2(const double* M, int64_t ld, int64_t rows, int64_t cols, double* out, hipStream_t s) {
  int64_t gx = (rows + 255) / 256;
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(colnorms2_kernel, dim3(static_cast<unsigned>(gx), static_cast<unsigned>(cols)), dim3(256), 0, s,
                     M, ld, rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_axpy_cols(double* X, int64_t ldx, const double* D, int64_t ldd, int64_t rows, int64_t cols,
                            hipStream_t s) {
  hipLaunchKernelGGL(axpy_cols_kernel, dim3(grid_of(rows * cols)), dim3(256), 0, s, X, ldx, D, ldd, rows, cols);
  return hipGetLastError();
}

}  // namespace tqr
