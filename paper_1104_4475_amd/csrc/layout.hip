// Layout conversions between column-major matrices and the tile layout.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace tqr {

// ---- layout conversions ------------------------------------------------------

// Column-major A (lda) -> tiles.  A column's rows in one tile row are a
// contiguous run both in A and in the tile, so block (g, y) copies the runs
// of columns g * 1024 / nb .. (1024 doubles) for tile rows y, y + gridDim.y,
// ...: four doubles per thread, each load instruction 64 consecutive
// doubles, all loads issued before the stores.  nb is a power of two <= 1024.
__global__ __launch_bounds__(256) void pack_kernel(const double* A, int64_t lda, double* tiles, int p, int q, int nb) {
  const int lg = __builtin_ctz(nb);
  const int64_t n = static_cast<int64_t>(q) << lg;
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * (1024 >> lg);
  for (int r = blockIdx.y; r < p; r += gridDim.y) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = threadIdx.x + 256 * k;
      const int64_t col = col0 + (e >> lg);
      v[k] = col < n ? A[col * lda + (static_cast<int64_t>(r) << lg) + (e & (nb - 1))] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = threadIdx.x + 256 * k;
      const int64_t col = col0 + (e >> lg);
      if (col < n)
        tiles[(((col >> lg) * p + r) << (2 * lg)) + ((col & (nb - 1)) << lg) + (e & (nb - 1))] = v[k];
    }
  }
}

// Batched pack: block g copies global tile g (problem found by binary
// search in tile_start) from its problem's column-major A.
__global__ __launch_bounds__(256) void pack_batched_kernel(const double* const* Aptr, const int64_t* lda,
                                                           const ProbDesc* prob, const int64_t* tile_start, int nprob) {
  const int64_t g = blockIdx.x;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (tile_start[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const ProbDesc& pd = prob[lo];
  const int64_t t = g - tile_start[lo];
  const int64_t r = t % pd.p, c = t / pd.p;
  const int nb = pd.nb;
  const double* A = Aptr[lo];
  const int64_t ld = lda[lo];
  double* dst = pd.tiles + (c * pd.p + r) * nb * nb;
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int cc = e / nb, rr = e - cc * nb;
    dst[e] = A[(c * nb + cc) * ld + r * nb + rr];
  }
}

// tiles -> column-major out (ld) for rows x cols (upper_only: zero below the
// diagonal, used for R).
__global__ void unpack_kernel(const double* tiles, double* out, int64_t ld, int p, int nb, int64_t rows, int64_t cols,
                              int upper_only) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t col = e / rows, row = e - col * rows;
    const int64_t r = row / nb, c = col / nb;
    double v = tiles[(c * p + r) * nb * nb + (col - c * nb) * nb + (row - r * nb)];
    if (upper_only && row > col) v = 0.0;
    out[col * ld + row] = v;
  }
}

__global__ void tau_kernel(const double* Tg, const double* Tp, double* tau, int p, int q, int nb) {
  const int64_t per = static_cast<int64_t>(p) * q * nb;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < 2 * per;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int which = e >= per;
    const int64_t x = e - which * per;
    const int64_t t = x / nb, j = x - t * nb;
    const double* T = (which ? Tp : Tg) + t * static_cast<int64_t>(IB) * nb;
    const int64_t b = j / IB, jj = j - b * IB;
    tau[e] = T[b * IB * IB + jj + jj * IB];
  }
}

// B (ldb, m x nrhs) -> p row tiles of nb x ncolB (ld nb), zero padded.
__global__ void pack_b_kernel(const double* B, int64_t ldb, int64_t nrhs, double* Bt, int p, int nb, int ncolB) {
  const int64_t total = static_cast<int64_t>(p) * nb * ncolB;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = e / (static_cast<int64_t>(nb) * ncolB);
    const int64_t x = e - r * nb * ncolB;
    const int64_t col = x / nb, row = x - col * nb;
    Bt[e] = col < nrhs ? B[col * ldb + r * nb + row] : 0.0;
  }
}

__global__ void unpack_b_kernel(const double* Bt, double* B, int64_t ldb, int64_t nrhs, int64_t rows, int nb,
                                int ncolB) {
  const int64_t total = rows * nrhs;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t col = e / rows, row = e - col * rows;
    const int64_t r = row / nb;
    B[col * ldb + row] = Bt[r * nb * ncolB + col * nb + (row - r * nb)];
  }
}

static int grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return static_cast<int>(g);
}

hipError_t launch_pack(const double* A, int64_t lda, double* tiles, int p, int q, int nb, hipStream_t s) {
  if (nb <= 0 || nb > 1024 || (nb & (nb - 1)) != 0) return hipErrorInvalidValue;
  if (p <= 0 || q <= 0) return hipSuccess;
  const int64_t groups = (static_cast<int64_t>(q) * nb + (1024 / nb) - 1) / (1024 / nb);
  const dim3 grid(static_cast<unsigned>(groups), static_cast<unsigned>(p < 65535 ? p : 65535));
  hipLaunchKernelGGL(pack_kernel, grid, dim3(256), 0, s, A, lda, tiles, p, q, nb);
  return hipGetLastError();
}
hipError_t launch_unpack(const double* tiles, double* out, int64_t ld, int p, int q, int nb, int rows, int cols,
                         int upper_only, hipStream_t s) {
  (void)q;
  hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(static_cast<int64_t>(rows) * cols)), dim3(256), 0, s, tiles, out,
                     ld, p, nb, static_cast<int64_t>(rows), static_cast<int64_t>(cols), upper_only);
  return hipGetLastError();
}
hipError_t launch_tau(const double* Tg, const double* Tp, double* tau, int p, int q, int nb, hipStream_t s) {
  hipLaunchKernelGGL(tau_kernel, dim3(grid_for(2LL * p * q * nb)), dim3(256), 0, s, Tg, Tp, tau, p, q, nb);
  return hipGetLastError();
}
hipError_t launch_pack_b(const double* B, int64_t ldb, int64_t nrhs, double* Bt, int p, int nb, int ncolB,
                         hipStream_t s) {
  hipLaunchKernelGGL(pack_b_kernel, dim3(grid_for(static_cast<int64_t>(p) * nb * ncolB)), dim3(256), 0, s, B, ldb,
                     nrhs, Bt, p, nb, ncolB);
  return hipGetLastError();
}
hipError_t launch_unpack_b(const double* Bt, double* B, int64_t ldb, int64_t nrhs, int rows, int nb, int ncolB,
                           hipStream_t s) {
  hipLaunchKernelGGL(unpack_b_kernel, dim3(grid_for(static_cast<int64_t>(rows) * nrhs)), dim3(256), 0, s, Bt, B, ldb,
                     nrhs, static_cast<int64_t>(rows), nb, ncolB);
  return hipGetLastError();
}

hipError_t launch_pack_batched(const double* const* Aptr, const int64_t* lda, const ProbDesc* prob,
                               const int64_t* tile_start, int nprob, int64_t ntiles, int nbmax, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  (void)nbmax;
  hipLaunchKernelGGL(pack_batched_kernel, dim3(static_cast<unsigned>(ntiles)), dim3(256), 0, s, Aptr, lda, prob,
                     tile_start, nprob);
  return hipGetLastError();
}

}  // namespace tqr
