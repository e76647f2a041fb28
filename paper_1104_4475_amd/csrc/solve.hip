// Least-squares helpers: triangular solve with the tiled R, FP64 residuals
// and column norms for the backward error of the refinement loop.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace tqr {

namespace {

__device__ __forceinline__ const double* rtile(const double* tiles, int p, int nb, int r, int c) {
  return tiles + (static_cast<size_t>(c) * p + r) * static_cast<size_t>(nb) * nb;
}

// Back substitution X = R^{-1} Y with the tiled upper triangular R (tiles
// (i, k), i <= k < q), in place in Y (rows i nb .. i nb + nb - 1 of tile row
// i).  One workgroup per tile row, block b taking row i = q - 1 - b, so a
// workgroup only waits for workgroups with smaller indices (already
// running): no residency assumption.  Row i applies Y_i -= R_ik X_k for
// k = q-1 .. i+1 as each X_k is published (flag k set to the launch's epoch),
// then solves R_ii X_i = Y_i: 32-row blocks from the bottom, each solved on
// one wave by sequential substitution with broadcasts by readlane, and
// subtracted from the rows above by all waves.  Up to TR_COLS right-hand
// sides per launch.  A wait longer than spin_ticks sets *err and the
// workgroup leaves.
constexpr int TR_THREADS = 512;
constexpr int TR_COLS = 16;

__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double readlane_d(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// ys[c * NB + row] -= sum_l op(M)[row][l0 + l] * xs[c * NB + l0 + l] for
// rows in [rlo, rhi), l < nl, columns < nc, with op(M) = M (element (r, c)
// at c * NB + r) or, with TRANS, M^T.  Thread t handles row t % NB and the
// l-range part t / NB of G = TR_THREADS / NB parts (loads issued 16 at a
// time); the G partial sums meet in ps and are added in a fixed order.
// Contains barriers: every thread calls it.
template <int NB, bool TRANS>
__device__ __forceinline__ void tr_update(double* ys, const double* xs, const double* M, int l0, int nl, int rlo,
                                          int rhi, int nc, double* ps) {
  constexpr int G = TR_THREADS / NB;
  const int row = threadIdx.x % NB, part = threadIdx.x / NB;
  const int per = (nl + G - 1) / G;
  const int la = part * per, lb = (la + per < nl) ? la + per : nl;
  const bool live = row >= rlo && row < rhi;
  double acc[TR_COLS];
#pragma unroll
  for (int c = 0; c < TR_COLS; ++c) acc[c] = 0.0;
  if (live) {
    for (int l = la; l < lb; l += 16) {
      double m[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const size_t idx = TRANS ? static_cast<size_t>(row) * NB + l0 + l + u
                                 : static_cast<size_t>(l0 + l + u) * NB + row;
        m[u] = (l + u < lb) ? M[idx] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (l + u < lb) {
#pragma unroll
          for (int c = 0; c < TR_COLS; ++c)
            if (c < nc) acc[c] += m[u] * xs[c * NB + l0 + l + u];
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < TR_COLS; ++c)
    if (c < nc) ps[(part * TR_COLS + c) * NB + row] = acc[c];
  __syncthreads();
  for (int e = threadIdx.x; e < TR_COLS * NB; e += TR_THREADS) {
    const int c = e / NB, r = e % NB;
    if (c < nc && r >= rlo && r < rhi) {
      double t = 0.0;
      for (int g = 0; g < G; ++g) t += ps[(g * TR_COLS + c) * NB + r];
      ys[c * NB + r] -= t;
    }
  }
}

// Whole-tile product ys[c * NB + r] -= sum_l op(M)[r][l] xs[c * NB + l]
// for all NB rows and columns c < nc, with coalesced loads of M:
//   op(M) = M:   wave w takes the tile columns l = w + 8 t (contiguous in
//                memory, lanes over rows), accumulates its partial sums for
//                every row and the 8 partials meet in ps (4 right-hand sides
//                per pass);
//   op(M) = M^T: wave w takes the output rows r = w + 8 t, whose entries are
//                tile column r (lanes over l), and reduces across the wave.
// Loads are issued TB columns at a time before their use.  Contains
// barriers: every thread calls it.
template <int NB, bool TRANS>
__device__ __forceinline__ void tile_gemv(double* ys, const double* xs, const double* M, int nc, double* ps) {
  constexpr int RJ = NB >= 64 ? NB / 64 : 1;  // entries of a column per lane
  constexpr int NW = TR_THREADS / 64;         // waves
  constexpr int PER = NB / NW;                // columns (rows for M^T) per wave
  constexpr int TB = PER < 8 ? PER : 8;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int c0 = 0; c0 < nc; c0 += 4) {
    if (!TRANS) {
      double acc[RJ][4];
#pragma unroll
      for (int j = 0; j < RJ; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[j][c] = 0.0;
      for (int t0 = 0; t0 < PER; t0 += TB) {
        double m[TB][RJ];
#pragma unroll
        for (int b = 0; b < TB; ++b)
#pragma unroll
          for (int j = 0; j < RJ; ++j) {
            const int r = lane + 64 * j;
            m[b][j] = r < NB ? M[static_cast<size_t>(w + NW * (t0 + b)) * NB + r] : 0.0;
          }
#pragma unroll
        for (int b = 0; b < TB; ++b) {
          const int l = w + NW * (t0 + b);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double x = (c0 + c < nc) ? xs[(c0 + c) * NB + l] : 0.0;
#pragma unroll
            for (int j = 0; j < RJ; ++j) acc[j][c] += m[b][j] * x;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        const int r = lane + 64 * j;
        if (r < NB) {
#pragma unroll
          for (int c = 0; c < 4; ++c) ps[(w * 4 + c) * NB + r] = acc[j][c];
        }
      }
      __syncthreads();
      for (int e = threadIdx.x; e < 4 * NB; e += TR_THREADS) {
        const int c = e / NB, r = e % NB;
        if (c0 + c < nc) {
          double t = 0.0;
#pragma unroll
          for (int v = 0; v < NW; ++v) t += ps[(v * 4 + c) * NB + r];
          ys[(c0 + c) * NB + r] -= t;
        }
      }
      __syncthreads();
    } else {
      for (int t0 = 0; t0 < PER; t0 += TB) {
        double m[TB][RJ];
#pragma unroll
        for (int b = 0; b < TB; ++b)
#pragma unroll
          for (int j = 0; j < RJ; ++j) {
            const int l = lane + 64 * j;
            m[b][j] = l < NB ? M[static_cast<size_t>(w + NW * (t0 + b)) * NB + l] : 0.0;
          }
#pragma unroll
        for (int b = 0; b < TB; ++b) {
          const int r = w + NW * (t0 + b);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (c0 + c >= nc) continue;
            double part = 0.0;
#pragma unroll
            for (int j = 0; j < RJ; ++j) {
              const int l = lane + 64 * j;
              if (l < NB) part += m[b][j] * xs[(c0 + c) * NB + l];
            }
            for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
            if (lane == 0) ys[(c0 + c) * NB + r] -= part;
          }
        }
      }
      __syncthreads();
    }
  }
}

// ys[c * NB + r] -= sum_l M[r][l] xs[c * NB + l] for the ROWS rows r =
// rlo .. rlo + ROWS - 1 only (ROWS = 64: one row per lane), columns split
// over the waves as in tile_gemv.  Contains barriers.
template <int NB, int ROWS>
__device__ __forceinline__ void rows_gemv(double* ys, const double* xs, const double* M, int rlo, int nc, double* ps) {
  static_assert(ROWS == 64, "one row per lane");
  constexpr int NW = TR_THREADS / 64;
  constexpr int PER = NB / NW;
  constexpr int TB = PER < 8 ? PER : 8;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = rlo + lane;
  for (int c0 = 0; c0 < nc; c0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int t0 = 0; t0 < PER; t0 += TB) {
      double m[TB];
#pragma unroll
      for (int b = 0; b < TB; ++b) m[b] = M[static_cast<size_t>(w + NW * (t0 + b)) * NB + r];
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int l = w + NW * (t0 + b);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += m[b] * ((c0 + c < nc) ? xs[(c0 + c) * NB + l] : 0.0);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) ps[(w * 4 + c) * ROWS + lane] = acc[c];
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * ROWS; e += TR_THREADS) {
      const int c = e / ROWS, rr = e % ROWS;
      if (c0 + c < nc) {
        double t = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) t += ps[(v * 4 + c) * ROWS + rr];
        ys[(c0 + c) * NB + rlo + rr] -= t;
      }
    }
    __syncthreads();
  }
}

// Inverse of diagonal block w (32 x 32, upper triangular) of the tile Rd
// on wave w < NB / 32: lane (rr, half) ends with row rr of the inverse
// (both halves alike); with TRANS, with row rr of the inverse's transpose
// (tb: 32 x 32 doubles of LDS per wave for the transposition).  Other waves
// keep the identity.
template <int NB, bool TRANS>
__device__ __forceinline__ void block_inverse(const double* Rd, int wave, int rr, int half, double (&xinv)[32],
                                              double* tb) {
#pragma unroll
  for (int c = 0; c < 32; ++c) xinv[c] = (c == rr) ? 1.0 : 0.0;
  if (wave >= NB / 32) return;
  const int base = 32 * wave;
  double ur[32];
#pragma unroll
  for (int l = 0; l < 32; ++l) ur[l] = Rd[static_cast<size_t>(base + l) * NB + base + rr];
#pragma unroll
  for (int st = 31; st >= 0; --st) {
    if (rr == st) {
      const double d = 1.0 / ur[st];
#pragma unroll
      for (int c = st; c < 32; ++c) xinv[c] *= d;
    }
#pragma unroll
    for (int c = st; c < 32; ++c) {
      const double v = readlane_d(xinv[c], st);
      if (rr < st) xinv[c] -= ur[st] * v;
    }
  }
  if (TRANS) {
    if (half == 0) {
#pragma unroll
      for (int c = 0; c < 32; ++c) tb[c * 32 + rr] = xinv[c];  // tb[c][rr] = inv[rr][c]
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < 32; ++c) xinv[c] = tb[rr * 32 + c];  // inv[c][rr]
  }
}

// Solve op(R_d) X = Y in place in ys (nc columns, NB rows) with the block
// inverses of block_inverse: 32-row blocks from the bottom for R, from the
// top for R^T; x_b = inv(op(R_bb)) y_b on wave b, then subtracted from the
// rows still to solve by all waves.  Contains barriers.
template <int NB, bool TRANS>
__device__ __forceinline__ void diag_solve(double* ys, const double* Rd, const double (&xinv)[32], double* ps, int nc,
                                           int wave, int rr, int half) {
  for (int s = 0; s < NB / 32; ++s) {
    const int b = TRANS ? s : NB / 32 - 1 - s;
    const int base = 32 * b;
    if (wave == b) {
      double xv[TR_COLS / 2];
#pragma unroll
      for (int u = 0; u < TR_COLS / 2; ++u) {
        xv[u] = 0.0;
        if (2 * u >= nc) continue;
        const double* yc = ys + (half + 2 * u) * NB + base;
#pragma unroll
        for (int l = 0; l < 32; ++l) xv[u] += xinv[l] * yc[l];
      }
#pragma unroll
      for (int u = 0; u < TR_COLS / 2; ++u)
        if (half + 2 * u < nc) ys[(half + 2 * u) * NB + base + rr] = xv[u];
    }
    __syncthreads();
    if (s + 1 < NB / 32) {
      if (TRANS)
        tr_update<NB, true>(ys, ys, Rd, base, 32, base + 32, NB, nc, ps);
      else
        tr_update<NB, false>(ys, ys, Rd, base, 32, 0, base, nc, ps);
      __syncthreads();
    }
  }
}

// Inverses of the diagonal tiles of the tiled upper triangular R: block
// (i, c) writes columns 16 c .. 16 c + 15 of inv(R_ii) (zero below the
// diagonal) into tile i of Rinv (q tiles of NB x NB, column-major), by the
// solve of R_ii X = I restricted to those columns.
template <int NB>
__global__ __launch_bounds__(TR_THREADS) void trinv_kernel(const double* tiles, int p, double* Rinv) {
  __shared__ double ys[NB * TR_COLS];
  __shared__ double ps[TR_THREADS * TR_COLS];
  const int i = blockIdx.x, c0 = blockIdx.y * TR_COLS;
  const int tid = threadIdx.x, lane = tid & 63, rr = lane & 31, half = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) {
    const int c = e / NB, r = e % NB;
    ys[e] = (r == c0 + c) ? 1.0 : 0.0;
  }
  const double* Rd = tiles + (static_cast<size_t>(i) * p + i) * NB * NB;
  double xinv[32];
  block_inverse<NB, false>(Rd, wave, rr, half, xinv, ps + wave * 32 * 32);
  __syncthreads();
  diag_solve<NB, false>(ys, Rd, xinv, ps, TR_COLS, wave, rr, half);
  double* out = Rinv + static_cast<size_t>(i) * NB * NB + static_cast<size_t>(c0) * NB;
  for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) out[e] = ys[e];
}

// Coupling tiles of the triangular solves: block (i, c) writes columns
// 16 c .. 16 c + 15 of Wn_i = -inv(op(R_ii)) N_i into tile i of Wn, where
// N_i is the tile coupling row i to the row solved dist rows before it: for
// R (back substitution) N_i = R_{i,i+dist}, i < q - dist; for R^T (forward)
// N_i = (R^T)_{i,i-dist}, tile (i, i - dist) of Rt, i >= dist.  Inv holds
// the inverses of the diagonal tiles (of R, or their transposes for R^T),
// so the tile is one product: the 16 columns of N_i in LDS, thread t forms
// row t % NB of TR_COLS / (TR_THREADS / NB) of them, reading the inverse's
// rows coalesced.
template <int NB, bool TRANS>
__global__ __launch_bounds__(TR_THREADS) void coupling_kernel(const double* tiles, const double* Rt,
                                                              const double* Inv, int p, int q, int dist, double* Wn) {
  constexpr int CG = TR_THREADS / NB;  // column groups
  constexpr int CPT = TR_COLS / CG;    // columns per thread
  static_assert(CG >= 1 && CPT >= 1 && CPT * CG == TR_COLS, "column split");
  __shared__ double ns[TR_COLS * NB];
  const int i = TRANS ? static_cast<int>(blockIdx.x) + dist : static_cast<int>(blockIdx.x);
  const int c0 = blockIdx.y * TR_COLS;
  const int tid = threadIdx.x, r = tid % NB, cg = tid / NB;
  const double* N = TRANS ? Rt + (static_cast<size_t>(i - dist) * q + i) * NB * NB
                          : tiles + (static_cast<size_t>(i + dist) * p + i) * NB * NB;
  for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) ns[e] = N[static_cast<size_t>(c0) * NB + e];
  __syncthreads();
  const double* M = Inv + static_cast<size_t>(i) * NB * NB;
  double acc[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) acc[c] = 0.0;
#pragma unroll 4
  for (int k = 0; k < NB; ++k) {
    const double a = M[static_cast<size_t>(k) * NB + r];
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc[c] += a * ns[(cg * CPT + c) * NB + k];
  }
  double* out = Wn + static_cast<size_t>(i) * NB * NB + static_cast<size_t>(c0) * NB;
#pragma unroll
  for (int c = 0; c < CPT; ++c) out[static_cast<size_t>(cg * CPT + c) * NB + r] = -acc[c];
}

// X = R^{-1} Y (TRANS = false) or X = R^{-T} Y (TRANS = true) in place in Y
// (rows i nb .. i nb + nb - 1 of tile row i), with the tiled upper
// triangular R (tiles (i, k), i <= k < q).  One workgroup per tile row,
// ordered so that a workgroup only waits for workgroups with smaller
// indices (already running): block b takes row q - 1 - b (back
// substitution) or row b (forward substitution with R^T).  Row i applies
// Y_i -= op(R)_ik X_k for every solved X_k (flag k set to the launch's
// epoch), then solves its diagonal tile: with Rinv (the inverses of the
// diagonal tiles from trinv_kernel) as one product X_i = op(inv(R_ii)) Y_i,
// else by diag_solve.  With TRANS and Rt (the tiles of R^T, from
// launch_transpose_r: tile (i, k), k <= i, of a q x q tile grid) the
// products read Rt and Rinv = the transposed inverses without transposition,
// so every load is coalesced.  INV: Rinv is given (a compile-time variant,
// so that the substitution's block inverses hold no registers in the
// product path).  With Wn (coupling tiles from coupling_kernel) as well,
// row i forms z_i = op(inv(R_ii)) (Y_i - sum over the rows solved before
// the last one) before it waits for that last row, then X_i = z_i + Wn_i
// X_last: one tile product per step on the solve's critical chain instead
// of two (trsm_part_kernel splits each row over several workgroups at
// NB >= 128).  Up to TR_COLS right-hand sides per launch.  A wait longer
// than spin_ticks sets *err and the workgroup leaves.
template <int NB, bool TRANS, bool INV>
__global__ __launch_bounds__(TR_THREADS) void trsm_wave_kernel(const double* tiles, const double* Rt,
                                                               const double* Rinv, const double* Wn, int p, int q,
                                                               double* Y, int64_t ldy, int nc, int32_t* flags,
                                                               int32_t epoch, int64_t spin_ticks, int32_t* err) {
  constexpr int GP = 1;
  __shared__ double ys[NB * TR_COLS];
  __shared__ double xs[NB * TR_COLS];
  __shared__ double ps[TR_THREADS * TR_COLS];  // partial sums of tr_update; block inverses for TRANS
  __shared__ int s_abort;
  const int blk = static_cast<int>(blockIdx.x) / GP, part = static_cast<int>(blockIdx.x) % GP;
  const int i = TRANS ? blk : q - 1 - blk;
  const int tid = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(i) * NB;
  for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) {
    const int c = e / NB, r = e % NB;
    ys[e] = c < nc ? Y[c * ldy + r0 + r] : 0.0;
  }
  if (tid == 0) s_abort = 0;
  const double* Rd = tiles + (static_cast<size_t>(i) * p + i) * NB * NB;
  const int lane = tid & 63, rr = lane & 31, half = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double xinv[32];
  if (!INV) block_inverse<NB, TRANS>(Rd, wave, rr, half, xinv, ps + wave * 32 * 32);
  __syncthreads();
  // Wait for the flags of row k (all its parts), then xs = X_k; false when
  // the wait failed.
  auto fetch = [&](int k) {
    if (tid == 0) {
      const uint64_t t0 = wall_clock64();
      for (int g = 0; g < GP && !s_abort; ++g) {
        while (__hip_atomic_load(flags + k * GP + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
          if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
              static_cast<int64_t>(wall_clock64() - t0) > spin_ticks) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_abort = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_abort)) return false;
    const int64_t k0 = static_cast<int64_t>(k) * NB;
    for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) {
      const int c = e / NB, r = e % NB;
      xs[e] = c < nc ? ld_coh(Y + c * ldy + k0 + r) : 0.0;
    }
    __syncthreads();
    return true;
  };
  // The row solved just before this one (coupled through Wn), if any.
  const bool coupled = INV && Wn && (TRANS ? i > 0 : i < q - 1);
  const int k_first = TRANS ? 0 : q - 1;
  const int k_end = coupled ? (TRANS ? i - 1 : i + 1) : i;
  for (int k = k_first; TRANS ? (k < k_end) : (k > k_end); k += TRANS ? 1 : -1) {
    if (!fetch(k)) return;
    // op(R)_ik: R_ik = tile (i, k) for the upper solve; (R_ki)^T for R^T.
    if (TRANS && Rt) {
      tile_gemv<NB, false>(ys, xs, Rt + (static_cast<size_t>(k) * q + i) * NB * NB, nc, ps);
    } else {
      const double* R = TRANS ? tiles + (static_cast<size_t>(i) * p + k) * NB * NB
                              : tiles + (static_cast<size_t>(k) * p + i) * NB * NB;
      tile_gemv<NB, TRANS>(ys, xs, R, nc, ps);
    }
  }
  double sign = 1.0;
  if (INV) {
    // xs = Y_i, ys = -op(inv(R_ii)) Y_i.
    for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) {
      xs[e] = ys[e];
      ys[e] = 0.0;
    }
    __syncthreads();
    if (TRANS && Rt)
      tile_gemv<NB, false>(ys, xs, Rinv + static_cast<size_t>(i) * NB * NB, nc, ps);
    else
      tile_gemv<NB, TRANS>(ys, xs, Rinv + static_cast<size_t>(i) * NB * NB, nc, ps);
    sign = -1.0;
    if (coupled) {
      // ys = -z_i - Wn_i X_last = -X_i.
      if (!fetch(k_end)) return;
      tile_gemv<NB, false>(ys, xs, Wn + static_cast<size_t>(i) * NB * NB, nc, ps);
    }
  } else {
    diag_solve<NB, TRANS>(ys, Rd, xinv, ps, nc, wave, rr, half);
  }
  constexpr int PR = NB / GP;  // rows stored by this workgroup
  for (int e = tid; e < PR * TR_COLS; e += TR_THREADS) {
    const int c = e / PR, r = part * PR + e % PR;
    if (c < nc) st_coh(Y + c * ldy + r0 + r, sign * ys[c * NB + r]);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) __hip_atomic_store(flags + i * GP + part, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The solve of trsm_wave_kernel with the inverses and two coupling tiles per
// row, at NB >= 128: GP = NB / 64 workgroups per tile row, part g owning
// rows 64 g .. 64 g + 63 of the row.  With Wn_i = -op(R_ii)^{-1} N_i (the
// row solved just before) and Wn2_i = -op(R_ii)^{-1} N2_i (the one before
// it):  X_i = op(R_ii)^{-1} w_i + Wn2_i X_{i+-2} + Wn_i X_{i+-1},  w_i = Y_i
// - sum of op(R)_ik X_k over the rows solved earlier still.  Each part
// forms its rows of w_i as those rows arrive (reading its 64 rows of each
// tile), publishes them (wbuf, wflags), gathers the whole w_i from the
// other parts and applies its rows of the inverse: all of this a step
// before X_{i+-1} is known.  After X_{i+-2} comes one 64-row product with
// Wn2_i, and after X_{i+-1} one with Wn_i: the only product on the solve's
// chain reads a quarter of a tile at NB = 256.  Y is solved in place: a
// part reads only its own rows of Y_i, which no other workgroup writes
// before every part of the row has published its partial sum.
template <int NB, bool TRANS, int GP>
__global__ __launch_bounds__(TR_THREADS) void trsm_part_kernel(const double* tiles, const double* Rt,
                                                               const double* Rinv, const double* Wn, const double* Wn2,
                                                               int p, int q, double* Y, int64_t ldy, int nc,
                                                               int32_t* flags,
                                                               int32_t* wflags, double* wbuf, int32_t epoch,
                                                               int64_t spin_ticks, int32_t* err) {
  static_assert(GP >= 2 && NB / GP == 64, "parts of 64 rows");
  __shared__ double ys[NB * TR_COLS];
  __shared__ double xs[NB * TR_COLS];
  __shared__ double ps[TR_THREADS * TR_COLS];
  __shared__ int s_abort;
  const int blk = static_cast<int>(blockIdx.x) / GP, part = static_cast<int>(blockIdx.x) % GP;
  const int i = TRANS ? blk : q - 1 - blk;
  const int tid = threadIdx.x, rlo = part * 64;
  const int64_t r0 = static_cast<int64_t>(i) * NB;
  for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) {
    const int c = e / NB, r = e % NB;
    ys[e] = (c < nc && r >= rlo && r < rlo + 64) ? Y[c * ldy + r0 + r] : 0.0;
  }
  if (tid == 0) s_abort = 0;
  __syncthreads();
  // Wait until every part of row k has set its flag in fl, then xs = the
  // NB x nc block at src (ld lds); false when the wait failed.
  auto gather = [&](const int32_t* fl, int k, const double* src, int64_t lds) {
    if (tid == 0) {
      const uint64_t t0 = wall_clock64();
      for (int g = 0; g < GP && !s_abort; ++g) {
        while (__hip_atomic_load(const_cast<int32_t*>(fl) + k * GP + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
               epoch) {
          if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
              static_cast<int64_t>(wall_clock64() - t0) > spin_ticks) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_abort = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_abort)) return false;
    for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) {
      const int c = e / NB, r = e % NB;
      xs[e] = c < nc ? ld_coh(src + c * lds + r) : 0.0;
    }
    __syncthreads();
    return true;
  };
  auto row_x = [&](int k) { return gather(flags, k, Y + static_cast<int64_t>(k) * NB, ldy); };
  // Stores this part's rows of ys (times sign) at dst (ld ldd), then sets
  // its flag in fl.
  auto publish = [&](double* dst, int64_t ldd, double sign, int32_t* fl) {
    for (int e = tid; e < 64 * TR_COLS; e += TR_THREADS) {
      const int c = e / 64, r = rlo + e % 64;
      if (c < nc) st_coh(dst + c * ldd + r, sign * ys[c * NB + r]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(fl + i * GP + part, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  // 1. This part's rows of w_i.
  const int near2 = TRANS ? i - 2 : i + 2;  // rows coupled through Wn2 / Wn
  const int near1 = TRANS ? i - 1 : i + 1;
  const int k_first = TRANS ? 0 : q - 1;
  for (int k = k_first; TRANS ? (k < near2) : (k > near2); k += TRANS ? 1 : -1) {
    if (!row_x(k)) return;
    const double* R = TRANS ? Rt + (static_cast<size_t>(k) * q + i) * NB * NB
                            : tiles + (static_cast<size_t>(k) * p + i) * NB * NB;
    rows_gemv<NB, 64>(ys, xs, R, rlo, nc, ps);
  }
  // 2. The whole w_i from every part, then ys = -(this part's rows of
  // op(R_ii)^{-1} w_i).
  double* wrow = wbuf + static_cast<int64_t>(i) * NB;
  const int64_t ldw = static_cast<int64_t>(q) * NB;
  publish(wrow, ldw, 1.0, wflags);
  if (!gather(wflags, i, wrow, ldw)) return;
  for (int e = tid; e < NB * TR_COLS; e += TR_THREADS) ys[e] = 0.0;
  __syncthreads();
  rows_gemv<NB, 64>(ys, xs, Rinv + static_cast<size_t>(i) * NB * NB, rlo, nc, ps);
  // 3. ys -= Wn2_i X_near2 and Wn_i X_near1 (this part's rows): ys = -X_i.
  if (TRANS ? near2 >= 0 : near2 < q) {
    if (!row_x(near2)) return;
    rows_gemv<NB, 64>(ys, xs, Wn2 + static_cast<size_t>(i) * NB * NB, rlo, nc, ps);
  }
  if (TRANS ? near1 >= 0 : near1 < q) {
    if (!row_x(near1)) return;
    rows_gemv<NB, 64>(ys, xs, Wn + static_cast<size_t>(i) * NB * NB, rlo, nc, ps);
  }
  publish(Y + r0, ldy, -1.0, flags);
}

// Tile transposes for the R^T solve: block (a, b), a >= b, writes
// dst tile (a, b) of a q x q grid = (src tile (b, a) of a p-row grid)^T;
// with diag, block (i, 0) writes dst tile i = (src tile i)^T (single tiles
// laid out one after the other).  64 x 64 sub-blocks through LDS.
template <int NB>
__global__ __launch_bounds__(256) void transpose_tiles_kernel(const double* src, int p, int q, double* dst, int diag) {
  __shared__ double buf[64][65];
  const int a = blockIdx.x, b = blockIdx.y;
  const double* S;
  double* D;
  if (diag) {
    if (b != 0) return;
    S = src + static_cast<size_t>(a) * NB * NB;
    D = dst + static_cast<size_t>(a) * NB * NB;
  } else {
    if (a < b) return;
    S = src + (static_cast<size_t>(a) * p + b) * NB * NB;
    D = dst + (static_cast<size_t>(b) * q + a) * NB * NB;
  }
  constexpr int SB = NB < 64 ? NB : 64;
  const int tx = threadIdx.x % SB, ty = threadIdx.x / SB;
  constexpr int RY = 256 / SB;
  for (int r0 = 0; r0 < NB; r0 += SB)
    for (int c0 = 0; c0 < NB; c0 += SB) {
      // buf[c][r] = S[r0 + r][c0 + c] (column-major S: (r, c) at c * NB + r).
      for (int c = ty; c < SB; c += RY) buf[c][tx] = S[static_cast<size_t>(c0 + c) * NB + r0 + tx];
      __syncthreads();
      // D[c0 + c][r0 + r] = S[r0 + r][c0 + c]: D column r0 + r, row c0 + c.
      for (int r = ty; r < SB; r += RY) D[static_cast<size_t>(r0 + r) * NB + c0 + tx] = buf[tx][r];
      __syncthreads();
    }
}

// out[c * ldo + j] = sign * sum_r A[j * lda + r] Y[c * ldy + r] for j < n,
// c < nrhs: one wave per GV_COLS consecutive columns (each load of Y serves
// all of them; the last wave's missing columns re-read column n - 1 and are
// not written), lanes over rows, eight rows per lane per pass with every
// load issued before the products, up to four right-hand sides per pass.
constexpr int GV_COLS = 4;
__global__ __launch_bounds__(256) void gemv_t_kernel(const double* A, int64_t lda, int64_t m, int64_t n,
                                                     const double* Y, int64_t ldy, int64_t nrhs, double* out,
                                                     int64_t ldo, double sign) {
  const int64_t j0 = ((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6) * GV_COLS;
  const int lane = threadIdx.x & 63;
  if (j0 >= n) return;
  const double* a[GV_COLS];
#pragma unroll
  for (int q = 0; q < GV_COLS; ++q) a[q] = A + (j0 + q < n ? j0 + q : n - 1) * lda;
  for (int64_t c0 = 0; c0 < nrhs; c0 += 4) {
    double s[GV_COLS][4] = {};
    int64_t r = lane;
    for (; r + 7 * 64 < m; r += 8 * 64) {
      double v[GV_COLS][8];
#pragma unroll
      for (int q = 0; q < GV_COLS; ++q)
#pragma unroll
        for (int u = 0; u < 8; ++u) v[q][u] = a[q][r + 64 * u];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if (c0 + h >= nrhs) continue;
        const double* y = Y + (c0 + h) * ldy + r;
        double yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) yv[u] = y[64 * u];
#pragma unroll
        for (int q = 0; q < GV_COLS; ++q)
#pragma unroll
          for (int u = 0; u < 8; ++u) s[q][h] += v[q][u] * yv[u];
      }
    }
    for (; r < m; r += 64) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if (c0 + h >= nrhs) continue;
        const double yv = Y[(c0 + h) * ldy + r];
#pragma unroll
        for (int q = 0; q < GV_COLS; ++q) s[q][h] += a[q][r] * yv;
      }
    }
#pragma unroll
    for (int q = 0; q < GV_COLS; ++q)
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        double t = s[q][h];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane == 0 && c0 + h < nrhs && j0 + q < n) out[(c0 + h) * ldo + j0 + q] = sign * t;
      }
  }
}

// Rv = B - A X for m x n A; grid (row blocks, column chunks), partial sums
// subtracted with FP64 atomics (Rv must hold B on entry).  The chunk's rows
// of X (four right-hand sides per pass) are staged once per workgroup in
// LDS, interleaved by right-hand side, and each thread streams its row of
// A sixteen columns at a time.  With fro2, the sum of squares of the
// elements of A read (each once, in the first pass) is added to *fro2: one
// atomic per workgroup.
constexpr int RES_CHUNK = 512;
constexpr int RES_STEP = 16;
__global__ __launch_bounds__(256) void residual_kernel(const double* A, int64_t lda, int64_t m, int64_t n,
                                                       const double* X, int64_t ldx, int64_t nrhs, double* Rv,
                                                       int64_t ldr, double* fro2) {
  __shared__ __attribute__((aligned(16))) double xs[4 * RES_CHUNK];
  __shared__ double red[4];
  double sq = 0.0;
  const int64_t row = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * RES_CHUNK;
  const int nc = static_cast<int>((c0 + RES_CHUNK < n) ? RES_CHUNK : n - c0);
  const double* arow = A + c0 * lda + (row < m ? row : 0);
  for (int64_t h0 = 0; h0 < nrhs; h0 += 4) {
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * RES_CHUNK; e += blockDim.x) {
      const int c = e >> 2, h = e & 3;
      xs[e] = (c < nc && h0 + h < nrhs) ? X[(h0 + h) * ldx + c0 + c] : 0.0;
    }
    __syncthreads();
    if (row >= m) continue;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int c = 0;
    for (; c + RES_STEP <= nc; c += RES_STEP) {
      double a[RES_STEP];
#pragma unroll
      for (int u = 0; u < RES_STEP; ++u) a[u] = arow[(c + u) * lda];
#pragma unroll
      for (int u = 0; u < RES_STEP; ++u) {
        const double* x = xs + 4 * (c + u);
#pragma unroll
        for (int h = 0; h < 4; ++h) s[h] += a[u] * x[h];
      }
      if (fro2 && h0 == 0) {
#pragma unroll
        for (int u = 0; u < RES_STEP; ++u) sq += a[u] * a[u];
      }
    }
    for (; c < nc; ++c) {
      const double a = arow[c * lda];
#pragma unroll
      for (int h = 0; h < 4; ++h) s[h] += a * xs[4 * c + h];
      if (h0 == 0) sq += a * a;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h)
      if (h0 + h < nrhs) atomicAdd(Rv + (h0 + h) * ldr + row, -s[h]);
  }
  if (fro2) {
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(fro2, red[0] + red[1] + red[2] + red[3]);
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
                                                        int64_t rows, int64_t cols, double alpha) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t c = e / rows, r = e - c * rows;
    X[c * ldx + r] += alpha * D[c * ldd + r];
  }
}

int grid_of(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 4096) g = 4096;
  return g < 1 ? 1 : static_cast<int>(g);
}

}  // namespace

template <bool TRANS>
static hipError_t trsm_launch(const double* tiles, const double* Rt, const double* Rinv, const double* Wn, int p, int q,
                              int nb, double* Y, int64_t ldy, int64_t nrhs, int32_t* flags, int32_t* epoch,
                              int32_t* err, int64_t spin_ticks, hipStream_t s) {
  // Parts per tile row: NB / 64 workgroups with the inverses and coupling
  // tiles at NB >= 128 (trsm_part_kernel, which exchanges partial sums
  // through wbuf, n x TR_COLS), else one (trsm_wave_kernel).
  const int gp = (Rinv && Wn && nb >= 128 && (!TRANS || Rt)) ? nb / 64 : 1;
  const int64_t n = static_cast<int64_t>(q) * nb;
  double* wbuf = nullptr;
  if (gp > 1) {
    const hipError_t e =
        hipMallocAsync(reinterpret_cast<void**>(&wbuf), static_cast<size_t>(n) * TR_COLS * sizeof(double), s);
    if (e != hipSuccess) return e;
  }
  hipError_t status = hipSuccess;
  for (int64_t c0 = 0; c0 < nrhs && status == hipSuccess; c0 += TR_COLS) {
    const int nc = static_cast<int>(nrhs - c0 < TR_COLS ? nrhs - c0 : TR_COLS);
    const int32_t ep = ++*epoch;
    double* Yc = Y + c0 * ldy;
    switch (nb * 4 + (Rinv ? 2 : 0) + (gp > 1 ? 1 : 0)) {
#define TQR_TRSM(NBV, INVV)                                                                                       \
  case NBV * 4 + INVV * 2:                                                                                        \
    hipLaunchKernelGGL((trsm_wave_kernel<NBV, TRANS, INVV>), dim3(q), dim3(TR_THREADS), 0, s, tiles, Rt, Rinv, Wn, \
                       p, q, Yc, ldy, nc, flags, ep, spin_ticks, err);                                           \
    break;
      TQR_TRSM(32, 0)
      TQR_TRSM(32, 1)
      TQR_TRSM(64, 0)
      TQR_TRSM(64, 1)
      TQR_TRSM(128, 0)
      TQR_TRSM(128, 1)
      TQR_TRSM(256, 0)
      TQR_TRSM(256, 1)
#undef TQR_TRSM
#define TQR_TRSM_PART(NBV, GPV)                                                                                \
  case NBV * 4 + 2 + 1:                                                                                        \
    hipLaunchKernelGGL((trsm_part_kernel<NBV, TRANS, GPV>), dim3(q * GPV), dim3(TR_THREADS), 0, s, tiles, Rt,   \
                       Rinv, Wn, Wn + static_cast<size_t>(q) * NBV * NBV, p, q, Yc, ldy, nc, flags, flags + 4 * q, \
                       wbuf, ep, spin_ticks, err);                                                             \
    break;
      TQR_TRSM_PART(128, 2)
      TQR_TRSM_PART(256, 4)
#undef TQR_TRSM_PART
      default:
        status = hipErrorInvalidValue;
    }
  }
  if (status == hipSuccess) status = hipGetLastError();
  if (wbuf) (void)hipFreeAsync(wbuf, s);
  return status;
}

hipError_t launch_trsm_upper(const double* tiles, const double* Rinv, const double* Wn, int p, int q, int nb, double* Y,
                             int64_t ldy, int64_t nrhs, int32_t* flags, int32_t* epoch, int32_t* err,
                             int64_t spin_ticks, hipStream_t s) {
  return trsm_launch<false>(tiles, nullptr, Rinv, Wn, p, q, nb, Y, ldy, nrhs, flags, epoch, err, spin_ticks, s);
}

hipError_t launch_trsm_upper_t(const double* tiles, const double* Rt, const double* Rinv, const double* Wn, int p,
                               int q, int nb, double* Y, int64_t ldy, int64_t nrhs, int32_t* flags, int32_t* epoch,
                               int32_t* err, int64_t spin_ticks, hipStream_t s) {
  return trsm_launch<true>(tiles, Rt, Rinv, Wn, p, q, nb, Y, ldy, nrhs, flags, epoch, err, spin_ticks, s);
}

hipError_t launch_coupling(const double* tiles, const double* Rt, const double* Inv, int p, int q, int nb, int trans,
                           double* Wn, hipStream_t s) {
  if (nb % TR_COLS != 0) return hipErrorInvalidValue;
  // Distance 1 into tiles 0 .. q - 1 of Wn; at nb >= 128 also distance 2
  // into tiles q .. 2q - 1 (the solves there couple two rows).
  const int maxd = nb >= 128 ? 2 : 1;
  for (int dist = 1; dist <= maxd && dist < q; ++dist) {
    const dim3 grid(static_cast<unsigned>(q - dist), static_cast<unsigned>(nb / TR_COLS));
    double* out = Wn + static_cast<size_t>(dist - 1) * q * nb * nb;
    switch (nb * 2 + (trans ? 1 : 0)) {
#define TQR_CPL(NBV, TV)                                                                                       \
  case NBV * 2 + TV:                                                                                           \
    hipLaunchKernelGGL((coupling_kernel<NBV, TV != 0>), grid, dim3(TR_THREADS), 0, s, tiles, Rt, Inv, p, q, dist, \
                       out);                                                                                   \
    break;
      TQR_CPL(32, 0)
      TQR_CPL(32, 1)
      TQR_CPL(64, 0)
      TQR_CPL(64, 1)
      TQR_CPL(128, 0)
      TQR_CPL(128, 1)
      TQR_CPL(256, 0)
      TQR_CPL(256, 1)
#undef TQR_CPL
      default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_transpose_r(const double* tiles, const double* Rinv, int p, int q, int nb, double* Rt,
                              double* RinvT, hipStream_t s) {
  switch (nb) {
#define TQR_TR(NBV)                                                                                          \
  case NBV:                                                                                                  \
    hipLaunchKernelGGL(transpose_tiles_kernel<NBV>, dim3(q, q), dim3(256), 0, s, tiles, p, q, Rt, 0);         \
    hipLaunchKernelGGL(transpose_tiles_kernel<NBV>, dim3(q, 1), dim3(256), 0, s, Rinv, p, q, RinvT, 1);       \
    break;
    TQR_TR(32)
    TQR_TR(64)
    TQR_TR(128)
    TQR_TR(256)
#undef TQR_TR
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_trinv(const double* tiles, int p, int q, int nb, double* Rinv, hipStream_t s) {
  if (nb % TR_COLS != 0) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(q), static_cast<unsigned>(nb / TR_COLS));
  switch (nb) {
    case 32: hipLaunchKernelGGL(trinv_kernel<32>, grid, dim3(TR_THREADS), 0, s, tiles, p, Rinv); break;
    case 64: hipLaunchKernelGGL(trinv_kernel<64>, grid, dim3(TR_THREADS), 0, s, tiles, p, Rinv); break;
    case 128: hipLaunchKernelGGL(trinv_kernel<128>, grid, dim3(TR_THREADS), 0, s, tiles, p, Rinv); break;
    case 256: hipLaunchKernelGGL(trinv_kernel<256>, grid, dim3(TR_THREADS), 0, s, tiles, p, Rinv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* Y, int64_t ldy,
                         int64_t nrhs, double* out, int64_t ldo, double sign, hipStream_t s) {
  const int64_t threads = (n + GV_COLS - 1) / GV_COLS * 64;
  if (threads == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(gemv_t_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s, A, lda, m,
                     n, Y, ldy, nrhs, out, ldo, sign);
  return hipGetLastError();
}

hipError_t launch_residual(const double* A, int64_t lda, int64_t m, int64_t n, const double* X, int64_t ldx,
                           const double* B, int64_t ldb, int64_t nrhs, double* Rv, int64_t ldr, hipStream_t s,
                           double* fro2) {
  hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_of(m * nrhs)), dim3(256), 0, s, B, ldb, Rv, ldr, m, nrhs);
  const dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>((n + RES_CHUNK - 1) / RES_CHUNK));
  hipLaunchKernelGGL(residual_kernel, grid, dim3(256), 0, s, A, lda, m, n, X, ldx, nrhs, Rv, ldr, fro2);
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
                            hipStream_t s, double alpha) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_cols_kernel, dim3(grid_of(rows * cols)), dim3(256), 0, s, X, ldx, D, ldd, rows, cols, alpha);
  return hipGetLastError();
}

hipError_t launch_copy_cols(const double* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                            hipStream_t s) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_of(rows * cols)), dim3(256), 0, s, S, lds, D, ldd, rows, cols);
  return hipGetLastError();
}

}  // namespace tqr
