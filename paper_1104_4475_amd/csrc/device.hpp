// Shared device/host definitions of the HIP tile kernels and executor.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "depcode.hpp"

namespace tqr {

constexpr int IB = 32;        // inner block size of every kernel (Sec. 4: ib = 32)
constexpr int NTHREADS = 512; // 8 waves of 64 lanes (two per SIMD)
constexpr int SLAB = 64;      // columns of C per update subtask (16 per wave)
constexpr int WIDE_SLAB = 128; // columns of a low-precision update subtask at nb >= 128

// Low-precision update subtasks at nb >= 128 read each block of reflectors
// from an image written by the panel subtask that computed it (FP32 or BF16
// reflectors and an FP32 T block, laid out as its padded LDS copy): bytes
// per ib-block for update precision upd (1 FP32, 2 BF16).
constexpr int image_bytes(int nb, int upd) {
  return upd == 1 ? IB * (nb + 4) * 4 + IB * 36 * 4 : IB * (nb + 8) * 2 + nb * 40 * 2 + IB * 36 * 4;
}
// Column slab of update subtasks for a tile size and update precision.
constexpr int update_slab(int nb, int upd) { return (upd != 0 && nb >= 128) ? WIDE_SLAB : SLAB; }

// Executor task kinds: the six tile kernels (Table 1) and the application of
// a panel task's reflectors to right-hand-side row tiles (apply_q).
enum DevKind : int32_t {
  D_GEQRT = 0, D_UNMQR = 1, D_TSQRT = 2, D_TSMQR = 3, D_TTQRT = 4, D_TTMQR = 5,
  D_APPLY_GE = 6,   // B_i <- Q_geqrt(i,k)^{T or N} B_i
  D_APPLY_TS = 7,   // [B_piv; B_i] <- Q_ts(i,k)^{T or N} [...]
  D_APPLY_TT = 8    // [B_piv; B_i] <- Q_tt(i,k)^{T or N} [...]
};

struct DevSub {
  int32_t kind, i, piv, k, j, slab, dep_begin, dep_end;
  int32_t sdep;   // streamed predecessor (C1 writer) or -1
  int32_t pdep;   // offset in deps of the streamed panel blocks, or -1
};

struct ExecArgs {
  double* tiles;        // p*q tiles of nb*nb, tile (r,c) at (c*p + r)*nb*nb
  double* Tg;           // GEQRT T factors, ib*nb per tile
  double* Tp;           // TS/TT T factors of the zeroed tile, ib*nb per tile
  double* B;            // apply_q: p row tiles of nb x ncolB (ld nb)
  const DevSub* sub;
  const int32_t* deps;
  int32_t* flags;       // one per subtask, set to epoch when done
  int32_t* prog;        // one per subtask: 64 epoch + blocks done (streamed updates)
  int32_t* ticket;      // dispatch counter (reset before each launch)
  int32_t* err;         // nonzero once any wait timed out
  int32_t nsub;
  int32_t epoch;
  int32_t p, q, nb;
  int32_t ncolB;        // columns of the B row tiles (multiple of 16)
  int32_t transB;       // apply_q: 1 = Q^T, 0 = Q
  int32_t upd;          // tqr_update_prec: precision of the update subtasks
  int64_t spin_ticks;   // wall-clock ticks a wait may last before giving up
  int64_t* trace;       // optional: per subtask (ticket, ready, end, workgroup)
  int32_t debug;        // diagnostics: bit 0 = clear the workgroup's LDS before each task
  int32_t fused;        // B set and the plan mixes factorization and Q^T B subtasks
  unsigned char* imgg;  // low-precision images of the GEQRT sets (nb >= 128, upd != FP64), nb/ib per tile
  unsigned char* imgp;  // the same for the TS/TT sets, indexed by the zeroed tile
};

// One problem of a batched launch: its tile storage and shape.
struct ProbDesc {
  double* tiles;
  double* Tg;
  double* Tp;
  int32_t p, q, nb, pad;
};

// Batched executor: the subtasks of all problems in one priority order;
// prob_of[t] names the problem of subtask t.  ctl holds the ticket, the
// error word and the epoch, which the reset kernel advances before every
// run (so a captured graph can be replayed).
struct BatchArgs {
  const ProbDesc* prob;
  const int32_t* prob_of;
  const DevSub* sub;
  const int32_t* deps;
  int32_t* flags;
  int32_t* ctl;         // [0] ticket, [1] err, [2] epoch
  int32_t nsub;
  int32_t upd;
  int64_t spin_ticks;
  int64_t* const* trace;  // device word holding the trace buffer (4 int64 per subtask), or null there
};

// Kernel launchers (defined in kernels.hip).
hipError_t launch_persistent(const ExecArgs& a, int grid, hipStream_t s);
hipError_t launch_level(const ExecArgs& a, const int32_t* order, int begin, int count, hipStream_t s);
hipError_t launch_reset(int32_t* ticket, int32_t* err, hipStream_t s);
hipError_t launch_pack(const double* A, int64_t lda, double* tiles, int p, int q, int nb, hipStream_t s);
hipError_t launch_unpack(const double* tiles, double* out, int64_t ld, int p, int q, int nb, int rows, int cols,
                         int upper_only, hipStream_t s);
hipError_t launch_tau(const double* Tg, const double* Tp, double* tau, int p, int q, int nb, hipStream_t s);
hipError_t launch_pack_b(const double* B, int64_t ldb, int64_t nrhs, double* Bt, int p, int nb, int ncolB,
                         hipStream_t s);
hipError_t launch_unpack_b(const double* Bt, double* B, int64_t ldb, int64_t nrhs, int rows, int nb, int ncolB,
                           hipStream_t s);
// X = R^{-1} Y in place (Y: n x nrhs, column-major).  Rinv: inverses of
// the q diagonal tiles from launch_trinv, or null (substitution inside the
// diagonal tiles).  Wn: coupling tiles from launch_coupling (trans 0), or
// null; used with Rinv only.  flags: 8 q int32 owned by the caller (per
// tile row and part of a row: the part's rows of X, then its partial sum),
// compared with the per-launch epoch (*epoch is advanced); err: set when a
// wait exceeds spin_ticks.
hipError_t launch_trsm_upper(const double* tiles, const double* Rinv, const double* Wn, int p, int q, int nb, double* Y,
                             int64_t ldy, int64_t nrhs, int32_t* flags, int32_t* epoch, int32_t* err,
                             int64_t spin_ticks, hipStream_t s);
// X = R^{-T} Y in place (same conventions).  Rt: the tiles of R^T from
// launch_transpose_r with Rinv then the transposed inverses, or null
// (transposed reads of R and Rinv).
hipError_t launch_trsm_upper_t(const double* tiles, const double* Rt, const double* Rinv, const double* Wn, int p,
                               int q, int nb, double* Y, int64_t ldy, int64_t nrhs, int32_t* flags, int32_t* epoch,
                               int32_t* err, int64_t spin_ticks, hipStream_t s);
// Wn = coupling tiles -op(R_ii)^{-1} N_i of the solve with R (trans 0: N_i
// = R_{i,i+d}) or R^T (trans 1: N_i = tile (i, i-d) of Rt): tiles 0 .. q - 1
// for d = 1 and, at nb >= 128, tiles q .. 2q - 1 for d = 2 (2q tiles).  Inv:
// the diagonal-tile inverses of launch_trinv (trans 0) or their transposes
// from launch_transpose_r (trans 1).
hipError_t launch_coupling(const double* tiles, const double* Rt, const double* Inv, int p, int q, int nb, int trans,
                           double* Wn, hipStream_t s);
// Rt (q x q tile grid, tiles (i, k) with k <= i) = tiles of R^T, and RinvT
// (q tiles) = transposes of the diagonal-tile inverses Rinv.
hipError_t launch_transpose_r(const double* tiles, const double* Rinv, int p, int q, int nb, double* Rt,
                              double* RinvT, hipStream_t s);
// Rinv (q tiles of nb x nb, column-major) = inverses of the diagonal tiles
// R_ii of the tiled R.
hipError_t launch_trinv(const double* tiles, int p, int q, int nb, double* Rinv, hipStream_t s);
// out (n x nrhs, ldo) = sign * A^T Y for A m x n (lda), Y m x nrhs (ldy).
hipError_t launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* Y, int64_t ldy,
                         int64_t nrhs, double* out, int64_t ldo, double sign, hipStream_t s);
// Rv = B - A X; with fro2, ||A||_F^2 is added to *fro2 (zeroed by the caller).
hipError_t launch_residual(const double* A, int64_t lda, int64_t m, int64_t n, const double* X, int64_t ldx,
                           const double* B, int64_t ldb, int64_t nrhs, double* Rv, int64_t ldr, hipStream_t s,
                           double* fro2 = nullptr);
hipError_t launch_colnorms2(const double* M, int64_t ld, int64_t rows, int64_t cols, double* out, hipStream_t s);
// X += alpha D (rows x cols); D -> copy of S.
hipError_t launch_axpy_cols(double* X, int64_t ldx, const double* D, int64_t ldd, int64_t rows, int64_t cols,
                            hipStream_t s, double alpha = 1.0);
hipError_t launch_copy_cols(const double* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                            hipStream_t s);
int persistent_occupancy(int nb, int upd);
hipError_t launch_batch_reset(int32_t* ctl, hipStream_t s);
hipError_t launch_batched(const BatchArgs& b, int grid, hipStream_t s);
int batched_occupancy(int upd);
// Double-complex factorization at nb = 32 (zkernels.hip): tiles and tau in
// interleaved complex layout, the executor's subtask table and flags; ctl
// holds the ticket and the error word (reset by the launch).  zpack copies
// a column-major complex matrix into tiles (unpack: back).
hipError_t launch_zqr(double* tiles, double* taug, double* taup, const DevSub* sub, const int32_t* deps,
                      int32_t* flags, int32_t* ctl, int32_t nsub, int32_t epoch, int32_t p, int64_t spin_ticks,
                      int grid, hipStream_t s, double* B = nullptr, int32_t ncolB = 0, int32_t transB = 1);
hipError_t launch_zpack(double* A, int64_t lda, double* tiles, int p, int q, bool unpack, hipStream_t s);
// X <- R^{-1} X (n x nrhs complex, ldx) for the complex R in the tiles of a
// p-row grid; n <= 4096 (else hipErrorInvalidValue).
hipError_t launch_zsolve_r(const double* tiles, int p, int n, double* X, int64_t ldx, int64_t nrhs, hipStream_t s);
// m x nrhs complex B to and from p row tiles of 32 x ncolB (zero padded).
hipError_t launch_zpack_b(double* Bm, int64_t ldb, int64_t nrhs, double* Bt, int p, int ncolB, bool unpack,
                          hipStream_t s);
int zqr_occupancy();
// All problems' column-major A (device pointer array Aptr, leading
// dimensions lda) into their tiles; tile_start[i] is the first global tile
// of problem i (nprob + 1 entries).
hipError_t launch_pack_batched(const double* const* Aptr, const int64_t* lda, const ProbDesc* prob,
                               const int64_t* tile_start, int nprob, int64_t ntiles, int nbmax, hipStream_t s);

}  // namespace tqr
