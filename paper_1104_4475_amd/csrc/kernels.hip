// HIP tile kernels (gfx950) and the DAG executor.
//
// The six kernels of Sec. 2.1 (Table 1) as LAPACK-style blocked Householder
// code with inner block ib = 32 and compact-WY T factors:
//   GEQRT  QR of one tile: R upper, V unit-lower below the diagonal.
//   TSQRT  zero a square tile under a triangle (V2 is the whole tile).
//   TTQRT  zero a triangle under a triangle (V2 upper triangular).
//   UNMQR / TSMQR / TTMQR  apply those reflectors to tiles further right.
// One workgroup of 4 waves runs one task.  Update tasks are split into
// column slabs of 64 (16 columns per wave); a wave keeps its nb x 16 block
// of C in FP64 MFMA accumulator layout for the whole task, so each ib-block
// of reflectors is applied with two FP64 16x16x4 MFMA contractions
// (W = V^T C and C -= V T^T W) without moving C.
//
// MFMA f64 16x16x4 operand layout (lane l, g = l / 16, n = l % 16; measured
// on gfx950 with one-hot operands):
//   A (16x4):  A[n][g]          B (4x16): B[g][n]
//   C/D (16x16): D[4i + g][n], i = 0..3 (four doubles per lane)
// For a fixed i the four lane groups hold the four consecutive rows
// 16 rb + 4 i + {0..3}, so a C block held as D feeds the B operand of a
// contraction over those rows directly.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace tqr {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ d4 zero4() { return d4{0.0, 0.0, 0.0, 0.0}; }

__device__ __forceinline__ double* tile_ptr(const ExecArgs& a, int r, int c) {
  return a.tiles + (static_cast<size_t>(c) * a.p + r) * static_cast<size_t>(a.nb) * a.nb;
}
__device__ __forceinline__ double* tg_ptr(const ExecArgs& a, int r, int c) {
  return a.Tg + (static_cast<size_t>(c) * a.p + r) * static_cast<size_t>(IB) * a.nb;
}
__device__ __forceinline__ double* tp_ptr(const ExecArgs& a, int r, int c) {
  return a.Tp + (static_cast<size_t>(c) * a.p + r) * static_cast<size_t>(IB) * a.nb;
}

enum { V_UNM = 0, V_TS = 1, V_TT = 2 };

// Apply one ib-block of reflectors (first column c0) to a wave's 16 columns.
// Vs (leading dimension ldv) holds the block's reflectors explicitly, zeros
// and unit diagonal included:
//   V_UNM  rows relative to the block's first row c0 (unit lower trapezoid);
//   V_TS   all nb rows of V2;
//   V_TT   rows 0..c0+ib-1 of V2, zero below each reflector's support.
// acc[rb][i] holds row 16 rb + 4 i + g of C (V_UNM) or of C2 (pairs).
// c1 points at the lane's column of C1 (pairs only); rows c0..c0+ib-1 of
// C1 take part.  trans: 1 applies Q^T (T^T), 0 applies Q (T).
template <int NB, int VAR>
__device__ __forceinline__ void apply_block(const double* Vs, int ldv, const double* Ts, int c0,
                                            d4 (&acc)[NB / 16], double* c1, int lane, int trans) {
  const int g = lane >> 4, n = lane & 15;
  const int rb_lo = (VAR == V_UNM) ? (c0 >> 4) : 0;
  const int rb_hi = (VAR == V_TT) ? ((c0 + IB) >> 4) : (NB >> 4);
  const int vbase = (VAR == V_UNM) ? c0 : 0;
  d4 w[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    if (VAR == V_UNM) {
      w[mb] = zero4();
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) w[mb][i] = c1[c0 + mb * 16 + 4 * i + g];
    }
  }
  // W += V^T C: lane (n, g) supplies V[16 rb + 4 i + g][16 mb + n].
  const double* va = Vs + (g - vbase) + n * ldv;
#pragma unroll
  for (int rb = 0; rb < NB / 16; ++rb) {
    if (rb < rb_lo || rb >= rb_hi) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) w[mb] = mfma(va[rb * 16 + 4 * i + mb * 16 * ldv], acc[rb][i], w[mb]);
    __builtin_amdgcn_sched_barrier(0);
  }
  // W' = T^T W (trans) or T W
  d4 wt[2] = {zero4(), zero4()};
#pragma unroll
  for (int ab = 0; ab < 2; ++ab) {
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      if (trans ? (jb > ab) : (jb < ab)) continue;  // T is upper triangular
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = jb * 16 + 4 * i + g, aa = ab * 16 + n;
        const double t = trans ? Ts[j + aa * IB] : Ts[aa + j * IB];
        wt[ab] = mfma(t, w[jb][i], wt[ab]);
      }
    }
  }
  if (VAR != V_UNM) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) c1[c0 + mb * 16 + 4 * i + g] -= wt[mb][i];
  }
  // C -= V W': lane (n, g) supplies V[16 rb + n][16 mb + 4 i + g].
  const double* vb = Vs + (n - vbase) + g * ldv;
#pragma unroll
  for (int rb = 0; rb < NB / 16; ++rb) {
    if (rb < rb_lo || rb >= rb_hi) continue;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[rb] = mfma(-vb[rb * 16 + (mb * 16 + 4 * i) * ldv], wt[mb][i], acc[rb]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Load / store a wave's nb x 16 column block (column col0 + n of a tile with
// leading dimension NB) in D layout, rows 16 rb .. for rb in [lo, hi).
template <int NB>
__device__ __forceinline__ void load_cols(d4 (&acc)[NB / 16], const double* C, int lane, int lo, int hi) {
  const int g = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < NB / 16; ++rb) {
    if (rb < lo || rb >= hi) {
      acc[rb] = zero4();
      continue;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[rb][i] = C[rb * 16 + 4 * i + g];
  }
}
template <int NB>
__device__ __forceinline__ void store_cols(const d4 (&acc)[NB / 16], double* C, int lane, int lo, int hi) {
  const int g = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < NB / 16; ++rb) {
    if (rb < lo || rb >= hi) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) C[rb * 16 + 4 * i + g] = acc[rb][i];
  }
}

// ---------------------------------------------------------------------------
// Panel factorization of ib columns held in LDS.
//
// Ps (ld ldp) holds the rows below the block's top: for GEQRT rows c0..nb-1
// of the panel (diagonal element of column jj at row jj); for the pair
// kernels the A2 rows 0..K-1, with the triangle block Rs (ib x ib) of R1 on
// top.  Column jj is owned by wave jj % 4, which computes its reflector
// (LAPACK convention: beta = -sign(alpha) ||(alpha, x)||, tau = (beta -
// alpha) / beta, v = x / (alpha - beta)); each wave then updates the panel
// columns it owns.
//
// PAIR = 0: GEQRT panel (alpha = Ps[jj][jj], x = Ps[jj+1.., jj]).
// PAIR = 1: alpha = Rs[jj][jj], x = Ps[0..len(jj)-1, jj] with len(jj) = K for
//           TS and c0 + jj + 1 for TT.
template <int PAIR>
__device__ __forceinline__ void panel_factor(double* Ps, int ldp, int K, double* Rs, double* tau, int tt, int c0) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int jj = 0; jj < IB; ++jj) {
    const int r0 = PAIR ? 0 : jj + 1;
    const int r1 = PAIR ? (tt ? c0 + jj + 1 : K) : K;
    double* colj = Ps + jj * ldp;
    if (wave == (jj & 3)) {
      double s = 0.0;
      for (int r = r0 + lane; r < r1; r += 64) s += colj[r] * colj[r];
      s = wave_sum(s);
      double* ap = PAIR ? (Rs + jj + jj * IB) : (colj + jj);
      const double alpha = *ap;
      double beta = alpha, t = 0.0, scale = 0.0;
      if (s != 0.0) {
        const double nrm = sqrt(alpha * alpha + s);
        beta = alpha >= 0.0 ? -nrm : nrm;
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int r = r0 + lane; r < r1; r += 64) colj[r] *= scale;
      if (lane == 0) {
        *ap = beta;
        tau[jj] = t;
      }
    }
    __syncthreads();
    const double t = tau[jj];
    if (t != 0.0) {
      for (int c = jj + 1; c < IB; ++c) {
        if ((c & 3) != wave) continue;
        double* colc = Ps + c * ldp;
        double d = 0.0;
        for (int r = r0 + lane; r < r1; r += 64) d += colj[r] * colc[r];
        double* top = PAIR ? (Rs + jj + c * IB) : (colc + jj);
        d = (wave_sum(d) + *top) * t;
        for (int r = r0 + lane; r < r1; r += 64) colc[r] -= colj[r] * d;
        if (lane == 0) *top -= d;
      }
    }
  }
  __syncthreads();
}

// T factor of the block (forward, columnwise, as LAPACK dlarft):
// T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] (V^T v_j)[0:j].
// G[a][j] = v_a^T v_j for a < j is computed first.
//   PAIR = 0: v_a = e_a + Ps[a+1.., a] (unit lower), rows relative to c0.
//   PAIR = 1: v_a = e_a (in R1) + Ps[0..K-1, a]; for TT the stored zeros
//             below the support make the full-length dot correct.
template <int PAIR>
__device__ __forceinline__ void build_t(const double* Ps, int ldp, int K, const double* tau, double* Gs, double* Ts) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int pr = wave; pr < IB * IB; pr += 4) {
    const int a = pr / IB, j = pr % IB;
    if (a >= j) continue;
    const double* va = Ps + a * ldp;
    const double* vj = Ps + j * ldp;
    double d = 0.0;
    const int r0 = PAIR ? 0 : j + 1;
    for (int r = r0 + lane; r < K; r += 64) d += va[r] * vj[r];
    d = wave_sum(d);
    if (lane == 0) Gs[a + j * IB] = d + (PAIR ? 0.0 : va[j]);
  }
  __syncthreads();
  if (wave == 0 && lane < IB) {
    const int a = lane;
    for (int j = 0; j < IB; ++j) {
      double v;
      if (a < j) {
        double s = 0.0;
        for (int b = a; b < j; ++b) s += Ts[a + b * IB] * Gs[b + j * IB];
        v = -tau[j] * s;
      } else {
        v = (a == j) ? tau[j] : 0.0;
      }
      Ts[a + j * IB] = v;
    }
  }
  __syncthreads();
}

template <int NB>
struct Smem {
  static constexpr int LDP = NB + 1;
  static constexpr int PS = LDP * IB;
  static constexpr int TOTAL = PS + 3 * IB * IB + IB;
};

// ---- GEQRT ---------------------------------------------------------------
template <int NB>
__device__ __forceinline__ void geqrt_task(double* A, double* T, double* sm) {
  constexpr int ldp = Smem<NB>::LDP;
  double* Ps = sm;
  double* Ts = Ps + Smem<NB>::PS;
  double* Gs = Ts + IB * IB;
  double* Rs = Gs + IB * IB;  // unused here
  double* tau = Rs + IB * IB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c0 = 0; c0 < NB; c0 += IB) {
    const int K = NB - c0;
    for (int idx = tid; idx < K * IB; idx += NTHREADS) {
      const int m = idx / K, kk = idx - m * K;
      Ps[kk + m * ldp] = A[(c0 + m) * NB + c0 + kk];
    }
    __syncthreads();
    panel_factor<0>(Ps, ldp, K, nullptr, tau, 0, c0);
    for (int idx = tid; idx < K * IB; idx += NTHREADS) {
      const int m = idx / K, kk = idx - m * K;
      A[(c0 + m) * NB + c0 + kk] = Ps[kk + m * ldp];
    }
    build_t<0>(Ps, ldp, K, tau, Gs, Ts);
    for (int e = tid; e < IB * IB; e += NTHREADS) {
      T[(c0 / IB) * IB * IB + e] = Ts[e];
      const int a = e % IB, c = e / IB;  // R has been stored: make V explicit
      if (a <= c) Ps[a + c * ldp] = (a == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int nch = (NB - c0 - IB) / 16;
    for (int ch = wave; ch < nch; ch += 4) {
      double* C = A + (c0 + IB + ch * 16 + (lane & 15)) * NB;
      d4 acc[NB / 16];
      load_cols<NB>(acc, C, lane, c0 / 16, NB / 16);
      apply_block<NB, V_UNM>(Ps, ldp, Ts, c0, acc, nullptr, lane, 1);
      store_cols<NB>(acc, C, lane, c0 / 16, NB / 16);
    }
    __syncthreads();
  }
}

// ---- TSQRT / TTQRT ----------------------------------------------------------
// R1: the pivot tile (upper triangle holds R), A2: the tile to zero.
template <int NB>
__device__ __forceinline__ void pair_qrt_task(double* R1, double* A2, double* T, double* sm, int tt) {
  constexpr int ldp = Smem<NB>::LDP;
  double* Ps = sm;
  double* Ts = Ps + Smem<NB>::PS;
  double* Gs = Ts + IB * IB;
  double* Rs = Gs + IB * IB;
  double* tau = Rs + IB * IB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c0 = 0; c0 < NB; c0 += IB) {
    const int K = tt ? c0 + IB : NB;
    for (int e = tid; e < IB * IB; e += NTHREADS) {
      const int a = e % IB, c = e / IB;
      Rs[e] = (a <= c) ? R1[(c0 + c) * NB + c0 + a] : 0.0;
    }
    for (int idx = tid; idx < K * IB; idx += NTHREADS) {
      const int m = idx / K, kk = idx - m * K;
      Ps[kk + m * ldp] = (!tt || kk <= c0 + m) ? A2[(c0 + m) * NB + kk] : 0.0;
    }
    __syncthreads();
    panel_factor<1>(Ps, ldp, K, Rs, tau, tt, c0);
    for (int e = tid; e < IB * IB; e += NTHREADS) {
      const int a = e % IB, c = e / IB;
      if (a <= c) R1[(c0 + c) * NB + c0 + a] = Rs[e];
    }
    for (int idx = tid; idx < K * IB; idx += NTHREADS) {
      const int m = idx / K, kk = idx - m * K;
      if (!tt || kk <= c0 + m) A2[(c0 + m) * NB + kk] = Ps[kk + m * ldp];
    }
    build_t<1>(Ps, ldp, K, tau, Gs, Ts);
    for (int e = tid; e < IB * IB; e += NTHREADS) T[(c0 / IB) * IB * IB + e] = Ts[e];
    const int nch = (NB - c0 - IB) / 16;
    const int hi = tt ? (c0 + IB) / 16 : NB / 16;
    for (int ch = wave; ch < nch; ch += 4) {
      const int col = c0 + IB + ch * 16 + (lane & 15);
      double* C2 = A2 + col * NB;
      d4 acc[NB / 16];
      load_cols<NB>(acc, C2, lane, 0, hi);
      if (tt)
        apply_block<NB, V_TT>(Ps, ldp, Ts, c0, acc, R1 + col * NB, lane, 1);
      else
        apply_block<NB, V_TS>(Ps, ldp, Ts, c0, acc, R1 + col * NB, lane, 1);
      store_cols<NB>(acc, C2, lane, 0, hi);
    }
    __syncthreads();
  }
}

// ---- UNMQR (and apply of a GEQRT set to B) --------------------------------
// V: the factored tile; T: its T factors; C: target with leading dim NB and
// ncol columns; the subtask covers columns col0..col0+63.
template <int NB>
__device__ __forceinline__ void unmqr_task(const double* V, const double* T, double* C, int col0, int ncol, double* sm, int trans) {
  constexpr int ldv = Smem<NB>::LDP;
  double* Vs = sm;
  double* Ts = Vs + Smem<NB>::PS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mycol = col0 + wave * 16;
  const bool active = mycol < ncol;
  double* Cw = C + static_cast<size_t>(mycol + (lane & 15)) * NB;
  d4 acc[NB / 16];
  if (active) load_cols<NB>(acc, Cw, lane, 0, NB / 16);
  for (int step = 0; step < NB / IB; ++step) {
    const int c0 = trans ? step * IB : NB - IB - step * IB;
    const int K = NB - c0;
    for (int idx = tid; idx < K * IB; idx += NTHREADS) {
      const int m = idx / K, kk = idx - m * K;
      Vs[kk + m * ldv] = kk > m ? V[(c0 + m) * NB + c0 + kk] : (kk == m ? 1.0 : 0.0);
    }
    for (int e = tid; e < IB * IB; e += NTHREADS) Ts[e] = T[(c0 / IB) * IB * IB + e];
    __syncthreads();
    if (active) apply_block<NB, V_UNM>(Vs, ldv, Ts, c0, acc, nullptr, lane, trans);
    __syncthreads();
  }
  if (active) store_cols<NB>(acc, Cw, lane, 0, NB / 16);
}

// ---- TSMQR / TTMQR (and apply of a pair set to B) --------------------------
template <int NB>
__device__ __forceinline__ void pair_mqr_task(const double* V2, const double* T, double* C1, double* C2, int col0, int ncol,
                              double* sm, int tt, int trans) {
  constexpr int ldv = Smem<NB>::LDP;
  double* Vs = sm;
  double* Ts = Vs + Smem<NB>::PS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mycol = col0 + wave * 16;
  const bool active = mycol < ncol;
  const size_t off = static_cast<size_t>(mycol + (lane & 15)) * NB;
  d4 acc[NB / 16];
  if (active) load_cols<NB>(acc, C2 + off, lane, 0, NB / 16);
  for (int step = 0; step < NB / IB; ++step) {
    const int c0 = trans ? step * IB : NB - IB - step * IB;
    const int K = tt ? c0 + IB : NB;
    for (int idx = tid; idx < K * IB; idx += NTHREADS) {
      const int m = idx / K, kk = idx - m * K;
      Vs[kk + m * ldv] = (!tt || kk <= c0 + m) ? V2[(c0 + m) * NB + kk] : 0.0;
    }
    for (int e = tid; e < IB * IB; e += NTHREADS) Ts[e] = T[(c0 / IB) * IB * IB + e];
    __syncthreads();
    if (active) {
      if (tt)
        apply_block<NB, V_TT>(Vs, ldv, Ts, c0, acc, C1 + off, lane, trans);
      else
        apply_block<NB, V_TS>(Vs, ldv, Ts, c0, acc, C1 + off, lane, trans);
    }
    __syncthreads();
  }
  if (active) store_cols<NB>(acc, C2 + off, lane, 0, NB / 16);
}

template <int NB>
__device__ __forceinline__ void run_sub(const ExecArgs& a, const DevSub& s, double* sm) {
  switch (s.kind) {
    case D_GEQRT:
      geqrt_task<NB>(tile_ptr(a, s.i, s.k), tg_ptr(a, s.i, s.k), sm);
      break;
    case D_UNMQR:
      unmqr_task<NB>(tile_ptr(a, s.i, s.k), tg_ptr(a, s.i, s.k), tile_ptr(a, s.i, s.j), s.slab * SLAB, NB, sm, 1);
      break;
    case D_TSQRT:
    case D_TTQRT:
      pair_qrt_task<NB>(tile_ptr(a, s.piv, s.k), tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), sm, s.kind == D_TTQRT);
      break;
    case D_TSMQR:
    case D_TTMQR:
      pair_mqr_task<NB>(tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), tile_ptr(a, s.piv, s.j), tile_ptr(a, s.i, s.j),
                        s.slab * SLAB, NB, sm, s.kind == D_TTMQR, 1);
      break;
    case D_APPLY_GE: {
      double* Bi = a.B + static_cast<size_t>(s.i) * NB * a.ncolB;
      unmqr_task<NB>(tile_ptr(a, s.i, s.k), tg_ptr(a, s.i, s.k), Bi, s.slab * SLAB, a.ncolB, sm, a.transB);
      break;
    }
    case D_APPLY_TS:
    case D_APPLY_TT: {
      double* Bp = a.B + static_cast<size_t>(s.piv) * NB * a.ncolB;
      double* Bi = a.B + static_cast<size_t>(s.i) * NB * a.ncolB;
      pair_mqr_task<NB>(tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), Bp, Bi, s.slab * SLAB, a.ncolB, sm,
                        s.kind == D_APPLY_TT, a.transB);
      break;
    }
    default:
      break;
  }
}

// ---- executors ---------------------------------------------------------------

// Persistent executor: workgroups take subtasks in dispatch order from an
// atomic ticket and wait for their predecessors' flags.  Every predecessor
// has a smaller index and was taken by a workgroup that is already running,
// so the smallest unfinished subtask can always proceed (no residency
// assumption).  A wait longer than spin_ticks sets *err, and every
// workgroup then leaves at its next wait or ticket.
template <int NB>
__global__ __launch_bounds__(NTHREADS) void exec_persistent(ExecArgs a) {
  __shared__ double sm[Smem<NB>::TOTAL];
  __shared__ int s_t;
  // Every branch that encloses or follows a barrier is on a wave-uniform
  // (scalar) value, so the compiler keeps the loop structured: wave 0 takes
  // the ticket and waits for the predecessors as a whole wave; only the
  // single atomic operations are guarded by lane == 0.
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (;;) {
    if (wave == 0) {
      int t = a.nsub;
      const int err0 = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (err0 == 0) {
        int tk = 0;
        if (lane == 0) tk = atomicAdd(a.ticket, 1);
        t = __builtin_amdgcn_readfirstlane(tk);
      }
      if (t < a.nsub) {
        const int db = a.sub[t].dep_begin, de = a.sub[t].dep_end;
        const uint64_t t0 = wall_clock64();
        for (int e = db; e < de && t < a.nsub; ++e) {
          int32_t* f = a.flags + a.deps[e];
          for (;;) {
            const int v = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
            if (v == a.epoch) break;
            const int err = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (err != 0 || static_cast<int64_t>(wall_clock64() - t0) > a.spin_ticks) {
              if (lane == 0) __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              t = a.nsub;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
      }
      if (lane == 0) s_t = t;
    }
    __syncthreads();
    // The ticket is the same for every thread; readfirstlane makes that
    // visible to the compiler (scalar loop exit and task dispatch).
    const int t = __builtin_amdgcn_readfirstlane(s_t);
    if (t >= a.nsub) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    run_sub<NB>(a, a.sub[t], sm);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave == 0 && lane == 0) __hip_atomic_store(a.flags + t, a.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Level-synchronous executor: one launch per DAG depth level, one subtask
// per workgroup (kernel boundaries order the levels).
template <int NB>
__global__ __launch_bounds__(NTHREADS) void exec_level(ExecArgs a, const int32_t* order, int begin) {
  __shared__ double sm[Smem<NB>::TOTAL];
  const int t = __builtin_amdgcn_readfirstlane(order[begin + blockIdx.x]);
  run_sub<NB>(a, a.sub[t], sm);
}

__global__ void reset_kernel(int32_t* ticket, int32_t* err) {
  *ticket = 0;
  *err = 0;
}

hipError_t launch_reset(int32_t* ticket, int32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, s, ticket, err);
  return hipGetLastError();
}

hipError_t launch_persistent(const ExecArgs& a, int grid, hipStream_t s) {
  switch (a.nb) {
    case 32: hipLaunchKernelGGL(exec_persistent<32>, dim3(grid), dim3(NTHREADS), 0, s, a); break;
    case 64: hipLaunchKernelGGL(exec_persistent<64>, dim3(grid), dim3(NTHREADS), 0, s, a); break;
    case 128: hipLaunchKernelGGL(exec_persistent<128>, dim3(grid), dim3(NTHREADS), 0, s, a); break;
    case 256: hipLaunchKernelGGL(exec_persistent<256>, dim3(grid), dim3(NTHREADS), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_level(const ExecArgs& a, const int32_t* order, int begin, int count, hipStream_t s) {
  switch (a.nb) {
    case 32: hipLaunchKernelGGL(exec_level<32>, dim3(count), dim3(NTHREADS), 0, s, a, order, begin); break;
    case 64: hipLaunchKernelGGL(exec_level<64>, dim3(count), dim3(NTHREADS), 0, s, a, order, begin); break;
    case 128: hipLaunchKernelGGL(exec_level<128>, dim3(count), dim3(NTHREADS), 0, s, a, order, begin); break;
    case 256: hipLaunchKernelGGL(exec_level<256>, dim3(count), dim3(NTHREADS), 0, s, a, order, begin); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int persistent_occupancy(int nb) {
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (nb) {
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_persistent<32>, NTHREADS, 0); break;
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_persistent<64>, NTHREADS, 0); break;
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_persistent<128>, NTHREADS, 0); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_persistent<256>, NTHREADS, 0); break;
    default: break;
  }
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

// ---- layout conversions ------------------------------------------------------

// Column-major A (lda) -> tiles.  One thread per element of the tile matrix.
__global__ void pack_kernel(const double* A, int64_t lda, double* tiles, int p, int q, int nb) {
  const int64_t m = static_cast<int64_t>(p) * nb;
  const int64_t total = m * q * nb;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t col = e / m, row = e - col * m;
    const int64_t r = row / nb, c = col / nb;
    tiles[(c * p + r) * nb * nb + (col - c * nb) * nb + (row - r * nb)] = A[col * lda + row];
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
  const int64_t total = static_cast<int64_t>(p) * nb * q * nb;
  hipLaunchKernelGGL(pack_kernel, dim3(grid_for(total)), dim3(256), 0, s, A, lda, tiles, p, q, nb);
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

}  // namespace tqr
