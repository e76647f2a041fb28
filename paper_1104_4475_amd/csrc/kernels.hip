// HIP tile kernels (gfx950) and the DAG executor.
//
// The six kernels of Sec. 2.1 (Table 1) as LAPACK-style blocked Householder
// code with inner block ib = 32 and compact-WY T factors:
//   GEQRT  QR of one tile: R upper, V unit-lower below the diagonal.
//   TSQRT  zero a square tile under a triangle (V2 is the whole tile).
//   TTQRT  zero a triangle under a triangle (V2 upper triangular).
//   UNMQR / TSMQR / TTMQR  apply those reflectors to tiles further right.
//
// One workgroup of 8 waves (two per SIMD) runs one task.  Update tasks are
// split into column slabs of 64.  The slab is shared by four column groups
// of 16 columns; the two waves of a group split the rows of C by 16-row
// block parity and keep them in FP64 MFMA accumulator layout for the whole
// task.  Each ib-block of reflectors is applied with two FP64 16x16x4 MFMA
// contractions, W = V^T C (partial sums of the two waves added through LDS)
// and C -= V (T^T W).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"
#include "hip_prims.hpp"

namespace tqr {

__device__ __forceinline__ double* tile_ptr(const ExecArgs& a, int r, int c) {
  return a.tiles + (static_cast<size_t>(c) * a.p + r) * static_cast<size_t>(a.nb) * a.nb;
}
__device__ __forceinline__ double* tg_ptr(const ExecArgs& a, int r, int c) {
  return a.Tg + (static_cast<size_t>(c) * a.p + r) * static_cast<size_t>(IB) * a.nb;
}
__device__ __forceinline__ double* tp_ptr(const ExecArgs& a, int r, int c) {
  return a.Tp + (static_cast<size_t>(c) * a.p + r) * static_cast<size_t>(IB) * a.nb;
}
// Image of block 0 of the GEQRT set of tile (r, c), or of the TS/TT set that
// zeroed it (blocks follow one another).
template <int NB, int P>
__device__ __forceinline__ unsigned char* imgg_ptr(const ExecArgs& a, int r, int c) {
  return a.imgg + (static_cast<size_t>(c) * a.p + r) * (NB / IB) * static_cast<size_t>(image_bytes(NB, P));
}
template <int NB, int P>
__device__ __forceinline__ unsigned char* imgp_ptr(const ExecArgs& a, int r, int c) {
  return a.imgp + (static_cast<size_t>(c) * a.p + r) * (NB / IB) * static_cast<size_t>(image_bytes(NB, P));
}

// LDS of one workgroup, in doubles.
// Precision of the update kernels' two large contractions (the panel
// kernels and everything else stay FP64).
enum { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };

// Low-precision copies of one ib-block of reflectors in LDS, in two layouts:
// column-major (reflector columns, rows contiguous; operand of V^T C) and
// row-major (the ib entries of a row contiguous; operand of V W).  The
// strides spread the 64 lanes of one LDS read over distinct banks.
template <int NB, int P>
struct LpV {
  using T = typename std::conditional<P == P_F32, float, __bf16>::type;
  static constexpr int LCM = (P == P_F32) ? NB + 3 : NB + 8;
  static constexpr int SRM = (P == P_F32) ? 33 : 40;
  static constexpr int CM = 0;
  static constexpr int RM = IB * LCM;
  static constexpr int BYTES = (IB * LCM + NB * SRM) * static_cast<int>(sizeof(T));
};

template <int NB>
struct Smem {
  static constexpr int LDP = NB + 1;            // odd leading dimension of blocks
  static constexpr int PS = 0;                  // reflector / panel block (LDP x IB), or the LpV copies
  static constexpr int PSZ = (LDP * IB * 8 > LpV<NB, P_F32>::BYTES ? LDP * IB : (LpV<NB, P_F32>::BYTES + 7) / 8);
  static_assert(LpV<NB, P_BF16>::BYTES <= PSZ * 8, "LDS region of the BF16 reflector copies");
  static constexpr int TS = PS + PSZ;           // T block
  static constexpr int GS = TS + IB * IB;       // Gram matrix V^T V
  static constexpr int RS = GS + IB * IB;       // triangle block of R1 (pair kernels)
  static constexpr int TAU = RS + IB * IB;      // tau of the panel
  static constexpr int VBUF = TAU + IB;         // current reflector, double buffered
  static constexpr int WX = VBUF + 2 * NB;      // W exchange: [group 4][half 2][8][64]
  static constexpr int TOTAL = WX + 4 * 2 * 8 * 64;
};

// ---------------------------------------------------------------------------
// Block staging between tiles (column-major, leading dimension NB) and LDS.
// Wave w handles columns w, w + 8, w + 16, w + 24 of the ib-wide block; a
// lane handles rows lane + 64 u, so each load instruction reads 64
// consecutive doubles of one column, and all loads are issued before the
// LDS writes.
//   ST_FULL       all K rows.
//   ST_UNIT_LOWER GEQRT reflectors: rows below the diagonal from src, 1 on
//                 the diagonal, 0 above (the stored R part is not read).
//   ST_UPPER      TT reflectors: rows 0..c0+m of column m from src, 0 below
//                 (the GEQRT reflectors below the diagonal are not read).
enum { ST_FULL = 0, ST_UNIT_LOWER = 1, ST_UPPER = 2 };
template <int NB, int MODE>
__device__ __forceinline__ void stage_block(double* Vs, int ldv, const double* src, int K, int c0) {
  constexpr int RCH = (NB + 63) / 64;
  const int lane = lane_id(), wave = wave_id();
  double v[4][RCH];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = wave + NWAVES * c;
#pragma unroll
    for (int u = 0; u < RCH; ++u) {
      const int kk = lane + 64 * u;
      bool use = kk < K;
      if (MODE == ST_UNIT_LOWER) use = use && kk > m;
      if (MODE == ST_UPPER) use = use && kk <= c0 + m;
      const double fill = (MODE == ST_UNIT_LOWER && kk == m) ? 1.0 : 0.0;
      v[c][u] = use ? gld(src + m * NB + kk) : fill;
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = wave + NWAVES * c;
#pragma unroll
    for (int u = 0; u < RCH; ++u) {
      const int kk = lane + 64 * u;
      if (kk < K) Vs[kk + m * ldv] = v[c][u];
    }
  }
}

// LDS block back to the tile; with UPPER_ONLY, rows 0..c0+m of column m.
template <int NB, bool UPPER_ONLY>
__device__ __forceinline__ void unstage_block(const double* Vs, int ldv, double* dst, int K, int c0) {
  constexpr int RCH = (NB + 63) / 64;
  const int lane = lane_id(), wave = wave_id();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = wave + NWAVES * c;
#pragma unroll
    for (int u = 0; u < RCH; ++u) {
      const int kk = lane + 64 * u;
      if (kk < K && (!UPPER_ONLY || kk <= c0 + m)) gst(dst + m * NB + kk, Vs[kk + m * ldv]);
    }
  }
}

// ib x ib T block (contiguous) into LDS.
__device__ __forceinline__ void stage_t(double* Ts, const double* T) {
  constexpr int PER = IB * IB / NTHREADS;
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) v[u] = gld(T + threadIdx.x + NTHREADS * u);
#pragma unroll
  for (int u = 0; u < PER; ++u) Ts[threadIdx.x + NTHREADS * u] = v[u];
}

// Register copy of a reflector block and its T block, loaded one block ahead
// so that the global-memory latency overlaps the current block's MFMAs.
template <int NB>
struct Prefetch {
  static constexpr int RCH = (NB + 63) / 64;
  static constexpr int TPER = IB * IB / NTHREADS;
  double v[4][RCH];
  double t[TPER];
};

template <int NB, int MODE>
__device__ __forceinline__ void prefetch_load(Prefetch<NB>& pf, const double* src, int K, int c0, const double* T) {
  const int lane = lane_nb<NB>(), wave = wave_id();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = wave + NWAVES * c;
#pragma unroll
    for (int u = 0; u < Prefetch<NB>::RCH; ++u) {
      const int kk = lane + 64 * u;
      bool use = kk < K;
      if (MODE == ST_UNIT_LOWER) use = use && kk > m;
      if (MODE == ST_UPPER) use = use && kk <= c0 + m;
      const double fill = (MODE == ST_UNIT_LOWER && kk == m) ? 1.0 : 0.0;
      pf.v[c][u] = use ? gld(src + m * NB + kk) : fill;
    }
  }
#pragma unroll
  for (int u = 0; u < Prefetch<NB>::TPER; ++u) pf.t[u] = gld(T + threadIdx.x + NTHREADS * u);
}

template <int NB>
__device__ __forceinline__ void prefetch_store(const Prefetch<NB>& pf, double* Vs, int ldv, int K, double* Ts) {
  const int lane = lane_nb<NB>(), wave = wave_id();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = wave + NWAVES * c;
#pragma unroll
    for (int u = 0; u < Prefetch<NB>::RCH; ++u) {
      const int kk = lane + 64 * u;
      if (kk < K) Vs[kk + m * ldv] = pf.v[c][u];
    }
  }
#pragma unroll
  for (int u = 0; u < Prefetch<NB>::TPER; ++u) Ts[threadIdx.x + NTHREADS * u] = pf.t[u];
}

// ---------------------------------------------------------------------------
// Block update.
enum { V_UNM = 0, V_TS = 1, V_TT = 2 };

// A wave of column group gw = wave % 4 and row half h = wave / 4 holds the
// 16-row blocks rb = 2 j + h of its 16 columns: acc[j][i] is row
// 16 rb + 4 i + g.  Load / store rows of blocks rb in [lo, hi).
template <int NB>
__device__ __forceinline__ void load_cols(d4 (&acc)[NB / 32], const double* C, int lo, int hi) {
  const int lane = lane_nb<NB>(), g = lane >> 4, h = wave_id() >> 2;
#pragma unroll
  for (int j = 0; j < NB / 32; ++j) {
    const int rb = 2 * j + h;
    if (rb < lo || rb >= hi) {
      acc[j] = zero4();
      continue;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[j][i] = gld(C + rb * 16 + 4 * i + g);
  }
}
template <int NB>
__device__ __forceinline__ void store_cols(const d4 (&acc)[NB / 32], double* C, int lo, int hi) {
  const int lane = lane_nb<NB>(), g = lane >> 4, h = wave_id() >> 2;
#pragma unroll
  for (int j = 0; j < NB / 32; ++j) {
    const int rb = 2 * j + h;
    if (rb < lo || rb >= hi) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) gst(C + rb * 16 + 4 * i + g, acc[j][i]);
  }
}

// Rows c0 + 16 mb + 4 i + g of the lane's column c1 of C1, the pair
// operand of apply_block.  The caller issues these loads before those of
// the next reflector block: vector memory loads complete in order, so the
// wait for C1 then leaves the prefetch in flight.  Both waves of a group
// read the rows before the exchange barrier of apply_block; the h = 0 wave
// writes them back only after it, so no read sees the update.
__device__ __forceinline__ void load_c1(d4 (&c1v)[2], const double* c1, int c0, bool active) {
  const int g = lane_id() >> 4;
  c1v[0] = zero4();
  c1v[1] = zero4();
  if (!active) return;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) c1v[mb][i] = gld(c1 + c0 + mb * 16 + 4 * i + g);
}

// Wait for every outstanding vector memory access of the wave.  Issued once
// after a task's C is loaded into registers: the compiler's wait placement
// otherwise carries those loads as possibly outstanding into the reflector
// loop and waits for all loads (the prefetched next block included) at the
// first use of C in every step.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// Apply one ib-block of reflectors (first column c0) to the column group's
// 16 columns.  Vs (leading dimension ldv) holds the block's reflectors
// explicitly (zeros and unit diagonal included):
//   V_UNM  rows relative to the block's first row c0 (unit lower trapezoid);
//   V_TS   all nb rows of V2;
//   V_TT   rows 0..c0+ib-1 of V2, zero below each reflector's support.
// c1 points at the lane's column of C1 (pairs only); rows c0..c0+ib-1 of
// C1 take part, read beforehand into c1v by load_c1.  wx is the group's W
// exchange area.  Every thread must call this (it contains a barrier);
// active says whether the group has columns.  trans: 1 applies Q^T (T^T),
// 0 applies Q (T).
template <int NB, int VAR>
__device__ __forceinline__ void apply_block(const double* Vs, int ldv, const double* Ts, int c0, d4 (&acc)[NB / 32],
                                            double* c1, const d4 (&c1v)[2], bool active, int trans, double* wx) {
  const int lane = lane_id(), g = lane >> 4, n = lane & 15;
  const int h = wave_id() >> 2;
  const int rb_lo = (VAR == V_UNM) ? (c0 >> 4) : 0;
  const int rb_hi = (VAR == V_TT) ? ((c0 + IB) >> 4) : (NB >> 4);
  const int vbase = (VAR == V_UNM) ? c0 : 0;
  // Partial W over this wave's row blocks: lane (n, g) supplies
  // V[16 rb + 4 i + g][16 mb + n]; two accumulators per mb.
  d4 w[2][2] = {{zero4(), zero4()}, {zero4(), zero4()}};
  if (active) {
    const double* va = Vs + (g - vbase) + n * ldv;
#pragma unroll
    for (int j = 0; j < NB / 32; ++j) {
      const int rb = 2 * j + h;
      if (rb < rb_lo || rb >= rb_hi) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
          w[mb][i & 1] = mfma(va[rb * 16 + 4 * i + mb * 16 * ldv], acc[j][i], w[mb][i & 1]);
      // Keep the operand loads of one row block together (bounds the
      // registers the scheduler spends on hoisted LDS reads).
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  d4 ws[2] = {w[0][0] + w[0][1], w[1][0] + w[1][1]};
  double* mine = wx + h * 8 * 64;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) mine[(mb * 4 + i) * 64 + lane] = ws[mb][i];
  __syncthreads();
  const double* other = wx + (1 - h) * 8 * 64;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) ws[mb][i] += other[(mb * 4 + i) * 64 + lane];
  if (!active) return;
  if (VAR != V_UNM) {
    ws[0] += c1v[0];
    ws[1] += c1v[1];
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
        const int jj = jb * 16 + 4 * i + g, aa = ab * 16 + n;
        const double t = trans ? Ts[jj + aa * IB] : Ts[aa + jj * IB];
        wt[ab] = mfma(t, ws[jb][i], wt[ab]);
      }
    }
  }
  if (VAR != V_UNM && h == 0) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) gst(c1 + c0 + mb * 16 + 4 * i + g, c1v[mb][i] - wt[mb][i]);
  }
  wt[0] = -wt[0];
  wt[1] = -wt[1];
  // C -= V W': lane (n, g) supplies V[16 rb + n][16 mb + 4 i + g]; the row
  // blocks are the inner loop so consecutive MFMAs are independent.
  const double* vb = Vs + (n - vbase) + g * ldv;
#pragma unroll
  for (int j = 0; j < NB / 32; ++j) {
    const int rb = 2 * j + h;
    if (rb < rb_lo || rb >= rb_hi) continue;
    d4 c = acc[j];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) c = mfma(vb[rb * 16 + (mb * 16 + 4 * i) * ldv], wt[mb][i], c);
    acc[j] = c;
  }
}

// ---------------------------------------------------------------------------
// Mixed-precision block update (P = P_F32 or P_BF16).  C stays FP64 in
// registers, here with acc[j][r] = row 16 rb + 4 g + r (the D layout of the
// FP32-output MFMAs).  V, C, W and T enter the MFMAs rounded to nearest
// (BF16 via FP32), products accumulate in FP32, and each correction is
// subtracted from the FP64 C.  The T-apply (W' = T^T W, 1/16 of the flops)
// runs in FP32 in both modes.
// Within each 16-row block the low-precision path keeps rows in the order
// lp_row(q) (q = 4 g + r, r = 0..3 the accumulator element of lane (g, n)):
// rows 2 g, 2 g + 1, 2 g + 8, 2 g + 9.  Each 16-byte access of a lane then
// holds two adjacent rows and the four lanes of a column cover 64
// contiguous bytes per instruction.  The reflectors of a block are kept in
// the same order within 16, so every contraction sees matching indices.
__device__ __forceinline__ int lp_row(int q) { return ((q >> 2) << 1) | (q & 1) | ((q & 2) << 2); }
__device__ __forceinline__ int lp_pos(int x) { return (((x >> 1) & 3) << 2) | (x & 1) | ((x >> 3) << 1); }

// Cg: first column of the wave's 16-column group (wave-uniform); lane
// (g, n) moves rows 16 rb + lp_row(4 g + r) of column n as two 16-byte
// accesses.
template <int NB>
__device__ __forceinline__ void load_cols_lp(d4 (&acc)[NB / 32], const double* Cg, int lo, int hi) {
  const int lane = lane_id(), g = lane >> 4, n = lane & 15, h = wave_id() >> 2;
  const auto r = rsrc(Cg, 16 * NB * 8);
#pragma unroll
  for (int j = 0; j < NB / 32; ++j) {
    const int rb = 2 * j + h;
    if (rb < lo || rb >= hi) {
      acc[j] = zero4();
      continue;
    }
    const int off = (n * NB + rb * 16 + 2 * g) * 8;
    const d2 a = gld2(r, off), b = gld2(r, off + 64);
    acc[j] = d4{a[0], a[1], b[0], b[1]};
  }
}
template <int NB>
__device__ __forceinline__ void store_cols_lp(const d4 (&acc)[NB / 32], double* Cg, int lo, int hi) {
  const int lane = lane_id(), g = lane >> 4, n = lane & 15, h = wave_id() >> 2;
  const auto r = rsrc(Cg, 16 * NB * 8);
#pragma unroll
  for (int j = 0; j < NB / 32; ++j) {
    const int rb = 2 * j + h;
    if (rb < lo || rb >= hi) continue;
    const int off = (n * NB + rb * 16 + 2 * g) * 8;
    gst2(r, off, d2{acc[j][0], acc[j][1]});
    gst2(r, off + 64, d2{acc[j][2], acc[j][3]});
  }
}

template <int P>
__device__ __forceinline__ typename LpV<32, P>::T to_lp(double x) {
  if constexpr (P == P_F32)
    return static_cast<float>(x);
  else
    return static_cast<__bf16>(static_cast<float>(x));
}

// Prefetched reflector block (FP64 registers) into both low-precision LDS
// copies, rows and reflectors in lp_row order within each 16-block; the T
// block stays FP64 in natural order.
template <int NB, int P>
__device__ __forceinline__ void prefetch_store_lp(const Prefetch<NB>& pf, unsigned char* vl, int K, double* Ts) {
  using L = LpV<NB, P>;
  using T = typename L::T;
  T* cm = reinterpret_cast<T*>(vl) + L::CM;
  T* rm = reinterpret_cast<T*>(vl) + L::RM;
  const int lane = lane_id(), wave = wave_id();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = wave + NWAVES * c;
    const int mp = (m & ~15) | lp_pos(m & 15);
#pragma unroll
    for (int u = 0; u < Prefetch<NB>::RCH; ++u) {
      const int kk = lane + 64 * u;
      const int kp = (kk & ~15) | lp_pos(kk & 15);
      if (kk < K) {
        const T v = to_lp<P>(pf.v[c][u]);
        cm[mp * L::LCM + kp] = v;
        rm[kp * L::SRM + mp] = v;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < Prefetch<NB>::TPER; ++u) Ts[threadIdx.x + NTHREADS * u] = pf.t[u];
}

// C1 rows c0 + 16 mb + lp_row(4 g + r) of the group's 16 columns (first
// column c1g) for apply_block_lp; issued before the next block's loads as
// for load_c1.
template <int NB>
__device__ __forceinline__ void load_c1_lp(d4 (&c1v)[2], const double* c1g, int c0, bool active) {
  const int lane = lane_id(), g = lane >> 4, n = lane & 15;
  c1v[0] = zero4();
  c1v[1] = zero4();
  if (!active) return;
  const auto c1r = rsrc(c1g, 16 * NB * 8);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    const int off = (n * NB + c0 + mb * 16 + 2 * g) * 8;
    const d2 a = gld2(c1r, off), b = gld2(c1r, off + 64);
    c1v[mb] = d4{a[0], a[1], b[0], b[1]};
  }
}

// Same contract as apply_block (rows, c1, barrier, trans); vl holds the
// LpV copies of the block's reflectors, wx is the group's exchange area.
template <int NB, int VAR, int P>
__device__ __forceinline__ void apply_block_lp(const unsigned char* vl, const double* Ts, int c0, d4 (&acc)[NB / 32],
                                               double* c1g, const d4 (&c1v)[2], bool active, int trans, float* wx) {
  using L = LpV<NB, P>;
  using T = typename L::T;
  const T* cm = reinterpret_cast<const T*>(vl) + L::CM;
  const T* rm = reinterpret_cast<const T*>(vl) + L::RM;
  const int lane = lane_id(), g = lane >> 4, n = lane & 15;
  const int h = wave_id() >> 2;
  const int rb_lo = (VAR == V_UNM) ? (c0 >> 4) : 0;
  const int rb_hi = (VAR == V_TT) ? ((c0 + IB) >> 4) : (NB >> 4);
  const int vbase = (VAR == V_UNM) ? c0 : 0;
  constexpr int NJ = NB / 32;
  // c1v: C1 rows c0 + 16 mb + lp_row(4 g + r) (pairs), from load_c1_lp.
  // In LDS position order (lp_row within 16) every index below reads as in
  // the natural order.
  const auto c1r = rsrc(c1g, 16 * NB * 8);
  // Partial W = V^T C over this wave's row blocks: w[mb] holds positions
  // 16 mb + 4 g + r of W.
  f4 w[2] = {zero4f(), zero4f()};
  if (active) {
    if constexpr (P == P_F32) {
      // k-slice r of row block rb: positions 16 rb + 4 g + r.
      f4 w1[2] = {zero4f(), zero4f()};
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int rb = 2 * j + h;
        if (rb < rb_lo || rb >= rb_hi) continue;
        const float* va = cm + n * L::LCM + (rb * 16 + 4 * g - vbase);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float b = static_cast<float>(acc[j][r]);
          if (r & 1) {
            w1[0] = mfma32(va[r], b, w1[0]);
            w1[1] = mfma32(va[16 * L::LCM + r], b, w1[1]);
          } else {
            w[0] = mfma32(va[r], b, w[0]);
            w[1] = mfma32(va[16 * L::LCM + r], b, w[1]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      w[0] += w1[0];
      w[1] += w1[1];
    } else {
      // One k-slice of 32 rows per pair of this wave's row blocks:
      // element e of lane (g, n) is row 16 rb_{e/4} + 4 g + e % 4.
      const bf4 zb = {static_cast<__bf16>(0.0f), static_cast<__bf16>(0.0f), static_cast<__bf16>(0.0f),
                      static_cast<__bf16>(0.0f)};
#pragma unroll
      for (int j = 0; j < NJ; j += 2) {
        const int j1 = (j + 1 < NJ) ? j + 1 : j;
        const int rb0 = 2 * j + h, rb1 = 2 * (j + 1) + h;
        const bool v0 = rb0 >= rb_lo && rb0 < rb_hi;
        const bool v1 = (j + 1 < NJ) && rb1 >= rb_lo && rb1 < rb_hi;
        if (!v0 && !v1) continue;
        bf8 b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          b[e] = v0 ? to_lp<P>(acc[j][e]) : static_cast<__bf16>(0.0f);
          b[4 + e] = v1 ? to_lp<P>(acc[j1][e]) : static_cast<__bf16>(0.0f);
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          const T* col = cm + (mb * 16 + n) * L::LCM + 4 * g - vbase;
          const bf4 a0 = v0 ? *reinterpret_cast<const bf4*>(col + rb0 * 16) : zb;
          const bf4 a1 = v1 ? *reinterpret_cast<const bf4*>(col + rb1 * 16) : zb;
          w[mb] = mfmabf(__builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7), b, w[mb]);
        }
      }
    }
  }
  float* mine = wx + h * 8 * 64;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) mine[(mb * 4 + r) * 64 + lane] = w[mb][r];
  __syncthreads();
  const float* other = wx + (1 - h) * 8 * 64;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) w[mb][r] += other[(mb * 4 + r) * 64 + lane];
  if (!active) return;
  if (VAR != V_UNM) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) w[mb][r] += static_cast<float>(c1v[mb][r]);
  }
  // W' = op(T) W in FP32: wt[ab] holds positions 16 ab + 4 g + r (T is
  // read at the reflectors those positions hold).
  f4 wt[2] = {zero4f(), zero4f()};
#pragma unroll
  for (int ab = 0; ab < 2; ++ab) {
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      if (trans ? (jb > ab) : (jb < ab)) continue;  // T is upper triangular
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kk = jb * 16 + lp_row(4 * g + r), aa = ab * 16 + lp_row(n);
        const double t = trans ? Ts[kk + aa * IB] : Ts[aa + kk * IB];
        wt[ab] = mfma32(static_cast<float>(t), w[jb][r], wt[ab]);
      }
    }
  }
  if (VAR != V_UNM && h == 0) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const int off = (n * NB + c0 + mb * 16 + 2 * g) * 8;
      gst2(c1r, off, d2{c1v[mb][0] - static_cast<double>(wt[mb][0]), c1v[mb][1] - static_cast<double>(wt[mb][1])});
      gst2(c1r, off + 64,
           d2{c1v[mb][2] - static_cast<double>(wt[mb][2]), c1v[mb][3] - static_cast<double>(wt[mb][3])});
    }
  }
  // C -= V W'.
  if constexpr (P == P_F32) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int rb = 2 * j + h;
      if (rb < rb_lo || rb >= rb_hi) continue;
      const float* vr = rm + (rb * 16 + n - vbase) * L::SRM + 4 * g;
      f4 d = zero4f();
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) d = mfma32(vr[mb * 16 + r], wt[mb][r], d);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[j][r] -= static_cast<double>(d[r]);
    }
  } else {
    // k-slice: element e of lane (g, n) is reflector 16 (e / 4) + 4 g + e % 4.
    bf8 bw;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      bw[e] = static_cast<__bf16>(wt[0][e]);
      bw[4 + e] = static_cast<__bf16>(wt[1][e]);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int rb = 2 * j + h;
      if (rb < rb_lo || rb >= rb_hi) continue;
      const T* vr = rm + (rb * 16 + n - vbase) * L::SRM + 4 * g;
      const bf4 a0 = *reinterpret_cast<const bf4*>(vr);
      const bf4 a1 = *reinterpret_cast<const bf4*>(vr + 16);
      const f4 d = mfmabf(__builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7), bw, zero4f());
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[j][r] -= static_cast<double>(d[r]);
    }
  }
}

// ---------------------------------------------------------------------------
// Wide low-precision update subtasks (nb >= 128, FP32 or BF16 updates).
//
// The panel subtask that computes an ib-block of reflectors rounds it once
// into an image in device memory; every update subtask that applies the
// block copies the image to LDS as it is (no conversion, and half the bytes
// of the FP64 reflectors).  An update subtask covers a slab of WSLAB = 128
// columns: wave w owns columns 16 w .. 16 w + 15 of the slab over all nb
// rows, so it forms W = V^T C for its columns alone (no exchange between
// waves), and a single barrier per block hands over the three LDS slots
// that hold consecutive images.
//
// Image of one block.  Rows and reflectors are kept in lp_row order within
// each 16 (position x of a group holds natural row, or reflector,
// lp_row(x)); V rows are the tile rows 0..nb-1, zero outside the block's
// support.  The image is laid out exactly as its LDS copy, padding
// included, so the copy is a plain transfer; the padded strides put the 64
// lanes of every operand read below on distinct banks.
//   FP32: cm[m'][k'] = V[k][m] as float, rows of LCM = nb + 4 floats;
//   BF16: cm as bf16, rows of LCM = nb + 8; then from RM, rm[k'][m'] =
//         V[k][m] as bf16, rows of SRM = 40;
//   both: from TO, Tq[kk'][aa'] = T[kk][aa] as float, rows of TLD = 36.
// BYTES is a whole number of KB (37 KB FP32, 41 KB BF16 at nb = 256).
constexpr int WSLAB = 128;

__device__ __forceinline__ int nat16(int x) { return (x & ~15) | lp_row(x & 15); }

template <int NB, int P>
struct Img {
  static constexpr int ESZ = (P == P_F32) ? 4 : 2;
  static constexpr int LCM = (P == P_F32) ? NB + 4 : NB + 8;
  static constexpr int RM = IB * LCM * ESZ;
  static constexpr int SRM = 40;
  static constexpr int TO = RM + ((P == P_F32) ? 0 : NB * SRM * 2);
  static constexpr int TLD = 36;
  static constexpr int BYTES = TO + IB * TLD * 4;
  static constexpr int NKB = BYTES / 1024;
};
static_assert(Img<256, P_F32>::BYTES == image_bytes(256, P_F32) && Img<128, P_F32>::BYTES == image_bytes(128, P_F32) &&
                  Img<256, P_BF16>::BYTES == image_bytes(256, P_BF16) &&
                  Img<128, P_BF16>::BYTES == image_bytes(128, P_BF16),
              "image size");
static_assert(Img<256, P_F32>::BYTES % 1024 == 0 && Img<128, P_F32>::BYTES % 1024 == 0 &&
                  Img<256, P_BF16>::BYTES % 1024 == 0 && Img<128, P_BF16>::BYTES % 1024 == 0,
              "image in whole KB");

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_b(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, 0x00020000);
}

// Image of the block whose explicit reflectors are in the FP64 LDS panel Ps
// (ld ldp, K rows, Ps row 0 = tile row vrow0) and whose T factor is in Ts
// (natural order, column-major), written with device-coherent stores (one
// thread per 16-byte piece; padding written as zeros).  Only reads LDS.
template <int NB, int P>
__device__ __forceinline__ void write_image(unsigned char* img, const double* Ps, int ldp, int vrow0, int K,
                                            const double* Ts) {
  using I = Img<NB, P>;
  const auto r = rsrc_b(img, I::BYTES);
  auto V = [&](int k, int m) -> double {
    const int kk = k - vrow0;
    return (kk >= 0 && kk < K) ? Ps[kk + m * ldp] : 0.0;
  };
  for (int c = threadIdx.x; c < I::BYTES / 16; c += NTHREADS) {
    const int o = 16 * c;
    u4 out = {0u, 0u, 0u, 0u};
    if (o < I::RM) {
      const int mp = o / (I::LCM * I::ESZ), kp = (o % (I::LCM * I::ESZ)) / I::ESZ;
      const int m = nat16(mp);
      if constexpr (P == P_F32) {
        if (kp < NB) {
          f4 f;
#pragma unroll
          for (int e = 0; e < 4; ++e) f[e] = static_cast<float>(V(nat16(kp + e), m));
          out = __builtin_bit_cast(u4, f);
        }
      } else {
        if (kp < NB) {
          bf8 h;
#pragma unroll
          for (int e = 0; e < 8; ++e) h[e] = to_lp<P_BF16>(V(nat16(kp + e), m));
          out = __builtin_bit_cast(u4, h);
        }
      }
    } else if (o < I::TO) {  // BF16 rm
      const int kp = (o - I::RM) / (I::SRM * 2), mp = ((o - I::RM) % (I::SRM * 2)) / 2;
      if (mp < IB) {
        const int k = nat16(kp);
        bf8 h;
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = to_lp<P_BF16>(V(k, nat16(mp + e)));
        out = __builtin_bit_cast(u4, h);
      }
    } else {
      const int t = (o - I::TO) / 4, kp = t / I::TLD, ap = t % I::TLD;
      if (ap < IB) {
        const int kk = nat16(kp);
        f4 f;
#pragma unroll
        for (int e = 0; e < 4; ++e) f[e] = static_cast<float>(Ts[kk + nat16(ap + e) * IB]);
        out = __builtin_bit_cast(u4, f);
      }
    }
    __builtin_amdgcn_raw_buffer_store_b128(out, r, o, 0, CPOL_SC1);
  }
}

// Copy of one image into an LDS slot by direct loads into LDS (device-
// coherent): each wave instruction moves 1 KB (lane l: bytes 16 l ..
// 16 l + 15 of it); wave w moves KB w, w + 8, ...  The data is in LDS once
// the wave's vector memory counter has drained.
// One direct load of 16 bytes per lane into LDS (lane l to lds + 16 l).  The
// builtin exists for the device target only; the host pass of this file
// needs no body.
__device__ __forceinline__ void lds_load16(__amdgpu_buffer_rsrc_t r, unsigned char* lds, int voff) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 16, voff, 0, 0, CPOL_SC1);
#endif
}

template <int NB, int P>
__device__ __forceinline__ void img_dma(const unsigned char* img, unsigned char* slot) {
  using I = Img<NB, P>;
  const auto r = rsrc_b(img, I::BYTES);
  const int lane = lane_id(), w = wave_id();
  // Every wave issues the same number of transfers (the last KB may be
  // moved twice, with the same data), so the count is known at compile time.
#pragma unroll
  for (int j0 = 0; j0 < I::NKB; j0 += NWAVES) {
    const int j = (j0 + w < I::NKB) ? j0 + w : I::NKB - 1;
    lds_load16(r, slot + 1024 * j, 1024 * j + 16 * lane);
  }
}

// Rows 16 rb + lp_row(4 g + r) of the lane's column (first column Cg of the
// wave's 16, lane (g, n) -> column n), all nb rows.
template <int NB>
__device__ __forceinline__ void load_strip_lp(d4 (&acc)[NB / 16], const double* Cg) {
  const int lane = lane_id(), g = lane >> 4, n = lane & 15;
  const auto r = rsrc(Cg, 16 * NB * 8);
#pragma unroll
  for (int rb = 0; rb < NB / 16; ++rb) {
    const int off = (n * NB + rb * 16 + 2 * g) * 8;
    const d2 a = gld2(r, off), b = gld2(r, off + 64);
    acc[rb] = d4{a[0], a[1], b[0], b[1]};
  }
}
template <int NB>
__device__ __forceinline__ void store_strip_lp(const d4 (&acc)[NB / 16], double* Cg) {
  const int lane = lane_id(), g = lane >> 4, n = lane & 15;
  const auto r = rsrc(Cg, 16 * NB * 8);
#pragma unroll
  for (int rb = 0; rb < NB / 16; ++rb) {
    const int off = (n * NB + rb * 16 + 2 * g) * 8;
    gst2(r, off, d2{acc[rb][0], acc[rb][1]});
    gst2(r, off + 64, d2{acc[rb][2], acc[rb][3]});
  }
}

// Block-by-block following of streamed predecessors (the planner's pdep and
// sdep edges).  A panel block publishes its completion flag (epoch); a wide
// pair update publishes 64 epoch + b + 1 in its progress word once its block
// b is stored (its C1 rows b ib .. b ib + ib - 1 are then final), a wide
// UNMQR 64 epoch + nb / ib once all its rows are stored.
struct StreamCtl {
  const int32_t* flags;  // completion flags
  const int32_t* prog;   // progress words
  int32_t* self;         // this subtask's progress word
  const int32_t* pblk;   // dispatch indices of the streamed panel blocks, or null
  int32_t sdep;          // streamed C1 writer, or -1
  int32_t epoch;
  int32_t* err;
  int64_t spin;
};

// Wave-level wait until ok(*w) (relaxed device-scope loads).  Gives up when
// the wait exceeds the executor's time limit or another workgroup has
// failed, and then sets the error word (the executor stops at its next wait).
template <class Ok>
__device__ __forceinline__ void wait_until(const int32_t* w, Ok ok, int32_t* err, int64_t spin) {
  const uint64_t t0 = wall_clock64();
  for (;;) {
    const int v = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(const_cast<int32_t*>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (ok(v)) return;
    const int e = __builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (e != 0 || static_cast<int64_t>(wall_clock64() - t0) > spin) {
      if (lane_id() == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}
template <class Ok>
__device__ __forceinline__ void wait_word(const int32_t* w, Ok ok, const StreamCtl& c) {
  wait_until(w, ok, c.err, c.spin);
}

// Early release of a panel block subtask (its predecessor entries carry
// stage fields): the waits before its look-ahead update (stage 1) and
// before the update of the rest of its tiles (stage 2), and the release
// after the look-ahead.  on = false for a whole panel task (or the batched
// executor): no waits and no release.
struct PanelSync {
  bool on;
  const int32_t* deps;
  int32_t db, de;
  const int32_t* flags;
  int32_t* self;  // this subtask's progress word
  int32_t epoch;
  int32_t* err;
  int64_t spin;
};

// Wave 0 waits for the completion of the stage-st predecessors; the
// workgroup then meets at a barrier.
__device__ __forceinline__ void panel_wait(const PanelSync& ps, int st) {
  if (ps.on && wave_id() == 0) {
    for (int e = ps.db; e < ps.de; ++e) {
      const int32_t d = __builtin_amdgcn_readfirstlane(ps.deps[e]);
      if (dep_stage(d) != st) continue;
      const int32_t ep = ps.epoch;
      wait_until(ps.flags + dep_index(d), [ep](int v) { return v == ep; }, ps.err, ps.spin);
    }
  }
  __syncthreads();
}

// Every store of the subtask so far has completed in every wave before the
// progress word announces the early release (as for the completion flag).
__device__ __forceinline__ void panel_release(const PanelSync& ps) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (ps.on && threadIdx.x == 0)
    __hip_atomic_store(ps.self, early_word(ps.epoch), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_panel_block(const StreamCtl& c, int b) {
  if (c.pblk) {
    const int32_t d = __builtin_amdgcn_readfirstlane(c.pblk[b]);
    if (dep_early(d)) {
      const int need = early_word(c.epoch);
      wait_word(c.prog + dep_index(d), [need](int v) { return v >= need; }, c);
    } else {
      const int e = c.epoch;
      wait_word(c.flags + dep_index(d), [e](int v) { return v == e; }, c);
    }
  }
}
__device__ __forceinline__ void wait_c1(const StreamCtl& c, int b) {
  if (c.sdep >= 0) {
    const int need = 64 * c.epoch + b + 1;
    wait_word(c.prog + c.sdep, [need](int v) { return v >= need; }, c);
  }
}

// Update subtask on columns col0 .. col0 + 127 of the target tile(s):
//   V_UNM  C2 <- Q^T C2 with the GEQRT set of a factored tile (C1 unused);
//   V_TS / V_TT  [C1; C2] <- Q^T [C1; C2] with a TS / TT set.
// img: image of block 0 of the set (blocks follow at Img<NB, P>::BYTES);
// lds: three slots of that size.  Only Q^T (the factorization).
template <int NB, int P, int VAR>
__device__ __forceinline__ void wide_update_task(const unsigned char* img, double* C1, double* C2, int col0,
                                                 unsigned char* lds, const StreamCtl& sc) {
  using I = Img<NB, P>;
  using T = typename LpV<32, P>::T;
  constexpr int NBLK = NB / IB, NJ = NB / 16, SLOT = I::BYTES;
  constexpr bool PAIR = VAR != V_UNM;
  const int lane = lane_id(), g = lane >> 4, n = lane & 15;
  const size_t colo = static_cast<size_t>(col0 + 16 * wave_id()) * NB;
  double* C2g = C2 + colo;
  double* C1g = PAIR ? C1 + colo : nullptr;
  // Three LDS slots: block b is read from slot b % 3 while the image of
  // block b + 2 lands in slot (b + 2) % 3, which block b - 1 read before the
  // barrier that ended it.  Streamed predecessors are polled only where this
  // wave has no memory access in flight (a poll waits for all of them): at
  // the start, and at the end of each block, for what the next block starts
  // with (the image two blocks ahead, the next C1 rows).  A block issues its
  // C1 rows first and the image copy second, so the wait for the C1 rows
  // after the first contraction leaves the copy in flight (the last two
  // blocks copy nothing: a separate instance of the block body, so that the
  // count of transfers in flight is known at compile time).
  wait_panel_block(sc, 0);
  if (NBLK > 1) wait_panel_block(sc, 1);
  if (NBLK > 2) wait_panel_block(sc, 2);
  if constexpr (PAIR) wait_c1(sc, 0);
  d4 c1v[2] = {zero4(), zero4()};
  if constexpr (PAIR) load_c1_lp<NB>(c1v, C1g, 0, true);
  img_dma<NB, P>(img, lds);
  if (NBLK > 1) img_dma<NB, P>(img + I::BYTES, lds + SLOT);
  d4 acc[NJ];
  load_strip_lp<NB>(acc, C2g);
  wait_vm();
  __syncthreads();
  int scur = 0;
  auto block = [&](int b, auto copy_tag) __attribute__((always_inline)) {
    constexpr bool COPY = decltype(copy_tag)::value;
    const int c0 = b * IB;
    const unsigned char* cur = lds + scur * SLOT;
    unsigned char* nxt = lds + ((scur == 0) ? 2 : scur - 1) * SLOT;
    scur = (scur == 2) ? 0 : scur + 1;
    if constexpr (PAIR) {
      if (b > 0) load_c1_lp<NB>(c1v, C1g, c0, true);
    }
    if constexpr (COPY) img_dma<NB, P>(img + static_cast<size_t>(b + 2) * I::BYTES, nxt);
    const int rb_lo = (VAR == V_UNM) ? (c0 >> 4) : 0;
    const int rb_hi = (VAR == V_TT) ? ((c0 + IB) >> 4) : NJ;
    // W = V^T C2 (+ C1 rows c0 .. c0 + 31): w[mb] holds positions
    // 16 mb + 4 g + r of W for column n.
    f4 w[2] = {zero4f(), zero4f()};
    if constexpr (P == P_F32) {
      // Lane (g, n) supplies V at reflector position 16 mb + n and row
      // positions 16 rb + 4 g + r (one 16-byte piece per mb).
      const float* cm = reinterpret_cast<const float*>(cur);
      f4 w1[2] = {zero4f(), zero4f()};
#pragma unroll
      for (int rb = 0; rb < NJ; ++rb) {
        if (rb < rb_lo || rb >= rb_hi) continue;
        const float* va = cm + n * I::LCM + rb * 16 + 4 * g;
        const f4 a0 = *reinterpret_cast<const f4*>(va);
        const f4 a1 = *reinterpret_cast<const f4*>(va + 16 * I::LCM);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float bb = static_cast<float>(acc[rb][r]);
          if (r & 1) {
            w1[0] = mfma32(a0[r], bb, w1[0]);
            w1[1] = mfma32(a1[r], bb, w1[1]);
          } else {
            w[0] = mfma32(a0[r], bb, w[0]);
            w[1] = mfma32(a1[r], bb, w[1]);
          }
        }
      }
      w[0] += w1[0];
      w[1] += w1[1];
    } else {
      // k-slice of 32 rows: element e of lane (g, n) is row position
      // 16 (rb + e / 4) + 4 g + e % 4.
      const bf4 zb = {static_cast<__bf16>(0.0f), static_cast<__bf16>(0.0f), static_cast<__bf16>(0.0f),
                      static_cast<__bf16>(0.0f)};
#pragma unroll
      for (int rb = 0; rb < NJ; rb += 2) {
        const bool v0 = rb >= rb_lo && rb < rb_hi, v1 = rb + 1 >= rb_lo && rb + 1 < rb_hi;
        if (!v0 && !v1) continue;
        bf8 bb;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          bb[e] = v0 ? to_lp<P>(acc[rb][e]) : static_cast<__bf16>(0.0f);
          bb[4 + e] = v1 ? to_lp<P>(acc[rb + 1][e]) : static_cast<__bf16>(0.0f);
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          const T* col = reinterpret_cast<const T*>(cur) + (mb * 16 + n) * I::LCM + 4 * g;
          const bf4 a0 = v0 ? *reinterpret_cast<const bf4*>(col + rb * 16) : zb;
          const bf4 a1 = v1 ? *reinterpret_cast<const bf4*>(col + (rb + 1) * 16) : zb;
          w[mb] = mfmabf(__builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7), bb, w[mb]);
        }
      }
    }
    if constexpr (PAIR) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) w[mb][r] += static_cast<float>(c1v[mb][r]);
    }
    // W' = T^T W in FP32 (T upper triangular): lane (g, n) supplies
    // T[kk][aa] for position 16 jb + 4 g + r of W and 16 ab + n of W'.
    const float* Tq = reinterpret_cast<const float*>(cur + I::TO);
    f4 wt[2] = {zero4f(), zero4f()};
#pragma unroll
    for (int ab = 0; ab < 2; ++ab)
#pragma unroll
      for (int jb = 0; jb <= ab; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) wt[ab] = mfma32(Tq[(jb * 16 + 4 * g + r) * I::TLD + ab * 16 + n], w[jb][r], wt[ab]);
    if constexpr (PAIR) {
      const auto c1r = rsrc(C1g, 16 * NB * 8);
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const int off = (n * NB + c0 + mb * 16 + 2 * g) * 8;
        gst2(c1r, off, d2{c1v[mb][0] - static_cast<double>(wt[mb][0]), c1v[mb][1] - static_cast<double>(wt[mb][1])});
        gst2(c1r, off + 64,
             d2{c1v[mb][2] - static_cast<double>(wt[mb][2]), c1v[mb][3] - static_cast<double>(wt[mb][3])});
      }
    }
    // C2 -= V W'.
    if constexpr (P == P_F32) {
      // Lane (g, n) supplies V at row position 16 rb + n and reflector
      // position 16 mb + 4 g + r (one float per MFMA).
#pragma unroll
      for (int rb = 0; rb < NJ; rb += 2) {
        const bool v0 = rb >= rb_lo && rb < rb_hi, v1 = rb + 1 >= rb_lo && rb + 1 < rb_hi;
        if (!v0 && !v1) continue;
        f4 d0 = zero4f(), d1 = zero4f();
        const float* vr = reinterpret_cast<const float*>(cur) + 4 * g * I::LCM + rb * 16 + n;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float* v = vr + (mb * 16 + r) * I::LCM;
            if (v0) d0 = mfma32(v[0], wt[mb][r], d0);
            if (v1) d1 = mfma32(v[16], wt[mb][r], d1);
          }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (v0) acc[rb][r] -= static_cast<double>(d0[r]);
          if (v1) acc[rb + 1][r] -= static_cast<double>(d1[r]);
        }
      }
    } else {
      // k-slice: element e of lane (g, n) is reflector position
      // 16 (e / 4) + 4 g + e % 4.
      bf8 bw;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        bw[e] = static_cast<__bf16>(wt[0][e]);
        bw[4 + e] = static_cast<__bf16>(wt[1][e]);
      }
#pragma unroll
      for (int rb = 0; rb < NJ; ++rb) {
        if (rb < rb_lo || rb >= rb_hi) continue;
        const T* vr = reinterpret_cast<const T*>(cur + I::RM) + (rb * 16 + n) * I::SRM + 4 * g;
        const bf4 a0 = *reinterpret_cast<const bf4*>(vr);
        const bf4 a1 = *reinterpret_cast<const bf4*>(vr + 16);
        const f4 d = mfmabf(__builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7), bw, zero4f());
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[rb][r] -= static_cast<double>(d[r]);
      }
    }
    // The image of block b + 1 (issued a block ago) has landed in every
    // wave's part of its slot, and this block's stores are complete, before
    // the barrier publishes both; then the streamed predecessors are far
    // enough for the next block.
    wait_vm();
    if (b + 3 < NBLK) wait_panel_block(sc, b + 3);
    if constexpr (PAIR) {
      if (b + 1 < NBLK) wait_c1(sc, b + 1);
    }
    __syncthreads();
    if constexpr (PAIR) {
      if (sc.self && threadIdx.x == 0)
        __hip_atomic_store(sc.self, 64 * sc.epoch + b + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
#pragma unroll 1
  for (int b = 0; b + 2 < NBLK; ++b) block(b, std::true_type{});
#pragma unroll 1
  for (int b = NBLK > 2 ? NBLK - 2 : 0; b < NBLK; ++b) block(b, std::false_type{});
  store_strip_lp<NB>(acc, C2g);
  if constexpr (!PAIR) {
    // An UNMQR keeps its rows in registers to the end: its followers see all
    // of them at once.
    wait_vm();
    __syncthreads();
    if (sc.self && threadIdx.x == 0)
      __hip_atomic_store(sc.self, 64 * sc.epoch + NBLK, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Panel factorization of ib columns (held in LDS on entry and exit, in
// registers in between).
//
// Ps (ld ldp) holds: for GEQRT (PAIR = 0) rows c0..nb-1 of the panel (K rows,
// diagonal of column jj at row jj); for the pair kernels (PAIR = 1) the A2
// rows 0..K-1, with the triangle block Rs (ib x ib) of R1 on top.  Wave w
// owns columns w, w + 8, ...; a lane holds rows lane + 64 u.  Column jj's
// reflector is computed by its owner (LAPACK convention: beta = -sign(alpha)
// ||(alpha, x)||, tau = (beta - alpha) / beta, v = x / (alpha - beta)) and
// broadcast through LDS; each wave then updates the columns it owns.  TT
// (PAIR = 1, tt) limits column jj's reflector to rows 0..c0+jj.
//
// Look-ahead: while reflector jj is applied, the owner of column jj + 1
// updates that column first and computes reflector jj + 1 at once, before
// its other columns, so one barrier per column separates consecutive
// reflectors and the chain between them is a single column update.  A
// wave's other columns take their dot products with v together and reduce
// them in one pass (wave_sum4).  For the pair kernels the rows of the
// triangle block stay in registers during the loop (lane a holds row a of
// each owned column) and go back to Rs at the end.
template <int NB, int PAIR>
__device__ __forceinline__ void panel_factor(double* Ps, int ldp, int K, double* Rs, double* tau, double* vbuf,
                                             int tt, int c0) {
  constexpr int RCH = (NB + 63) / 64;
  const int lane = lane_id(), wave = wave_id();
  double pc[4][RCH];
  double rs[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int u = 0; u < RCH; ++u) {
      const int r = lane + 64 * u;
      pc[q][u] = r < K ? Ps[r + (wave + NWAVES * q) * ldp] : 0.0;
    }
    rs[q] = (PAIR && lane < IB) ? Rs[lane + (wave + NWAVES * q) * IB] : 0.0;
  }

  // Reflector of column jj (owned by this wave, held in register slot q):
  // writes v to vbuf[jj & 1], tau[jj], and (pairs) beta to row jj of the
  // triangle.  jj < 64, so the diagonal row jj of a GEQRT panel is in row
  // chunk 0.
  auto reflector = [&](int jj, int q) {
    double (&x)[RCH] = pc[q];
    const int r0 = PAIR ? 0 : jj + 1;
    const int r1 = PAIR ? (tt ? c0 + jj + 1 : K) : K;
    double* vb = vbuf + (jj & 1) * NB;
    double ssq = 0.0;
#pragma unroll
    for (int u = 0; u < RCH; ++u) {
      const int r = lane + 64 * u;
      if (r >= r0 && r < r1) ssq += x[u] * x[u];
    }
    ssq = wave_sum(ssq);
    const double alpha = PAIR ? lane_d(rs[q], jj) : lane_d(x[0], jj);
    double beta = alpha, t = 0.0, scale = 0.0;
    if (ssq != 0.0) {
      const double nrm = sqrt(alpha * alpha + ssq);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
#pragma unroll
    for (int u = 0; u < RCH; ++u) {
      const int r = lane + 64 * u;
      const bool in = r >= r0 && r < r1;
      if (in) x[u] *= scale;
      if (!PAIR && u == 0 && r == jj) x[u] = beta;
      if (r < NB) vb[r] = in ? x[u] : 0.0;
    }
    if (PAIR && lane == jj) rs[q] = beta;
    if (lane == 0) tau[jj] = t;
  };

  // Reflector jj (v, t) applied to this wave's column slot q2, given the
  // wavefront sum d of v . (its rows in registers).
  auto apply_col = [&](int jj, int q2, const double (&v)[RCH], double d, double t) {
    d += PAIR ? lane_d(rs[q2], jj) : lane_d(pc[q2][0], jj);
    d *= t;
#pragma unroll
    for (int u = 0; u < RCH; ++u) {
      pc[q2][u] -= v[u] * d;
      if (!PAIR && u == 0 && lane == jj) pc[q2][u] -= d;
    }
    if (PAIR && lane == jj) rs[q2] -= d;
  };
  auto dot = [&](int q2, const double (&v)[RCH]) {
    double d = 0.0;
#pragma unroll
    for (int u = 0; u < RCH; ++u) d += v[u] * pc[q2][u];
    return d;
  };

  if (wave == 0) reflector(0, 0);
  // Column jj = 8 q + w: slot q of wave w.  The owner of column jj + 1
  // (wave w + 1, slot q; or wave 0, slot q + 1) updates it first, computes
  // its reflector at raised priority, then updates its other columns.
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll 1
    for (int w = 0; w < NWAVES; ++w) {
      const int jj = NWAVES * q + w;
      __syncthreads();
      const double t = uniform_d(tau[jj]);
      const int nxt = jj + 1;
      const int nq = (w + 1 < NWAVES) ? q : q + 1;  // slot of column nxt
      const bool own_next = nxt < IB && wave == (nxt & 7);
      double v[RCH];
#pragma unroll
      for (int u = 0; u < RCH; ++u) {
        const int r = lane + 64 * u;
        v[u] = r < NB ? vbuf[(jj & 1) * NB + r] : 0.0;
      }
      if (own_next) {
        __builtin_amdgcn_s_setprio(3);
        if (nq == q) {
          if (t != 0.0) apply_col(jj, q, v, wave_sum(dot(q, v)), t);
          reflector(nxt, q);
        } else if (q + 1 < 4) {
          const int qn = (q + 1 < 4) ? q + 1 : q;
          if (t != 0.0) apply_col(jj, qn, v, wave_sum(dot(qn, v)), t);
          reflector(nxt, qn);
        }
        __builtin_amdgcn_s_setprio(0);
      }
      if (t != 0.0) {
        // this wave's columns right of nxt: the dot products first, then
        // one reduction of all of them, then the updates
        double dd[4];
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) dd[q2] = q2 < q ? 0.0 : dot(q2, v);
        if (q < 3)
          wave_sum4(dd);
        else
          dd[3] = wave_sum(dd[3]);
#pragma unroll
        for (int q2 = q; q2 < 4; ++q2) {
          const int c = wave + NWAVES * q2;
          if (c > nxt) apply_col(jj, q2, v, dd[q2], t);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int u = 0; u < RCH; ++u) {
      const int r = lane + 64 * u;
      if (r < K) Ps[r + (wave + NWAVES * q) * ldp] = pc[q][u];
    }
    if (PAIR && lane < IB) Rs[lane + (wave + NWAVES * q) * IB] = rs[q];
  }
  __syncthreads();
}

// T factor of the block (forward, columnwise, as LAPACK dlarft):
// T[j][j] = tau_j and T[0:j, j] = -tau_j T[0:j, 0:j] (V^T v_j)[0:j].
// Ps holds the block's reflectors explicitly (K rows); the Gram matrix
// G = V^T V comes from FP64 MFMAs (upper 16 x 16 blocks).  The two diagonal
// 16 x 16 blocks of T follow the recurrence on their own reflectors (one
// row of T per lane), and the coupling block is T12 = -T11 (V1^T V2) T22,
// two 16 x 16 MFMA products.  The Gram blocks run on waves 0..2, the
// diagonal blocks on waves 0 and 1 and the coupling block on wave 0, with a
// barrier after each phase.
template <int NB>
__device__ __forceinline__ void build_t(const double* Ps, int ldp, int K, const double* tau, double* Gs, double* Ts) {
  const int lane = lane_id(), wave = wave_id(), g = lane >> 4, n = lane & 15;
  auto gram = [&](int gb) {
    const int ab = (gb == 2) ? 1 : 0, jb = (gb == 0) ? 0 : 1;
    d4 a0 = zero4(), a1 = zero4();
    const double* pa = Ps + g + (ab * 16 + n) * ldp;
    const double* pb = Ps + g + (jb * 16 + n) * ldp;
    for (int k0 = 0; k0 < K; k0 += 8) {
      a0 = mfma(pa[k0], pb[k0], a0);
      a1 = mfma(pa[k0 + 4], pb[k0 + 4], a1);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) Gs[(ab * 16 + 4 * i + g) + (jb * 16 + n) * IB] = a0[i] + a1[i];
  };
  auto tdiag = [&](int half, int a) {
    const int off = 16 * half;
    double trow[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < j; ++b) s += trow[b] * Gs[(off + b) + (off + j) * IB];
      const double tj = tau[off + j];
      trow[j] = (a < j) ? -tj * s : (a == j ? tj : 0.0);
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) Ts[(off + a) + (off + j) * IB] = trow[j];
    if (half == 1) {
#pragma unroll
      for (int j = 0; j < 16; ++j) Ts[(16 + a) + j * IB] = 0.0;  // T21 = 0
    }
  };
  auto t12 = [&]() {
    // P = G12 T22 (D layout: P[4 i + g][n] in p[i]), then T12 = -T11 P.
    d4 pm = zero4(), e = zero4();
#pragma unroll
    for (int st = 0; st < 4; ++st)
      pm = mfma(Gs[n + (16 + 4 * st + g) * IB], Ts[(16 + 4 * st + g) + (16 + n) * IB], pm);
#pragma unroll
    for (int st = 0; st < 4; ++st) e = mfma(Ts[n + (4 * st + g) * IB], pm[st], e);
#pragma unroll
    for (int i = 0; i < 4; ++i) Ts[(4 * i + g) + (16 + n) * IB] = -e[i];
  };
  if (wave < 3) gram(wave);
  __syncthreads();
  if (wave < 2 && lane < 16) tdiag(wave, lane);
  __syncthreads();
  if (wave == 0) t12();
  __syncthreads();
}

// The reflectors of an ib-block, explicit in the FP64 LDS panel Ps (K rows),
// rewritten in place as the low-precision LDS copies of LpV<NB, P> (via
// registers; contains barriers).  The T block in Ts is kept.
template <int NB, int P>
__device__ __forceinline__ void panel_to_lp(double* Ps, int ldp, int K, double* Ts) {
  const int lane = lane_id(), wave = wave_id();
  Prefetch<NB> pf;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = wave + NWAVES * c;
#pragma unroll
    for (int u = 0; u < Prefetch<NB>::RCH; ++u) {
      const int kk = lane + 64 * u;
      pf.v[c][u] = kk < K ? Ps[kk + m * ldp] : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < Prefetch<NB>::TPER; ++u) pf.t[u] = Ts[threadIdx.x + NTHREADS * u];
  __syncthreads();
  prefetch_store_lp<NB, P>(pf, reinterpret_cast<unsigned char*>(Ps), K, Ts);
  __syncthreads();
}

// ---- GEQRT ---------------------------------------------------------------
// P: precision of the block update of the rest of the tile (the reflector
// generation, norms, scaling and T, is FP64 in every mode).
// The inner blocks c0 = cb, cb + ib, ... < ce are factored (all of them, or
// one when the planner splits the task into block subtasks).
template <int NB, int P>
__device__ __forceinline__ void geqrt_task(double* A, double* T, double* sm, int cb, int ce, unsigned char* img,
                                           const PanelSync& ps) {
  constexpr int ldp = Smem<NB>::LDP;
  double* Ps = sm + Smem<NB>::PS;
  double* Ts = sm + Smem<NB>::TS;
  double* Gs = sm + Smem<NB>::GS;
  double* tau = sm + Smem<NB>::TAU;
  double* vbuf = sm + Smem<NB>::VBUF;
  const int tid = threadIdx.x, lane = lane_id(), gw = wave_id() & 3;
  double* wx = sm + Smem<NB>::WX + gw * 16 * 64;
#pragma unroll 1
  for (int c0 = cb; c0 < ce; c0 += IB) {
    const int K = NB - c0;
    stage_block<NB, ST_FULL>(Ps, ldp, A + c0 * NB + c0, K, c0);
    __syncthreads();
    panel_factor<NB, 0>(Ps, ldp, K, nullptr, tau, vbuf, 0, c0);
    unstage_block<NB, false>(Ps, ldp, A + c0 * NB + c0, K, c0);
    __syncthreads();
    // R has been stored: make the reflectors explicit (unit diagonal).
    for (int e = tid; e < IB * IB; e += NTHREADS) {
      const int a = e % IB, c = e / IB;
      if (a <= c) Ps[a + c * ldp] = (a == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    build_t<NB>(Ps, ldp, K, tau, Gs, Ts);
    for (int e = tid; e < IB * IB; e += NTHREADS) gst(T + (c0 / IB) * IB * IB + e, Ts[e]);
    if constexpr (P != P_F64 && NB >= 128) write_image<NB, P>(img + (c0 / IB) * Img<NB, P>::BYTES, Ps, ldp, c0, K, Ts);
    const int nch = (NB - c0 - IB) / 16;
    if constexpr (P != P_F64) {
      if (nch > 0) panel_to_lp<NB, P>(Ps, ldp, K, Ts);
    }
    // The rest of the tile in chunks of 16 columns, four at a time.  With
    // early release: the next block's columns (chunks 0 and 1) first, then
    // the release, then the rest.
    const int la = ps.on ? (nch < 2 ? nch : 2) : nch;
#pragma unroll 1
    for (int ph = 0; ph < (ps.on ? 2 : 1); ++ph) {
      if (ps.on) {
        if (ph == 1) panel_release(ps);
        panel_wait(ps, ph + 1);
      }
      const int ch1 = ph == 0 ? la : nch;
#pragma unroll 1
      for (int base = ph == 0 ? 0 : la; base < ch1; base += 4) {
        const int ch = base + gw;
        const bool active = ch < ch1;
        d4 acc[NB / 32];
        const d4 none[2] = {zero4(), zero4()};
        if constexpr (P == P_F64) {
          double* C = A + (c0 + IB + ch * 16 + (lane & 15)) * NB;
          if (active) load_cols<NB>(acc, C, c0 / 16, NB / 16);
          apply_block<NB, V_UNM>(Ps, ldp, Ts, c0, acc, nullptr, none, active, 1, wx);
          if (active) store_cols<NB>(acc, C, c0 / 16, NB / 16);
        } else {
          double* Cg = A + static_cast<size_t>(c0 + IB + ch * 16) * NB;
          if (active) load_cols_lp<NB>(acc, Cg, c0 / 16, NB / 16);
          apply_block_lp<NB, V_UNM, P>(reinterpret_cast<const unsigned char*>(Ps), Ts, c0, acc, nullptr, none, active, 1,
                                       reinterpret_cast<float*>(wx));
          if (active) store_cols_lp<NB>(acc, Cg, c0 / 16, NB / 16);
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// ---- TSQRT / TTQRT ----------------------------------------------------------
// R1: the pivot tile (upper triangle holds R), A2: the tile to zero.
// TT: 1 for TTQRT (A2 upper triangular), 0 for TSQRT.
// Inner blocks cb <= c0 < ce as for geqrt_task.
template <int NB, int P, int TT>
__device__ __forceinline__ void pair_qrt_task(double* R1, double* A2, double* T, double* sm, int cb, int ce,
                                              unsigned char* img, const PanelSync& ps) {
  constexpr int tt = TT;
  constexpr int ldp = Smem<NB>::LDP;
  double* Ps = sm + Smem<NB>::PS;
  double* Ts = sm + Smem<NB>::TS;
  double* Gs = sm + Smem<NB>::GS;
  double* Rs = sm + Smem<NB>::RS;
  double* tau = sm + Smem<NB>::TAU;
  double* vbuf = sm + Smem<NB>::VBUF;
  const int tid = threadIdx.x, lane = lane_id(), gw = wave_id() & 3;
  double* wx = sm + Smem<NB>::WX + gw * 16 * 64;
#pragma unroll 1
  for (int c0 = cb; c0 < ce; c0 += IB) {
    const int K = tt ? c0 + IB : NB;
    for (int e = tid; e < IB * IB; e += NTHREADS) {
      const int a = e % IB, c = e / IB;
      Rs[e] = (a <= c) ? gld(R1 + (c0 + c) * NB + c0 + a) : 0.0;
    }
    if (tt)
      stage_block<NB, ST_UPPER>(Ps, ldp, A2 + c0 * NB, K, c0);
    else
      stage_block<NB, ST_FULL>(Ps, ldp, A2 + c0 * NB, K, c0);
    __syncthreads();
    panel_factor<NB, 1>(Ps, ldp, K, Rs, tau, vbuf, tt, c0);
    for (int e = tid; e < IB * IB; e += NTHREADS) {
      const int a = e % IB, c = e / IB;
      if (a <= c) gst(R1 + (c0 + c) * NB + c0 + a, Rs[e]);
    }
    if (tt)
      unstage_block<NB, true>(Ps, ldp, A2 + c0 * NB, K, c0);
    else
      unstage_block<NB, false>(Ps, ldp, A2 + c0 * NB, K, c0);
    build_t<NB>(Ps, ldp, K, tau, Gs, Ts);
    for (int e = tid; e < IB * IB; e += NTHREADS) gst(T + (c0 / IB) * IB * IB + e, Ts[e]);
    if constexpr (P != P_F64 && NB >= 128) write_image<NB, P>(img + (c0 / IB) * Img<NB, P>::BYTES, Ps, ldp, 0, K, Ts);
    const int nch = (NB - c0 - IB) / 16;
    const int hi = tt ? (c0 + IB) / 16 : NB / 16;
    if constexpr (P != P_F64) {
      if (nch > 0) panel_to_lp<NB, P>(Ps, ldp, K, Ts);
    }
    // As for geqrt_task: look-ahead chunks first with early release.
    const int la = ps.on ? (nch < 2 ? nch : 2) : nch;
#pragma unroll 1
    for (int ph = 0; ph < (ps.on ? 2 : 1); ++ph) {
      if (ps.on) {
        if (ph == 1) panel_release(ps);
        panel_wait(ps, ph + 1);
      }
      const int ch1 = ph == 0 ? la : nch;
#pragma unroll 1
      for (int base = ph == 0 ? 0 : la; base < ch1; base += 4) {
        const int ch = base + gw;
        const bool active = ch < ch1;
        d4 acc[NB / 32], c1v[2];
        if constexpr (P == P_F64) {
          const int col = c0 + IB + ch * 16 + (lane & 15);
          double* C2 = A2 + col * NB;
          load_c1(c1v, R1 + col * NB, c0, active);
          if (active) load_cols<NB>(acc, C2, 0, hi);
          if (tt)
            apply_block<NB, V_TT>(Ps, ldp, Ts, c0, acc, R1 + col * NB, c1v, active, 1, wx);
          else
            apply_block<NB, V_TS>(Ps, ldp, Ts, c0, acc, R1 + col * NB, c1v, active, 1, wx);
          if (active) store_cols<NB>(acc, C2, 0, hi);
        } else {
          const size_t colg = static_cast<size_t>(c0 + IB + ch * 16) * NB;
          const unsigned char* vl = reinterpret_cast<const unsigned char*>(Ps);
          float* wxf = reinterpret_cast<float*>(wx);
          load_c1_lp<NB>(c1v, R1 + colg, c0, active);
          if (active) load_cols_lp<NB>(acc, A2 + colg, 0, hi);
          if (tt)
            apply_block_lp<NB, V_TT, P>(vl, Ts, c0, acc, R1 + colg, c1v, active, 1, wxf);
          else
            apply_block_lp<NB, V_TS, P>(vl, Ts, c0, acc, R1 + colg, c1v, active, 1, wxf);
          if (active) store_cols_lp<NB>(acc, A2 + colg, 0, hi);
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// ---- UNMQR (and application of a GEQRT set to B) ---------------------------
// V: the factored tile; T: its T factors; C: target with leading dimension
// NB and ncol columns; the subtask covers columns col0..col0+63.
template <int NB, int P>
__device__ __forceinline__ void unmqr_task(const double* V, const double* T, double* C, int col0, int ncol, double* sm,
                                           int trans) {
  constexpr int ldv = Smem<NB>::LDP;
  double* Vs = sm + Smem<NB>::PS;
  double* Ts = sm + Smem<NB>::TS;
  const int lane = lane_nb<NB>(), gw = wave_id() & 3;
  double* wx = sm + Smem<NB>::WX + gw * 16 * 64;
  const int mycol = col0 + gw * 16;
  const bool active = mycol < ncol;
  double* Cw = C + static_cast<size_t>(mycol + (lane & 15)) * NB;
  Prefetch<NB> pf;
  {
    const int c0 = trans ? 0 : NB - IB;
    prefetch_load<NB, ST_UNIT_LOWER>(pf, V + c0 * NB + c0, NB - c0, c0, T + (c0 / IB) * IB * IB);
  }
  unsigned char* vl = reinterpret_cast<unsigned char*>(sm + Smem<NB>::PS);
  d4 acc[NB / 32];
  const d4 none[2] = {zero4(), zero4()};
  if (active) {
    if constexpr (P == P_F64)
      load_cols<NB>(acc, Cw, 0, NB / 16);
    else
      load_cols_lp<NB>(acc, C + static_cast<size_t>(mycol) * NB, 0, NB / 16);
  }
  wait_vm();
#pragma unroll 1
  for (int step = 0; step < NB / IB; ++step) {
    const int c0 = trans ? step * IB : NB - IB - step * IB;
    const int K = NB - c0;
    if constexpr (P == P_F64)
      prefetch_store<NB>(pf, Vs, ldv, K, Ts);
    else
      prefetch_store_lp<NB, P>(pf, vl, K, Ts);
    __syncthreads();
    if (step + 1 < NB / IB) {
      const int n0 = trans ? c0 + IB : c0 - IB;
      prefetch_load<NB, ST_UNIT_LOWER>(pf, V + n0 * NB + n0, NB - n0, n0, T + (n0 / IB) * IB * IB);
    }
    if constexpr (P == P_F64)
      apply_block<NB, V_UNM>(Vs, ldv, Ts, c0, acc, nullptr, none, active, trans, wx);
    else
      apply_block_lp<NB, V_UNM, P>(vl, Ts, c0, acc, nullptr, none, active, trans, reinterpret_cast<float*>(wx));
    __syncthreads();
  }
  if (active) {
    if constexpr (P == P_F64)
      store_cols<NB>(acc, Cw, 0, NB / 16);
    else
      store_cols_lp<NB>(acc, C + static_cast<size_t>(mycol) * NB, 0, NB / 16);
  }
}

// ---- Q application to narrow right-hand sides (16 columns) ----------------
// With only 16 columns the four column groups of the update kernels would
// leave three quarters of the waves idle, so here every wave takes the same
// 16 columns and its own 16-row blocks rb = wave + 8 j (FP64 accumulator
// layout).  The eight partial W = V^T B are added through LDS by every wave,
// each wave forms W' = op(T) W itself, and B -= V W' on its rows.
template <int NB>
constexpr int narrow_nj() { return (NB / 16 + NWAVES - 1) / NWAVES; }

template <int NB>
__device__ __forceinline__ void load_rows_narrow(d4 (&acc)[narrow_nj<NB>()], const double* Bc, int lo, int hi) {
  const int lane = lane_nb<NB>(), g = lane >> 4, wave = wave_id();
#pragma unroll
  for (int j = 0; j < narrow_nj<NB>(); ++j) {
    const int rb = wave + NWAVES * j;
    if (rb >= NB / 16 || rb < lo || rb >= hi) {
      acc[j] = zero4();
      continue;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[j][i] = gld(Bc + rb * 16 + 4 * i + g);
  }
}
template <int NB>
__device__ __forceinline__ void store_rows_narrow(const d4 (&acc)[narrow_nj<NB>()], double* Bc, int lo, int hi) {
  const int lane = lane_nb<NB>(), g = lane >> 4, wave = wave_id();
#pragma unroll
  for (int j = 0; j < narrow_nj<NB>(); ++j) {
    const int rb = wave + NWAVES * j;
    if (rb >= NB / 16 || rb < lo || rb >= hi) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) gst(Bc + rb * 16 + 4 * i + g, acc[j][i]);
  }
}

// One ib-block (first column c0) applied to the narrow B; c1 (pairs): the
// lane's column of B1 (read by every wave before the barrier, written by
// wave 0 after it).  wx: 8 x 8 x 64 doubles.  Contains a barrier.
template <int NB, int VAR>
__device__ __forceinline__ void apply_block_narrow(const double* Vs, int ldv, const double* Ts, int c0,
                                                   d4 (&acc)[narrow_nj<NB>()], double* c1, int trans, double* wx) {
  const int lane = lane_nb<NB>(), g = lane >> 4, n = lane & 15, wave = wave_id();
  const int rb_lo = (VAR == V_UNM) ? (c0 >> 4) : 0;
  const int rb_hi = (VAR == V_TT) ? ((c0 + IB) >> 4) : (NB >> 4);
  const int vbase = (VAR == V_UNM) ? c0 : 0;
  d4 w[2] = {zero4(), zero4()};
  {
    const double* va = Vs + (g - vbase) + n * ldv;
#pragma unroll
    for (int j = 0; j < narrow_nj<NB>(); ++j) {
      const int rb = wave + NWAVES * j;
      if (rb >= NB / 16 || rb < rb_lo || rb >= rb_hi) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) w[mb] = mfma(va[rb * 16 + 4 * i + mb * 16 * ldv], acc[j][i], w[mb]);
    }
  }
  d4 c1v[2] = {zero4(), zero4()};
  if (VAR != V_UNM) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) c1v[mb][i] = gld(c1 + c0 + mb * 16 + 4 * i + g);
  }
  double* mine = wx + wave * 8 * 64;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) mine[(mb * 4 + i) * 64 + lane] = w[mb][i];
  __syncthreads();
  d4 ws[2] = {c1v[0], c1v[1]};
#pragma unroll
  for (int o = 0; o < NWAVES; ++o) {
    const double* part = wx + o * 8 * 64;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) ws[mb][i] += part[(mb * 4 + i) * 64 + lane];
  }
  d4 wt[2] = {zero4(), zero4()};
#pragma unroll
  for (int ab = 0; ab < 2; ++ab) {
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      if (trans ? (jb > ab) : (jb < ab)) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int jj = jb * 16 + 4 * i + g, aa = ab * 16 + n;
        const double t = trans ? Ts[jj + aa * IB] : Ts[aa + jj * IB];
        wt[ab] = mfma(t, ws[jb][i], wt[ab]);
      }
    }
  }
  if (VAR != V_UNM && wave == 0) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) gst(c1 + c0 + mb * 16 + 4 * i + g, c1v[mb][i] - wt[mb][i]);
  }
  wt[0] = -wt[0];
  wt[1] = -wt[1];
  const double* vb = Vs + (n - vbase) + g * ldv;
#pragma unroll
  for (int j = 0; j < narrow_nj<NB>(); ++j) {
    const int rb = wave + NWAVES * j;
    if (rb >= NB / 16 || rb < rb_lo || rb >= rb_hi) continue;
    d4 c = acc[j];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) c = mfma(vb[rb * 16 + (mb * 16 + 4 * i) * ldv], wt[mb][i], c);
    acc[j] = c;
  }
}

// Reflector block c (first column) of a Q application task into registers.
template <int NB>
__device__ __forceinline__ void apply_load_block(Prefetch<NB>& pf, int kind, const double* V, const double* T, int c) {
  if (kind == D_APPLY_GE)
    prefetch_load<NB, ST_UNIT_LOWER>(pf, V + c * NB + c, NB - c, c, T + (c / IB) * IB * IB);
  else if (kind == D_APPLY_TT)
    prefetch_load<NB, ST_UPPER>(pf, V + c * NB, c + IB, c, T + (c / IB) * IB * IB);
  else
    prefetch_load<NB, ST_FULL>(pf, V + c * NB, NB, c, T + (c / IB) * IB * IB);
}

// Q application task on 16-column row tiles: kind D_APPLY_GE (B1 unused),
// D_APPLY_TS or D_APPLY_TT.  V: the factored (GE) or zeroed (TS/TT) tile.
// pf holds the first reflector block on entry (apply_load_block with
// c = 0 for Q^T, nb - ib for Q).
template <int NB>
__device__ __forceinline__ void apply_narrow_task(int kind, const double* V, const double* T, double* B1, double* B2,
                                                  double* sm, int trans, Prefetch<NB>& pf) {
  constexpr int ldv = Smem<NB>::LDP;
  double* Vs = sm + Smem<NB>::PS;
  double* Ts = sm + Smem<NB>::TS;
  double* wx = sm + Smem<NB>::WX;
  const int lane = lane_nb<NB>();
  const bool ge = kind == D_APPLY_GE, tt = kind == D_APPLY_TT;
  double* c1 = ge ? nullptr : B1 + (lane & 15) * NB;
  double* Bc = B2 + (lane & 15) * NB;
  d4 acc[narrow_nj<NB>()];
  load_rows_narrow<NB>(acc, Bc, 0, NB / 16);
#pragma unroll 1
  for (int step = 0; step < NB / IB; ++step) {
    const int c0 = trans ? step * IB : NB - IB - step * IB;
    const int K = ge ? NB - c0 : (tt ? c0 + IB : NB);
    prefetch_store<NB>(pf, Vs, ldv, K, Ts);
    __syncthreads();
    if (step + 1 < NB / IB) apply_load_block<NB>(pf, kind, V, T, trans ? c0 + IB : c0 - IB);
    if (ge)
      apply_block_narrow<NB, V_UNM>(Vs, ldv, Ts, c0, acc, c1, trans, wx);
    else if (tt)
      apply_block_narrow<NB, V_TT>(Vs, ldv, Ts, c0, acc, c1, trans, wx);
    else
      apply_block_narrow<NB, V_TS>(Vs, ldv, Ts, c0, acc, c1, trans, wx);
    __syncthreads();
  }
  store_rows_narrow<NB>(acc, Bc, 0, NB / 16);
}

// ---- TSMQR / TTMQR (and application of a pair set to B) --------------------
// TT: 1 for a TT set (triangular V2), 0 for a TS set; a compile-time
// parameter so that each loop holds the registers of one variant only.
template <int NB, int P, int TT>
__device__ __forceinline__ void pair_mqr_task(const double* V2, const double* T, double* C1, double* C2, int col0,
                                              int ncol, double* sm, int trans) {
  constexpr bool tt = TT != 0;
  constexpr int ldv = Smem<NB>::LDP;
  double* Vs = sm + Smem<NB>::PS;
  double* Ts = sm + Smem<NB>::TS;
  const int lane = lane_nb<NB>(), gw = wave_id() & 3;
  double* wx = sm + Smem<NB>::WX + gw * 16 * 64;
  const int mycol = col0 + gw * 16;
  const bool active = mycol < ncol;
  const size_t off = static_cast<size_t>(mycol + (lane & 15)) * NB;
  Prefetch<NB> pf;
  {
    const int c0 = trans ? 0 : NB - IB;
    if (tt)
      prefetch_load<NB, ST_UPPER>(pf, V2 + c0 * NB, c0 + IB, c0, T + (c0 / IB) * IB * IB);
    else
      prefetch_load<NB, ST_FULL>(pf, V2 + c0 * NB, NB, c0, T + (c0 / IB) * IB * IB);
  }
  unsigned char* vl = reinterpret_cast<unsigned char*>(sm + Smem<NB>::PS);
  d4 acc[NB / 32], c1v[2];
  double* c1g = C1 + static_cast<size_t>(mycol) * NB;
  if (active) {
    if constexpr (P == P_F64)
      load_cols<NB>(acc, C2 + off, 0, NB / 16);
    else
      load_cols_lp<NB>(acc, C2 + static_cast<size_t>(mycol) * NB, 0, NB / 16);
  }
  wait_vm();
#pragma unroll 1
  for (int step = 0; step < NB / IB; ++step) {
    const int c0 = trans ? step * IB : NB - IB - step * IB;
    const int K = tt ? c0 + IB : NB;
    if constexpr (P == P_F64)
      prefetch_store<NB>(pf, Vs, ldv, K, Ts);
    else
      prefetch_store_lp<NB, P>(pf, vl, K, Ts);
    __syncthreads();
    // This block's C1 rows before the next block's reflectors (in-order
    // completion: the C1 wait leaves the prefetch in flight).
    if constexpr (P == P_F64)
      load_c1(c1v, C1 + off, c0, active);
    else
      load_c1_lp<NB>(c1v, c1g, c0, active);
    if (step + 1 < NB / IB) {
      const int n0 = trans ? c0 + IB : c0 - IB;
      if (tt)
        prefetch_load<NB, ST_UPPER>(pf, V2 + n0 * NB, n0 + IB, n0, T + (n0 / IB) * IB * IB);
      else
        prefetch_load<NB, ST_FULL>(pf, V2 + n0 * NB, NB, n0, T + (n0 / IB) * IB * IB);
    }
    if constexpr (P == P_F64) {
      if (tt)
        apply_block<NB, V_TT>(Vs, ldv, Ts, c0, acc, C1 + off, c1v, active, trans, wx);
      else
        apply_block<NB, V_TS>(Vs, ldv, Ts, c0, acc, C1 + off, c1v, active, trans, wx);
    } else {
      float* wxf = reinterpret_cast<float*>(wx);
      if (tt)
        apply_block_lp<NB, V_TT, P>(vl, Ts, c0, acc, c1g, c1v, active, trans, wxf);
      else
        apply_block_lp<NB, V_TS, P>(vl, Ts, c0, acc, c1g, c1v, active, trans, wxf);
    }
    __syncthreads();
  }
  if (active) {
    if constexpr (P == P_F64)
      store_cols<NB>(acc, C2 + off, 0, NB / 16);
    else
      store_cols_lp<NB>(acc, C2 + static_cast<size_t>(mycol) * NB, 0, NB / 16);
  }
}

// P: precision of the update subtasks (UNMQR, TSMQR, TTMQR); the panel
// subtasks and the application of Q to right-hand sides are FP64.
template <int NB, int P>
__device__ __forceinline__ void run_sub(const ExecArgs& a, const DevSub& s, double* sm, int t) {
  // Low-precision updates at nb >= 128 run as wide subtasks from reflector
  // images (the planner splits them into WIDE_SLAB-column slabs).
  constexpr bool kWide = P != P_F64 && NB >= 128;
  static_assert(!kWide || 3 * Img<NB, P>::BYTES <= Smem<NB>::TOTAL * 8, "LDS of the wide update");
  static_assert(WSLAB == WIDE_SLAB && WSLAB == 16 * NWAVES, "wide slab width");
  StreamCtl sc{};
  if constexpr (kWide) {
    const int pd = __builtin_amdgcn_readfirstlane(s.pdep), sd = __builtin_amdgcn_readfirstlane(s.sdep);
    sc = StreamCtl{a.flags, a.prog, a.prog ? a.prog + t : nullptr, pd >= 0 ? a.deps + pd : nullptr,
                   sd, a.epoch, a.err, a.spin_ticks};
  }
  // Panel subtasks: slab = the inner block to factor, or -1 for all.
  const int cb = s.slab < 0 ? 0 : s.slab * IB, ce = s.slab < 0 ? NB : cb + IB;
  PanelSync ps{};
  if ((s.kind == D_GEQRT || s.kind == D_TSQRT || s.kind == D_TTQRT) && s.slab >= 0 && a.prog)
    ps = PanelSync{true, a.deps, __builtin_amdgcn_readfirstlane(s.dep_begin), __builtin_amdgcn_readfirstlane(s.dep_end),
                   a.flags, a.prog + t, a.epoch, a.err, a.spin_ticks};
  switch (s.kind) {
    case D_GEQRT:
      geqrt_task<NB, P>(tile_ptr(a, s.i, s.k), tg_ptr(a, s.i, s.k), sm, cb, ce,
                        kWide ? imgg_ptr<NB, P>(a, s.i, s.k) : nullptr, ps);
      break;
    case D_UNMQR:
      if constexpr (kWide) {
        wide_update_task<NB, P, V_UNM>(imgg_ptr<NB, P>(a, s.i, s.k), nullptr, tile_ptr(a, s.i, s.j), s.slab * WSLAB,
                                       reinterpret_cast<unsigned char*>(sm), sc);
        break;
      }
      unmqr_task<NB, P>(tile_ptr(a, s.i, s.k), tg_ptr(a, s.i, s.k), tile_ptr(a, s.i, s.j), s.slab * SLAB, NB, sm, 1);
      break;
    case D_TSQRT:
    case D_TTQRT:
      if (s.kind == D_TTQRT)
        pair_qrt_task<NB, P, 1>(tile_ptr(a, s.piv, s.k), tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), sm, cb, ce,
                                kWide ? imgp_ptr<NB, P>(a, s.i, s.k) : nullptr, ps);
      else
        pair_qrt_task<NB, P, 0>(tile_ptr(a, s.piv, s.k), tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), sm, cb, ce,
                                kWide ? imgp_ptr<NB, P>(a, s.i, s.k) : nullptr, ps);
      break;
    case D_TSMQR:
    case D_TTMQR:
      if constexpr (kWide) {
        unsigned char* lds = reinterpret_cast<unsigned char*>(sm);
        if (s.kind == D_TTMQR)
          wide_update_task<NB, P, V_TT>(imgp_ptr<NB, P>(a, s.i, s.k), tile_ptr(a, s.piv, s.j), tile_ptr(a, s.i, s.j),
                                        s.slab * WSLAB, lds, sc);
        else
          wide_update_task<NB, P, V_TS>(imgp_ptr<NB, P>(a, s.i, s.k), tile_ptr(a, s.piv, s.j), tile_ptr(a, s.i, s.j),
                                        s.slab * WSLAB, lds, sc);
        break;
      }
      if (s.kind == D_TTMQR)
        pair_mqr_task<NB, P, 1>(tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), tile_ptr(a, s.piv, s.j),
                                tile_ptr(a, s.i, s.j), s.slab * SLAB, NB, sm, 1);
      else
        pair_mqr_task<NB, P, 0>(tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), tile_ptr(a, s.piv, s.j),
                                tile_ptr(a, s.i, s.j), s.slab * SLAB, NB, sm, 1);
      break;
    case D_APPLY_GE:
    case D_APPLY_TS:
    case D_APPLY_TT:
      if (s.kind == D_APPLY_GE) {
        double* Bi = a.B + static_cast<size_t>(s.i) * NB * a.ncolB;
        unmqr_task<NB, P_F64>(tile_ptr(a, s.i, s.k), tg_ptr(a, s.i, s.k), Bi, s.slab * SLAB, a.ncolB, sm, a.transB);
        break;
      }
      {
        double* Bp = a.B + static_cast<size_t>(s.piv) * NB * a.ncolB;
        double* Bi = a.B + static_cast<size_t>(s.i) * NB * a.ncolB;
        if (s.kind == D_APPLY_TT)
          pair_mqr_task<NB, P_F64, 1>(tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), Bp, Bi, s.slab * SLAB, a.ncolB, sm,
                                      a.transB);
        else
          pair_mqr_task<NB, P_F64, 0>(tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), Bp, Bi, s.slab * SLAB, a.ncolB, sm,
                                      a.transB);
      }
      break;
    default:
      break;
  }
}

// ---- executors ---------------------------------------------------------------

// Ticket loop of the persistent executors: workgroups take subtasks in
// dispatch order from an atomic ticket and wait for their predecessors'
// flags.  Every predecessor has a smaller index and was taken by a
// workgroup that is already running, so the smallest unfinished subtask can
// always proceed (no residency assumption).  A wait longer than spin_ticks
// sets *err, and every workgroup then leaves at its next wait or ticket.
// run(t) executes subtask t with the whole workgroup.
struct LoopCtl {
  const DevSub* sub;
  const int32_t* deps;
  int32_t* flags;
  const int32_t* prog;  // progress words (early releases), or null
  int32_t* ticket;
  int32_t* err;
  int32_t nsub;
  int32_t epoch;
  int64_t spin_ticks;
  int64_t* trace;
};

// Wave 0 of a workgroup waits until every predecessor of subtask t that is
// due before it starts has published its flag (or, for an early entry, its
// early release); returns t, or c.nsub after a timeout (which sets *err) or
// when another workgroup has set *err.
__device__ __forceinline__ int wait_deps(const LoopCtl& c, int t, int lane) {
  const int db = c.sub[t].dep_begin, de = c.sub[t].dep_end;
  const uint64_t t0 = wall_clock64();
  if (c.trace && lane == 0) c.trace[4 * static_cast<int64_t>(t)] = static_cast<int64_t>(t0);
  for (int e = db; e < de && t < c.nsub; ++e) {
    const int32_t d = __builtin_amdgcn_readfirstlane(c.deps[e]);
    if (dep_stage(d) != 0) continue;  // waited for inside the panel subtask
    const bool early = dep_early(d) && c.prog;
    const int32_t* f = (early ? c.prog : c.flags) + dep_index(d);
    const int32_t need = early ? early_word(c.epoch) : c.epoch;
    for (;;) {
      const int v = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(const_cast<int32_t*>(f), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (early ? v >= need : v == need) break;
      const int err = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (err != 0 || static_cast<int64_t>(wall_clock64() - t0) > c.spin_ticks) {
        if (lane == 0) __hip_atomic_store(c.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = c.nsub;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return t;
}

// After run(t): every data store of the task is device-coherent, so once
// each wave has seen its stores complete the flag can be published.
// The end tick is read before the flag is published, so a successor's ready
// tick (read after it has seen the flag) is never earlier than it.
__device__ __forceinline__ void finish_task(const LoopCtl& c, int t, int wave, int lane) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (wave == 0 && lane == 0) {
    if (c.trace) {
      c.trace[4 * static_cast<int64_t>(t) + 2] = static_cast<int64_t>(wall_clock64());
      c.trace[4 * static_cast<int64_t>(t) + 3] = blockIdx.x;
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // keep the clock read before the flag store
    }
    __hip_atomic_store(c.flags + t, c.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <class Run>
__device__ __forceinline__ void exec_loop(const LoopCtl& c, Run run) {
  __shared__ int s_t;
  // Every branch that encloses or follows a barrier is on a wave-uniform
  // (scalar) value, so the compiler keeps the loop structured: wave 0 takes
  // the ticket and waits for the predecessors as a whole wave; only the
  // single atomic operations are guarded by lane == 0.
  const int lane = lane_id();
  const int wave = wave_id();
  for (;;) {
    if (wave == 0) {
      int t = c.nsub;
      const int err0 = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (err0 == 0) {
        int tk = 0;
        if (lane == 0) tk = atomicAdd(c.ticket, 1);
        t = __builtin_amdgcn_readfirstlane(tk);
      }
      if (t < c.nsub) t = wait_deps(c, t, lane);
      if (lane == 0) s_t = t;
    }
    __syncthreads();
    // The ticket is the same for every thread; readfirstlane makes that
    // visible to the compiler (scalar loop exit and task dispatch).
    const int t = __builtin_amdgcn_readfirstlane(s_t);
    if (t >= c.nsub) break;
    if (c.trace && threadIdx.x == 0) c.trace[4 * static_cast<int64_t>(t) + 1] = static_cast<int64_t>(wall_clock64());
    run(t);
    finish_task(c, t, wave, lane);
  }
}

// The same loop, with pre(t) run by every wave after the ticket is known and
// before the predecessors are waited for (for loads of data that no
// predecessor writes, so their latency overlaps the wait).
template <class Pre, class Run>
__device__ __forceinline__ void exec_loop_pre(const LoopCtl& c, Pre pre, Run run) {
  __shared__ int s_t, s_go;
  const int lane = lane_id();
  const int wave = wave_id();
  for (;;) {
    if (wave == 0) {
      int t = c.nsub;
      const int err0 = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (err0 == 0) {
        int tk = 0;
        if (lane == 0) tk = atomicAdd(c.ticket, 1);
        t = __builtin_amdgcn_readfirstlane(tk);
      }
      if (lane == 0) s_t = t;
    }
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_t);
    if (t >= c.nsub) break;
    pre(t);
    if (wave == 0) {
      const int tw = wait_deps(c, t, lane);
      if (lane == 0) s_go = (tw == t) ? 1 : 0;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_go) == 0) break;
    if (c.trace && threadIdx.x == 0) c.trace[4 * static_cast<int64_t>(t) + 1] = static_cast<int64_t>(wall_clock64());
    run(t);
    finish_task(c, t, wave, lane);
  }
}

template <int NB, int P>
__global__ __launch_bounds__(NTHREADS) void exec_persistent(ExecArgs a) {
  __shared__ double sm[Smem<NB>::TOTAL];
  const LoopCtl c{a.sub, a.deps, a.flags, a.prog, a.ticket, a.err, a.nsub, a.epoch, a.spin_ticks, a.trace};
  exec_loop(c, [&](int t) {
    if (a.debug & 1) {
      for (int e = threadIdx.x; e < Smem<NB>::TOTAL; e += NTHREADS) sm[e] = 0.0;
      __syncthreads();
    }
    run_sub<NB, P>(a, a.sub[t], sm, t);
  });
}

// Executor of a Q application plan (apply_q kinds only, FP64): a kernel of
// its own, so that it carries only the register budget of the update tasks.
template <int NB>
__global__ __launch_bounds__(NTHREADS) void exec_apply(ExecArgs a) {
  __shared__ double sm[Smem<NB>::TOTAL];
  const LoopCtl c{a.sub, a.deps, a.flags, a.prog, a.ticket, a.err, a.nsub, a.epoch, a.spin_ticks, a.trace};
  if (a.ncolB == 16) {
    // Narrow right-hand sides: the first reflector block (written by the
    // factorization, never by a predecessor) is loaded before the wait.
    Prefetch<NB> pf;
    auto tk = [&](int t) {
      const DevSub& s = a.sub[t];
      const int kind = __builtin_amdgcn_readfirstlane(s.kind);
      const double* Tk = (kind == D_APPLY_GE) ? tg_ptr(a, s.i, s.k) : tp_ptr(a, s.i, s.k);
      return Tk;
    };
    exec_loop_pre(
        c,
        [&](int t) {
          const DevSub& s = a.sub[t];
          const int kind = __builtin_amdgcn_readfirstlane(s.kind);
          apply_load_block<NB>(pf, kind, tile_ptr(a, s.i, s.k), tk(t), a.transB ? 0 : NB - IB);
        },
        [&](int t) {
          const DevSub& s = a.sub[t];
          const int kind = __builtin_amdgcn_readfirstlane(s.kind);
          double* Bp = (kind == D_APPLY_GE) ? nullptr : a.B + static_cast<size_t>(s.piv) * NB * a.ncolB;
          double* Bi = a.B + static_cast<size_t>(s.i) * NB * a.ncolB;
          apply_narrow_task<NB>(kind, tile_ptr(a, s.i, s.k), tk(t), Bp, Bi, sm, a.transB, pf);
        });
    return;
  }
  exec_loop(c, [&](int t) {
    const DevSub& s = a.sub[t];
    const int kind = __builtin_amdgcn_readfirstlane(s.kind);
    if (kind == D_APPLY_GE) {
      double* Bi = a.B + static_cast<size_t>(s.i) * NB * a.ncolB;
      unmqr_task<NB, P_F64>(tile_ptr(a, s.i, s.k), tg_ptr(a, s.i, s.k), Bi, s.slab * SLAB, a.ncolB, sm, a.transB);
    } else {
      double* Bp = a.B + static_cast<size_t>(s.piv) * NB * a.ncolB;
      double* Bi = a.B + static_cast<size_t>(s.i) * NB * a.ncolB;
      if (kind == D_APPLY_TT)
        pair_mqr_task<NB, P_F64, 1>(tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), Bp, Bi, s.slab * SLAB, a.ncolB, sm,
                                    a.transB);
      else
        pair_mqr_task<NB, P_F64, 0>(tile_ptr(a, s.i, s.k), tp_ptr(a, s.i, s.k), Bp, Bi, s.slab * SLAB, a.ncolB, sm,
                                    a.transB);
    }
  });
}

// Batched executor: subtasks of many problems (tile sizes 32 or 64) in one
// launch; each subtask runs on its problem's tiles.
template <int P>
__global__ __launch_bounds__(NTHREADS, 4) void exec_batched(BatchArgs b) {
  __shared__ double sm[Smem<64>::TOTAL];
  const int epoch = __builtin_amdgcn_readfirstlane(
      __hip_atomic_load(b.ctl + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  // The trace buffer is read from device memory, so that a captured graph
  // of the launch can be traced or not without capturing it again.
  int64_t* const tr = b.trace ? *b.trace : nullptr;
  const LoopCtl c{b.sub, b.deps, b.flags, nullptr, b.ctl, b.ctl + 1, b.nsub, epoch, b.spin_ticks, tr};
  exec_loop(c, [&](int t) {
    const ProbDesc& pd = b.prob[__builtin_amdgcn_readfirstlane(b.prob_of[t])];
    ExecArgs a{};
    a.tiles = pd.tiles;
    a.Tg = pd.Tg;
    a.Tp = pd.Tp;
    a.p = __builtin_amdgcn_readfirstlane(pd.p);
    a.q = __builtin_amdgcn_readfirstlane(pd.q);
    a.nb = __builtin_amdgcn_readfirstlane(pd.nb);
    a.upd = P;
    if (a.nb == 32)
      run_sub<32, P>(a, b.sub[t], sm, t);
    else
      run_sub<64, P>(a, b.sub[t], sm, t);
  });
}

__global__ void batch_reset_kernel(int32_t* ctl) {
  ctl[0] = 0;
  ctl[1] = 0;
  ctl[2] = ctl[2] + 1;
}

hipError_t launch_batch_reset(int32_t* ctl, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, ctl);
  return hipGetLastError();
}

hipError_t launch_batched(const BatchArgs& b, int grid, hipStream_t s) {
  switch (b.upd) {
    case P_F64: hipLaunchKernelGGL((exec_batched<P_F64>), dim3(grid), dim3(NTHREADS), 0, s, b); break;
    case P_F32: hipLaunchKernelGGL((exec_batched<P_F32>), dim3(grid), dim3(NTHREADS), 0, s, b); break;
    case P_BF16: hipLaunchKernelGGL((exec_batched<P_BF16>), dim3(grid), dim3(NTHREADS), 0, s, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int batched_occupancy(int upd) {
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (upd) {
    case P_F64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_batched<P_F64>, NTHREADS, 0); break;
    case P_F32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_batched<P_F32>, NTHREADS, 0); break;
    case P_BF16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_batched<P_BF16>, NTHREADS, 0); break;
    default: break;
  }
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

// Level-synchronous executor: one launch per DAG depth level, one subtask
// per workgroup (kernel boundaries order the levels).
template <int NB, int P>
__global__ __launch_bounds__(NTHREADS) void exec_level(ExecArgs a, const int32_t* order, int begin) {
  __shared__ double sm[Smem<NB>::TOTAL];
  const int t = __builtin_amdgcn_readfirstlane(order[begin + blockIdx.x]);
  run_sub<NB, P>(a, a.sub[t], sm, t);
  // Streamed and early-release waits inside later levels read the flags.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(a.flags + t, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void reset_kernel(int32_t* ticket, int32_t* err) {
  *ticket = 0;
  *err = 0;
}

hipError_t launch_reset(int32_t* ticket, int32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, s, ticket, err);
  return hipGetLastError();
}

template <int NB>
static hipError_t launch_persistent_nb(const ExecArgs& a, int grid, hipStream_t s) {
  if (a.B && !a.fused) {
    hipLaunchKernelGGL((exec_apply<NB>), dim3(grid), dim3(NTHREADS), 0, s, a);
    return hipGetLastError();
  }
  switch (a.upd) {
    case P_F64: hipLaunchKernelGGL((exec_persistent<NB, P_F64>), dim3(grid), dim3(NTHREADS), 0, s, a); break;
    case P_F32: hipLaunchKernelGGL((exec_persistent<NB, P_F32>), dim3(grid), dim3(NTHREADS), 0, s, a); break;
    case P_BF16: hipLaunchKernelGGL((exec_persistent<NB, P_BF16>), dim3(grid), dim3(NTHREADS), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_persistent(const ExecArgs& a, int grid, hipStream_t s) {
  switch (a.nb) {
    case 32: return launch_persistent_nb<32>(a, grid, s);
    case 64: return launch_persistent_nb<64>(a, grid, s);
    case 128: return launch_persistent_nb<128>(a, grid, s);
    case 256: return launch_persistent_nb<256>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NB>
static hipError_t launch_level_nb(const ExecArgs& a, const int32_t* order, int begin, int count, hipStream_t s) {
  switch (a.upd) {
    case P_F64: hipLaunchKernelGGL((exec_level<NB, P_F64>), dim3(count), dim3(NTHREADS), 0, s, a, order, begin); break;
    case P_F32: hipLaunchKernelGGL((exec_level<NB, P_F32>), dim3(count), dim3(NTHREADS), 0, s, a, order, begin); break;
    case P_BF16: hipLaunchKernelGGL((exec_level<NB, P_BF16>), dim3(count), dim3(NTHREADS), 0, s, a, order, begin); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_level(const ExecArgs& a, const int32_t* order, int begin, int count, hipStream_t s) {
  switch (a.nb) {
    case 32: return launch_level_nb<32>(a, order, begin, count, s);
    case 64: return launch_level_nb<64>(a, order, begin, count, s);
    case 128: return launch_level_nb<128>(a, order, begin, count, s);
    case 256: return launch_level_nb<256>(a, order, begin, count, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NB>
static int occupancy_nb(int upd) {
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (upd) {
    case P_F64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_persistent<NB, P_F64>, NTHREADS, 0); break;
    case P_F32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_persistent<NB, P_F32>, NTHREADS, 0); break;
    case P_BF16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_persistent<NB, P_BF16>, NTHREADS, 0); break;
    default: break;
  }
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

int persistent_occupancy(int nb, int upd) {
  switch (nb) {
    case 32: return occupancy_nb<32>(upd);
    case 64: return occupancy_nb<64>(upd);
    case 128: return occupancy_nb<128>(upd);
    case 256: return occupancy_nb<256>(upd);
    default: return 1;
  }
}

}  // namespace tqr
