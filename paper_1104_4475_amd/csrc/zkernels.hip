// Double-complex tile kernels (the paper's ZGEQRT family, Sec. 5) and their
// executor, nb = 32.
//
// The six kernels of Sec. 2.1 in complex arithmetic with LAPACK's complex
// elementary reflector: H = I - tau u u^H, u = (1, v), H^H (alpha, x) =
// (beta, 0) with beta = -sign(Re alpha) sqrt(|alpha|^2 + ||x||^2) real,
// tau = (beta - alpha) / beta, v = x / (alpha - beta); H = I only when x = 0
// and alpha is real.  The factorization applies H^H from the left, so an
// update subtracts conj(tau) u (u^H c) from each column c.
//
// Storage: a complex tile is nb x nb column-major with interleaved real and
// imaginary parts (tile (r, c) of a p x q grid at 2 (c p + r) nb^2
// doubles); tau of the GEQRT set of tile (r, c) at 2 (c p + r) nb doubles
// of taug, of the TS/TT set that zeroed it likewise in taup.
//
// One task runs on two waves (a workgroup of 128 lanes).  Wave w holds
// columns 16 w .. 16 w + 15 of the tile it updates, four lanes per column,
// eight rows per lane (lane l: column 16 w + l % 16, rows 8 (l / 16) ..
// 8 (l / 16) + 7); the four lanes of a column add their partial sums with
// the 16- and 32-lane swaps.  Reflectors are generated and applied one at a
// time: the owner lanes of column j write it to LDS, the norm is a
// wavefront sum over one row per lane, the reflector goes back to LDS, and
// every lane forms its column's dot product u^H c and rank-1 update.  A
// finished column's lanes keep the column as it was when its reflector was
// generated; v is that column times its scale, written at the end.
//
// The executor walks the same subtask tables as the real executor (one
// subtask per task at this tile size; the Q application plans with one
// 32-column slab of the right-hand side per subtask) with a ticket loop of
// its own:
// subtasks are taken in dispatch order and wait for their predecessors'
// completion flags (epoch-tagged, so no reset between runs).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "hip_prims.hpp"

namespace tqr {
namespace {

constexpr int ZNB = 32;
constexpr int ZTHREADS = 128;
constexpr int ZCPW = 16;  // columns per wave
constexpr int ZRPL = 8;   // rows per lane
constexpr int ZNCH = ZNB / 8;

struct cd {
  double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cconj(cd a) { return cd{a.re, -a.im}; }
// a -= w v
__device__ __forceinline__ void csub_mul(cd& a, cd w, cd v) {
  a.re = fma(-w.re, v.re, fma(w.im, v.im, a.re));
  a.im = fma(-w.re, v.im, fma(-w.im, v.re, a.im));
}
// s += conj(v) a
__device__ __forceinline__ void cacc_conj(cd& s, cd v, cd a) {
  s.re = fma(v.re, a.re, fma(v.im, a.im, s.re));
  s.im = fma(v.re, a.im, fma(-v.im, a.re, s.im));
}

// LDS of one task, in doubles.
struct ZLds {
  static constexpr int XB = 0;               // owner's column, one complex row per lane
  static constexpr int VB = 2 * 64;          // reflector, one complex row per lane
  static constexpr int TAU = 4 * 64;         // tau of the task's reflectors
  static constexpr int R1S = TAU + 2 * ZNB;  // 8 rows of the pivot tile (complex)
  static constexpr int VS = 0;               // 8 reflectors, one complex row per lane
  static constexpr int C1S = 2 * 8 * ZNB;    // 8 rows of C1 (complex)
  static constexpr int TSC = 4 * 8 * ZNB;    // their tau
  static constexpr int TOTAL = R1S + 2 * 8 * ZNB > TSC + 16 ? R1S + 2 * 8 * ZNB : TSC + 16;
};

struct ZPos {
  int lane, wave, c, h, r0;
  __device__ __forceinline__ ZPos() {
    lane = lane_id();
    wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    c = ZCPW * wave + lane % ZCPW;
    h = lane / ZCPW;
    r0 = h * ZRPL;
  }
};

__device__ __forceinline__ cd zcol_sum(cd x) {
  return cd{add_swapped<32>(add_swapped<16>(x.re)), add_swapped<32>(add_swapped<16>(x.im))};
}

__device__ __forceinline__ cd zld(const double* p) { return cd{gld(p), gld(p + 1)}; }
__device__ __forceinline__ void zst(double* p, cd v) {
  gst(p, v.re);
  gst(p + 1, v.im);
}
__device__ __forceinline__ cd lds_cd(const double* p) {
  const d2 v = *reinterpret_cast<const d2*>(p);
  return cd{v[0], v[1]};
}
__device__ __forceinline__ void lds_st(double* p, cd v) { *reinterpret_cast<d2*>(p) = d2{v.re, v.im}; }

// Rows r0 .. r0 + 7 of column col of a complex tile.
__device__ __forceinline__ void zload_col(cd (&a)[ZRPL], const double* tile, int col, int r0) {
  const auto R = rsrc(tile, ZNB * ZNB * 16);
  const int base = (col * ZNB + r0) * 16;
#pragma unroll
  for (int k = 0; k < ZRPL; ++k) {
    const d2 v = gld2(R, base + 16 * k);
    a[k] = cd{v[0], v[1]};
  }
}
__device__ __forceinline__ void zstore_col(const cd (&a)[ZRPL], double* tile, int col, int r0) {
  const auto R = rsrc(tile, ZNB * ZNB * 16);
  const int base = (col * ZNB + r0) * 16;
#pragma unroll
  for (int k = 0; k < ZRPL; ++k) gst2(R, base + 16 * k, d2{a[k].re, a[k].im});
}

struct ZRefl {
  double beta;
  cd tau, scale;
};
// Complex reflector of (alpha, x) with ||x||^2 = ssq (uniform inputs).
__device__ __forceinline__ ZRefl zmake_refl(cd alpha, double ssq) {
  ZRefl f{alpha.re, cd{0.0, 0.0}, cd{0.0, 0.0}};
  if (ssq != 0.0 || alpha.im != 0.0) {
    const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + ssq);
    f.beta = alpha.re >= 0.0 ? -nrm : nrm;
    f.tau = cd{(f.beta - alpha.re) / f.beta, -alpha.im / f.beta};
    const double dr = alpha.re - f.beta, di = alpha.im, den = dr * dr + di * di;
    f.scale = cd{dr / den, -di / den};  // 1 / (alpha - beta)
  }
  return f;
}

__device__ __forceinline__ cd uniform_cd(cd v) { return cd{uniform_d(v.re), uniform_d(v.im)}; }

// Dot product u^H c over this lane's rows, summed over the column's lanes.
__device__ __forceinline__ cd zdot(const double* vb, const cd (&a)[ZRPL], int r0) {
  cd s0{0.0, 0.0}, s1{0.0, 0.0};
#pragma unroll
  for (int k = 0; k < ZRPL; k += 2) {
    cacc_conj(s0, lds_cd(vb + 2 * (r0 + k)), a[k]);
    cacc_conj(s1, lds_cd(vb + 2 * (r0 + k + 1)), a[k + 1]);
  }
  return zcol_sum(cd{s0.re + s1.re, s0.im + s1.im});
}
__device__ __forceinline__ void zupdate(const double* vb, cd (&a)[ZRPL], int r0, cd w) {
#pragma unroll
  for (int k = 0; k < ZRPL; ++k) csub_mul(a[k], w, lds_cd(vb + 2 * (r0 + k)));
}

// ---- ZGEQRT ----------------------------------------------------------------
__device__ void zgeqrt_task(double* A, double* tau, double* L) {
  const ZPos P;
  const int lane = P.lane, c = P.c, r0 = P.r0;
  double* xb = L + ZLds::XB;
  double* vb = L + ZLds::VB;
  cd a[ZRPL];
  zload_col(a, A, c, r0);
  cd myscale{0.0, 0.0}, mytau{0.0, 0.0};
  double mybeta = 0.0;
#pragma unroll 1
  for (int j = 0; j < ZNB; ++j) {
    if (c == j) {
#pragma unroll
      for (int k = 0; k < ZRPL; ++k) lds_st(xb + 2 * (r0 + k), a[k]);
    }
    __syncthreads();
    const cd x = lane < ZNB ? lds_cd(xb + 2 * lane) : cd{0.0, 0.0};
    const cd alpha = uniform_cd(lds_cd(xb + 2 * j));
    const double xs = (lane > j && lane < ZNB) ? x.re * x.re + x.im * x.im : 0.0;
    const ZRefl f = zmake_refl(alpha, wave_sum(xs));
    if (P.wave == 0 && lane < ZNB)
      lds_st(vb + 2 * lane, lane > j ? cmul(x, f.scale) : cd{lane == j ? 1.0 : 0.0, 0.0});
    __syncthreads();
    const cd d = zdot(vb, a, r0);
    const cd w = c > j ? cmul(cconj(f.tau), d) : cd{0.0, 0.0};
    zupdate(vb, a, r0, w);
    if (c == j) {
      myscale = f.scale;
      mytau = f.tau;
      mybeta = f.beta;
    }
  }
  // R above the diagonal, beta on it, v = scale x below it; tau.
  cd o[ZRPL];
#pragma unroll
  for (int k = 0; k < ZRPL; ++k) {
    const int r = r0 + k;
    o[k] = r < c ? a[k] : (r == c ? cd{mybeta, 0.0} : cmul(a[k], myscale));
  }
  zstore_col(o, A, c, r0);
  if (P.h == 0) zst(tau + 2 * c, mytau);
}

// ---- ZTSQRT / ZTTQRT ---------------------------------------------------------
// R1: pivot tile (upper triangle R), A2: the tile to zero (TT: its upper
// triangle).  Row j of R1 is needed only at step j: 8 rows at a time in LDS.
template <int TT>
__device__ void zpair_task(double* R1, double* A2, double* tau, double* L) {
  const ZPos P;
  const int lane = P.lane, c = P.c, h = P.h, r0 = P.r0;
  double* xb = L + ZLds::XB;
  double* vb = L + ZLds::VB;
  double* r1s = L + ZLds::R1S;
  cd a[ZRPL];
  zload_col(a, A2, c, r0);
  if (TT) {
#pragma unroll
    for (int k = 0; k < ZRPL; ++k)
      if (r0 + k > c) a[k] = cd{0.0, 0.0};
  }
  cd myscale{0.0, 0.0}, mytau{0.0, 0.0};
#pragma unroll 1
  for (int b = 0; b < ZNCH; ++b) {
    if (h == 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int row = 8 * b + i;
        lds_st(r1s + 2 * (i * ZNB + c), row <= c ? zld(R1 + 2 * (c * ZNB + row)) : cd{0.0, 0.0});
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int j = 8 * b; j < 8 * b + 8; ++j) {
      const int jj = j & 7;
      if (c == j) {
#pragma unroll
        for (int k = 0; k < ZRPL; ++k) lds_st(xb + 2 * (r0 + k), a[k]);
      }
      __syncthreads();
      const bool in = lane < ZNB && (TT ? lane <= j : true);
      const cd x = in ? lds_cd(xb + 2 * lane) : cd{0.0, 0.0};
      const cd alpha = uniform_cd(lds_cd(r1s + 2 * (jj * ZNB + j)));
      const ZRefl f = zmake_refl(alpha, wave_sum(x.re * x.re + x.im * x.im));
      if (P.wave == 0 && lane < ZNB) lds_st(vb + 2 * lane, cmul(x, f.scale));
      __syncthreads();
      const cd dot = zdot(vb, a, r0);
      const cd top = lds_cd(r1s + 2 * (jj * ZNB + c));  // R1[j][c] (0 below the diagonal)
      const cd w = c > j ? cmul(cconj(f.tau), cd{top.re + dot.re, top.im + dot.im}) : cd{0.0, 0.0};
      zupdate(vb, a, r0, w);
      if (h == 0 && c >= j) lds_st(r1s + 2 * (jj * ZNB + c), c == j ? cd{f.beta, 0.0} : cd{top.re - w.re, top.im - w.im});
      if (c == j) {
        myscale = f.scale;
        mytau = f.tau;
      }
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int row = 8 * b + i;
        if (row <= c) zst(R1 + 2 * (c * ZNB + row), lds_cd(r1s + 2 * (i * ZNB + c)));
      }
    }
    __syncthreads();
  }
  // V2 = scale x (TT: its upper triangle).
#pragma unroll
  for (int k = 0; k < ZRPL; ++k) {
    const int r = r0 + k;
    if (!TT || r <= c) zst(A2 + 2 * (c * ZNB + r), cmul(a[k], myscale));
  }
  if (h == 0) zst(tau + 2 * c, mytau);
}

// ---- ZUNMQR / ZTSMQR / ZTTMQR --------------------------------------------------
// KIND 0: reflectors of a ZGEQRT tile (unit diagonal, rows below it); 1: of
// a ZTSQRT tile (every row); 2: of a ZTTQRT tile (upper triangle).  C1 (pair
// kinds: the pivot row's tile, row j touched by reflector j only), C2: the
// target tile.  CONJ: Q^H, reflector 0 first with conj(tau); else Q, the
// last reflector first with tau.
template <int KIND, bool CONJ>
__device__ void zupdate_task(const double* V, const double* tau, double* C1, double* C2, double* L) {
  constexpr bool PAIR = KIND != 0;
  const ZPos P;
  const int lane = P.lane, c = P.c, h = P.h, r0 = P.r0;
  double* vs = L + ZLds::VS;
  double* c1s = L + ZLds::C1S;
  double* tsc = L + ZLds::TSC;
  cd a[ZRPL];
  zload_col(a, C2, c, r0);
#pragma unroll 1
  for (int qq = 0; qq < ZNCH; ++qq) {
    const int q = CONJ ? qq : ZNCH - 1 - qq;
    if (P.wave == 0) {
      if (lane < ZNB) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int jv = 8 * q + i;
          const cd x = zld(V + 2 * (jv * ZNB + lane));
          const cd vv = KIND == 0 ? (lane > jv ? x : cd{lane == jv ? 1.0 : 0.0, 0.0})
                                  : (KIND == 2 ? (lane <= jv ? x : cd{0.0, 0.0}) : x);
          lds_st(vs + 2 * (i * ZNB + lane), vv);
        }
      }
      if (lane < 8) lds_st(tsc + 2 * lane, zld(tau + 2 * (8 * q + lane)));
    }
    if (PAIR && h == 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) lds_st(c1s + 2 * (i * ZNB + c), zld(C1 + 2 * (c * ZNB + 8 * q + i)));
    }
    __syncthreads();
#pragma unroll 1
    for (int ii = 0; ii < 8; ++ii) {
      const int i = CONJ ? ii : 7 - ii;
      const double* vb = vs + 2 * i * ZNB;
      const cd dot = zdot(vb, a, r0);
      const cd top = PAIR ? lds_cd(c1s + 2 * (i * ZNB + c)) : cd{0.0, 0.0};
      const cd t = lds_cd(tsc + 2 * i);
      const cd w = cmul(CONJ ? cconj(t) : t, cd{top.re + dot.re, top.im + dot.im});
      zupdate(vb, a, r0, w);
      if (PAIR && h == 0) lds_st(c1s + 2 * (i * ZNB + c), cd{top.re - w.re, top.im - w.im});
    }
    __syncthreads();
    if (PAIR && h == 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) zst(C1 + 2 * (c * ZNB + 8 * q + i), lds_cd(c1s + 2 * (i * ZNB + c)));
    }
  }
  zstore_col(a, C2, c, r0);
}

struct ZArgs {
  double* tiles;
  double* taug;
  double* taup;
  const DevSub* sub;
  const int32_t* deps;
  int32_t* flags;
  int32_t* ticket;
  int32_t* err;
  int32_t nsub, epoch, p;
  int64_t spin_ticks;
  double* B;       // Q application: p row tiles of 32 x ncolB complex (ld 32)
  int32_t ncolB;   // columns of the row tiles, a multiple of 32 (one 32-column slab per subtask)
  int32_t transB;  // 1: Q^H B, 0: Q B
};

__device__ __forceinline__ double* ztile(const ZArgs& a, int r, int c) {
  return a.tiles + (static_cast<size_t>(c) * a.p + r) * 2 * ZNB * ZNB;
}
__device__ __forceinline__ double* ztau(double* base, const ZArgs& a, int r, int c) {
  return base + (static_cast<size_t>(c) * a.p + r) * 2 * ZNB;
}

__global__ __launch_bounds__(ZTHREADS) void exec_zqr(ZArgs a) {
  __shared__ __attribute__((aligned(16))) double L[ZLds::TOTAL];
  __shared__ int s_t;
  const int lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (;;) {
    if (wave == 0) {
      int t = a.nsub;
      const int e0 = __builtin_amdgcn_readfirstlane(__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (e0 == 0) {
        int tk = 0;
        if (lane == 0) tk = atomicAdd(a.ticket, 1);
        t = __builtin_amdgcn_readfirstlane(tk);
      }
      if (t < a.nsub) {
        // every predecessor entry is a plain completion flag at this tile size
        const uint64_t t0 = wall_clock64();
        for (int e = a.sub[t].dep_begin; e < a.sub[t].dep_end && t < a.nsub; ++e) {
          const int32_t d = dep_index(__builtin_amdgcn_readfirstlane(a.deps[e]));
          for (;;) {
            const int v = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(a.flags + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (v == a.epoch) break;
            const int er = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (er != 0 || static_cast<int64_t>(wall_clock64() - t0) > a.spin_ticks) {
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
    const int t = __builtin_amdgcn_readfirstlane(s_t);
    if (t >= a.nsub) break;
    const DevSub& s = a.sub[t];
    const int kind = __builtin_amdgcn_readfirstlane(s.kind);
    const int i = __builtin_amdgcn_readfirstlane(s.i), piv = __builtin_amdgcn_readfirstlane(s.piv);
    const int k = __builtin_amdgcn_readfirstlane(s.k), j = __builtin_amdgcn_readfirstlane(s.j);
    switch (kind) {
      case D_GEQRT: zgeqrt_task(ztile(a, i, k), ztau(a.taug, a, i, k), L); break;
      case D_UNMQR: zupdate_task<0, true>(ztile(a, i, k), ztau(a.taug, a, i, k), nullptr, ztile(a, i, j), L); break;
      case D_TSQRT: zpair_task<0>(ztile(a, piv, k), ztile(a, i, k), ztau(a.taup, a, i, k), L); break;
      case D_TTQRT: zpair_task<1>(ztile(a, piv, k), ztile(a, i, k), ztau(a.taup, a, i, k), L); break;
      case D_TSMQR:
        zupdate_task<1, true>(ztile(a, i, k), ztau(a.taup, a, i, k), ztile(a, piv, j), ztile(a, i, j), L);
        break;
      case D_TTMQR:
        zupdate_task<2, true>(ztile(a, i, k), ztau(a.taup, a, i, k), ztile(a, piv, j), ztile(a, i, j), L);
        break;
      case D_APPLY_GE:
      case D_APPLY_TS:
      case D_APPLY_TT: {
        const size_t off = 2 * static_cast<size_t>(__builtin_amdgcn_readfirstlane(s.slab)) * ZNB * ZNB;
        double* Bi = a.B + 2 * static_cast<size_t>(i) * ZNB * a.ncolB + off;
        double* Bp = a.B + 2 * static_cast<size_t>(piv) * ZNB * a.ncolB + off;
        const double* V = ztile(a, i, k);
        if (kind == D_APPLY_GE) {
          if (a.transB)
            zupdate_task<0, true>(V, ztau(a.taug, a, i, k), nullptr, Bi, L);
          else
            zupdate_task<0, false>(V, ztau(a.taug, a, i, k), nullptr, Bi, L);
        } else if (kind == D_APPLY_TS) {
          if (a.transB)
            zupdate_task<1, true>(V, ztau(a.taup, a, i, k), Bp, Bi, L);
          else
            zupdate_task<1, false>(V, ztau(a.taup, a, i, k), Bp, Bi, L);
        } else {
          if (a.transB)
            zupdate_task<2, true>(V, ztau(a.taup, a, i, k), Bp, Bi, L);
          else
            zupdate_task<2, false>(V, ztau(a.taup, a, i, k), Bp, Bi, L);
        }
        break;
      }
      default: break;
    }
    // publish once every lane's stores are complete
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (wave == 0 && lane == 0) __hip_atomic_store(a.flags + t, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void zreset_kernel(int32_t* ticket, int32_t* err) {
  *ticket = 0;
  *err = 0;
}

// Column-major complex A (m x n, leading dimension lda in complex elements)
// to and from the tile layout.
__global__ void zpack_kernel(double* A, int64_t lda, double* tiles, int p, int q, bool unpack) {
  const int64_t total = static_cast<int64_t>(p) * q * ZNB * ZNB;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t t = e / (ZNB * ZNB), w = e % (ZNB * ZNB);
    const int64_t tc = t / p, tr = t % p, cc = w / ZNB, rr = w % ZNB;
    const int64_t col = tc * ZNB + cc, row = tr * ZNB + rr;
    double* T = tiles + 2 * e;
    double* M = A + 2 * (col * lda + row);
    if (unpack) {
      M[0] = T[0];
      M[1] = T[1];
    } else {
      T[0] = M[0];
      T[1] = M[1];
    }
  }
}

// m x nrhs column-major complex B (ldb) to and from p row tiles of 32 x
// ncolB (ld 32; columns nrhs .. ncolB - 1 zero when packing).
__global__ void zpack_b_kernel(double* Bm, int64_t ldb, int64_t nrhs, double* Bt, int p, int ncolB, bool unpack) {
  const int64_t total = static_cast<int64_t>(p) * ZNB * ncolB;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t t = e / (static_cast<int64_t>(ZNB) * ncolB), w = e % (static_cast<int64_t>(ZNB) * ncolB);
    const int64_t col = w / ZNB, row = t * ZNB + w % ZNB;
    double* T = Bt + 2 * e;
    if (col >= nrhs) {
      if (!unpack) {
        T[0] = 0.0;
        T[1] = 0.0;
      }
      continue;
    }
    double* M = Bm + 2 * (col * ldb + row);
    if (unpack) {
      M[0] = T[0];
      M[1] = T[1];
    } else {
      T[0] = M[0];
      T[1] = M[1];
    }
  }
}

// X <- R^{-1} X for the upper triangular n x n complex R held in the tiles
// (top q tile rows): one workgroup per right-hand side, the column in LDS,
// back substitution with the column of R below the pivot applied by all
// threads (n <= ZSOLVE_MAX).
constexpr int ZSOLVE_MAX = 4096;
__global__ __launch_bounds__(256) void zsolve_r_kernel(const double* tiles, int p, int n, double* X, int64_t ldx) {
  __shared__ __attribute__((aligned(16))) double xs[2 * ZSOLVE_MAX];
  double* x = X + 2 * static_cast<int64_t>(blockIdx.x) * ldx;
  for (int r = threadIdx.x; r < n; r += blockDim.x) lds_st(xs + 2 * r, cd{x[2 * r], x[2 * r + 1]});
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    const int ti = i / ZNB, ci = i % ZNB;
    const double* colt = tiles;  // column i of R: tiles (tr, ti), tr <= ti
    const cd rii = zld(colt + 2 * ((static_cast<size_t>(ti) * p + ti) * ZNB * ZNB + ci * ZNB + ci));
    const cd bi = lds_cd(xs + 2 * i);
    const double den = rii.re * rii.re + rii.im * rii.im;
    const cd xi = cd{(bi.re * rii.re + bi.im * rii.im) / den, (bi.im * rii.re - bi.re * rii.im) / den};
    __syncthreads();
    if (threadIdx.x == 0) lds_st(xs + 2 * i, xi);
    for (int r = threadIdx.x; r < i; r += blockDim.x) {
      const cd rri = zld(colt + 2 * ((static_cast<size_t>(ti) * p + r / ZNB) * ZNB * ZNB + ci * ZNB + r % ZNB));
      cd b = lds_cd(xs + 2 * r);
      csub_mul(b, xi, rri);
      lds_st(xs + 2 * r, b);
    }
    __syncthreads();
  }
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    const cd v = lds_cd(xs + 2 * r);
    x[2 * r] = v.re;
    x[2 * r + 1] = v.im;
  }
}

}  // namespace

hipError_t launch_zsolve_r(const double* tiles, int p, int n, double* X, int64_t ldx, int64_t nrhs, hipStream_t s) {
  if (n > ZSOLVE_MAX || nrhs < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zsolve_r_kernel, dim3(static_cast<unsigned>(nrhs)), dim3(256), 0, s, tiles, p, n, X, ldx);
  return hipGetLastError();
}

hipError_t launch_zpack_b(double* Bm, int64_t ldb, int64_t nrhs, double* Bt, int p, int ncolB, bool unpack,
                          hipStream_t s) {
  const int64_t total = static_cast<int64_t>(p) * ZNB * ncolB;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zpack_b_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, Bm, ldb, nrhs, Bt, p,
                     ncolB, unpack);
  return hipGetLastError();
}

hipError_t launch_zqr(double* tiles, double* taug, double* taup, const DevSub* sub, const int32_t* deps,
                      int32_t* flags, int32_t* ctl, int32_t nsub, int32_t epoch, int32_t p, int64_t spin_ticks,
                      int grid, hipStream_t s, double* B, int32_t ncolB, int32_t transB) {
  hipLaunchKernelGGL(zreset_kernel, dim3(1), dim3(1), 0, s, ctl, ctl + 1);
  ZArgs a{tiles, taug, taup, sub, deps, flags, ctl, ctl + 1, nsub, epoch, p, spin_ticks, B, ncolB, transB};
  hipLaunchKernelGGL(exec_zqr, dim3(grid), dim3(ZTHREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zpack(double* A, int64_t lda, double* tiles, int p, int q, bool unpack, hipStream_t s) {
  const int64_t total = static_cast<int64_t>(p) * q * ZNB * ZNB;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zpack_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A, lda, tiles, p, q, unpack);
  return hipGetLastError();
}

int zqr_occupancy() {
  int blocks = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, exec_zqr, ZTHREADS, 0);
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

}  // namespace tqr
