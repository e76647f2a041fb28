// Device primitives shared by the tile kernels: vector types, FP64 MFMA,
// device-coherent loads and stores, wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace tqr {

// MFMA f64 16x16x4 operand layout (lane l, g = l / 16, n = l % 16; measured
// on gfx950 with one-hot operands):
//   A (16x4):  A[n][g]          B (4x16): B[g][n]
//   C/D (16x16): D[4i + g][n], i = 0..3 (four doubles per lane)
// For a fixed i the four lane groups hold the four consecutive rows
// 16 rb + 4 i + {0..3}, so a C block held as D feeds the B operand of a
// contraction over those rows directly.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int NWAVES = NTHREADS / 64;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 zero4() { return d4{0.0, 0.0, 0.0, 0.0}; }
__device__ __forceinline__ f4 zero4f() { return f4{0.0f, 0.0f, 0.0f, 0.0f}; }
// FP32 MFMA 16x16x4 and BF16 MFMA 16x16x32 (FP32 accumulation).  Measured
// on gfx950: both write D[4 g + r][n] (lane l = 16 g + n, register r), and
// the k index of an A element is that of the B element in the same lane
// and position, so any consistent assignment of k to (g, e) contracts
// correctly.
__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfmabf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// The lane index, opaque to the optimizer: the empty asm statement keeps
// lane-derived addresses from being hoisted out of the persistent task loops,
// where they would stay live across every task and spill to scratch (they
// are recomputed at each use instead).
__device__ __forceinline__ int lane_id() {
  int v = threadIdx.x & 63;
  asm volatile("" : "+v"(v));
  return v;
}
// The lane index for the FP64 update and prefetch helpers: plain at
// NB >= 128, where the FP64 executor holds its addresses without spilling
// and the opaque index would only add recomputation; opaque below.
template <int NB>
__device__ __forceinline__ int lane_nb() {
  if constexpr (NB >= 128)
    return threadIdx.x & 63;
  else
    return lane_id();
}

// Tile, T and right-hand-side data move with device-coherent (sc1) loads and
// stores.  The eight XCDs have L2 caches that are not coherent with each
// other; with every data access coherent at device scope, a task publishes
// its results by waiting for its stores to complete, without writing back
// and invalidating the whole L2 of its XCD around every task.
__device__ __forceinline__ double gld(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gst(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 16-byte device-coherent accesses through a buffer resource (the base
// pointer is wave-uniform, the byte offset per lane): buffer loads and
// stores with the sc1 cache policy, as the scalar accesses above.
typedef double d2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
constexpr int CPOL_SC1 = 16;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const double* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0, bytes, 0x00020000);
}
__device__ __forceinline__ d2 gld2(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CPOL_SC1));
}
__device__ __forceinline__ void gst2(__amdgpu_buffer_rsrc_t r, int off, d2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, off, 0, CPOL_SC1);
}
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(b));
  const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double lane_d(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// One DPP move of a double (two 32-bit halves); lanes outside row_mask or
// reading an invalid source get 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Sum over the 64 lanes of a wave, returned to every lane: quad swaps and
// row rotations give each row of 16 its sum, row_bcast:15 / row_bcast:31
// carry the row sums into the last row, and lane 63 holds the total.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x124, 0xf>(v);  // row_ror:4
  v += dpp_d<0x128, 0xf>(v);  // row_ror:8
  v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return lane_d(v, 63);
}

// x[l] + x[l ^ 16] (SWAP = 16) or x[l] + x[l ^ 32] (SWAP = 32) in every lane.
// The gfx950 lane swaps exchange the odd rows of their first operand with
// the even rows of their second (16) or the upper half of the first with
// the lower half of the second (32); with both operands x, the two results
// hold, in every lane, x[l] and x[l ^ SWAP] in some order (measured).
template <int SWAP>
__device__ __forceinline__ double add_swapped(double x) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = static_cast<unsigned>(b), hi = static_cast<unsigned>(b >> 32);
  const auto l2 = SWAP == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                             : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h2 = SWAP == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                             : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double f = __longlong_as_double((static_cast<long long>(h2[0]) << 32) | l2[0]);
  const double g = __longlong_as_double((static_cast<long long>(h2[1]) << 32) | l2[1]);
  return f + g;
}

// The four sums over the 64 lanes of a wave of a[0..3], returned in a
// (uniform).  A butterfly over each quad leaves lane l with the quad's sum
// of value m(l) = 2 (l & 1) + ((l >> 1) & 1): lanes exchange the two values
// they do not keep, so four values cost two steps instead of eight.  Row
// rotations by 4 and 8 then add the lanes of the row with the same l & 3,
// and the 16- and 32-lane swaps the other rows: lanes 0, 2, 1, 3 then hold
// the totals of values 0, 1, 2, 3.
__device__ __forceinline__ void wave_sum4(double (&a)[4]) {
  const int l = lane_id();
  const bool odd = (l & 1) != 0, up = (l & 2) != 0;
  // lane pairs (xor 1): even lanes keep values 0 and 1, odd lanes 2 and 3
  const double b0 = (odd ? a[2] : a[0]) + dpp_d<0xb1, 0xf>(odd ? a[0] : a[2]);
  const double b1 = (odd ? a[3] : a[1]) + dpp_d<0xb1, 0xf>(odd ? a[1] : a[3]);
  // lane pairs (xor 2): lanes with bit 1 clear keep b0, the others b1
  double c = (up ? b1 : b0) + dpp_d<0x4e, 0xf>(up ? b0 : b1);
  c += dpp_d<0x124, 0xf>(c);  // row_ror:4
  c += dpp_d<0x128, 0xf>(c);  // row_ror:8
  c = add_swapped<16>(c);
  c = add_swapped<32>(c);
  a[0] = lane_d(c, 0);
  a[1] = lane_d(c, 2);
  a[2] = lane_d(c, 1);
  a[3] = lane_d(c, 3);
}

}  // namespace tqr
