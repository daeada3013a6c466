// Device helpers shared by the one-sweep kernels (internal): the 16-byte row
// groups, the element views of float32 and bfloat16 rows, the wave sum, the
// LDS-only barrier and the raw buffer resource word.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"

namespace gkb {
namespace fdev {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 64 lanes of a wave through DPP moves (no LDS round trips),
// in one fixed tree: quad pairs, quad halves, half-row mirror, row mirror,
// then rows 0 + 1 and 2 + 3 (row broadcast of lane 15), then the two halves
// (row broadcast of lane 31); the total is lane 63's, returned to every lane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double wsum_dpp(double v) {
  v += dpp_move<0xb1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4e, 0xf>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_move<0x140, 0xf>(v);   // row_mirror
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, 63), hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), 63);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// A row is read as 16-byte groups: 4 float32, 8 bfloat16 (widened exactly
// to float32) or 2 float64 elements.
template <typename TA> struct Elems;
template <> struct Elems<double> {
  static constexpr int VN = 2;
  static constexpr bool F32DOT = false;
  __device__ __forceinline__ static double at(const f4& v, int e) { return __builtin_bit_cast(d2, v)[e]; }
};
template <> struct Elems<float> {
  static constexpr int VN = 4;
  static constexpr bool F32DOT = false;   // row dot products in float64
  __device__ __forceinline__ static float at(const f4& v, int e) { return v[e]; }
};
template <> struct Elems<bf16> {
  static constexpr int VN = 8;
  // per-thread dot products in float32 (as the two-product bfloat16 path
  // accumulates), then float64 across threads: halves the arithmetic per
  // element, which bounds this form; A^T w stays float64 and is exact for
  // whatever w is computed, so the recovery is unaffected
  static constexpr bool F32DOT = true;
  __device__ __forceinline__ static float at(const f4& v, int e) {
    const uint32_t b = __float_as_uint(v[e >> 1]);
    return __uint_as_float((e & 1) ? (b & 0xffff0000u) : (b << 16));
  }
};

// LDS writes complete, then the workgroup barrier.  Unlike __syncthreads()
// this does not order global memory, so the row loads in flight stay in
// flight across it (every value exchanged at these barriers is in LDS).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Word 3 of a raw buffer resource on gfx9 (32-bit data format, no swizzle).
constexpr int RSRC_WORD3 = 0x00020000;

}  // namespace fdev
}  // namespace gkb
