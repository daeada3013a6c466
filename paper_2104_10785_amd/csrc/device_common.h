// Device helpers shared by the kernel sources: accumulation types, 16-byte
// packs of the matrix element types, streaming loads and fixed-order
// wave/block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gemv.h"

namespace gkb {

static inline unsigned nblocks(int64_t work, int64_t per) { return (unsigned)((work + per - 1) / per); }

// ---------------------------------------------------------------- types
template <typename TA> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = float; };
template <> struct Acc<bf16> { using type = float; };

__device__ __forceinline__ double to_acc(double x) { return x; }
__device__ __forceinline__ float to_acc(float x) { return x; }
__device__ __forceinline__ float to_acc(bf16 x) { return __uint_as_float(((uint32_t)x.bits) << 16); }

// Unpack a 16-byte load into VN accumulator values.
template <typename TA> struct Pack;
template <> struct Pack<double> {
  static constexpr int VN = 2;
  __device__ __forceinline__ static void unpack(const uint4& u, double* o) {
    o[0] = __hiloint2double((int)u.y, (int)u.x);
    o[1] = __hiloint2double((int)u.w, (int)u.z);
  }
};
template <> struct Pack<float> {
  static constexpr int VN = 4;
  __device__ __forceinline__ static void unpack(const uint4& u, float* o) {
    o[0] = __uint_as_float(u.x);
    o[1] = __uint_as_float(u.y);
    o[2] = __uint_as_float(u.z);
    o[3] = __uint_as_float(u.w);
  }
};
template <> struct Pack<bf16> {
  static constexpr int VN = 8;
  __device__ __forceinline__ static void unpack(const uint4& u, float* o) {
    o[0] = __uint_as_float(u.x << 16);
    o[1] = __uint_as_float(u.x & 0xffff0000u);
    o[2] = __uint_as_float(u.y << 16);
    o[3] = __uint_as_float(u.y & 0xffff0000u);
    o[4] = __uint_as_float(u.z << 16);
    o[5] = __uint_as_float(u.z & 0xffff0000u);
    o[6] = __uint_as_float(u.w << 16);
    o[7] = __uint_as_float(u.w & 0xffff0000u);
  }
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_stream(const void* p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

// n consecutive basis values from a 16-byte aligned address, as the
// accumulator type (zeros when !ok).
template <typename TB, int VN, typename ACC>
__device__ __forceinline__ void load_vec(const TB* ptr, bool ok, ACC* out) {
  if constexpr ((VN * sizeof(TB)) % 16 == 0) {
    constexpr int NQ = VN * sizeof(TB) / 16;
    uint4 raw[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) raw[i] = ok ? reinterpret_cast<const uint4*>(ptr)[i] : make_uint4(0, 0, 0, 0);
    const TB* vals = reinterpret_cast<const TB*>(raw);
#pragma unroll
    for (int e = 0; e < VN; ++e) out[e] = (ACC)vals[e];
  } else {
#pragma unroll
    for (int e = 0; e < VN; ++e) out[e] = ok ? (ACC)ptr[e] : (ACC)0;
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block (256 threads) sum in a fixed order; result valid in every thread.
__device__ __forceinline__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = (red[0] + red[1]) + (red[2] + red[3]);
  return t;
}

// The normalisation step's norm and tests.  The norm is the square root of
// the sum of nparts partial sums of squares, added in a fixed order by the
// 256 threads, so every workgroup obtains the same value and takes the same
// branch.  A NaN or Inf norm sets flag = {3, index}; a norm <= thr (thr =
// eps * sig_in[0] when relative, else eps) is a breakdown: flag = {code,
// index}, sig_out = sig_in.  Otherwise sig_out = max(sig_in, norm) (sig_in
// when !track).  The lead thread writes coef_out, sig_out and flag.  Returns
// the norm when the vector is to be scaled, else -1; *sig_new (if given)
// receives the value written to sig_out.
__device__ __forceinline__ double norm_test(const double* __restrict__ normpart, int nparts,
                                            const double* __restrict__ sig_in, double* __restrict__ sig_out,
                                            double eps, int relative, int track, int* __restrict__ flag, int code,
                                            int index, double* __restrict__ coef_out, bool lead, double* red,
                                            double* sig_new = nullptr) {
  double s = 0.0;
  for (int p = threadIdx.x; p < nparts; p += 256) s += normpart[p];
  const double tot = block_sum256(s, red);
  const double nrm = sqrt(tot);
  const double sin = *sig_in;
  const double thr = relative ? eps * sin : eps;
  if (!(nrm < INFINITY)) {  // NaN or Inf
    if (lead) {
      flag[0] = 3;
      flag[1] = index;
      *coef_out = nrm;
    }
    return -1.0;
  }
  if (nrm <= thr) {
    if (lead) {
      flag[0] = code;
      flag[1] = index;
      *coef_out = nrm;
      *sig_out = sin;
    }
    return -1.0;
  }
  const double so = track ? fmax(sin, nrm) : sin;
  if (lead) {
    *coef_out = nrm;
    *sig_out = so;
  }
  if (sig_new != nullptr) *sig_new = so;
  return nrm;
}

}  // namespace gkb
