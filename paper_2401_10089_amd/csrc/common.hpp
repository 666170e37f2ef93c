// Device helpers shared by the HIP kernels of the logm library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace logm {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One CDNA matrix-core step: D(16x16) += A(16x4) * B(4x16) in fp64.
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; lane l receives
// D[4 * r + l / 16][l % 16] in element r of the result.
__device__ __forceinline__ f64x4 mfma_f64_16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The fp32 matrix-core step of the same 16 x 16 x 4 shape: same operand layout,
// but lane l receives D[4 * (l / 16) + r][l % 16] in element r.
__device__ __forceinline__ f32x4 mfma_f32_16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma_16x16x4(double a, double b, f64x4 c) { return mfma_f64_16x16x4(a, b, c); }
__device__ __forceinline__ f32x4 mfma_16x16x4(float a, float b, f32x4 c) { return mfma_f32_16x16x4(a, b, c); }

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Wave-wide sum (64 lanes), every lane gets the result.  Fixed butterfly order,
// so the result is reproducible run to run.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Wave-wide argmax of v (>= 0 or -1 for "no candidate"), ties to the smallest
// index.  Every lane gets (value, index).
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    double ov = __shfl_xor(v, off, 64);
    int oi = __shfl_xor(idx, off, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// One DPP row/bank-masked move of a double (two 32-bit halves).  Lanes whose
// source is outside the row or masked off keep `old`.
template <int CTRL, int ROWMASK, int BANKMASK>
__device__ __forceinline__ double dpp_double(double old, double src) {
  const long long o = __double_as_longlong(old);
  const long long s = __double_as_longlong(src);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, CTRL, ROWMASK, BANKMASK, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), CTRL, ROWMASK, BANKMASK, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide maximum of v using DPP row shifts and row broadcasts (gfx9 family);
// the full maximum lands in lane 63 and is returned to every lane.
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_double<0x111, 0xf, 0xf>(v, v));  // row_shr:1
  v = fmax(v, dpp_double<0x112, 0xf, 0xf>(v, v));  // row_shr:2
  v = fmax(v, dpp_double<0x113, 0xf, 0xf>(v, v));  // row_shr:3
  v = fmax(v, dpp_double<0x114, 0xf, 0xe>(v, v));  // row_shr:4, banks 1-3
  v = fmax(v, dpp_double<0x118, 0xf, 0xc>(v, v));  // row_shr:8, banks 2-3
  v = fmax(v, dpp_double<0x142, 0xa, 0xf>(v, v));  // row_bcast:15, rows 1 and 3
  v = fmax(v, dpp_double<0x143, 0xc, 0xf>(v, v));  // row_bcast:31, rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}


// Lane `lane` (wave-uniform) of a double, as a uniform value.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide maximum of an unsigned key (DPP row shifts and broadcasts, the full
// maximum lands in lane 63), returned to every lane.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x113, 0xf, 0xf, false));  // row_shr:3
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xe, false));  // row_shr:4
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xc, false));  // row_shr:8
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Reciprocal for the multipliers: hardware estimate and two Newton steps (within
// an ulp or so of 1/a); 0 for a zero pivot, whose singularity the root reports.
__device__ __forceinline__ double pivot_recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  return (a != 0.0) ? r : 0.0;
}

}  // namespace logm
