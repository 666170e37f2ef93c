// Device helpers shared by the HIP kernels of the logm library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace logm {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// One CDNA matrix-core step: D(16x16) += A(16x4) * B(4x16) in fp64.
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; lane l receives
// D[4 * r + l / 16][l % 16] in element r of the result.
__device__ __forceinline__ f64x4 mfma_f64_16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

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

}  // namespace logm
