// Elementary functions called by the generated element code, for T = float
// and T = double (device only).
#pragma once

#include <hip/hip_runtime.h>

__device__ __forceinline__ float sx_log(float a) { return logf(a); }
__device__ __forceinline__ double sx_log(double a) { return log(a); }
__device__ __forceinline__ float sx_sqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double sx_sqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float sx_abs(float a) { return fabsf(a); }
__device__ __forceinline__ double sx_abs(double a) { return fabs(a); }

template <int N, typename T>
__device__ __forceinline__ T sx_pown(T a) {
  T r = a;
#pragma unroll
  for (int k = 1; k < N; ++k) r *= a;
  return r;
}
