// Matrix-core (MFMA 16x16x4) helpers for gfx950.
//
// Operand layout of v_mfma_{f64,f32}_16x16x4 (D = A B + C, A 16x4, B 4x16):
// lane l supplies A[l%16][l/16] and B[l/16][l%16]; it receives four
// accumulator values of column l%16, at rows 4v + l/16 for FP64 (interleaved)
// and 4(l/16) + v for FP32 (blocked), v = 0..3.
#pragma once
#include <hip/hip_runtime.h>

namespace sem {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  using V4 = d4;
  __device__ static constexpr int row(int v, int g) { return 4 * v + g; }
  __device__ static V4 op(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <>
struct Mfma<float> {
  using V4 = f4;
  __device__ static constexpr int row(int v, int g) { return 4 * g + v; }
  __device__ static V4 op(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// Global-address-space views: pointers read from argument blocks or device
// descriptors are otherwise accessed through flat instructions, whose
// completion the compiler can only wait for together with LDS traffic.
#define SEM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ inline const SEM_GLOBAL T* gview(const T* p) {
  return (const SEM_GLOBAL T*)p;
}

// Workgroup barrier that orders LDS accesses only: global loads still in
// flight (prefetches) and global stores are not waited for, as they are at
// __syncthreads().  For kernels whose waves exchange data through LDS alone.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Index of the calling wavefront in its workgroup, as a wave-uniform
// (scalar) value, so that branches on it are not taken per lane.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

}  // namespace sem
