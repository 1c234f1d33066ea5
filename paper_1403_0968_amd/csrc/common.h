// Device helpers shared by the HIP kernels of libsem.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sem {

// bfloat16 stored as uint16_t: the upper half of an IEEE float
__device__ __host__ inline float bf16_to_f32(uint16_t h) {
  union {
    uint32_t u;
    float f;
  } c;
  c.u = (uint32_t)h << 16;
  return c.f;
}
// round to nearest even (finite inputs)
__device__ __host__ inline uint16_t f32_to_bf16(float f) {
  union {
    uint32_t u;
    float f;
  } c;
  c.f = f;
  uint32_t u = c.u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <class TS, class TC> struct Cvt;
template <> struct Cvt<double, double> {
  __device__ static double ld(double v) { return v; }
};
template <> struct Cvt<float, float> {
  __device__ static float ld(float v) { return v; }
};
template <> struct Cvt<uint16_t, float> {
  __device__ static float ld(uint16_t v) { return bf16_to_f32(v); }
};
template <> struct Cvt<float, double> {
  __device__ static double ld(float v) { return (double)v; }
};
template <> struct Cvt<double, float> {
  __device__ static float ld(double v) { return (float)v; }
};

// Global-memory pointer.  A pointer read from device memory (a work item's
// or a solve's descriptor) has no known address space, and loads and stores
// through it compile to FLAT instructions, which wait on both memory
// counters and keep fewer loads in flight; kernels whose buffers are global
// memory (all device buffers here) access them through gp pointers.
template <class T> using gp = T __attribute__((address_space(1))) *;

// orders a wave's LDS writes before its later LDS reads of other lanes'
// entries: the lanes of a wave execute together and a wave's LDS
// operations complete in issue order, so only the compiler has to be kept
// from moving accesses across this point (for LDS regions that one wave
// owns; a workgroup barrier would also wait for the other waves)
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// wave64 sum in a fixed order (butterfly over lanes), deterministic
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block sum, deterministic for a fixed block size; result valid in thread 0
template <int THREADS>
__device__ inline double block_sum(double v, double *smem /* THREADS/64 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < THREADS / 64; ++q) s += smem[q];
  }
  __syncthreads();
  return s;
}

}  // namespace sem
