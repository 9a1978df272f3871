// Small gfx950 device helpers shared by the kernels (wave64 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pulsar {

// Hardware transcendental approximations (about 1 ulp on normal inputs).
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Workgroups are dispatched to the chip's 8 XCDs (each with its own L2) in
// round-robin order. xcd_block maps dispatched block b of nb active blocks to
// a logical block such that each XCD gets one contiguous run of logical
// blocks: neighbouring logical blocks, which share cache lines of their
// inputs and outputs, then meet in the same L2. A bijection on [0, nb).
constexpr uint32_t kXcds = 8;

// s_waitcnt operand (gfx9 encoding) that waits for every outstanding vector
// memory operation, global-to-LDS loads included, and nothing else.
constexpr int kWaitVmem0 = 0x0F70;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t x = b % kXcds, s = b / kXcds;
  const uint32_t q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + s;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Inclusive prefix sum across the 64 lanes.
__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    unsigned long long o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

// Scene of element x: the largest b in [0, B) with start[b] <= x, for an
// ascending start array with start[0] = 0 (empty scenes are skipped because
// a later scene with the same start wins).
__device__ __forceinline__ int find_scene(const uint32_t* __restrict__ start, int B, uint32_t x) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
  return (uint64_t(1) << lane) - 1u;
}

}  // namespace pulsar
