// Device helpers shared by the MI355X kernels (wave64, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MM_WAVE 64

namespace mm {

// ---------------------------------------------------------------- SplitMix64
// Counter form of SplitMix64 (Steele, Lea, Flood 2014): output number i of the
// generator started at `state` is mix(state + (i + 1) * golden_gamma).
__host__ __device__ inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm64_at(uint64_t state, uint64_t i) {
  return sm64_mix(state + (i + 1) * 0x9E3779B97F4A7C15ull);
}
// Stream selection: seed ^ (level << 48) ^ (tag << 32).
__host__ __device__ inline uint64_t rng_stream(uint64_t seed, uint32_t level, uint32_t tag) {
  return seed ^ ((uint64_t)level << 48) ^ ((uint64_t)tag << 32);
}
// Top 24 bits as a unit draw in [0, 1); exact in FP32 and FP64.
__host__ __device__ inline double unit24(uint64_t r) { return (double)(r >> 40) * 0x1p-24; }

enum RngTag : uint32_t { TAG_INIT = 1, TAG_PROLONG = 2, TAG_LP = 16 };

// ---------------------------------------------------------------- wave ops
__device__ inline int lane_id() { return __lane_id(); }

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ inline T group_sum(T v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}
template <typename T>
__device__ inline T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
// Inclusive prefix sum over the wave.
template <typename T>
__device__ inline T wave_incl_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T w = __shfl_up(v, o, 64);
    if (l >= o) v += w;
  }
  return v;
}
// int32: the same inclusive sum from DPP row shifts (1, 2, 4, 8 within rows
// of 16 lanes) and row broadcasts (lane 15 into rows 1 and 3, lane 31 into
// rows 2 and 3): VALU data movement instead of six LDS-crossbar shuffles.
// Lanes whose source lies outside their row keep the identity 0.
template <>
__device__ inline int32_t wave_incl_scan<int32_t>(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}
// Minimum over the wave (int32, every lane active): DPP min-scan as above
// (identity INT32_MAX), then lane 63's value, uniform across the wave.
template <>
__device__ inline int32_t wave_min<int32_t>(int32_t v) {
  constexpr int32_t hi = 0x7fffffff;
  v = min(v, __builtin_amdgcn_update_dpp(hi, v, 0x111, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(hi, v, 0x112, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(hi, v, 0x114, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(hi, v, 0x118, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(hi, v, 0x142, 0xa, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(hi, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}
// Inclusive max over the wave (int32, DPP as above; identity INT32_MIN).
__device__ inline int32_t wave_incl_max(int32_t v) {
  constexpr int32_t lo = -2147483647 - 1;
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x111, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x112, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x114, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x118, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x142, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x143, 0xc, 0xf, false));
  return v;
}
// Issue priority of the calling wave above the default.  The far-field
// kernels run beside the sweep kernel on a second stream; the sweep keeps
// every SIMD's vector unit busy, so at default priority the far field's
// waves, and with them its chain of short dependent kernels, would advance
// only in the sweep's idle cycles.
__device__ inline void raise_wave_priority() { __builtin_amdgcn_s_setprio(3); }

__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Exclusive block scan (blockDim multiple of 64, <= 1024). Returns the
// exclusive prefix of v; *total receives the block sum. `sh` needs
// blockDim/64 + 1 entries.
template <typename T>
__device__ inline T block_excl_scan(T v, T* sh, T* total) {
  const int l = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T inc = wave_incl_scan(v);
  if (l == 63) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int i = 0; i < nw; ++i) { T t = sh[i]; sh[i] = run; run += t; }
    sh[nw] = run;
  }
  __syncthreads();
  T res = sh[w] + inc - v;
  *total = sh[nw];
  __syncthreads();
  return res;
}

}  // namespace mm
