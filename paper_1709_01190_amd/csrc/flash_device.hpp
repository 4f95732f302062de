// Device-side building blocks of the FLASH kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flashk {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kWave = 64;

// MurmurHash3's 32-bit finaliser: the column permutation pi of Eq. 1
// (applied to col ^ s_h) and the densification probe hash.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// splitmix64 output function: seed expansion and reservoir priorities.
__host__ __device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Seeds {
  uint32_t s_h;  // column permutation
  uint32_t s_d;  // densification probes
  uint64_t s_p;  // reservoir priorities
};

// One user seed -> three seeds: the first three outputs of the splitmix64
// sequence started at `seed`.
inline Seeds expand_seed(uint64_t seed) {
  const uint64_t g = 0x9E3779B97F4A7C15ull;
  Seeds s;
  s.s_h = (uint32_t)splitmix_out(seed + g);
  s.s_d = (uint32_t)splitmix_out(seed + 2 * g);
  s.s_p = splitmix_out(seed + 3 * g);
  return s;
}

// Reservoir priority of row `id` in table `t`: 32 pseudo-random bits above the
// id, so priorities are distinct and their order is a uniform random order.
__device__ __forceinline__ uint64_t priority(uint64_t s_p, uint32_t t, uint32_t id) {
  const uint64_t x = splitmix_out(s_p ^ (((uint64_t)t << 32) | (uint64_t)id));
  return (x & 0xFFFFFFFF00000000ull) | (uint64_t)id;
}

__device__ __forceinline__ uint32_t pow2_ceil(uint32_t x) {
  return x <= 1 ? 1u : 1u << (32 - __clz(x - 1));
}

// Ascending bitonic sort of buf[0, P) (P a power of two) by one 64-thread
// block.  Each compare-exchange pair (i, i ^ j) is owned by its lower index,
// so pairs of one step are disjoint.
__device__ inline void block64_bitonic_sort(uint64_t* buf, uint32_t P) {
  const uint32_t lane = threadIdx.x;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = lane; i < P; i += kWave) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = buf[i], b = buf[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            buf[i] = b;
            buf[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

}  // namespace flashk
