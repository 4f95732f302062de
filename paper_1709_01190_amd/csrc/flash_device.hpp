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

// The same finaliser, callable on the host too.
__host__ __device__ __forceinline__ uint32_t fmix32_hd(uint32_t h) {
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
  uint32_t s_r;  // bucket -> shared reservoir map
};

// One user seed -> four seeds: the first four outputs of the splitmix64
// sequence started at `seed`.
inline Seeds expand_seed(uint64_t seed) {
  const uint64_t g = 0x9E3779B97F4A7C15ull;
  Seeds s;
  s.s_h = (uint32_t)splitmix_out(seed + g);
  s.s_d = (uint32_t)splitmix_out(seed + 2 * g);
  s.s_p = splitmix_out(seed + 3 * g);
  s.s_r = (uint32_t)splitmix_out(seed + 4 * g);
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

// Cross-lane primitives on DPP (row_shr / row_bcast, GFX9 encodings) and
// ds_swizzle, so that scans and exchanges need no LDS address arithmetic.
// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false); // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false); // row_bcast:31
  return v;
}

// Inclusive prefix maximum across the wave (values are unsigned; 0 is the identity).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
  uint32_t o;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);
  v = v > o ? v : o;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);
  v = v > o ? v : o;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
  v = v > o ? v : o;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
  v = v > o ? v : o;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v = v > o ? v : o;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  v = v > o ? v : o;
  return v;
}

// Sum over the wave, the same in every lane.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

// Value of lane (lane ^ j) for a power of two j < 64 (j folds to a constant
// after unrolling): quad permutes for 1 and 2, swizzles up to 16, bpermute for 32.
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, uint32_t j) {
  switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);
    case 4: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (4 << 10) | 0x1f);
    case 8: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (8 << 10) | 0x1f);
    case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (16 << 10) | 0x1f);
    default: return (uint32_t)__shfl_xor((int)v, (int)j, kWave);
  }
}

__device__ __forceinline__ uint64_t xor_lane64(uint64_t v, uint32_t j) {
  return ((uint64_t)xor_lane((uint32_t)(v >> 32), j) << 32) | xor_lane((uint32_t)v, j);
}

}  // namespace flashk
