// Adding phase (paper Alg. 2) with fixed-size reservoirs (Sec. 2.4, Alg. 1),
// read as bottom-R priority sampling so that the tables do not depend on the
// order in which GPU atomics land.
//
//   count   : counts[t][m] += 1 for every (row, t); the returned old value is
//             the arrival's rank inside its bucket (Alg. 2's ReservoirCounter)
//   scan    : seg = exclusive prefix sum of counts over all L*M buckets
//   scatter : staged[seg[t][m] + rank] = row
//   select  : per bucket, the min(count, R) arrivals with the smallest
//             priority, in ascending priority, into ids[t][m][0..)
//             - buckets of <= 8 arrivals: one thread, ranks in registers
//             - larger buckets: one wave; all arrivals sorted in LDS when few,
//               else a priority threshold keeps ~2R candidates (bisected until
//               between R and the LDS capacity), which are then sorted.
// Every step is a deterministic function of the keys, so the result is
// bit-identical for any scheduling.
#include "launch.hpp"

namespace flashk {

namespace {

constexpr int kSmall = 8;          // arrivals handled by one thread
constexpr uint32_t kWaveCap = 2048; // LDS priorities per wave (16 KiB)
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kTile = kScanThreads * kScanItems;

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void insert_count_kernel(const uint32_t* __restrict__ keys, uint32_t n_elems, uint32_t L,
                                    uint32_t M, uint32_t* counts, uint32_t* __restrict__ rank) {
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n_elems; e += gridDim.x * blockDim.x) {
    const uint32_t k = keys[e];
    uint32_t r = kEmpty;
    if (k < M) r = atomicAdd(&counts[(uint64_t)(e % L) * M + k], 1u);
    rank[e] = r;
  }
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* total, uint32_t* sh /*[4]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wid) before += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  *total = tot;
  return before + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums_kernel(const uint32_t* in, uint64_t n,
                                                                      uint32_t* tile_sums) {
  __shared__ uint32_t sh[4];
  const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t tot;
  block_excl_scan(s, &tot, sh);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// One block: exclusive scan of the tile sums, in place.
__global__ __launch_bounds__(kScanThreads) void scan_tile_offsets_kernel(uint32_t* tile_sums,
                                                                         uint32_t n_tiles) {
  __shared__ uint32_t sh[4];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < n_tiles; base += kScanThreads) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < n_tiles ? tile_sums[i] : 0;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(v, &tot, sh);
    if (i < n_tiles) tile_sums[i] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(const uint32_t* in, uint64_t n,
                                                                  const uint32_t* tile_offsets,
                                                                  uint32_t* out) {
  __shared__ uint32_t sh[4];
  const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(s, &tot, sh) + tile_offsets[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

__global__ void insert_scatter_kernel(const uint32_t* __restrict__ keys,
                                      const uint32_t* __restrict__ rank, uint32_t n_elems, uint32_t L,
                                      uint32_t M, const uint32_t* __restrict__ seg,
                                      int32_t* __restrict__ staged) {
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n_elems; e += gridDim.x * blockDim.x) {
    const uint32_t r = rank[e];
    if (r == kEmpty) continue;
    const uint32_t k = keys[e];
    staged[seg[(uint64_t)(e % L) * M + k] + r] = (int32_t)(e / L);
  }
}

struct SelectArgs {
  const uint32_t* counts;
  const uint32_t* seg;
  const int32_t* staged;
  int32_t* ids;
  uint32_t* worklist;
  uint32_t* wl_len;
  uint64_t n_buckets;
  uint64_t s_p;
  uint32_t M;
  int R;
};

// Buckets with at most kSmall arrivals: rank each arrival against the others
// in registers.  Larger buckets go to the wave-level worklist.
__global__ void bucket_select_small_kernel(SelectArgs a) {
  for (uint64_t bk = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; bk < a.n_buckets;
       bk += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t n = a.counts[bk];
    if (n == 0) continue;
    if (n > (uint32_t)kSmall) {
      const uint32_t pos = atomicAdd(a.wl_len, 1u);
      a.worklist[pos] = (uint32_t)bk;
      continue;
    }
    const uint32_t t = (uint32_t)(bk / a.M);
    const uint32_t start = a.seg[bk];
    uint64_t pk[kSmall];
#pragma unroll
    for (int i = 0; i < kSmall; ++i)
      pk[i] = (uint32_t)i < n ? priority(a.s_p, t, (uint32_t)a.staged[start + i]) : ~0ull;
#pragma unroll
    for (int i = 0; i < kSmall; ++i) {
      if ((uint32_t)i >= n) break;
      int r = 0;
#pragma unroll
      for (int j = 0; j < kSmall; ++j) r += pk[j] < pk[i];
      if (r < a.R) a.ids[bk * (uint64_t)a.R + r] = (int32_t)(uint32_t)pk[i];
    }
  }
}

// One wave per worklist bucket.
__global__ __launch_bounds__(64) void bucket_select_wave_kernel(SelectArgs a) {
  __shared__ uint64_t buf[kWaveCap];
  __shared__ uint32_t cnt_sh;
  const uint32_t lane = threadIdx.x;
  const uint32_t len = *a.wl_len;
  const uint32_t R = (uint32_t)a.R;
  const uint32_t sort_all = (2 * R > 256u ? 2 * R : 256u) < kWaveCap ? (2 * R > 256u ? 2 * R : 256u)
                                                                       : kWaveCap;
  for (uint32_t w = blockIdx.x; w < len; w += gridDim.x) {
    const uint32_t bk = a.worklist[w];
    const uint32_t n = a.counts[bk];
    const uint32_t t = bk / a.M;
    const uint32_t start = a.seg[bk];
    const int32_t* src = a.staged + start;
    uint32_t c;
    if (n <= sort_all) {
      c = n;
      for (uint32_t i = lane; i < n; i += kWave) buf[i] = priority(a.s_p, t, (uint32_t)src[i]);
    } else {
      // keep priorities whose top 32 bits are below thr; aim for
      // min(2R, (R + cap) / 2) of them, bisect until R <= kept <= cap
      const uint64_t target = (2 * R < (R + kWaveCap) / 2) ? 2 * R : (R + kWaveCap) / 2;
      uint64_t lo = 0, hi = 1ull << 32;
      bool hi_known = false;
      uint64_t thr = (target << 32) / n + 1;
      if (thr > hi) thr = hi;
      for (int iter = 0; iter < 96; ++iter) {
        if (lane == 0) cnt_sh = 0;
        __syncthreads();
        for (uint32_t i = lane; i < n; i += kWave) {
          const uint64_t pk = priority(a.s_p, t, (uint32_t)src[i]);
          if ((pk >> 32) < thr) {
            const uint32_t pos = atomicAdd(&cnt_sh, 1u);
            if (pos < kWaveCap) buf[pos] = pk;
          }
        }
        __syncthreads();
        c = cnt_sh;
        __syncthreads();
        if (c >= R && c <= kWaveCap) break;
        if (c < R) {
          lo = thr;
          thr = hi_known ? (lo + hi + 1) / 2 : (thr * 2 < (1ull << 32) ? thr * 2 : (1ull << 32));
        } else {
          hi = thr;
          hi_known = true;
          thr = (lo + hi) / 2;
        }
        if (c > kWaveCap) c = kWaveCap;  // only reached if the loop ends without success
      }
    }
    const uint32_t P = pow2_ceil(c);
    for (uint32_t i = c + lane; i < P; i += kWave) buf[i] = ~0ull;
    __syncthreads();
    block64_bitonic_sort(buf, P);
    const uint32_t keep = n < R ? n : R;
    for (uint32_t i = lane; i < keep; i += kWave)
      a.ids[(uint64_t)bk * R + i] = (int32_t)(uint32_t)buf[i];
    __syncthreads();
  }
}

int grid_for(uint64_t n, int threads, int per_cu) {
  const uint64_t want = (uint64_t)device_info().cus * per_cu;
  const uint64_t need = (n + threads - 1) / threads;
  return (int)(need < want ? (need ? need : 1) : want);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256, 8)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

size_t insert_ws_bytes(const Cfg& c, int64_t n_rows) {
  const uint64_t ne = (uint64_t)n_rows * c.L, nb = (uint64_t)c.L * c.M;
  const uint64_t tiles = (nb + kTile - 1) / kTile;
  return align256(4 * ne) * 2 + align256(4 * nb) * 2 + align256(4 * (tiles + 1)) + align256(4);
}

InsertWs insert_ws_carve(const Cfg& c, int64_t n_rows, void* ws) {
  const uint64_t ne = (uint64_t)n_rows * c.L, nb = (uint64_t)c.L * c.M;
  const uint64_t tiles = (nb + kTile - 1) / kTile;
  char* p = (char*)ws;
  InsertWs w;
  w.rank = (uint32_t*)p;
  p += align256(4 * ne);
  w.staged = (int32_t*)p;
  p += align256(4 * ne);
  w.seg = (uint32_t*)p;
  p += align256(4 * nb);
  w.worklist = (uint32_t*)p;
  p += align256(4 * nb);
  w.tile_sums = (uint32_t*)p;
  p += align256(4 * (tiles + 1));
  w.wl_len = (uint32_t*)p;
  return w;
}

hipError_t launch_insert(const Cfg& c, int64_t n_rows, const uint32_t* keys, uint32_t* counts,
                         int32_t* ids, const InsertWs& w, hipStream_t s) {
  const uint64_t nb = (uint64_t)c.L * c.M;
  const uint32_t ne = (uint32_t)((uint64_t)n_rows * c.L);
  hipError_t e;
  // initialisation: clear the counters (the reservoirs need no clearing)
  if ((e = launch_fill_u32(counts, nb, 0u, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(w.wl_len, 1, 0u, s)) != hipSuccess) return e;
  if (ne == 0) return hipSuccess;
  hipLaunchKernelGGL(insert_count_kernel, dim3(grid_for(ne, 256, 16)), dim3(256), 0, s, keys, ne,
                     (uint32_t)c.L, c.M, counts, w.rank);
  const uint32_t tiles = (uint32_t)((nb + kTile - 1) / kTile);
  hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(tiles), dim3(kScanThreads), 0, s, counts, nb,
                     w.tile_sums);
  hipLaunchKernelGGL(scan_tile_offsets_kernel, dim3(1), dim3(kScanThreads), 0, s, w.tile_sums,
                     tiles);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(tiles), dim3(kScanThreads), 0, s, counts, nb,
                     w.tile_sums, w.seg);
  hipLaunchKernelGGL(insert_scatter_kernel, dim3(grid_for(ne, 256, 16)), dim3(256), 0, s, keys,
                     w.rank, ne, (uint32_t)c.L, c.M, w.seg, w.staged);
  SelectArgs a;
  a.counts = counts;
  a.seg = w.seg;
  a.staged = w.staged;
  a.ids = ids;
  a.worklist = w.worklist;
  a.wl_len = w.wl_len;
  a.n_buckets = nb;
  a.s_p = c.seeds.s_p;
  a.M = c.M;
  a.R = c.R;
  hipLaunchKernelGGL(bucket_select_small_kernel, dim3(grid_for(nb, 256, 16)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(bucket_select_wave_kernel, dim3(device_info().cus * 16), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace flashk
