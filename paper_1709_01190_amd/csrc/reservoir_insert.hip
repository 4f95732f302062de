// Adding phase (paper Alg. 2) with fixed-size reservoirs (Sec. 2.4, Alg. 1),
// read as bottom-R priority sampling so that the tables do not depend on the
// order in which arrivals are processed.
//
// A counting sort of the (table, key) arrivals, privatised in LDS so that no
// global atomics are needed:
//   transpose : keys[N][L] -> keysT[L][Np] (table-major, rows padded to 64)
//   count     : block (t, chunk, slice) histograms the keys of table t that
//               fall in its chunk of CH buckets, over its slice of rows, in
//               LDS; part[(t*M + m) * S + slice] = that count
//   scan      : partoff = exclusive prefix sum of part (bucket-major, slice
//               minor), so every (bucket, slice) owns a run of `staged`
//   totals    : counts[t][m] = sum over slices (Alg. 2's ReservoirCounter),
//               seg[t][m] = first staged slot of the bucket
//   scatter   : the same blocks place each arrival's row id at an LDS cursor
//   select    : per bucket, the min(count, R) arrivals with the smallest
//               priority, in ascending priority, into ids[t][m][0..)
//               - buckets of <= 8 arrivals: one thread, ranks in registers
//               - 9..64 arrivals: the wave of the bucket's thread, one arrival
//                 per lane, a bitonic sort across the lanes in registers
//               - 65..256 arrivals: one wave per bucket, two or four arrivals
//                 per lane, a bitonic sort in registers (no LDS)
//               - larger buckets: one wave; all arrivals sorted in LDS when few,
//                 else a priority threshold keeps ~2R candidates (bisected until
//                 between R and the LDS capacity), which are then sorted.
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

__global__ void fill_strided_u32_kernel(uint32_t* p, uint64_t n, uint32_t stride, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i * stride] = v;
}

constexpr uint32_t kChunk = 16384;  // buckets per LDS histogram (64 KiB)
constexpr int kPartThreads = 512;
constexpr int kPartUnroll = 4;

// With shared reservoirs each key is replaced by its reservoir (keys >= M,
// the empty key included, stay empty).
struct ShareMap {
  int shared;
  uint32_t s_r, M;
  uint64_t P;
};

__device__ __forceinline__ uint32_t shared_reservoir(const ShareMap& sm, uint32_t t, uint32_t key) {
  if (key == kEmpty || key >= sm.M) return kEmpty;
  return (uint32_t)reservoir_of(true, sm.s_r, sm.P, sm.M, t, key);
}

// Table-major copy of the keys.  With shared reservoirs each key becomes its
// reservoir, and a row that reaches one reservoir from several tables keeps
// only the first such table's entry (the others become empty): a reservoir
// then sees every row at most once.
__global__ __launch_bounds__(256) void keys_transpose_kernel(const uint32_t* __restrict__ keys, uint32_t n,
                                                             uint32_t L, uint32_t np,
                                                             uint32_t* __restrict__ keys_t, ShareMap sm) {
  __shared__ uint32_t tile[64][65];
  const uint32_t row0 = blockIdx.x * 64, t0 = blockIdx.y * 64;
  for (uint32_t i = threadIdx.x; i < 64 * 64; i += 256) {
    const uint32_t r = i >> 6, c = i & 63, row = row0 + r, t = t0 + c;
    uint32_t key = (row < n && t < L) ? keys[(uint64_t)row * L + t] : kEmpty;
    if (sm.shared) key = shared_reservoir(sm, t, key);
    tile[r][c] = key;
  }
  if (sm.shared) {
    __syncthreads();
    // earlier tables of the same row: inside this tile from LDS, before it
    // (t0 > 0) recomputed from the keys
    uint32_t keep[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t i = threadIdx.x + 256u * (uint32_t)e;
      const uint32_t r = i >> 6, c = i & 63, row = row0 + r;
      uint32_t v = tile[r][c];
      if (v != kEmpty) {
        for (uint32_t c2 = 0; c2 < c; ++c2)
          if (tile[r][c2] == v) v = kEmpty;
        if (v != kEmpty && row < n)
          for (uint32_t t2 = 0; t2 < t0; ++t2)
            if (shared_reservoir(sm, t2, keys[(uint64_t)row * L + t2]) == v) v = kEmpty;
      }
      keep[e] = v;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t i = threadIdx.x + 256u * (uint32_t)e;
      tile[i >> 6][i & 63] = keep[e];
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < 64 * 64; i += 256) {
    const uint32_t c = i >> 6, r = i & 63, row = row0 + r, t = t0 + c;
    if (t < L && row < np) keys_t[(uint64_t)t * np + row] = tile[r][c];
  }
}

struct PartArgs {
  const uint32_t* keys_t;  // [L][np]
  uint32_t* part;          // [L * M * S]
  const uint32_t* partoff; // [L * M * S]
  int32_t* staged;
  uint32_t np, M, ch, n_chunks, n_slices, slice_vecs;
  uint32_t id_base;        // id of row 0 of this batch
  uint32_t row_mod;        // shared reservoirs: the L key rows are one row of
                           // L * row_mod entries, and entry e is row e % row_mod
};

// Buckets of the chunk starting at bucket lo: ch, or fewer in the last chunk
// when the partition's bucket count (a shared pool) is not a multiple of ch.
__device__ __forceinline__ uint32_t chunk_len(const PartArgs& a, uint32_t lo) {
  return a.M - lo < a.ch ? a.M - lo : a.ch;
}

// Workgroups go to the 8 XCDs round-robin by blockIdx.x.  This bijection
// renumbers them so that consecutive logical blocks run on one XCD: the
// slices of one (table, chunk) then write their interleaved runs of `staged`
// through the same L2, where the partial lines merge.
__device__ __forceinline__ uint32_t xcd_local_block(uint32_t p, uint32_t g) {
  const uint32_t x = p & 7, q = g >> 3, r = g & 7;
  return x * q + (x < r ? x : r) + (p >> 3);
}

// Block (t, chunk, slice): histogram of the keys of table t inside the chunk,
// over the slice's rows, in LDS.
__global__ __launch_bounds__(kPartThreads) void part_count_kernel(PartArgs a) {
  extern __shared__ uint32_t h[];
  const uint32_t lb = xcd_local_block(blockIdx.x, gridDim.x);
  const uint32_t sl = lb % a.n_slices;
  const uint32_t ck = (lb / a.n_slices) % a.n_chunks;
  const uint32_t t = lb / (a.n_slices * a.n_chunks);
  const uint32_t lo = ck * a.ch;
  const uint32_t cl = chunk_len(a, lo);
  for (uint32_t j = threadIdx.x; j < cl; j += kPartThreads) h[j] = 0;
  __syncthreads();
  const uint4* rowv = reinterpret_cast<const uint4*>(a.keys_t + (uint64_t)t * a.np);
  const uint32_t v0 = sl * a.slice_vecs;
  uint32_t v1 = v0 + a.slice_vecs;
  if (v1 > a.np / 4) v1 = a.np / 4;
  // kPartUnroll 16-byte loads per thread are in flight before their keys are
  // counted (one workgroup per CU: the loads' latency is hidden by the
  // thread's own later loads, not by other waves)
  for (uint32_t vb = v0 + threadIdx.x; vb < v1; vb += kPartUnroll * kPartThreads) {
    uint4 x[kPartUnroll];
#pragma unroll
    for (int u = 0; u < kPartUnroll; ++u) {
      const uint32_t v = vb + (uint32_t)u * kPartThreads;
      x[u] = v < v1 ? rowv[v] : make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
    }
#pragma unroll
    for (int u = 0; u < kPartUnroll; ++u) {
      const uint32_t d0 = x[u].x - lo, d1 = x[u].y - lo, d2 = x[u].z - lo, d3 = x[u].w - lo;
      if (d0 < cl) atomicAdd(&h[d0], 1u);
      if (d1 < cl) atomicAdd(&h[d1], 1u);
      if (d2 < cl) atomicAdd(&h[d2], 1u);
      if (d3 < cl) atomicAdd(&h[d3], 1u);
    }
  }
  __syncthreads();
  const uint64_t b0 = (uint64_t)t * a.M + lo;
  for (uint32_t j = threadIdx.x; j < cl; j += kPartThreads)
    a.part[(b0 + j) * a.n_slices + sl] = h[j];
}

// Same blocks: each arrival's row id goes to the next free slot of its
// (bucket, slice) run; LDS cursors start at partoff.
__global__ __launch_bounds__(kPartThreads) void part_scatter_kernel(PartArgs a) {
  extern __shared__ uint32_t cur[];
  const uint32_t lb = xcd_local_block(blockIdx.x, gridDim.x);
  const uint32_t sl = lb % a.n_slices;
  const uint32_t ck = (lb / a.n_slices) % a.n_chunks;
  const uint32_t t = lb / (a.n_slices * a.n_chunks);
  const uint32_t lo = ck * a.ch;
  const uint32_t cl = chunk_len(a, lo);
  const uint64_t b0 = (uint64_t)t * a.M + lo;
  for (uint32_t j = threadIdx.x; j < cl; j += kPartThreads)
    cur[j] = a.partoff[(b0 + j) * a.n_slices + sl];
  __syncthreads();
  const uint4* rowv = reinterpret_cast<const uint4*>(a.keys_t + (uint64_t)t * a.np);
  const uint32_t v0 = sl * a.slice_vecs;
  uint32_t v1 = v0 + a.slice_vecs;
  if (v1 > a.np / 4) v1 = a.np / 4;
  for (uint32_t vb = v0 + threadIdx.x; vb < v1; vb += kPartUnroll * kPartThreads) {
    uint4 x[kPartUnroll];
#pragma unroll
    for (int u = 0; u < kPartUnroll; ++u) {
      const uint32_t v = vb + (uint32_t)u * kPartThreads;
      x[u] = v < v1 ? rowv[v] : make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
    }
#pragma unroll
    for (int u = 0; u < kPartUnroll; ++u) {
      const uint32_t v = vb + (uint32_t)u * kPartThreads;
      const uint32_t kk[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
      const uint32_t row0 = a.row_mod ? (4 * v) % a.row_mod : 4 * v;  // row_mod is a multiple of 64
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t d = kk[j] - lo;
        if (d < cl) a.staged[atomicAdd(&cur[d], 1u)] = (int32_t)(a.id_base + row0 + (uint32_t)j);
      }
    }
  }
}

// newcnt[b] = the batch's arrivals in bucket b (sum over its slices), seg[b]
// = their first staged slot.
__global__ void bucket_totals_kernel(const uint32_t* part, const uint32_t* partoff, uint64_t nb,
                                     uint32_t n_slices, uint32_t* newcnt, uint32_t* seg) {
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
       b += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t c = 0;
    for (uint32_t s = 0; s < n_slices; ++s) c += part[b * n_slices + s];
    newcnt[b] = c;
    seg[b] = partoff[b * n_slices];
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

struct SelectArgs {
  int32_t* index;          // reservoir b: count at index[b * S] (in when appending, and out),
                           // slot i at index[b * S + kSlot0 + i]
  uint32_t S;
  const uint32_t* newcnt;  // the batch's arrivals per bucket
  const uint32_t* seg;     // their first staged slot
  const int32_t* staged;
  uint4* work;          // [nb] {bucket, first staged slot, candidates, old slots}
                        // of the large buckets, from the back
  uint32_t* wl_len;     // [2] buckets listed: [0] mid-size (from the front of
                        // `work`), [1] large (from the back)
  uint64_t n_buckets;
  uint64_t s_p;
  uint32_t M;
  int R;
  int append;           // 1: merge with the reservoirs already in the index
};

// Candidate i of bucket bk: its first `occ` are the ids already in the
// reservoir (appending), the rest the batch's arrivals.
__device__ __forceinline__ uint32_t candidate(const SelectArgs& a, uint64_t bk, uint32_t start, uint32_t occ,
                                              uint32_t i) {
  return i < occ ? (uint32_t)a.index[bk * (uint64_t)a.S + kSlot0 + i] : (uint32_t)a.staged[start + i - occ];
}

constexpr uint32_t kMid = 64;   // arrivals handled by one wave in registers, one per lane
constexpr uint32_t kRegMax = 256;  // arrivals sorted in registers, up to four per lane

// Appends for the lanes where pred holds, with one atomic per wave; returns
// each such lane's slot.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool pred) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return 0;
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if ((threadIdx.x & 63) == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = (uint32_t)__builtin_amdgcn_readlane((int)base, (int)leader);
  return base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Ascending sort of one 64-bit value per lane within each aligned segment of
// SEG lanes (SEG a power of two <= 64), all segments at once.
template <uint32_t SEG>
__device__ __forceinline__ uint64_t segment_bitonic_sort(uint64_t v) {
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (uint32_t k = 2; k <= SEG; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      const uint64_t o = xor_lane64(v, j);
      const uint64_t mn = v < o ? v : o, mx = v < o ? o : v;
      const bool up = k == SEG || (lane & k) == 0;
      v = (((lane & j) == 0) == up) ? mn : mx;
    }
  }
  return v;
}

// The wave sorts the buckets of its lanes whose sizes are in (lo, SEG], 64 /
// SEG at a time, one per segment of SEG lanes, one arrival per lane, and
// writes their reservoirs.  `n`, `start`, `occ` are the candidates, their
// position (as `fetch` takes it) and the old slots of each lane's own bucket
// bk (any bucket per lane); fetch(bucket, start, occ, i) gives candidate i.
template <uint32_t SEG, class Fetch>
__device__ __forceinline__ void sort_buckets_by_segments(const SelectArgs& a, uint64_t bk, uint32_t n,
                                                         uint32_t start, uint32_t occ, uint32_t lo,
                                                         const Fetch& fetch) {
  constexpr uint32_t G = 64 / SEG;
  const uint32_t lane = threadIdx.x & 63, seg = lane / SEG, sl = lane % SEG;
  const uint32_t R = (uint32_t)a.R;
  uint64_t mm = __ballot(n > lo && n <= SEG);
  while (mm) {
    // pop up to G buckets; segment g takes the g-th (segments past the last get none)
    uint32_t my_src = 64;
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) {
      const uint32_t src = mm ? (uint32_t)__ffsll((unsigned long long)mm) - 1 : 64u;
      if (mm) mm &= mm - 1;
      if (seg == g) my_src = src;
    }
    const bool has = my_src < 64;
    const uint32_t bn = (uint32_t)__shfl((int)n, has ? (int)my_src : 0, 64);
    const uint32_t bs = (uint32_t)__shfl((int)start, has ? (int)my_src : 0, 64);
    const uint32_t bo = (uint32_t)__shfl((int)occ, has ? (int)my_src : 0, 64);
    // (bucket indices are below 2^32)
    const uint64_t bb = (uint32_t)__shfl((int)(uint32_t)bk, has ? (int)my_src : 0, 64);
    const uint32_t t = (uint32_t)(bb / a.M);
    const bool live = has && sl < bn;
    const uint64_t v = live ? priority(a.s_p, t, fetch(bb, bs, bo, sl)) : ~0ull;
    const uint64_t sorted = segment_bitonic_sort<SEG>(v);
    if (live && sl < R) a.index[bb * a.S + kSlot0 + sl] = (int32_t)(uint32_t)sorted;
  }
}

// Thread per bucket.  Buckets with at most kSmall arrivals: each thread ranks
// its arrivals against each other in registers.  Buckets with kSmall < n <=
// kMid: the wave sorts them in registers, one arrival per lane, four at a
// time up to 16 arrivals and two at a time up to 32.  Larger buckets are listed (with
// their start and size) for the LDS kernel; they are rare, so their appends
// are few.
// The select of one bucket per lane; every lane of the wave calls it (the
// appends and the lane-segment sorts work across the wave).  fetch(bucket,
// start, occ, i) gives candidate i of a bucket (start, occ: as the lane
// passed them); the work items of mid-size and large buckets carry gstart,
// the bucket's first slot in `staged`, where their kernels read them.
template <class Fetch>
__device__ __forceinline__ void select_lanes(const SelectArgs& a, uint64_t bk, bool in, uint32_t nn, uint32_t old,
                                             uint32_t start, uint32_t gstart, const Fetch& fetch) {
  const uint32_t R = (uint32_t)a.R;
  const uint32_t occ = old < R ? old : R;   // reservoir slots that take part
  const uint32_t n = nn ? occ + nn : 0u;    // candidates (none: the bucket is unchanged)
  int32_t* res = a.index + bk * (uint64_t)a.S;
  const bool small = n >= 1 && n <= (uint32_t)kSmall;
  // (a small bucket writes its header with its slots below)
  if (in && !small) res[0] = (int32_t)(old + nn);
  const bool mid = n > kMid && n <= kRegMax;
  const bool big = n > kRegMax;
  const uint32_t pm = wave_append(&a.wl_len[0], mid);
  if (mid) a.work[pm] = make_uint4((uint32_t)bk, gstart, n, occ);
  const uint32_t pb = wave_append(&a.wl_len[1], big);
  if (big) a.work[a.n_buckets - 1 - pb] = make_uint4((uint32_t)bk, gstart, n, occ);
  if (small) {
    const uint32_t t = (uint32_t)(bk / a.M);
    // every candidate is fetched before any is used (past the last one the
    // last is fetched again)
    uint32_t idc[kSmall];
#pragma unroll
    for (int i = 0; i < kSmall; ++i) idc[i] = fetch(bk, start, occ, (uint32_t)i < n ? (uint32_t)i : n - 1);
    uint64_t pk[kSmall];
#pragma unroll
    for (int i = 0; i < kSmall; ++i) pk[i] = (uint32_t)i < n ? priority(a.s_p, t, idc[i]) : ~0ull;
    // Batcher's odd-even merge network for 8 (19 compare-exchanges; the
    // priorities are distinct, absent ones ~0 sort last)
    constexpr int kNet[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2},
                                 {5, 6}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4},
                                 {5, 6}};
#pragma unroll
    for (int c = 0; c < 19; ++c) {
      const uint64_t x = pk[kNet[c][0]], y = pk[kNet[c][1]];
      pk[kNet[c][0]] = x < y ? x : y;
      pk[kNet[c][1]] = x < y ? y : x;
    }
    // header, then slots 0..7 (words past min(n, R) are not part of the
    // index; S >= 32 words, so all twelve lie inside the reservoir): three
    // 16-byte stores into one line
    uint4* r4 = reinterpret_cast<uint4*>(res);
    r4[0] = make_uint4(old + nn, 0u, 0u, 0u);
    r4[1] = make_uint4((uint32_t)pk[0], (uint32_t)pk[1], (uint32_t)pk[2], (uint32_t)pk[3]);
    if (n > 4 && R > 4) r4[2] = make_uint4((uint32_t)pk[4], (uint32_t)pk[5], (uint32_t)pk[6], (uint32_t)pk[7]);
  }
  // every lane of the wave is still here: the mid-size buckets, several per
  // wave when they are small enough
  sort_buckets_by_segments<16>(a, bk, n, start, occ, (uint32_t)kSmall, fetch);
  sort_buckets_by_segments<32>(a, bk, n, start, occ, 16u, fetch);
  sort_buckets_by_segments<64>(a, bk, n, start, occ, 32u, fetch);
}

__global__ __launch_bounds__(256) void bucket_select_small_kernel(SelectArgs a) {
  const uint64_t bk = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = bk < a.n_buckets;
  const uint32_t nn = in ? a.newcnt[bk] : 0u;
  const uint32_t old = (in && a.append) ? (uint32_t)a.index[bk * (uint64_t)a.S] : 0u;
  const uint32_t start = in ? a.seg[bk] : 0u;
  select_lanes(a, bk, in, nn, old, start, start,
               [&](uint64_t b, uint32_t st, uint32_t oc, uint32_t i) { return candidate(a, b, st, oc, i); });
}

// ---- two-level partition (buckets that receive few arrivals each)
//   tile    : block (t, tile of kTileE entries of keys_t[t]) counting-sorts
//             its entries by chunk of CH buckets in LDS and writes them back
//             in that order (contiguous writes), with each chunk's offsets
//             in the tile and its count added to the chunk's total
//   scan    : chunk_base = exclusive prefix of the chunk totals (table-major)
//   chunk   : block (t, chunk) reads the chunk's run of every tile, histograms
//             it by bucket in LDS, writes newcnt and seg of its CH buckets,
//             then places each row id in the chunk's region of `staged`
//             (assembled in LDS when it fits); when the index is replaced
//             (no append) the same block then selects its buckets, reading
//             their candidates from that region, as bucket_select_small does
// It produces the same newcnt, seg and (up to the order inside a bucket's
// run) staged as the one-level partition.
constexpr uint32_t kTileE = 8192;        // entries per tile (13 bits of row offset)
constexpr uint32_t kMaxChunks2 = 256;    // chunks per table (one scan value per thread)
constexpr uint32_t kMaxCh2 = 4096;       // buckets per chunk (LDS histogram)

struct TwoArgs {
  const uint32_t* keys_t;   // [Lp][np_part]
  uint32_t* ent;            // [Lp][n_tiles][kTileE] entries (row offset << chb | bucket in chunk)
  uint32_t* tile_off;       // [Lp][n_tiles][n_chunks + 1] chunk offsets inside each tile
  uint32_t* chunk_tot;      // [Lp * n_chunks] arrivals per chunk (zeroed before the tile kernel)
  const uint32_t* chunk_base;  // [Lp * n_chunks] their first staged slot
  uint32_t* newcnt;
  uint32_t* seg;
  int32_t* staged;
  uint32_t np, M;           // row length and buckets of the partition
  uint32_t chb, n_chunks, n_tiles;
  uint32_t id_base, row_mod;
  uint32_t out_cap;         // ids a chunk may assemble in LDS
  int fused;                // select the chunk's buckets here (no append)
  SelectArgs sel;
};

__global__ __launch_bounds__(256) void tile_partition_kernel(TwoArgs a) {
  extern __shared__ uint32_t sm2[];
  __shared__ uint32_t sh[4];
  uint32_t* cnt = sm2;                     // [n_chunks + 1] counts, then offsets
  uint32_t* ent = sm2 + kMaxChunks2 + 4;   // [kTileE]
  const uint32_t tile = blockIdx.x, t = blockIdx.y;
  const uint32_t ch = 1u << a.chb;
  for (uint32_t c = threadIdx.x; c <= a.n_chunks; c += 256) cnt[c] = 0;
  __syncthreads();
  constexpr int kPer = kTileE / 256 / 4;   // 16-byte loads per thread
  const uint32_t e0 = tile * kTileE;
  const uint4* rowv = reinterpret_cast<const uint4*>(a.keys_t + (uint64_t)t * a.np);
  uint32_t key[4 * kPer], rk[4 * kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const uint32_t v = e0 / 4 + threadIdx.x + (uint32_t)u * 256;
    const uint4 x = 4 * v < a.np ? rowv[v] : make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
    key[4 * u] = x.x;
    key[4 * u + 1] = x.y;
    key[4 * u + 2] = x.z;
    key[4 * u + 3] = x.w;
  }
#pragma unroll
  for (int j = 0; j < 4 * kPer; ++j) {
    rk[j] = 0;
    if (key[j] < a.M) rk[j] = atomicAdd(&cnt[key[j] >> a.chb], 1u);
  }
  __syncthreads();
  const uint32_t my = threadIdx.x < a.n_chunks ? cnt[threadIdx.x] : 0u;
  uint32_t total;
  const uint32_t off = block_excl_scan(my, &total, sh);
  uint32_t* toff = a.tile_off + ((uint64_t)t * a.n_tiles + tile) * (a.n_chunks + 1);
  if (threadIdx.x < a.n_chunks) {
    cnt[threadIdx.x] = off;
    toff[threadIdx.x] = off;
    if (my) atomicAdd(&a.chunk_tot[(uint64_t)t * a.n_chunks + threadIdx.x], my);
  }
  if (threadIdx.x == 0) toff[a.n_chunks] = total;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4 * kPer; ++j) {
    if (key[j] < a.M) {
      const uint32_t e = 4 * (threadIdx.x + (uint32_t)(j / 4) * 256) + (uint32_t)(j % 4);  // offset in the tile
      ent[cnt[key[j] >> a.chb] + rk[j]] = (e << a.chb) | (key[j] & (ch - 1));
    }
  }
  __syncthreads();
  uint32_t* out = a.ent + ((uint64_t)t * a.n_tiles + tile) * kTileE;
  for (uint32_t i = threadIdx.x; i < total; i += 256) out[i] = ent[i];
}

constexpr uint32_t kTB = 512;   // tiles whose run bounds sit in LDS at a time

__global__ __launch_bounds__(256) void chunk_scatter_kernel(TwoArgs a) {
  // [ch] counts, then cursors; [2 * kTB] run bounds; [out_cap] the chunk's
  // region of `staged`, assembled before it is written
  extern __shared__ uint32_t hc[];
  __shared__ uint32_t sh[4];
  const uint32_t c = blockIdx.x, t = blockIdx.y;
  const uint32_t ch = 1u << a.chb, lo = c * ch;
  const uint32_t cl = a.M - lo < ch ? a.M - lo : ch;
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t* tb = hc + ch;
  for (uint32_t j = threadIdx.x; j < ch; j += 256) hc[j] = 0;
  const uint64_t tb0 = (uint64_t)t * a.n_tiles;
  // Calls fn(entry, tile) for every entry of the chunk's run in every tile.
  // The run bounds of kTB tiles are loaded into LDS at once; a wave takes
  // four tiles per step and has the loads of all four (two entries per lane
  // each) in flight before using any.
  auto for_each_entry = [&](auto&& fn) {
    for (uint32_t g0 = 0; g0 < a.n_tiles; g0 += kTB) {
      const uint32_t gn = a.n_tiles - g0 < kTB ? a.n_tiles - g0 : kTB;
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < gn; i += 256) {
        const uint32_t* toff = a.tile_off + (tb0 + g0 + i) * (a.n_chunks + 1) + c;
        tb[2 * i] = toff[0];
        tb[2 * i + 1] = toff[1];
      }
      __syncthreads();
      for (uint32_t i0 = wv; i0 < gn; i0 += 16) {
        uint32_t x[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t i = i0 + 4u * (uint32_t)u;
          const uint32_t b0 = i < gn ? tb[2 * i] : 0u, b1 = i < gn ? tb[2 * i + 1] : 0u;
          const uint32_t* run = a.ent + (tb0 + g0 + i) * kTileE;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const uint32_t j = b0 + 64u * (uint32_t)h + lane;
            x[2 * u + h] = j < b1 ? run[j] : kEmpty;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (x[2 * u + h] != kEmpty) fn(x[2 * u + h], g0 + i0 + 4u * (uint32_t)u);
        // runs longer than 128 entries
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t i = i0 + 4u * (uint32_t)u;
          if (i < gn) {
            const uint32_t b0 = tb[2 * i], b1 = tb[2 * i + 1];
            const uint32_t* run = a.ent + (tb0 + g0 + i) * kTileE;
            for (uint32_t j = b0 + 128 + lane; j < b1; j += 64) fn(run[j], g0 + i);
          }
        }
      }
    }
  };
  // 1. histogram of the chunk's buckets
  for_each_entry([&](uint32_t x, uint32_t) { atomicAdd(&hc[x & (ch - 1)], 1u); });
  __syncthreads();
  // 2. counts and first slots of the chunk's buckets (thread i owns buckets
  // i * q .. i * q + q - 1); the counts become cursors
  constexpr uint32_t kPer = kMaxCh2 / 256;
  const uint32_t q = ch >= 256 ? ch / 256 : 1u;
  uint32_t v[kPer], loff[kPer];
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t i = 0; i < kPer; ++i) {
    const uint32_t j = threadIdx.x * q + i;
    v[i] = (i < q && j < cl) ? hc[j] : 0u;
    sum += v[i];
  }
  uint32_t total;
  uint32_t run_off = block_excl_scan(sum, &total, sh);
  const uint32_t base = a.chunk_base[(uint64_t)t * a.n_chunks + c];
  const uint64_t b0 = (uint64_t)t * a.M + lo;
  __syncthreads();
#pragma unroll
  for (uint32_t i = 0; i < kPer; ++i) {
    const uint32_t j = threadIdx.x * q + i;
    loff[i] = run_off;
    if (i < q && j < cl) {
      a.newcnt[b0 + j] = v[i];
      a.seg[b0 + j] = base + run_off;
      hc[j] = run_off;
    }
    run_off += v[i];
  }
  // 3. each arrival's row id at its bucket's cursor (the bounds are loaded
  // again behind a barrier inside for_each_entry): into LDS and then out with
  // contiguous stores, or straight to `staged` when the chunk holds more than
  // the LDS region
  uint32_t* outb = tb + 2 * kTB;
  const bool in_lds = total <= a.out_cap;
  for_each_entry([&](uint32_t x, uint32_t tile) {
    const uint32_t e = tile * kTileE + (x >> a.chb);
    const uint32_t row = a.row_mod ? e % a.row_mod : e;
    const uint32_t pos = atomicAdd(&hc[x & (ch - 1)], 1u);
    if (in_lds)
      outb[pos] = a.id_base + row;
    else
      a.staged[base + pos] = (int32_t)(a.id_base + row);
  });
  if (in_lds) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < total; i += 256) a.staged[base + i] = (int32_t)outb[i];
  }
  if (!a.fused) return;
  // 4. the select of the chunk's buckets, candidates from the LDS region (or
  // from `staged`, which the barrier makes visible to the workgroup); the
  // mid-size and large buckets go on to their kernels through the work lists
  __syncthreads();
#pragma unroll
  for (uint32_t i = 0; i < kPer; ++i) {
    if (i >= q) break;
    const uint32_t j = threadIdx.x * q + i;
    const bool in = j < cl;
    if (in_lds)
      select_lanes(a.sel, b0 + j, in, in ? v[i] : 0u, 0u, loff[i], base + loff[i],
                   [&](uint64_t, uint32_t st, uint32_t, uint32_t k) { return outb[st + k]; });
    else
      select_lanes(a.sel, b0 + j, in, in ? v[i] : 0u, 0u, loff[i], base + loff[i],
                   [&](uint64_t, uint32_t st, uint32_t, uint32_t k) { return (uint32_t)a.staged[base + st + k]; });
  }
}

// Ascending bitonic sort of the wave's 64 * KPL values, element e = lane * KPL
// + i in v[i] of lane `lane`: exchanges with a partner element e ^ j inside
// the lane when j < KPL, else with the same register of lane (lane ^ j / KPL).
template <int KPL>
__device__ __forceinline__ void wave_sort_u64(uint64_t (&v)[KPL]) {
  const uint32_t lane = threadIdx.x & 63;
  constexpr uint32_t N = 64u * KPL;
#pragma unroll
  for (uint32_t k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= (uint32_t)KPL) {
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
          const uint32_t e = lane * KPL + (uint32_t)i;
          const uint64_t o = xor_lane64(v[i], j / KPL);
          const uint64_t mn = v[i] < o ? v[i] : o, mx = v[i] < o ? o : v[i];
          v[i] = (((e & j) == 0) == ((e & k) == 0)) ? mn : mx;
        }
      } else {
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
          if ((i & (int)j) == 0) {
            const int i2 = i | (int)j;
            const bool asc = ((lane * KPL + (uint32_t)i) & k) == 0;
            const uint64_t x = v[i], y = v[i2];
            const bool sw = asc ? (x > y) : (x < y);
            v[i] = sw ? y : x;
            v[i2] = sw ? x : y;
          }
        }
      }
    }
  }
}

// One bucket with kMid < n <= 64 * KPL candidates: all in registers, sorted,
// the first min(n, R) written.
template <int KPL>
__device__ __forceinline__ void select_in_registers(const SelectArgs& a, uint32_t bk, uint32_t start, uint32_t n,
                                                    uint32_t occ) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t t = bk / a.M;
  uint32_t idc[KPL];
  if (!a.append) {
    // one run of `staged`: all loads issued together (past its end the last
    // candidate is read again)
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
      const uint32_t e = lane * KPL + (uint32_t)i;
      idc[i] = (uint32_t)a.staged[start + (e < n ? e : n - 1)];
    }
  } else {
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
      const uint32_t e = lane * KPL + (uint32_t)i;
      idc[i] = e < n ? candidate(a, bk, start, occ, e) : 0u;
    }
  }
  uint64_t v[KPL];
#pragma unroll
  for (int i = 0; i < KPL; ++i) v[i] = lane * KPL + (uint32_t)i < n ? priority(a.s_p, t, idc[i]) : ~0ull;
  wave_sort_u64<KPL>(v);
  // every candidate was read above: the reservoir can be overwritten
  const uint32_t keep = n < (uint32_t)a.R ? n : (uint32_t)a.R;
  int32_t* slots = a.index + (uint64_t)bk * a.S + kSlot0;
#pragma unroll
  for (int i = 0; i < KPL; ++i) {
    const uint32_t e = lane * KPL + (uint32_t)i;
    if (e < keep) slots[e] = (int32_t)(uint32_t)v[i];
  }
}

// One wave per mid-size bucket (kMid < n <= kRegMax), no LDS, so the CUs keep
// as many waves as their registers allow.
__global__ __launch_bounds__(64) void bucket_select_mid_kernel(SelectArgs a) {
  const uint32_t len = a.wl_len[0];
  for (uint32_t w = blockIdx.x; w < len; w += gridDim.x) {
    const uint4 e = a.work[w];
    if (e.z <= 128u)
      select_in_registers<2>(a, e.x, e.y, e.z, e.w);
    else
      select_in_registers<4>(a, e.x, e.y, e.z, e.w);
  }
}

// One wave per large bucket (n > kRegMax).  CAP priorities fit in LDS: 1024
// when R <= 256 (the threshold keeps about 2R <= 512, between R and CAP), so
// that twice as many waves fit a CU; 2048 above.
template <uint32_t CAP>
__global__ __launch_bounds__(64) void bucket_select_big_kernel(SelectArgs a) {
  constexpr uint32_t kWaveCap = CAP;
  __shared__ uint64_t buf[kWaveCap];
  __shared__ uint32_t cnt_sh;
  const uint32_t lane = threadIdx.x;
  const uint32_t len = a.wl_len[1];
  const uint32_t R = (uint32_t)a.R;
  const uint32_t sort_all = (2 * R > 256u ? 2 * R : 256u) < kWaveCap ? (2 * R > 256u ? 2 * R : 256u)
                                                                       : kWaveCap;
  for (uint32_t w = blockIdx.x; w < len; w += gridDim.x) {
    const uint4 e = a.work[a.n_buckets - 1 - w];
    const uint32_t bk = e.x, n = e.z, occ = e.w;
    const uint32_t t = bk / a.M;
    uint32_t c;
    if (n <= sort_all) {
      c = n;
      for (uint32_t i = lane; i < n; i += kWave) buf[i] = priority(a.s_p, t, candidate(a, bk, e.y, occ, i));
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
          const uint64_t pk = priority(a.s_p, t, candidate(a, bk, e.y, occ, i));
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
    // every candidate was read above: the reservoir can be overwritten
    const uint32_t keep = n < R ? n : R;
    for (uint32_t i = lane; i < keep; i += kWave)
      a.index[(uint64_t)bk * a.S + kSlot0 + i] = (int32_t)(uint32_t)buf[i];
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

hipError_t launch_fill_strided_u32(uint32_t* p, uint64_t n, uint32_t stride, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_strided_u32_kernel, dim3(grid_for(n, 256, 8)), dim3(256), 0, s, p, n, stride, v);
  return hipGetLastError();
}

namespace {

// Shape of the LDS-privatised counting sort for n rows.  With shared
// reservoirs the L key rows form one row of L * np entries over P buckets.
struct Geo {
  uint32_t np;                 // rows padded to 64
  uint32_t Lp, np_part;        // partition tables and their row length
  uint64_t Mp;                 // partition buckets per table
  uint32_t ch, n_chunks, n_slices, slice_vecs;
  uint64_t nb, nparts, tiles;
  // two-level partition (two_level): chunks of 2^chb buckets, tiles of kTileE entries
  bool two_level;
  uint32_t chb, n_chunks2, n_tiles2;
  uint64_t tiles2;              // scan tiles over the Lp * n_chunks2 chunk totals
};

Geo geometry(const Cfg& c, int64_t n_rows) {
  Geo g;
  g.np = (uint32_t)(((uint64_t)(n_rows > 0 ? n_rows : 1) + 63) / 64 * 64);
  g.Lp = c.shared ? 1u : (uint32_t)c.L;
  g.Mp = c.shared ? c.P : (uint64_t)c.M;
  g.np_part = c.shared ? g.np * (uint32_t)c.L : g.np;
  g.ch = g.Mp < kChunk ? (uint32_t)g.Mp : kChunk;
  g.n_chunks = (uint32_t)((g.Mp + g.ch - 1) / g.ch);  // a shared pool may end in a short chunk
  const uint32_t base_blocks = g.Lp * g.n_chunks;
  // about one partition block per CU: more row slices interleave more runs
  // of `staged` (partial-line writes), fewer leave CUs idle
  const uint32_t cus = (uint32_t)device_info().cus;
  uint32_t s = (cus + base_blocks - 1) / base_blocks;
  const uint32_t max_s = g.np_part / 16384 > 1 ? g.np_part / 16384 : 1;  // slices of >= 16384 rows
  if (s > max_s) s = max_s;
  if (s < 1) s = 1;
  g.n_slices = s;
  g.slice_vecs = (g.np_part / 4 + s - 1) / s;
  g.nb = (uint64_t)g.Lp * g.Mp;
  g.nparts = g.nb * s;
  g.tiles = (g.nparts + kTile - 1) / kTile;
  // Two-level partition when the buckets receive few arrivals: chunks of
  // at least Mp / 128 buckets (runs of ~64 entries per tile; twice that
  // measured slower, the chunk workgroups then hold twice the LDS), halved
  // down to Mp / 256 while a chunk's region of `staged` exceeds 64 KiB;
  // taken if that region is at most 128 KiB and the histogram fits LDS.
  const double per_bucket = (double)g.np_part / (double)g.Mp;
  uint32_t chb = 6;
  while ((1ull << chb) * 128 < g.Mp) ++chb;
  while (chb > 6 && (double)(1ull << chb) * per_bucket * 4.0 > 65536.0 && (1ull << (chb - 1)) * kMaxChunks2 >= g.Mp)
    --chb;
  g.chb = chb;
  g.n_chunks2 = (uint32_t)((g.Mp + (1ull << chb) - 1) >> chb);
  g.n_tiles2 = (g.np_part + kTileE - 1) / kTileE;
  g.two_level = (1u << chb) <= kMaxCh2 && g.n_chunks2 <= kMaxChunks2 &&
                (double)(1ull << chb) * per_bucket * 4.0 <= 131072.0 && g.Mp < (1ull << 31);
  g.tiles2 = ((uint64_t)g.Lp * g.n_chunks2 + kTile - 1) / kTile;
  return g;
}

// Bytes of the partition's own buffers: part and partoff (one level), or the
// entries, tile offsets, chunk totals and chunk bases (two levels).
uint64_t part_bytes(const Geo& g) {
  if (!g.two_level) return 2 * align256(4 * g.nparts);
  const uint64_t chunks = (uint64_t)g.Lp * g.n_chunks2;
  return align256(4ull * g.Lp * g.n_tiles2 * kTileE) + align256(4ull * g.Lp * g.n_tiles2 * (g.n_chunks2 + 1)) +
         2 * align256(4 * chunks);
}

}  // namespace

size_t insert_ws_bytes(const Cfg& c, int64_t n_rows) {
  const Geo g = geometry(c, n_rows);
  const uint64_t ne = (uint64_t)(n_rows > 0 ? n_rows : 1) * c.L;
  const uint64_t tiles = g.two_level ? g.tiles2 : g.tiles;
  return align256(4 * (uint64_t)c.L * g.np) + align256(4 * ne) + part_bytes(g) +
         2 * align256(4 * g.nb) + align256(16 * g.nb) + align256(4 * (tiles + 1)) + align256(8);
}

InsertWs insert_ws_carve(const Cfg& c, int64_t n_rows, void* ws) {
  const Geo g = geometry(c, n_rows);
  const uint64_t ne = (uint64_t)(n_rows > 0 ? n_rows : 1) * c.L;
  char* p = (char*)ws;
  InsertWs w;
  w.keys_t = (uint32_t*)p;
  p += align256(4 * (uint64_t)c.L * g.np);
  w.staged = (int32_t*)p;
  p += align256(4 * ne);
  if (g.two_level) {
    const uint64_t chunks = (uint64_t)g.Lp * g.n_chunks2;
    w.part = w.partoff = nullptr;
    w.ent = (uint32_t*)p;
    p += align256(4ull * g.Lp * g.n_tiles2 * kTileE);
    w.tile_off = (uint32_t*)p;
    p += align256(4ull * g.Lp * g.n_tiles2 * (g.n_chunks2 + 1));
    w.chunk_tot = (uint32_t*)p;
    p += align256(4 * chunks);
    w.chunk_base = (uint32_t*)p;
    p += align256(4 * chunks);
  } else {
    w.ent = w.tile_off = w.chunk_tot = w.chunk_base = nullptr;
    w.part = (uint32_t*)p;
    p += align256(4 * g.nparts);
    w.partoff = (uint32_t*)p;
    p += align256(4 * g.nparts);
  }
  w.seg = (uint32_t*)p;
  p += align256(4 * g.nb);
  w.newcnt = (uint32_t*)p;
  p += align256(4 * g.nb);
  w.work = (uint4*)p;
  p += align256(16 * g.nb);
  w.tile_sums = (uint32_t*)p;
  p += align256(4 * ((g.two_level ? g.tiles2 : g.tiles) + 1));
  w.wl_len = (uint32_t*)p;
  return w;
}

hipError_t launch_insert(const Cfg& c, int64_t n_rows, const uint32_t* keys, uint32_t id_base, bool append,
                         int32_t* index, const InsertWs& w, hipStream_t s) {
  const Geo g = geometry(c, n_rows);
  hipError_t e;
  // (with rows, the select below writes every reservoir's count)
  if (n_rows <= 0) return append ? hipSuccess : launch_fill_strided_u32((uint32_t*)index, g.nb, c.S, 0u, s);
  if ((e = launch_fill_u32(w.wl_len, 2, 0u, s)) != hipSuccess) return e;
  // table-major keys
  ShareMap sm;
  sm.shared = c.shared ? 1 : 0;
  sm.s_r = c.s_r;
  sm.M = c.M;
  sm.P = c.P;
  hipLaunchKernelGGL(keys_transpose_kernel, dim3(g.np / 64, (c.L + 63) / 64), dim3(256), 0, s, keys,
                     (uint32_t)n_rows, (uint32_t)c.L, g.np, w.keys_t, sm);
  SelectArgs a;
  a.index = index;
  a.S = c.S;
  a.newcnt = w.newcnt;
  a.seg = w.seg;
  a.staged = w.staged;
  a.work = w.work;
  a.wl_len = w.wl_len;
  a.n_buckets = g.nb;
  a.s_p = c.seeds.s_p;
  a.M = c.shared ? 1u : c.M;  // priority salt: the table, or the shared reservoir itself
  a.R = c.R;
  a.append = append ? 1 : 0;
  // The chunk blocks select their own buckets when those receive many
  // arrivals each (most go on to the wave-per-bucket kernels anyway); with
  // few arrivals a thread per bucket across the whole index is faster than
  // a chunk block's threads taking several buckets each.
  const bool fused = g.two_level && !append && (double)g.np_part >= 16.0 * (double)g.Mp;
  if (g.two_level) {
    const uint64_t chunks = (uint64_t)g.Lp * g.n_chunks2;
    if ((e = launch_fill_u32(w.chunk_tot, chunks, 0u, s)) != hipSuccess) return e;
    TwoArgs ta;
    ta.keys_t = w.keys_t;
    ta.ent = w.ent;
    ta.tile_off = w.tile_off;
    ta.chunk_tot = w.chunk_tot;
    ta.chunk_base = w.chunk_base;
    ta.newcnt = w.newcnt;
    ta.seg = w.seg;
    ta.staged = w.staged;
    ta.np = g.np_part;
    ta.M = (uint32_t)g.Mp;
    ta.chb = g.chb;
    ta.n_chunks = g.n_chunks2;
    ta.n_tiles = g.n_tiles2;
    ta.id_base = id_base;
    ta.row_mod = c.shared ? g.np : 0u;
    const size_t lds_tile = sizeof(uint32_t) * (kMaxChunks2 + 4 + kTileE);
    hipLaunchKernelGGL(tile_partition_kernel, dim3(g.n_tiles2, g.Lp), dim3(256), lds_tile, s, ta);
    const uint32_t tiles2 = (uint32_t)g.tiles2;
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(tiles2), dim3(kScanThreads), 0, s, w.chunk_tot, chunks,
                       w.tile_sums);
    hipLaunchKernelGGL(scan_tile_offsets_kernel, dim3(1), dim3(kScanThreads), 0, s, w.tile_sums, tiles2);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(tiles2), dim3(kScanThreads), 0, s, w.chunk_tot, chunks,
                       w.tile_sums, w.chunk_base);
    // LDS for 1.25 times a chunk's expected arrivals, rounded up to a power
    // of two, if that is at most 8K ids (32 KiB: four blocks per CU); larger
    // chunks store straight to `staged`, which measured faster than two
    // blocks per CU
    const double per_chunk = (double)(1u << g.chb) * (double)g.np_part / (double)g.Mp;
    uint32_t cap = 1024;
    while (cap <= 8192 && (double)cap < 1.25 * per_chunk) cap <<= 1;
    if (cap > 8192) cap = 0;
    ta.out_cap = cap;
    ta.fused = fused ? 1 : 0;
    ta.sel = a;
    const size_t lds_chunk = sizeof(uint32_t) * ((1u << g.chb) + 2 * kTB + cap);
    if ((e = allow_lds(reinterpret_cast<const void*>(&chunk_scatter_kernel), lds_chunk)) != hipSuccess) return e;
    hipLaunchKernelGGL(chunk_scatter_kernel, dim3(g.n_chunks2, g.Lp), dim3(256), lds_chunk, s, ta);
  } else {
  PartArgs pa;
  pa.keys_t = w.keys_t;
  pa.part = w.part;
  pa.partoff = w.partoff;
  pa.staged = w.staged;
  pa.np = g.np_part;
  pa.M = (uint32_t)g.Mp;
  pa.ch = g.ch;
  pa.n_chunks = g.n_chunks;
  pa.n_slices = g.n_slices;
  pa.slice_vecs = g.slice_vecs;
  pa.id_base = id_base;
  pa.row_mod = c.shared ? g.np : 0u;
  const uint32_t blocks = g.Lp * g.n_chunks * g.n_slices;
  const size_t lds = sizeof(uint32_t) * g.ch;
  hipLaunchKernelGGL(part_count_kernel, dim3(blocks), dim3(kPartThreads), lds, s, pa);
  // exclusive scan of the (bucket, slice) counts
  const uint32_t tiles = (uint32_t)g.tiles;
  hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(tiles), dim3(kScanThreads), 0, s, w.part, g.nparts,
                     w.tile_sums);
  hipLaunchKernelGGL(scan_tile_offsets_kernel, dim3(1), dim3(kScanThreads), 0, s, w.tile_sums, tiles);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(tiles), dim3(kScanThreads), 0, s, w.part, g.nparts,
                     w.tile_sums, w.partoff);
  hipLaunchKernelGGL(bucket_totals_kernel, dim3(grid_for(g.nb, 256, 16)), dim3(256), 0, s, w.part,
                     w.partoff, g.nb, g.n_slices, w.newcnt, w.seg);
  hipLaunchKernelGGL(part_scatter_kernel, dim3(blocks), dim3(kPartThreads), lds, s, pa);
  }
  if (!fused)
    hipLaunchKernelGGL(bucket_select_small_kernel, dim3((uint32_t)((g.nb + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(bucket_select_mid_kernel, dim3(device_info().cus * 32), dim3(64), 0, s, a);
  if (c.R <= 256)
    hipLaunchKernelGGL(bucket_select_big_kernel<1024>, dim3(device_info().cus * 32), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(bucket_select_big_kernel<kWaveCap>, dim3(device_info().cus * 32), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace flashk
