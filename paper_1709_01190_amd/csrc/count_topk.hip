// Querying phase (paper Alg. 3, Sec. 3.2 item 3): gather the L reservoirs a
// query hits, count how many of them hold each id, and return the k ids with
// the highest counts (ties: smaller id first).
//
// One wavefront per query (count_topk_kernel):
//   1. lane t reads key t and the bucket's count; one packed DPP scan gives
//      every table its first candidate and its first task (a task is 4
//      consecutive occupied slots, one 16-byte load);
//   2. the wave walks the tasks 256 at a time: each table's first task is
//      marked in LDS and a DPP prefix-max assigns every lane its table, so
//      four 16-byte loads per lane are in flight at once;
//   3. each id goes into an LDS open-addressing table whose slot packs
//      (id << cbits | count): one CAS claims an empty slot, a matching id
//      adds 1 (count_ids16: all first probes at once, then up to two
//      colliding ids per lane retried with double hashing);
//   4. one sweep compacts the distinct entries to the front of the table and
//      histograms their counts, which gives the threshold count c*; if too
//      many ids tie at c*, an id threshold is guessed from the uniform spread
//      of ids and bisected until between k and k + slack entries survive;
//   5. the survivors are sorted in registers and written; the table is
//      cleared on the way.
// Queries with more candidates than a launch's table takes are handed on to
// the next launch (a larger table).  A last stage with a table of 32-64 KB
// runs one workgroup of several waves per query (count_topk_block_kernel).
#include "launch.hpp"

namespace flashk {

namespace {

struct QueryArgs {
  const int32_t* index;       // reservoir b: count at index[b * S], slot i at index[b * S + kSlot0 + i]
  const uint32_t* qkeys;
  const int32_t* self_ids;
  int32_t* out_ids;
  int32_t* out_counts;
  const uint32_t* qlist;      // process qlist[0 .. *qlist_len) if not null
  const uint32_t* qlist_len;
  uint32_t* ovf_list;         // queries with total > max_total go here (null: never)
  uint32_t* ovf_len;
  int64_t n_queries;
  int64_t n_indexed;
  uint32_t M;
  int L, R, k, self_mode, cbits;   // k: the row stride of the outputs (the largest k)
  const int32_t* k_per_query;       // per-query k (clamped to [1, k]) if not null
  uint32_t S;                 // words per reservoir (a multiple of 32, so every task is one
                              // aligned 16-byte load)
  uint32_t max_total;         // candidates this launch's table accepts
  uint32_t sb;                // survivor buffer entries
  int shared;                 // reservoirs shared through the seeded map
  uint32_t s_r;
  uint64_t P;                 // reservoirs in the index
};

__host__ __device__ inline uint32_t slack_for(uint32_t need) { return need / 8 > 16 ? need / 8 : 16; }

__host__ __device__ inline size_t smem_bytes(int cap, int L, uint32_t sb) {
  const size_t scratch = sb > 256 ? sb : 256;
  return (size_t)cap * 4 + scratch * 4 + (size_t)L * 16 + (size_t)(L + 1) * 4 + 16;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x; }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t rl(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

// value of a per-table register array (table t held by lane t & 63, chunk t >> 6)
template <int LCH>
__device__ __forceinline__ uint32_t tab_reg(const uint32_t (&r)[LCH], uint32_t t) {
  if (LCH == 1) return rl(r[0], t);
  const uint32_t c = t >> 6, l = t & 63;
  uint32_t v = rl(r[0], l);
  if (LCH > 1 && c == 1) v = rl(r[LCH > 1 ? 1 : 0], l);
  if (LCH > 2 && c == 2) v = rl(r[LCH > 2 ? 2 : 0], l);
  if (LCH > 3 && c == 3) v = rl(r[LCH > 3 ? 3 : 0], l);
  return v;
}

template <int LCH>
__device__ __forceinline__ void tab_reg_add(uint32_t (&r)[LCH], uint32_t t, uint32_t add) {
  const uint32_t c = t >> 6, l = t & 63;
  if (lane_id() == l) {
#pragma unroll
    for (int i = 0; i < LCH; ++i)
      if ((uint32_t)i == c) r[i] += add;
  }
}

// The lane index, read so that the compiler cannot hoist what is derived from
// it out of the query loop (the sorts' per-stage lane masks would otherwise
// all stay live in scalar registers and spill).
__device__ __forceinline__ uint32_t opaque_lane() {
  uint32_t l;
  asm volatile("v_and_b32 %0, 63, %1" : "=v"(l) : "v"((uint32_t)threadIdx.x));
  return l;
}

// Sort m <= 64 * KPL keys held in scratch (ascending) across the wave, KPL
// keys per lane (element i = lane * KPL + r), and write the first k as
// (id, count); positions past m get (-1, 0).
template <int KPL>
__device__ __forceinline__ void sort_write(const uint32_t* scratch, uint32_t m, uint32_t k, uint32_t L,
                                           uint32_t idshift, uint32_t idmask, int32_t* out_ids,
                                           int32_t* out_counts) {
  const uint32_t lane = opaque_lane();
  uint32_t x[KPL];
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    const uint32_t i = lane * KPL + (uint32_t)r;
    x[r] = i < m ? scratch[i] : 0xFFFFFFFFu;
  }
#pragma unroll
  for (uint32_t kk = 2; kk <= 64u * KPL; kk <<= 1) {
#pragma unroll
    for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
      if (j < (uint32_t)KPL) {
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          if ((r & j) != 0) continue;
          const uint32_t i = lane * KPL + (uint32_t)r;
          const uint32_t p = x[r], q = x[r ^ j];
          const bool up = (i & kk) == 0;
          const uint32_t mn = p < q ? p : q, mx = p < q ? q : p;
          x[r] = up ? mn : mx;
          x[r ^ j] = up ? mx : mn;
        }
      } else {
        const uint32_t lj = j / KPL;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          const uint32_t i = lane * KPL + (uint32_t)r;
          const uint32_t o = xor_lane(x[r], lj);
          const bool up = (i & kk) == 0, lower = (lane & lj) == 0;
          const uint32_t mn = x[r] < o ? x[r] : o, mx = x[r] < o ? o : x[r];
          x[r] = (lower == up) ? mn : mx;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    const uint32_t i = lane * KPL + (uint32_t)r;
    if (i < k) {
      const bool real = i < m;
      out_ids[i] = real ? (int32_t)(x[r] & idmask) : -1;
      out_counts[i] = real ? (int32_t)L - (int32_t)(x[r] >> idshift) : 0;
    }
  }
  for (uint32_t i = 64u * KPL + lane; i < k; i += kWave) {
    out_ids[i] = -1;
    out_counts[i] = 0;
  }
}

// Same result for any m: each key's rank is the number of smaller keys.
__device__ __forceinline__ void rank_write(const uint32_t* scratch, uint32_t m, uint32_t k, uint32_t L,
                                           uint32_t idshift, uint32_t idmask, int32_t* out_ids,
                                           int32_t* out_counts) {
  const uint32_t lane = threadIdx.x & 63;
  for (uint32_t j0 = 0; j0 < m; j0 += 4 * kWave) {
    uint32_t key[4], rank[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t j = j0 + (uint32_t)r * kWave + lane;
      key[r] = j < m ? scratch[j] : 0xFFFFFFFFu;
      rank[r] = 0;
    }
    uint32_t i = 0;
    for (; i + 4 <= m; i += 4) {
      const uint4 o = *reinterpret_cast<const uint4*>(scratch + i);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        rank[r] += (o.x < key[r]) + (o.y < key[r]) + (o.z < key[r]) + (o.w < key[r]);
    }
    for (; i < m; ++i) {
      const uint32_t o = scratch[i];
#pragma unroll
      for (int r = 0; r < 4; ++r) rank[r] += o < key[r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t j = j0 + (uint32_t)r * kWave + lane;
      if (j < m && rank[r] < k) {
        out_ids[rank[r]] = (int32_t)(key[r] & idmask);
        out_counts[rank[r]] = (int32_t)L - (int32_t)(key[r] >> idshift);
      }
    }
  }
  for (uint32_t j = m + lane; j < k; j += kWave) {
    out_ids[j] = -1;
    out_counts[j] = 0;
  }
}

// Output length of query q: its own k clamped to [1, kmax], else kmax.
__device__ __forceinline__ uint32_t query_k(const QueryArgs& a, uint64_t q, uint32_t kmax) {
  if (!a.k_per_query) return kmax;
  const int32_t kk = a.k_per_query[q];
  return kk < 1 ? 1u : ((uint32_t)kk > kmax ? kmax : (uint32_t)kk);
}

// Appends the n pending hand-on queries (lane i holds the i-th) to the
// overflow list with one atomic; returns 0.
__device__ __forceinline__ uint32_t flush_overflow(const QueryArgs& a, uint32_t buf, uint32_t n) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t pos = 0;
  if (lane == 0) pos = atomicAdd(a.ovf_len, n);
  pos = rl(pos, 0);
  if (lane < n) a.ovf_list[pos + lane] = buf;
  return 0;
}

// Orders this wave's earlier LDS accesses before its later ones, for data
// that lanes of the same wave exchange through LDS.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Adds 16 candidate ids per lane (bit j of `valid`: idv[j] takes part) to
// the LDS table of CAP packed (id << cb | count) slots, with double hashing
// (an odd stride per id, so a probe run visits every slot of the power-of-two
// table; the table is at most half full).  All 16 first probes go out at
// once; after that each lane retries one colliding id at a time, so every
// retry instruction carries as many lanes as still have work.
template <int CAP>
__device__ __forceinline__ void count_ids16(uint32_t* tab, const uint32_t (&idv)[16], uint32_t valid,
                                            uint32_t cb) {
  constexpr int kLog = __builtin_ctz(CAP);
  uint32_t old[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint32_t slot = (idv[j] * 0x9E3779B1u) >> (32 - kLog);
    old[j] = ((valid >> j) & 1u) ? atomicCAS(&tab[slot], kEmpty, (idv[j] << cb) | 1u) : kEmpty;
  }
  uint32_t pend = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (!((valid >> j) & 1u) || old[j] == kEmpty) continue;
    if ((old[j] >> cb) == idv[j]) {
      atomicAdd(&tab[(idv[j] * 0x9E3779B1u) >> (32 - kLog)], 1u);
    } else {
      pend |= 1u << j;
    }
  }
  // two colliding ids per lane are retried at once
  constexpr int P = 2;
  bool act[P];
  uint32_t cid[P], cslot[P], cstep[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    act[r] = false;
    cid[r] = cslot[r] = cstep[r] = 0;
  }
  for (;;) {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      if (!act[r] && pend) {
        const uint32_t j = (uint32_t)__ffs(pend) - 1;
        pend &= pend - 1;
        uint32_t v = idv[0];
#pragma unroll
        for (int i = 1; i < 16; ++i) v = j == (uint32_t)i ? idv[i] : v;
        cid[r] = v;
        cstep[r] = ((v * 0x85EBCA77u) >> (32 - kLog)) | 1u;
        cslot[r] = (((v * 0x9E3779B1u) >> (32 - kLog)) + cstep[r]) & (CAP - 1);
        act[r] = true;
      }
    }
    bool any = false;
#pragma unroll
    for (int r = 0; r < P; ++r) any = any || act[r];
    if (!__any(any)) break;
    uint32_t o[P];
#pragma unroll
    for (int r = 0; r < P; ++r) o[r] = act[r] ? atomicCAS(&tab[cslot[r]], kEmpty, (cid[r] << cb) | 1u) : kEmpty;
#pragma unroll
    for (int r = 0; r < P; ++r) {
      if (!act[r]) continue;
      if (o[r] == kEmpty) {
        act[r] = false;
      } else if ((o[r] >> cb) == cid[r]) {
        atomicAdd(&tab[cslot[r]], 1u);
        act[r] = false;
      } else {
        cslot[r] = (cslot[r] + cstep[r]) & (CAP - 1);
      }
    }
  }
}

template <int CAP, int LCH>
__global__ __launch_bounds__(64) void count_topk_kernel(QueryArgs a) {
  constexpr int U = 4;                 // tasks (of 4 candidates) per lane per window
  constexpr int W = kWave * U;         // tasks per window
  constexpr int kLog = __builtin_ctz(CAP);
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* tab = (uint32_t*)smem;                         // [CAP] packed (id << cbits | count)
  uint32_t* scratch = tab + CAP;                           // [max(W, sb)] window marks, then survivors
  uint4* tinfo = reinterpret_cast<uint4*>(scratch + (a.sb > (uint32_t)W ? a.sb : (uint32_t)W));  // [L]
  uint32_t* hist = reinterpret_cast<uint32_t*>(tinfo + a.L);  // [L + 1]

  const uint32_t lane = lane_id();
  const uint32_t L = (uint32_t)a.L;
  const uint32_t R = (uint32_t)a.R;
  const uint32_t cb = (uint32_t)a.cbits;
  const uint32_t cmask = (1u << cb) - 1u;
  const uint32_t kmax = (uint32_t)a.k;
  const uint32_t idshift = 32u - cb;   // survivor key = (L - count) << idshift | id
  uint4* tab4 = reinterpret_cast<uint4*>(tab);
  for (uint32_t i = lane; i < (uint32_t)CAP / 4; i += kWave) tab4[i] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
  for (uint32_t i = lane; i < (uint32_t)W; i += kWave) scratch[i] = kEmpty;
  __syncthreads();

  uint32_t ovf_buf = 0, ovf_n = 0;  // pending hand-ons: lane i holds the i-th
  const uint64_t nq = a.qlist ? (uint64_t)*a.qlist_len : (uint64_t)a.n_queries;
  for (uint64_t w = blockIdx.x; w < nq; w += gridDim.x) {
    const uint64_t q = a.qlist ? (uint64_t)a.qlist[w] : w;
    const int64_t self = a.self_mode == 1 ? (int64_t)a.self_ids[q] : (a.self_mode == 2 ? (int64_t)q : -1);
    const uint32_t k = query_k(a, q, kmax);

    // 1. occupancy of the L buckets.  Each bucket's occupied slots are cut
    // into tasks of 4 consecutive slots (one 16-byte load); one packed scan
    // gives every table its first candidate (high half) and first task (low
    // half).  tinfo[t] = {slot base - 4 * first task (64-bit), first task * 4
    // + occupancy}, so task j of the query reads ids[base' + 4 j + i] for
    // 4 j + i < end.
    uint32_t tstart[LCH], tcnt[LCH];
    uint32_t carry = 0;
#pragma unroll
    for (int c = 0; c < LCH; ++c) {
      const uint32_t t = (uint32_t)c * 64 + lane;
      uint32_t nt = 0;
      uint64_t base = 0;
      if (t < L) {
        const uint32_t key = a.qkeys[q * (uint64_t)L + t];
        if (key < a.M) {
          const uint64_t bucket = reservoir_of(a.shared != 0, a.s_r, a.P, a.M, t, key);
          const uint32_t cnt = (uint32_t)a.index[bucket * a.S];
          nt = cnt < R ? cnt : R;
          base = bucket * a.S + kSlot0;
        }
      }
      const uint32_t ct = (nt + 3) >> 2;
      const uint32_t packed = (nt << 16) | ct;
      const uint32_t inc = wave_incl_scan(packed);
      const uint32_t pre = carry + inc - packed;
      tstart[c] = pre & 0xFFFFu;
      tcnt[c] = ct;
      if (t < L)
        tinfo[t] = make_uint4((uint32_t)(base - 4ull * tstart[c]), (uint32_t)((base - 4ull * tstart[c]) >> 32),
                              4u * tstart[c] + nt, 0u);
      carry += rl(inc, 63);
    }
    const uint32_t total = carry >> 16, n_tasks = carry & 0xFFFFu;
    if (total > a.max_total) {
      // hand the query on; appends are batched 64 at a time (one atomic each)
      if (lane == ovf_n) ovf_buf = (uint32_t)q;
      if (++ovf_n == (uint32_t)kWave) ovf_n = flush_overflow(a, ovf_buf, ovf_n);
      continue;
    }
    for (uint32_t c = lane; c <= L; c += kWave) hist[c] = 0;
    __syncthreads();

    // 2-3. gather and count, W tasks (4 W candidates) per window
    for (uint32_t base = 0; base < n_tasks; base += W) {
      // mark where each table's tasks start inside the window; the table
      // holding the window's first task is marked at position 0
      uint32_t tf = 0;
#pragma unroll
      for (int c = 0; c < LCH; ++c) {
        const uint32_t t = (uint32_t)c * 64 + lane;
        const bool ne = tcnt[c] > 0;
        if (ne && tstart[c] > base && tstart[c] < base + W) scratch[tstart[c] - base] = t;
        const uint64_t bal = __ballot(ne && tstart[c] <= base);
        if (bal) tf = (uint32_t)c * 64 + 63 - (uint32_t)__clzll((long long)bal);
      }
      if (lane == 0) scratch[0] = tf;
      __syncthreads();
      uint32_t tcarry = 0;
      uint4 ids4[U];
      uint32_t vmask[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t mk = scratch[u * kWave + lane];
        scratch[u * kWave + lane] = kEmpty;
        uint32_t tt = wave_incl_max(mk == kEmpty ? 0u : mk + 1);  // 0 = no mark yet
        tt = tt > tcarry ? tt : tcarry;
        tcarry = rl(tt, 63);
        // every lane loads: a lane past the last task reads the last task
        // again (always in bounds) and masks all four candidates off
        const uint32_t task = base + (uint32_t)u * kWave + lane;
        const uint32_t tc = task < n_tasks ? task : n_tasks - 1;
        const uint4 ti = tinfo[tt - 1];
        const uint64_t addr = (((uint64_t)ti.y << 32) | ti.x) + 4ull * tc;
        const uint32_t room = ti.z - 4u * tc;  // occupied slots of this bucket from here, >= 1
        vmask[u] = task < n_tasks ? (room >= 4 ? 0xFu : ((1u << room) - 1u)) : 0u;
        ids4[u] = *reinterpret_cast<const uint4*>(a.index + addr);
      }
      uint32_t idv[16];
      uint32_t valid = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        idv[4 * u + 0] = ids4[u].x;
        idv[4 * u + 1] = ids4[u].y;
        idv[4 * u + 2] = ids4[u].z;
        idv[4 * u + 3] = ids4[u].w;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (((vmask[u] >> j) & 1u) && (int64_t)idv[4 * u + j] != self) valid |= 1u << (4 * u + j);
      }
      count_ids16<CAP>(tab, idv, valid, cb);
      __syncthreads();
    }

    // 4. compact the distinct entries to tab[0, nd) in place (each chunk is
    // read and cleared before compacted entries are written into it) and
    // histogram their counts on the way: count 1 in registers, larger counts
    // in LDS.  Everything past nd is left empty.
    uint32_t nd = 0, ones = 0;
    for (uint32_t i0 = 0; i0 < (uint32_t)CAP / 4; i0 += kWave) {
      const uint4 v4 = tab4[i0 + lane];
      tab4[i0 + lane] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
      const uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
      uint32_t n4 = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (v[j] == kEmpty) continue;
        ++n4;
        const uint32_t c = v[j] & cmask;
        if (c == 1) ++ones;
        else atomicAdd(&hist[c], 1u);
      }
      const uint32_t inc = wave_incl_scan(n4);
      uint32_t pos = nd + inc - n4;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (v[j] != kEmpty) tab[pos++] = v[j];
      nd += rl(inc, 63);
    }
    ones = wave_sum(ones);
    if (lane == 0) hist[1] += ones;
    __syncthreads();
    const uint32_t nd4 = (nd + 3) / 4;  // sweeps read tab4[0, nd4); the tail is empty

    uint32_t cstar = 0, thr = 0xFFFFFFFFu;
    if (nd > k) {
      // c*: the largest count with at least k ids at or above it
      uint32_t above = 0;
      bool found = false;
      for (int c0 = (int)L; c0 >= 1 && !found; c0 -= kWave) {
        const int c = c0 - (int)lane;
        const uint32_t h = c >= 1 ? hist[c] : 0u;
        const uint32_t inc = wave_incl_scan(h);
        const uint64_t hit = __ballot(above + inc >= k);
        if (hit) {
          const uint32_t f = (uint32_t)__ffsll((unsigned long long)hit) - 1;
          cstar = (uint32_t)(c0 - (int)f);
          above += rl(inc - h, f);
          found = true;
        } else {
          above += rl(inc, 63);
        }
      }
      const uint32_t need = k - above;
      const uint32_t ties = hist[cstar];
      const uint32_t slack = slack_for(need);
      if (ties > need + slack) {
        // id threshold with need <= #(ties with id < thr) <= need + slack,
        // guessed from the uniform spread of ids, then bisected
        const uint64_t span = (uint64_t)a.n_indexed;
        uint64_t lo = 0, hi = span;
        uint64_t g = (uint64_t)((float)(need + slack / 2) * ((float)span / (float)ties)) + 1;
        if (g >= hi) g = hi - 1;
        if (g <= lo) g = lo + 1;
        for (int it = 0; it < 64; ++it) {
          // empty slots never match: their count field is cmask > L >= c*
          uint32_t cnt = 0;
          for (uint32_t i = lane; i < nd4; i += kWave) {
            const uint4 v4 = tab4[i];
            cnt += ((v4.x & cmask) == cstar && (uint64_t)(v4.x >> cb) < g) +
                   ((v4.y & cmask) == cstar && (uint64_t)(v4.y >> cb) < g) +
                   ((v4.z & cmask) == cstar && (uint64_t)(v4.z >> cb) < g) +
                   ((v4.w & cmask) == cstar && (uint64_t)(v4.w >> cb) < g);
          }
          cnt = wave_sum(cnt);
          if (cnt < need) {
            lo = g;
          } else if (cnt > need + slack) {
            hi = g;
          } else {
            break;
          }
          g = (lo + hi) / 2;
          if (g == lo) break;  // cannot happen for distinct ids; keeps the loop finite
        }
        thr = (uint32_t)g;
      }
    }

    // 5. survivors -> scratch, four entries per lane (tab[0, nd) is cleared
    // on the way), then sort and write
    uint32_t m = 0;
    for (uint32_t i0 = 0; i0 < nd4; i0 += kWave) {
      const uint32_t i = i0 + lane;
      uint4 v4 = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
      if (i < nd4) {
        v4 = tab4[i];
        tab4[i] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
      }
      const uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
      bool sel[4];
      uint32_t n_sel = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t c = v[j] & cmask, idv = v[j] >> cb;
        sel[j] = v[j] != kEmpty && (c > cstar || (c == cstar && idv < thr));
        n_sel += sel[j];
      }
      const uint32_t inc = wave_incl_scan(n_sel);
      uint32_t pos = m + inc - n_sel;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!sel[j]) continue;
        if (pos < a.sb) scratch[pos] = ((L - (v[j] & cmask)) << idshift) | (v[j] >> cb);
        ++pos;
      }
      m += rl(inc, 63);
    }
    if (m > a.sb) m = a.sb;
    __syncthreads();
    const uint64_t orow = q * (uint64_t)kmax;
    for (uint32_t j = k + lane; j < kmax; j += kWave) {
      a.out_ids[orow + j] = -1;
      a.out_counts[orow + j] = 0;
    }
    const uint32_t idmask = (idshift >= 32) ? 0xFFFFFFFFu : ((1u << idshift) - 1u);
    if (m <= 64) {
      sort_write<1>(scratch, m, k, L, idshift, idmask, a.out_ids + orow, a.out_counts + orow);
    } else if (m <= 128) {
      sort_write<2>(scratch, m, k, L, idshift, idmask, a.out_ids + orow, a.out_counts + orow);
    } else if (m <= 256) {
      sort_write<4>(scratch, m, k, L, idshift, idmask, a.out_ids + orow, a.out_counts + orow);
    } else {
      rank_write(scratch, m, k, L, idshift, idmask, a.out_ids + orow, a.out_counts + orow);
    }
    __syncthreads();
    // leave the window marks empty for the next query
    for (uint32_t i = lane; i < (uint32_t)W; i += kWave) scratch[i] = kEmpty;
  }
  if (ovf_n) flush_overflow(a, ovf_buf, ovf_n);
}

// LDS bytes of the workgroup kernel: table, per-wave window marks (reused for
// the survivors), table info, histogram and 8 control words.
__host__ __device__ inline uint32_t block_scratch(uint32_t sb, int nw) {
  return sb > (uint32_t)(nw * 256) ? sb : (uint32_t)(nw * 256);
}
__host__ __device__ inline size_t block_smem_bytes(int cap, int L, uint32_t sb, int nw) {
  return (size_t)cap * 4 + (size_t)block_scratch(sb, nw) * 4 + (size_t)L * 16 + (size_t)(L + 1) * 4 + 32;
}

// The same query steps for queries with many candidates, by a workgroup of
// NW wavefronts that share one LDS table, so that a CU keeps 8-16 waves in
// flight although the table takes 32-64 KB.  Waves take the gather windows in
// turn; the table is swept in place (no compaction) with the sweeps split
// over all threads; block-wide sums go through LDS words.  Wave 0 sorts and
// writes the survivors.
template <int CAP, int LCH, int NW>
__global__ __launch_bounds__(64 * NW) void count_topk_block_kernel(QueryArgs a) {
  constexpr int U = 4;                 // tasks (of 4 candidates) per lane per window
  constexpr int W = kWave * U;         // tasks per window
  constexpr uint32_t NT = kWave * NW;  // threads
  constexpr int kLog = __builtin_ctz(CAP);
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t scr_n = block_scratch(a.sb, NW);
  uint32_t* tab = (uint32_t*)smem;                                    // [CAP]
  uint32_t* scratch = tab + CAP;                                      // [scr_n]
  uint4* tinfo = reinterpret_cast<uint4*>(scratch + scr_n);           // [L]
  uint32_t* hist = reinterpret_cast<uint32_t*>(tinfo + a.L);          // [L + 1]
  uint32_t* ctrl = hist + a.L + 1;  // [0] distinct ids, [1..3] bisection counts, [4] survivors

  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t* marks = scratch + wv * W;                                 // this wave's window marks
  const uint32_t L = (uint32_t)a.L;
  const uint32_t R = (uint32_t)a.R;
  const uint32_t cb = (uint32_t)a.cbits;
  const uint32_t cmask = (1u << cb) - 1u;
  const uint32_t kmax = (uint32_t)a.k;
  const uint32_t idshift = 32u - cb;
  uint4* tab4 = reinterpret_cast<uint4*>(tab);
  for (uint32_t i = tid; i < (uint32_t)CAP / 4; i += NT) tab4[i] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
  for (uint32_t i = tid; i < scr_n; i += NT) scratch[i] = kEmpty;
  __syncthreads();

  const uint64_t nq = a.qlist ? (uint64_t)*a.qlist_len : (uint64_t)a.n_queries;
  for (uint64_t w = blockIdx.x; w < nq; w += gridDim.x) {
    const uint64_t q = a.qlist ? (uint64_t)a.qlist[w] : w;
    const int64_t self = a.self_mode == 1 ? (int64_t)a.self_ids[q] : (a.self_mode == 2 ? (int64_t)q : -1);
    const uint32_t k = query_k(a, q, kmax);

    // 1. occupancy (every wave keeps the per-table registers; wave 0 publishes tinfo)
    uint32_t tstart[LCH], tcnt[LCH];
    uint32_t carry = 0;
#pragma unroll
    for (int c = 0; c < LCH; ++c) {
      const uint32_t t = (uint32_t)c * 64 + lane;
      uint32_t nt = 0;
      uint64_t base = 0;
      if (t < L) {
        const uint32_t key = a.qkeys[q * (uint64_t)L + t];
        if (key < a.M) {
          const uint64_t bucket = reservoir_of(a.shared != 0, a.s_r, a.P, a.M, t, key);
          const uint32_t cnt = (uint32_t)a.index[bucket * a.S];
          nt = cnt < R ? cnt : R;
          base = bucket * a.S + kSlot0;
        }
      }
      const uint32_t ct = (nt + 3) >> 2;
      const uint32_t packed = (nt << 16) | ct;
      const uint32_t inc = wave_incl_scan(packed);
      const uint32_t pre = carry + inc - packed;
      tstart[c] = pre & 0xFFFFu;
      tcnt[c] = ct;
      if (wv == 0 && t < L)
        tinfo[t] = make_uint4((uint32_t)(base - 4ull * tstart[c]), (uint32_t)((base - 4ull * tstart[c]) >> 32),
                              4u * tstart[c] + nt, 0u);
      carry += rl(inc, 63);
    }
    const uint32_t n_tasks = carry & 0xFFFFu;
    if (wv == 0) {
      for (uint32_t c = lane; c <= L; c += kWave) hist[c] = 0;
      if (lane < 8) ctrl[lane] = 0;
    }
    __syncthreads();

    // 2-3. gather and count; wave wv takes windows wv, wv + NW, ...
    for (uint32_t base = wv * (uint32_t)W; base < n_tasks; base += NW * (uint32_t)W) {
      uint32_t tf = 0;
#pragma unroll
      for (int c = 0; c < LCH; ++c) {
        const uint32_t t = (uint32_t)c * 64 + lane;
        const bool ne = tcnt[c] > 0;
        if (ne && tstart[c] > base && tstart[c] < base + W) marks[tstart[c] - base] = t;
        const uint64_t bal = __ballot(ne && tstart[c] <= base);
        if (bal) tf = (uint32_t)c * 64 + 63 - (uint32_t)__clzll((long long)bal);
      }
      if (lane == 0) marks[0] = tf;
      wave_lds_sync();
      uint32_t tcarry = 0;
      uint4 ids4[U];
      uint32_t vmask[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t mk = marks[u * kWave + lane];
        marks[u * kWave + lane] = kEmpty;
        uint32_t tt = wave_incl_max(mk == kEmpty ? 0u : mk + 1);
        tt = tt > tcarry ? tt : tcarry;
        tcarry = rl(tt, 63);
        const uint32_t task = base + (uint32_t)u * kWave + lane;
        const uint32_t tc = task < n_tasks ? task : n_tasks - 1;
        const uint4 ti = tinfo[tt - 1];
        const uint64_t addr = (((uint64_t)ti.y << 32) | ti.x) + 4ull * tc;
        const uint32_t room = ti.z - 4u * tc;
        vmask[u] = task < n_tasks ? (room >= 4 ? 0xFu : ((1u << room) - 1u)) : 0u;
        ids4[u] = *reinterpret_cast<const uint4*>(a.index + addr);
      }
      uint32_t idv[16];
      uint32_t valid = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        idv[4 * u + 0] = ids4[u].x;
        idv[4 * u + 1] = ids4[u].y;
        idv[4 * u + 2] = ids4[u].z;
        idv[4 * u + 3] = ids4[u].w;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (((vmask[u] >> j) & 1u) && (int64_t)idv[4 * u + j] != self) valid |= 1u << (4 * u + j);
      }
      count_ids16<CAP>(tab, idv, valid, cb);
      wave_lds_sync();
    }
    __syncthreads();

    // 4. histogram of the counts over the whole table (count 1 in registers)
    uint32_t ones = 0, nd = 0;
    for (uint32_t i = tid; i < (uint32_t)CAP / 4; i += NT) {
      const uint4 v4 = tab4[i];
      const uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (v[j] == kEmpty) continue;
        ++nd;
        const uint32_t c = v[j] & cmask;
        if (c == 1) ++ones;
        else atomicAdd(&hist[c], 1u);
      }
    }
    ones = wave_sum(ones);
    nd = wave_sum(nd);
    if (lane == 0) {
      if (ones) atomicAdd(&hist[1], ones);
      atomicAdd(&ctrl[0], nd);
    }
    __syncthreads();
    nd = ctrl[0];

    // 5. c* (every wave computes the same value), then the id threshold for
    // ties, bisected on block-wide counts (ctrl[1 + it % 3]: the word for the
    // round after next is cleared while this one is summed)
    uint32_t cstar = 0, thr = 0xFFFFFFFFu;
    if (nd > k) {
      uint32_t above = 0;
      bool found = false;
      for (int c0 = (int)L; c0 >= 1 && !found; c0 -= kWave) {
        const int c = c0 - (int)lane;
        const uint32_t h = c >= 1 ? hist[c] : 0u;
        const uint32_t inc = wave_incl_scan(h);
        const uint64_t hit = __ballot(above + inc >= k);
        if (hit) {
          const uint32_t f = (uint32_t)__ffsll((unsigned long long)hit) - 1;
          cstar = (uint32_t)(c0 - (int)f);
          above += rl(inc - h, f);
          found = true;
        } else {
          above += rl(inc, 63);
        }
      }
      const uint32_t need = k - above;
      const uint32_t ties = hist[cstar];
      const uint32_t slack = slack_for(need);
      if (ties > need + slack) {
        const uint64_t span = (uint64_t)a.n_indexed;
        uint64_t lo = 0, hi = span;
        uint64_t g = (uint64_t)((float)(need + slack / 2) * ((float)span / (float)ties)) + 1;
        if (g >= hi) g = hi - 1;
        if (g <= lo) g = lo + 1;
        for (int it = 0; it < 64; ++it) {
          uint32_t cnt = 0;
          for (uint32_t i = tid; i < (uint32_t)CAP / 4; i += NT) {
            const uint4 v4 = tab4[i];
            cnt += ((v4.x & cmask) == cstar && (uint64_t)(v4.x >> cb) < g) +
                   ((v4.y & cmask) == cstar && (uint64_t)(v4.y >> cb) < g) +
                   ((v4.z & cmask) == cstar && (uint64_t)(v4.z >> cb) < g) +
                   ((v4.w & cmask) == cstar && (uint64_t)(v4.w >> cb) < g);
          }
          cnt = wave_sum(cnt);
          uint32_t* word = ctrl + 1 + it % 3;
          if (lane == 0 && cnt) atomicAdd(word, cnt);
          if (tid == 0) ctrl[1 + (it + 1) % 3] = 0;
          __syncthreads();
          cnt = *word;
          if (cnt < need) {
            lo = g;
          } else if (cnt > need + slack) {
            hi = g;
          } else {
            break;
          }
          g = (lo + hi) / 2;
          if (g == lo) break;
        }
        thr = (uint32_t)g;
      }
    }

    // 6. survivors -> scratch[0, m), four entries per lane (the table is
    // cleared on the way)
    for (uint32_t i = tid; i < (uint32_t)CAP / 4; i += NT) {
      const uint4 v4 = tab4[i];
      tab4[i] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
      const uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
      bool sel[4];
      uint32_t n_sel = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t c = v[j] & cmask, idv = v[j] >> cb;
        sel[j] = v[j] != kEmpty && (c > cstar || (c == cstar && idv < thr));
        n_sel += sel[j];
      }
      const uint32_t inc = wave_incl_scan(n_sel);
      const uint32_t tot = rl(inc, 63);
      if (tot) {
        uint32_t pos0 = 0;
        if (lane == 0) pos0 = atomicAdd(&ctrl[4], tot);
        uint32_t pos = rl(pos0, 0) + inc - n_sel;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (!sel[j]) continue;
          if (pos < a.sb) scratch[pos] = ((L - (v[j] & cmask)) << idshift) | (v[j] >> cb);
          ++pos;
        }
      }
    }
    __syncthreads();

    // 7. wave 0 sorts and writes, then restores the marks it overwrote
    if (wv == 0) {
      uint32_t m = ctrl[4];
      if (m > a.sb) m = a.sb;
      const uint64_t orow = q * (uint64_t)kmax;
      for (uint32_t j = k + lane; j < kmax; j += kWave) {
        a.out_ids[orow + j] = -1;
        a.out_counts[orow + j] = 0;
      }
      const uint32_t idmask = (idshift >= 32) ? 0xFFFFFFFFu : ((1u << idshift) - 1u);
      if (m <= 64) {
        sort_write<1>(scratch, m, k, L, idshift, idmask, a.out_ids + orow, a.out_counts + orow);
      } else if (m <= 128) {
        sort_write<2>(scratch, m, k, L, idshift, idmask, a.out_ids + orow, a.out_counts + orow);
      } else if (m <= 256) {
        sort_write<4>(scratch, m, k, L, idshift, idmask, a.out_ids + orow, a.out_counts + orow);
      } else {
        rank_write(scratch, m, k, L, idshift, idmask, a.out_ids + orow, a.out_counts + orow);
      }
      wave_lds_sync();
      for (uint32_t i = lane; i < m; i += kWave) scratch[i] = kEmpty;
    }
  }
}

// ---------------------------------------------------------------------------
// First stage for queries of at most 2048 candidates whose ids are nearly all
// distinct (the usual case: a query meets a few ids in several tables and
// many once).  One wave per query keeps all its candidates in registers (up
// to 32 per lane) and needs no full counting table:
//   a. every candidate sets its three bits (in one word) of a 32K-bit LDS
//      filter; one whose three bits were all set already is a suspect (a
//      repeated id, or an id whose bits other ids set).  Three bits instead
//      of one cut these false suspects about twenty-fold at 2048
//      candidates (from ~64 to ~3), still with one LDS atomic per candidate;
//   b. the suspects go into a small exact table, and a second pass counts
//      every candidate that is in it.  A candidate not in it occurs exactly
//      once: had its id occurred before, that earlier occurrence would have
//      set its bits and made this one a suspect;
//   c. the ids of count >= 2 (all in the table) come first; the rest of the
//      k places go to the smallest ids of count 1, found by a radix select
//      over id bins (the bin holding the cut is ranked directly, or refined
//      when crowded).
// Queries with more candidates or suspects than the stage holds, or with at
// least k ids of count >= 2 (the threshold count is then above 1), are
// handed on to the counting-table stages.
constexpr int kFastU = 8;                  // tasks of 4 candidates per lane
constexpr uint32_t kFastCap = 64 * 4 * kFastU;
constexpr uint32_t kBmWords = 1024;        // filter bits: 32 * 1024
constexpr uint32_t kTs = 256;              // suspect table slots
constexpr uint32_t kSusp = 128;            // suspects a query may have
constexpr int kNB = 512;                   // radix bins
constexpr uint32_t kCut = 64;              // a cut bin of at most this many ids is ranked directly

// window marks: one 16-bit entry (table + 1; 0: none) per task of the window
constexpr uint32_t kMarkWords = 64 * kFastU / 2;
static_assert(kMarkWords <= (uint32_t)kNB, "the window marks live in the radix bins");
// the suspects' own filter (8K bits): a candidate whose bit is clear there is
// no suspect, so only about one in a hundred probes the suspect table
constexpr uint32_t kB2Words = 256;
constexpr uint32_t kStageK = 256;   // rows of up to this k are assembled in LDS
constexpr uint32_t kSmallK = 128;   // up to this k the survivor keys fit the suspects' filter's words
static_assert(256 + 2 * kTs + kB2Words == kBmWords, "suspect table and suspects' filter fill the filter's words");
static_assert(kSusp <= (uint32_t)kNB - kMarkWords, "the suspect list follows the marks in the bins");

// LDS words: filter, table info, radix bins, the cut bin's ids, and (k above
// kSmallK only) survivor keys and tie groups.  Buffers whose lifetimes do not
// overlap share words:
//   - the window marks (gather) are the first bins: once read they are zero
//     again, as the bins must be when counting starts;
//   - the suspect list (filter, suspect table) is the last 128 bins, cleared
//     after use;
//   - once every candidate has passed the filter its words are free: words
//     256..767 hold the suspect table (ids, then counts) and 768..1023 the
//     suspects' filter, both set up before use; with k <= kSmallK the survivor
//     keys and tie groups then take the suspects' filter's words;
//   - with k <= kStageK the output row (ids, then counts) is assembled in the
//     first 2k words once the suspect table has been read for the last time.
// The filter and the bins are zero between queries.
__host__ __device__ inline uint32_t fast_lds_words(int L, uint32_t kmax) {
  const uint32_t k4 = (kmax + 3u) & ~3u;
  return kBmWords + 4u * (uint32_t)L + (uint32_t)kNB + kCut + (kmax <= kSmallK ? 0u : 2 * k4);
}

// One multiplicative hash per id serves all three structures: the filter
// word is its top 10 bits and the word's three bits are bits 17..21, 12..16
// and 7..11, the suspect table slot is its top 8 bits, and the suspects'
// filter bit its top 13 (word = the slot, so one address reaches both).  An
// id that shares a suspect's top bits costs at most a longer probe; results
// never depend on the hash.  The multiply takes the
// id's low 24 bits (a full-rate 24-bit multiply instead of a quarter-rate
// 32-bit one): ids 2^24 apart share a hash, which costs the same.
__device__ __forceinline__ uint32_t id_hash(uint32_t id) { return __umul24(id, 0x3779B1u); }
__device__ __forceinline__ uint32_t ts_slot_of(uint32_t h) { return h >> 24; }

// Bins [0, 512): lane l holds bins 8l .. 8l+7.  Returns the bin b* where the
// running count first reaches `need` (1 <= need <= total), with *before =
// the count of the bins below it and *inb = its own.  With `prefix`, every
// bin below b* is replaced by its exclusive prefix (the start of its group).
// With `all` != 0 the last bin is not counted in LDS: it holds all minus
// the other bins.
__device__ __forceinline__ uint32_t find_cut_bin(uint32_t* bins, uint32_t need, uint32_t* before, uint32_t* inb,
                                                 bool prefix, uint32_t all = 0) {
  const uint32_t lane = threadIdx.x & 63;
  uint4* b4 = reinterpret_cast<uint4*>(bins + 8 * lane);
  const uint4 b0 = b4[0];
  const uint4 b1 = b4[1];
  uint32_t v[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
  if (all) {
    uint32_t part = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) part += v[i];
    const uint32_t rest = all - wave_sum(part);
    if (lane == 63) v[7] += rest;
  }
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) sum += v[i];
  const uint32_t incl = wave_incl_scan(sum);
  const uint32_t excl = incl - sum;
  const uint64_t hit = __ballot(excl < need && need <= incl);
  const uint32_t f = hit ? (uint32_t)__ffsll((unsigned long long)hit) - 1 : 63u;
  uint32_t run = excl, bin = 0, bef = 0, own = 0;
  bool done = false;
  uint32_t pre[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    pre[i] = run;
    if (!done && run + v[i] >= need) {
      bin = 8 * lane + (uint32_t)i;
      bef = run;
      own = v[i];
      done = true;
    }
    run += v[i];
  }
  if (prefix) {
    b4[0] = make_uint4(pre[0], pre[1], pre[2], pre[3]);
    b4[1] = make_uint4(pre[4], pre[5], pre[6], pre[7]);
  }
  *before = rl(bef, f);
  *inb = rl(own, f);
  return rl(bin, f);
}

__device__ __forceinline__ uint32_t bitlen64(uint64_t x) { return x ? 64u - (uint32_t)__clzll((long long)x) : 0u; }

template <int LCH>
// At most 96 VGPRs (five waves per SIMD): the stage waits on memory, and
// 20 waves per CU keep more loads in flight than 16 with fewer spills.
__global__ __launch_bounds__(64, 5) void count_topk_fast_kernel(QueryArgs a) {
  constexpr int U = kFastU;
  constexpr int W = kWave * U;
  constexpr int NJ = 4 * U;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t kmax = (uint32_t)a.k;
  const uint32_t k4 = (kmax + 3u) & ~3u;
  uint32_t* bm = (uint32_t*)smem;                         // [kBmWords] filter
  uint32_t* tsk = bm + 256;                                // [kTs] suspect ids
  uint32_t* tsc = tsk + kTs;                               // [kTs] their counts
  uint4* tinfo = reinterpret_cast<uint4*>(bm + kBmWords);  // [L]
  uint32_t* bins = reinterpret_cast<uint32_t*>(tinfo + a.L);  // [kNB] radix bins
  uint32_t* cutb = bins + kNB;                             // [kCut] ids of the cut bin
  uint16_t* marks = reinterpret_cast<uint16_t*>(bins);    // [W] window marks (table + 1; 0: none)
  uint32_t* susp = bins + kNB - kSusp;                     // [kSusp] suspect list
  uint32_t* b2 = bm + kBmWords - kB2Words;                 // [kB2Words] the suspects' filter
  const bool staged = kmax <= kStageK;                     // output rows assembled in bm[0, 2k)
  uint32_t* surv = kmax <= kSmallK ? b2 : cutb + kCut;    // [kmax] survivor keys / ids of count >= 2
  uint32_t* grp = surv + k4;                               // [kmax] ties grouped by bin

  const uint32_t lane = threadIdx.x;
  const uint32_t L = (uint32_t)a.L;
  const uint32_t R = (uint32_t)a.R;
  const uint32_t cb = (uint32_t)a.cbits;
  const uint32_t idshift = 32u - cb;
  const uint32_t idmask = (idshift >= 32) ? 0xFFFFFFFFu : ((1u << idshift) - 1u);
  uint4* bm4 = reinterpret_cast<uint4*>(bm);
  uint4* bins4 = reinterpret_cast<uint4*>(bins);
  for (uint32_t i = lane; i < kBmWords / 4; i += kWave) bm4[i] = make_uint4(0, 0, 0, 0);
  for (uint32_t i = lane; i < (uint32_t)kNB / 4; i += kWave) bins4[i] = make_uint4(0, 0, 0, 0);
  __syncthreads();

  uint32_t ovf_buf = 0, ovf_n = 0;
  const uint64_t nq = a.qlist ? (uint64_t)*a.qlist_len : (uint64_t)a.n_queries;
  // the next query's keys are loaded while the current one is processed:
  // key[c] of lane t = table c * 64 + t.  The bucket counts are read when the
  // query starts: a count loaded a query ahead brings in the reservoir's first
  // line (the header shares it with the first slots), which the L2 has mostly
  // evicted again by the time the gather reads the slots.
  uint32_t pkey[LCH];
  auto load_keys = [&](uint64_t wq) {
    const uint64_t qq = wq < nq ? (a.qlist ? (uint64_t)a.qlist[wq] : wq) : 0;
#pragma unroll
    for (int c = 0; c < LCH; ++c) {
      const uint32_t t = (uint32_t)c * 64 + lane;
      pkey[c] = (wq < nq && t < L) ? a.qkeys[qq * (uint64_t)L + t] : kEmpty;
    }
  };
  load_keys(blockIdx.x);
  for (uint64_t w = blockIdx.x; w < nq; w += gridDim.x) {
    const uint64_t q = a.qlist ? (uint64_t)a.qlist[w] : w;
    const int64_t self = a.self_mode == 1 ? (int64_t)a.self_ids[q] : (a.self_mode == 2 ? (int64_t)q : -1);
    const uint32_t k = query_k(a, q, kmax);

    // 1. occupancy, as in the counting-table stages
    uint32_t tstart[LCH], tcnt[LCH];
    uint32_t carry = 0;
#pragma unroll
    for (int c = 0; c < LCH; ++c) {
      const uint32_t t = (uint32_t)c * 64 + lane;
      uint32_t nt = 0;
      uint64_t base = 0;
      if (pkey[c] < a.M) {
        const uint64_t bucket = reservoir_of(a.shared != 0, a.s_r, a.P, a.M, t, pkey[c]);
        const uint32_t cnt = (uint32_t)a.index[bucket * a.S];
        nt = cnt < R ? cnt : R;
        base = bucket * a.S + kSlot0;
      }
      const uint32_t ct = (nt + 3) >> 2;
      const uint32_t packed = (nt << 16) | ct;
      const uint32_t inc = wave_incl_scan(packed);
      const uint32_t pre = carry + inc - packed;
      tstart[c] = pre & 0xFFFFu;
      tcnt[c] = ct;
      if (t < L)
        tinfo[t] = make_uint4((uint32_t)(base - 4ull * tstart[c]), (uint32_t)((base - 4ull * tstart[c]) >> 32),
                              4u * tstart[c] + nt, 0u);
      carry += rl(inc, 63);
    }
    const uint32_t total = carry >> 16, n_tasks = carry & 0xFFFFu;
    load_keys(w + gridDim.x);
    bool hand_on = total > kFastCap || n_tasks > (uint32_t)W;
    const bool touched = !hand_on;
    uint32_t idv[NJ];
    uint32_t nsus = 0;
    // radix bins of the first level (filled with the count-1 ids below): 511
    // bins over [0, wid), sized so that about twice the share of ids
    // expected below the cut (ids spread evenly, cut near k) is covered, and
    // bin 511 for every id above
    const uint64_t span = (uint64_t)(a.n_indexed > 0 ? a.n_indexed : 1);
    uint64_t est = total > k ? 2ull * k * span / total + 64 : span;
    if (est > span) est = span;
    uint32_t s0 = bitlen64(est - 1) > 9 ? bitlen64(est - 1) - 9 : 0;
    const uint32_t wid0 = (uint32_t)(kNB - 1) << s0;
    if (!hand_on) {
      // 2. gather every candidate (the tasks fit one window); an absent or
      // excluded candidate becomes kEmpty
#pragma unroll
      for (int c = 0; c < LCH; ++c) {
        const uint32_t t = (uint32_t)c * 64 + lane;
        if (tcnt[c] > 0 && tstart[c] > 0) marks[tstart[c]] = (uint16_t)(t + 1);
      }
      uint32_t tf = 0;
#pragma unroll
      for (int c = 0; c < LCH; ++c) {
        const uint64_t bal = __ballot(tcnt[c] > 0 && tstart[c] == 0);
        if (bal) tf = (uint32_t)c * 64 + (uint32_t)__ffsll((unsigned long long)bal) - 1;
      }
      if (lane == 0) marks[0] = (uint16_t)(tf + 1);
      wave_lds_sync();
      // every task's 16-byte load is issued before any is used
      uint32_t tcarry = 0;
      uint4 v4[U];
      uint32_t room[U];   // occupied slots of the task's bucket from its first (0: no task)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        room[u] = 0;
        v4[u] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
        if ((uint32_t)u * kWave < n_tasks) {
          const uint32_t mk = marks[u * kWave + lane];
          marks[u * kWave + lane] = 0;
          uint32_t tt = wave_incl_max(mk);   // table + 1 of the latest mark at or before this task
          tt = tt > tcarry ? tt : tcarry;
          tcarry = rl(tt, 63);
          const uint32_t task = (uint32_t)u * kWave + lane;
          const uint32_t tc = task < n_tasks ? task : n_tasks - 1;
          const uint4 ti = tinfo[tt - 1];
          const uint64_t addr = (((uint64_t)ti.y << 32) | ti.x) + 4ull * tc;
          room[u] = task < n_tasks ? ti.z - 4u * tc : 0u;
          v4[u] = *reinterpret_cast<const uint4*>(a.index + addr);
        }
      }
      // the query's own id (never a real id when absent: kEmpty is no candidate)
      const uint32_t self32 = self >= 0 ? (uint32_t)self : kEmpty;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t vv[4] = {v4[u].x, v4[u].y, v4[u].z, v4[u].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) idv[4 * u + i] = (room[u] > (uint32_t)i && vv[i] != self32) ? vv[i] : kEmpty;
      }
      // 3a. filter: a candidate whose three bits are set already is a suspect.  The
      // four atomics of a task are all issued before any result is used, so
      // they are waited for once (absent candidates take no part: a shared
      // word would serialise them).
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if ((uint32_t)u * kWave < n_tasks) {
          uint32_t bit[4], old[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t x = idv[4 * u + i];
            const uint32_t h = id_hash(x);
            bit[i] = (1u << ((h >> 17) & 31u)) | (1u << ((h >> 12) & 31u)) | (1u << ((h >> 7) & 31u));
            old[i] = 0;
            if (x != kEmpty) old[i] = atomicOr(&bm[h >> 22], bit[i]);
          }
          bool seen[4];
          uint64_t m[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            seen[i] = (old[i] & bit[i]) == bit[i];
            m[i] = __ballot(seen[i]);
          }
          if (m[0] | m[1] | m[2] | m[3]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const uint32_t p = nsus + mbcnt(m[i]);
              if (seen[i] && p < kSusp) susp[p] = idv[4 * u + i];
              nsus += (uint32_t)__popcll(m[i]);
            }
          }
        }
      }
      hand_on = nsus > kSusp;
    }
    uint32_t nmulti = 0, nsing = 0;
    if (!hand_on) {
      if (nsus) {
        // the suspect table and the suspects' filter take the filter's words
        reinterpret_cast<uint4*>(tsk)[lane] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
        reinterpret_cast<uint4*>(tsc)[lane] = make_uint4(0, 0, 0, 0);
        reinterpret_cast<uint4*>(b2)[lane] = make_uint4(0, 0, 0, 0);
      }
      wave_lds_sync();
      // 3b. the suspects into the exact table (ids only; linear probing, at
      // most half full), and their bits into the suspects' filter
      for (uint32_t i = lane; i < nsus; i += kWave) {
        const uint32_t x = susp[i];
        const uint32_t h = id_hash(x);
        uint32_t sl = ts_slot_of(h);
        atomicOr(&b2[sl], 1u << ((h >> 19) & 31u));
        for (;;) {
          const uint32_t o = atomicCAS(&tsk[sl], kEmpty, x);
          if (o == kEmpty || o == x) break;
          sl = (sl + 1) & (kTs - 1);
        }
      }
      wave_lds_sync();
      // the suspect list sits in the bins, which count from here on
      if (nsus && lane < kSusp / 4) reinterpret_cast<uint4*>(susp)[lane] = make_uint4(0, 0, 0, 0);
      wave_lds_sync();
      // 3c. count every candidate that is a suspect; the others occur once
      // and go into the first level's radix bins
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if ((uint32_t)u * kWave < n_tasks) {
          // the suspects' filter word and the table slot of every candidate,
          // read together (unused when the query has no suspects)
          uint32_t sl[4], w2[4], o[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t h = id_hash(idv[4 * u + i]);
            sl[i] = ts_slot_of(h);
            w2[i] = __builtin_amdgcn_ubfe(b2[sl[i]], h >> 19, 1u);   // bit (h >> 19) mod 32
            o[i] = tsk[sl[i]];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t x = idv[4 * u + i];
            // (an absent candidate may pass: it then finds no equal entry)
            const bool f2 = nsus && w2[i] != 0;
            uint32_t s2 = sl[i], o2 = f2 ? o[i] : kEmpty;
            if (o2 != x && o2 != kEmpty) {   // another id holds the slot: walk on
              do {
                s2 = (s2 + 1) & (kTs - 1);
                o2 = tsk[s2];
              } while (o2 != x && o2 != kEmpty);
            }
            const bool hit = o2 == x && x != kEmpty;
            if (hit) atomicAdd(&tsc[s2], 1u);
            const uint32_t y = hit ? kEmpty : x;
            idv[4 * u + i] = y;
            if (y < wid0) atomicAdd(&bins[y >> s0], 1u);   // the ids above are counted as a remainder
            nsing += (uint32_t)__popcll(__ballot(y != kEmpty));
          }
        }
      }
      wave_lds_sync();
      // the table's ids of count >= 2, and of count 1 (they occur once: their
      // bit was set by another id; they join the bins)
      uint32_t nm = 0, n1 = 0;
      if (nsus) {
        for (uint32_t i = lane; i < kTs; i += kWave) {
          const uint32_t x = tsk[i];
          const uint32_t c = x != kEmpty ? tsc[i] : 0u;
          nm += c >= 2;
          n1 += c == 1;
          if (c == 1 && x < wid0) atomicAdd(&bins[x >> s0], 1u);
        }
      }
      nmulti = wave_sum(nm);
      nsing += wave_sum(n1);
      hand_on = nmulti >= k;
    }
    if (hand_on) {
      if (lane == ovf_n) ovf_buf = (uint32_t)q;
      if (++ovf_n == (uint32_t)kWave) ovf_n = flush_overflow(a, ovf_buf, ovf_n);
    } else {
      // 4. the ids of count >= 2 all survive, ahead of the rest; then the
      // `need` smallest ids of count 1
      const uint32_t D = nsing + nmulti;
      const uint32_t need = (D <= k ? D : k) - nmulti;
      const uint64_t orow = q * (uint64_t)kmax;
      int32_t* oid = a.out_ids + orow;
      int32_t* ocnt = a.out_counts + orow;
      wave_lds_sync();
      uint32_t bstar = 0, before = 0, inb = 0;
      if (need < nsing) bstar = find_cut_bin(bins, need, &before, &inb, true, nsing);
      if (need < nsing && inb <= kCut && bstar < (uint32_t)kNB - 1) {
        // 5a. one radix level settles it: the ties of bins below b* survive,
        // and the smallest `need - before` of bin b*.  Output place of a
        // survivor = ids of count >= 2 + the start of its bin's group + its
        // rank in the group (bins are id ranges), so no sort is needed.
        // The bins below b* now hold the start of their groups; scattering
        // advances each to the group's end.
        uint32_t ncut = 0;
        // four ids per lane at a time: their cursor atomics are all issued
        // before any result is used.  An absent id (kEmpty) falls in the
        // last bin, which is above b*.
        auto place4 = [&](const uint32_t (&y)[4]) {
          uint32_t b[4], pos[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            b[i] = y[i] < wid0 ? y[i] >> s0 : (uint32_t)(kNB - 1);
            pos[i] = 0;
            if (b[i] < bstar) pos[i] = atomicAdd(&bins[b[i]], 1u);
          }
          uint64_t mp[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (b[i] < bstar) grp[pos[i]] = y[i];
            mp[i] = __ballot(b[i] == bstar);
          }
          if (mp[0] | mp[1] | mp[2] | mp[3]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const uint32_t p = ncut + mbcnt(mp[i]);
              if (b[i] == bstar && p < kCut) cutb[p] = y[i];
              ncut += (uint32_t)__popcll(mp[i]);
            }
          }
        };
#pragma unroll
        for (int u = 0; u < U; ++u)
          if ((uint32_t)u * kWave < n_tasks) {
            const uint32_t y4[4] = {idv[4 * u], idv[4 * u + 1], idv[4 * u + 2], idv[4 * u + 3]};
            place4(y4);
          }
        uint32_t nmc = 0;
        if (nsus) {
          for (uint32_t i0 = 0; i0 < kTs; i0 += 4 * kWave) {
            uint32_t x4[4], c4[4], y4[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              x4[j] = tsk[i0 + j * kWave + lane];
              c4[j] = x4[j] != kEmpty ? tsc[i0 + j * kWave + lane] : 0u;
              y4[j] = c4[j] == 1 ? x4[j] : kEmpty;
            }
            place4(y4);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint32_t x = x4[j], c = c4[j];
              // ids of count >= 2: key (L - count, id)
              const bool mult = c >= 2;
              const uint64_t mm = __ballot(mult);
              if (mult) surv[nmc + mbcnt(mm)] = ((L - c) << idshift) | x;
              nmc += (uint32_t)__popcll(mm);
            }
          }
        }
        wave_lds_sync();
        // each survivor's place is known: the row is assembled in the first
        // filter's words (free now; ids, then counts) and stored with
        // coalesced writes, or written in place when k is above 512
        auto put = [&](uint32_t pos, uint32_t id, uint32_t cnt) {
          if (staged) {
            bm[pos] = id;
            bm[kmax + pos] = cnt;
          } else {
            oid[pos] = (int32_t)id;
            ocnt[pos] = (int32_t)cnt;
          }
        };
        // ids of count >= 2: rank among themselves by (count desc, id asc)
        for (uint32_t j0 = 0; j0 < nmulti; j0 += kWave) {
          const uint32_t j = j0 + lane;
          const uint32_t key = j < nmulti ? surv[j] : 0xFFFFFFFFu;
          uint32_t rank = 0;
          for (uint32_t i = 0; i < nmulti; ++i) rank += surv[i] < key;
          if (j < nmulti) put(rank, key & idmask, L - (key >> idshift));
        }
        // ties below the cut bin: rank inside the bin's group
        for (uint32_t p = lane; p < before; p += kWave) {
          const uint32_t y = grp[p];
          const uint32_t b = y >> s0;   // below the cut bin: y < wid0
          const uint32_t g0 = b ? bins[b - 1] : 0u, g1 = bins[b];
          uint32_t rank = 0;
          for (uint32_t i = g0; i < g1; ++i) rank += grp[i] < y;
          put(nmulti + g0 + rank, y, 1u);
        }
        // the cut bin: its `need - before` smallest
        if (lane < ncut) {
          const uint32_t y = cutb[lane];
          uint32_t rank = 0;
          for (uint32_t i = 0; i < ncut; ++i) rank += cutb[i] < y;
          if (rank < need - before) put(nmulti + before + rank, y, 1u);
        }
        const uint32_t m = nmulti + need;
        if (staged) {
          wave_lds_sync();
          for (uint32_t j = lane; j < kmax; j += kWave) {
            oid[j] = j < m ? (int32_t)bm[j] : -1;
            ocnt[j] = j < m ? (int32_t)bm[kmax + j] : 0;
          }
        } else {
          for (uint32_t j = m + lane; j < kmax; j += kWave) {
            oid[j] = -1;
            ocnt[j] = 0;
          }
        }
      } else {
        // 5b. all ids of count 1 survive, or the cut needs finer bins:
        // ids below x_lo survive with the smallest `cut` of [x_lo, x_hi),
        // found level by level (32-bit ranges: ids are below 2^31, so
        // 0xFFFFFFFF stands for 2^32), then every survivor key is sorted
        uint32_t x_lo = kEmpty, x_hi = kEmpty;
        uint32_t cut = 0;
        if (need < nsing) {
          uint32_t s = s0, lo = 0, wid = wid0, needl = need;
          uint32_t bs = bstar, bef = before, in_b = inb;
          for (int level = 0;; ++level) {
            if (level > 0) {
              for (uint32_t i = lane; i < (uint32_t)kNB / 4; i += kWave) bins4[i] = make_uint4(0, 0, 0, 0);
              wave_lds_sync();
              auto bin_of = [&](uint32_t x) {
                const uint32_t d = x - lo;   // wraps above wid for x < lo (lo + wid <= 2^32)
                if (x != kEmpty && d < wid) atomicAdd(&bins[d >> s], 1u);
              };
#pragma unroll
              for (int u = 0; u < U; ++u)
                if ((uint32_t)u * kWave < n_tasks) {
#pragma unroll
                  for (int i = 0; i < 4; ++i) bin_of(idv[4 * u + i]);
                }
              if (nsus)
                for (uint32_t i = lane; i < kTs; i += kWave) bin_of(tsc[i] == 1 ? tsk[i] : kEmpty);
              wave_lds_sync();
              bs = find_cut_bin(bins, needl, &bef, &in_b, false);
            }
            uint32_t nlo, nwid;
            if (level == 0 && bs == (uint32_t)kNB - 1) {
              nlo = wid;
              nwid = kEmpty - wid;   // [wid, 2^32)
            } else {
              nlo = lo + (bs << s);
              const uint32_t rest = wid - (bs << s);
              nwid = (1u << s) < rest ? (1u << s) : rest;
            }
            needl -= bef;
            // each level narrows the range 2^9-fold: ids below 2^32 need at
            // most four levels; the bound only guards the loop
            if (in_b <= kCut || level >= 5) {
              x_lo = nlo;
              x_hi = nlo + nwid;
              if (x_hi < nlo) x_hi = kEmpty;
              cut = needl;
              break;
            }
            lo = nlo;
            wid = nwid;
            s = bitlen64(wid - 1) > 9 ? bitlen64(wid - 1) - 9 : 0;
            wave_lds_sync();
          }
        }
        uint32_t m = 0, ncut = 0;
        auto take = [&](uint32_t x, uint32_t c) {
          const bool all = x != kEmpty && (c >= 2 || x < x_lo);
          const bool part = x != kEmpty && c == 1 && x >= x_lo && x < x_hi;
          const uint64_t mm = __ballot(all);
          if (all) surv[m + mbcnt(mm)] = ((L - c) << idshift) | x;
          m += (uint32_t)__popcll(mm);
          const uint64_t mp = __ballot(part);
          if (mp) {
            if (part && ncut + mbcnt(mp) < kCut) cutb[ncut + mbcnt(mp)] = x;
            ncut += (uint32_t)__popcll(mp);
          }
        };
        if (nsus)
          for (uint32_t i0 = 0; i0 < kTs; i0 += kWave) {
            const uint32_t x = tsk[i0 + lane];
            take(x, x != kEmpty ? tsc[i0 + lane] : 0u);
          }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if ((uint32_t)u * kWave < n_tasks) {
#pragma unroll
            for (int i = 0; i < 4; ++i) take(idv[4 * u + i], 1u);
          }
        wave_lds_sync();
        if (ncut > kCut) ncut = kCut;   // not reached: the cut bin holds at most kCut ids
        if (ncut) {
          const uint32_t mine = lane < ncut ? cutb[lane] : 0u;
          uint32_t rank = 0;
          for (uint32_t j = 0; j < ncut; ++j) rank += cutb[j] < mine;
          const bool sel = lane < ncut && rank < cut;
          const uint64_t mm = __ballot(sel);
          if (sel) surv[m + mbcnt(mm)] = ((L - 1u) << idshift) | mine;
          m += (uint32_t)__popcll(mm);
          wave_lds_sync();
        }
        for (uint32_t j = k + lane; j < kmax; j += kWave) {
          oid[j] = -1;
          ocnt[j] = 0;
        }
        if (m <= 64) {
          sort_write<1>(surv, m, k, L, idshift, idmask, oid, ocnt);
        } else if (m <= 128) {
          sort_write<2>(surv, m, k, L, idshift, idmask, oid, ocnt);
        } else if (m <= 256) {
          sort_write<4>(surv, m, k, L, idshift, idmask, oid, ocnt);
        } else {
          rank_write(surv, m, k, L, idshift, idmask, oid, ocnt);
        }
      }
    }
    // 6. leave the filter, the suspect table, the bins and the marks empty
    // for the next query (the marks were cleared as they were read; clearing
    // them all again costs one store per lane)
    wave_lds_sync();
    if (touched) {
      for (uint32_t i = lane; i < kBmWords / 4; i += kWave) bm4[i] = make_uint4(0, 0, 0, 0);
      for (uint32_t i = lane; i < (uint32_t)kNB / 4; i += kWave) bins4[i] = make_uint4(0, 0, 0, 0);
    }
    wave_lds_sync();
  }
  if (ovf_n) flush_overflow(a, ovf_buf, ovf_n);
}

template <int LCH>
hipError_t launch_fast(const QueryArgs& a, int grid, hipStream_t st) {
  const size_t lds = 4 * (size_t)fast_lds_words(a.L, (uint32_t)a.k);
  const hipError_t e = allow_lds(reinterpret_cast<const void*>(&count_topk_fast_kernel<LCH>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((count_topk_fast_kernel<LCH>), dim3(grid), dim3(64), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_fast_any(const QueryArgs& a, int grid, hipStream_t st) {
  switch ((a.L + 63) / 64) {
    case 1: return launch_fast<1>(a, grid, st);
    case 2: return launch_fast<2>(a, grid, st);
    case 3: return launch_fast<3>(a, grid, st);
    case 4: return launch_fast<4>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

template <int CAP, int LCH>
hipError_t launch_cap(const QueryArgs& a, int grid, hipStream_t st) {
  const size_t lds = smem_bytes(CAP, a.L, a.sb);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const hipError_t e = allow_lds(reinterpret_cast<const void*>(&count_topk_kernel<CAP, LCH>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((count_topk_kernel<CAP, LCH>), dim3(grid), dim3(64), lds, st, a);
  return hipGetLastError();
}

template <int LCH>
hipError_t launch_lch(int cap, const QueryArgs& a, int grid, hipStream_t st) {
  switch (cap) {
    case 1024: return launch_cap<1024, LCH>(a, grid, st);
    case 2048: return launch_cap<2048, LCH>(a, grid, st);
    case 4096: return launch_cap<4096, LCH>(a, grid, st);
    case 8192: return launch_cap<8192, LCH>(a, grid, st);
    case 16384: return launch_cap<16384, LCH>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_any(int cap, const QueryArgs& a, int grid, hipStream_t st) {
  switch ((a.L + 63) / 64) {
    case 1: return launch_lch<1>(cap, a, grid, st);
    case 2: return launch_lch<2>(cap, a, grid, st);
    case 3: return launch_lch<3>(cap, a, grid, st);
    case 4: return launch_lch<4>(cap, a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

template <int CAP, int LCH, int NW>
hipError_t launch_block_kernel(const QueryArgs& a, int grid, hipStream_t st) {
  const size_t lds = block_smem_bytes(CAP, a.L, a.sb, NW);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const hipError_t e = allow_lds(reinterpret_cast<const void*>(&count_topk_block_kernel<CAP, LCH, NW>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((count_topk_block_kernel<CAP, LCH, NW>), dim3(grid), dim3(64 * NW), lds, st, a);
  return hipGetLastError();
}

template <int LCH, int NW>
hipError_t launch_block_cap(int cap, const QueryArgs& a, int grid, hipStream_t st) {
  switch (cap) {
    case 8192: return launch_block_kernel<8192, LCH, NW>(a, grid, st);
    case 16384: return launch_block_kernel<16384, LCH, NW>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

template <int NW>
hipError_t launch_block_lch(int cap, const QueryArgs& a, int grid, hipStream_t st) {
  switch ((a.L + 63) / 64) {
    case 1: return launch_block_cap<1, NW>(cap, a, grid, st);
    case 2: return launch_block_cap<2, NW>(cap, a, grid, st);
    case 3: return launch_block_cap<3, NW>(cap, a, grid, st);
    case 4: return launch_block_cap<4, NW>(cap, a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_block_any(int nw, int cap, const QueryArgs& a, int grid, hipStream_t st) {
  switch (nw) {
    case 4: return launch_block_lch<4>(cap, a, grid, st);
    case 8: return launch_block_lch<8>(cap, a, grid, st);
    case 16: return launch_block_lch<16>(cap, a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// Supported table size at or below v (powers of two, 1024 .. 16384).
int supported_cap(int v) {
  int c = 1024;
  while (c < 16384 && 2 * c <= v) c <<= 1;
  return c;
}

}  // namespace

size_t query_ws_bytes(const Cfg&, int64_t n_queries) {
  const uint64_t q = (uint64_t)(n_queries > 0 ? n_queries : 1);
  return 2 * align256(4 * q) + align256(16);
}

QueryWs query_ws_carve(const Cfg&, int64_t n_queries, void* ws) {
  const uint64_t q = (uint64_t)(n_queries > 0 ? n_queries : 1);
  QueryWs w;
  w.ovf_list[0] = (uint32_t*)ws;
  w.ovf_list[1] = (uint32_t*)((char*)ws + align256(4 * q));
  w.ovf_len = (uint32_t*)((char*)ws + 2 * align256(4 * q));
  return w;
}

// Query stages: each launch takes the queries whose candidate total fits its
// table at <= 3/4 load (the last takes every query) and hands the rest on.
hipError_t launch_query(const Cfg& c, const int32_t* index,
                        int64_t n_indexed, int64_t n_queries, const uint32_t* qkeys,
                        const int32_t* self_ids, int self_mode, int32_t k, const int32_t* k_per_query,
                        int32_t* out_ids, int32_t* out_counts, const QueryWs& w, hipStream_t st) {
  if (n_queries <= 0) return hipSuccess;
  QueryArgs a = {};
  a.index = index;
  a.S = c.S;
  a.qkeys = qkeys;
  a.self_ids = self_ids;
  a.out_ids = out_ids;
  a.out_counts = out_counts;
  a.n_queries = n_queries;
  a.n_indexed = n_indexed > 0 ? n_indexed : 1;
  a.M = c.M;
  a.L = c.L;
  a.R = c.R;
  a.k = k;
  a.shared = c.shared ? 1 : 0;
  a.s_r = c.s_r;
  a.P = c.P;
  a.self_mode = self_mode;
  a.k_per_query = k_per_query;
  a.cbits = 32 - __builtin_clz((unsigned)c.L + 1u);

  const uint32_t full = (uint32_t)c.L * (uint32_t)c.R;  // most candidates a query can have
  uint32_t last = 1024;
  while (last < 2 * full) last <<= 1;                   // table that takes any query at load 1/2
  const Tuning tu = tuning();
  // When the index holds at least R arrivals per bucket on average, its
  // buckets are nearly all full and nearly every query brings about L * R
  // candidates: a stage whose table cannot take that many would only hand
  // its queries on, so it is left out.
  const double per_bucket = c.shared ? (double)n_indexed * (double)c.L / (double)c.P
                                     : (double)n_indexed / (double)c.M;
  const bool skip_small = tu.query_skip_full != 0 && per_bucket >= (double)c.R;
  int caps[3];
  int n_stage = 0;
  // first and second table sizes (0: no such stage), rounded to a supported size
  for (int v : {tu.query_cap1, tu.query_cap2}) {
    if (v <= 0) continue;
    const int cap = supported_cap(v);
    if ((uint32_t)cap >= last) break;
    if (skip_small && (uint32_t)cap * 3 / 4 < full) continue;
    if (n_stage == 0 || cap > caps[n_stage - 1]) caps[n_stage++] = cap;
  }
  caps[n_stage++] = (int)last;
  // the last stage runs as one workgroup of NW waves per query when its table is large
  const int nw = (last >= 8192 && tu.query_big_waves > 1) ? tu.query_big_waves : 1;

  const int cus = device_info().cus;
  const int per_cu = tu.query_blocks_per_cu > 0 ? tu.query_blocks_per_cu : 512;
  // the filter stage goes first unless every query is sure to exceed it
  // (full buckets with more than its 2048 candidates)
  const bool filter = tu.query_filter != 0 && !(skip_small && full > kFastCap);
  const int first = filter ? 1 : 0;   // stage index of the first counting-table stage
  hipError_t e;
  if ((n_stage + first) > 1 && (e = launch_fill_u32(w.ovf_len, 4, 0u, st)) != hipSuccess) return e;
  if (filter) {
    QueryArgs b = a;
    b.ovf_list = w.ovf_list[0];
    b.ovf_len = w.ovf_len;
    const int64_t want = (int64_t)cus * per_cu;
    if ((e = launch_fast_any(b, (int)(n_queries < want ? n_queries : want), st)) != hipSuccess) return e;
  }
  for (int s = first; s < n_stage + first; ++s) {
    QueryArgs b = a;
    const int cs = s - first;   // index into caps
    const bool final_stage = s == n_stage + first - 1;
    b.max_total = final_stage ? full : (uint32_t)caps[cs] * 3 / 4;
    const uint32_t need_sb = (uint32_t)k + slack_for((uint32_t)k);
    b.sb = need_sb < b.max_total ? need_sb : (b.max_total > (uint32_t)k ? b.max_total : (uint32_t)k);
    b.sb = (b.sb + 3) & ~3u;  // keeps tinfo 16-byte aligned
    if (s > 0) {
      b.qlist = w.ovf_list[(s - 1) & 1];
      b.qlist_len = w.ovf_len + ((s - 1) & 1);
    }
    if (!final_stage) {
      b.ovf_list = w.ovf_list[s & 1];
      b.ovf_len = w.ovf_len + (s & 1);
      // the list this stage fills was last read by the stage before
      if (s >= 2 && (e = launch_fill_u32(w.ovf_len + (s & 1), 1, 0u, st)) != hipSuccess) return e;
    }
    if (final_stage && nw > 1) {
      // as many workgroups as fit on the CUs at once (LDS and 32 waves per CU)
      const size_t lds = block_smem_bytes(caps[cs], c.L, b.sb, nw);
      int per = (int)((160 * 1024) / lds);
      if (per > 32 / nw) per = 32 / nw;
      if (per < 1) per = 1;
      const int64_t want = (int64_t)cus * per;
      const int grid = (int)(n_queries < want ? n_queries : want);
      if ((e = launch_block_any(nw, caps[cs], b, grid, st)) != hipSuccess) return e;
      continue;
    }
    int64_t want = (int64_t)cus * per_cu;
    if (s > 0) want = (int64_t)cus * 8;
    const int grid = (int)(n_queries < want ? n_queries : want);
    if ((e = launch_any(caps[cs], b, grid, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace flashk
