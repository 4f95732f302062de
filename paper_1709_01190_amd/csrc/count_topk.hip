// Querying phase (paper Alg. 3, Sec. 3.2 item 3): gather the L reservoirs a
// query hits, count how many of them hold each id, and return the k ids with
// the highest counts (ties: smaller id first).
//
// One wavefront per query:
//   1. lane t reads key t and counts[t][key]; a wave scan gives each table's
//      offset in the flattened candidate list (total = sum of occupancies);
//   2. lanes walk the flattened list (a per-lane table cursor that only moves
//      forward), load ids from HBM four at a time and add them to an LDS
//      open-addressing table whose slot packs (id << cbits | count); the
//      slots touched are recorded so that later passes and the final clear
//      cost O(distinct candidates), not O(table size);
//   3. a histogram of counts gives the threshold count c*; ids with count c*
//      are cut by a radix select on the id (8 bits per pass);
//   4. the k survivors are sorted by (count desc, id asc) with an LDS bitonic
//      sort and written out.
// Queries whose occupancy exceeds half the table go to an overflow list that
// a second launch with a larger table handles.
#include "launch.hpp"

namespace flashk {

namespace {

struct QueryArgs {
  const uint32_t* counts;
  const int32_t* ids;
  const uint32_t* qkeys;
  const int32_t* self_ids;
  int32_t* out_ids;
  int32_t* out_counts;
  const uint32_t* qlist;      // process qlist[0 .. *qlist_len) if not null
  const uint32_t* qlist_len;
  uint32_t* ovf_list;         // spill queries with total > CAP/2 here if not null
  uint32_t* ovf_len;
  int64_t n_queries;
  uint32_t M;
  int L, R, k, self_mode, cbits, top_shift;
  uint32_t ks;                // power of two >= k
};

struct Smem {
  uint64_t* outk;  // [ks]
  uint32_t* tab;   // [CAP]
  uint16_t* used;  // [CAP / 2]
  uint32_t* keysh; // [L]
  uint32_t* pref;  // [L + 1]
  uint32_t* hist;  // [max(L + 1, 256)]
  uint32_t* scal;  // [4]: nused, nout
};

__host__ __device__ inline size_t smem_bytes(int cap, int L, uint32_t ks) {
  const int nh = (L + 1) > 256 ? (L + 1) : 256;
  return (size_t)ks * 8 + (size_t)cap * 4 + (size_t)cap + (size_t)L * 4 + (size_t)(L + 1) * 4 +
         (size_t)nh * 4 + 16;
}

template <int CAP>
__device__ __forceinline__ void count_insert(const Smem& s, uint32_t id, int cbits) {
  constexpr int kLog = __builtin_ctz(CAP);
  uint32_t slot = (id * 0x9E3779B1u) >> (32 - kLog);
  const uint32_t mine = (id << cbits) | 1u;
  while (true) {
    uint32_t cur = s.tab[slot];
    if (cur == kEmpty) {
      cur = atomicCAS(&s.tab[slot], kEmpty, mine);
      if (cur == kEmpty) {
        s.used[atomicAdd(&s.scal[0], 1u)] = (uint16_t)slot;
        return;
      }
    }
    if ((cur >> cbits) == id) {
      atomicAdd(&s.tab[slot], 1u);
      return;
    }
    slot = (slot + 1) & (CAP - 1);
  }
}

template <int CAP>
__global__ __launch_bounds__(64) void count_topk_kernel(QueryArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  Smem s;
  {
    unsigned char* p = smem;
    s.outk = (uint64_t*)p;
    p += (size_t)a.ks * 8;
    s.tab = (uint32_t*)p;
    p += (size_t)CAP * 4;
    s.used = (uint16_t*)p;
    p += (size_t)CAP;
    s.keysh = (uint32_t*)p;
    p += (size_t)a.L * 4;
    s.pref = (uint32_t*)p;
    p += (size_t)(a.L + 1) * 4;
    s.hist = (uint32_t*)p;
    p += (size_t)((a.L + 1) > 256 ? (a.L + 1) : 256) * 4;
    s.scal = (uint32_t*)p;
  }
  const uint32_t lane = threadIdx.x;
  const int L = a.L;
  const uint32_t cmask = (1u << a.cbits) - 1u;
  const uint32_t R = (uint32_t)a.R;
  for (uint32_t i = lane; i < (uint32_t)CAP; i += kWave) s.tab[i] = kEmpty;

  const uint64_t nq = a.qlist ? (uint64_t)*a.qlist_len : (uint64_t)a.n_queries;
  for (uint64_t w = blockIdx.x; w < nq; w += gridDim.x) {
    const uint64_t q = a.qlist ? (uint64_t)a.qlist[w] : w;
    const int64_t self = a.self_mode == 1 ? (int64_t)a.self_ids[q] : (a.self_mode == 2 ? (int64_t)q : -1);

    // 1. occupancy of the L buckets and their offsets
    uint32_t carry = 0;
    for (int t0 = 0; t0 < L; t0 += kWave) {
      const int t = t0 + (int)lane;
      uint32_t nt = 0;
      if (t < L) {
        const uint32_t key = a.qkeys[q * (uint64_t)L + t];
        if (key < a.M) {
          const uint32_t c = a.counts[(uint64_t)t * a.M + key];
          nt = c < R ? c : R;
        }
        s.keysh[t] = key;
      }
      const uint32_t inc = wave_incl_scan(nt);
      if (t < L) s.pref[t] = carry + inc - nt;
      carry += __shfl(inc, kWave - 1, kWave);
    }
    const uint32_t total = carry;
    if (lane == 0) {
      s.pref[L] = total;
      s.scal[0] = 0;
      s.scal[1] = 0;
    }
    __syncthreads();
    if (total > (uint32_t)CAP / 2) {
      if (lane == 0) a.ovf_list[atomicAdd(a.ovf_len, 1u)] = (uint32_t)q;
      __syncthreads();
      continue;
    }

    // 2. gather and count
    {
      uint32_t tc = 0;
      constexpr int U = 4;
      for (uint32_t base = 0; base < total; base += kWave * U) {
        int32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t e = base + lane + kWave * u;
          v[u] = -1;
          if (e < total) {
            while (s.pref[tc + 1] <= e) ++tc;
            const uint64_t bucket = (uint64_t)tc * a.M + s.keysh[tc];
            v[u] = a.ids[bucket * R + (e - s.pref[tc])];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (v[u] >= 0 && (int64_t)v[u] != self) count_insert<CAP>(s, (uint32_t)v[u], a.cbits);
      }
    }
    for (int c = (int)lane; c <= L; c += kWave) s.hist[c] = 0;
    __syncthreads();
    const uint32_t nd = s.scal[0];

    // 3. threshold count c* and tie cut
    for (uint32_t i = lane; i < nd; i += kWave) atomicAdd(&s.hist[s.tab[s.used[i]] & cmask], 1u);
    __syncthreads();
    uint32_t cstar = 0, thr_id = 0xFFFFFFFFu;
    if (nd > (uint32_t)a.k) {
      uint32_t above = 0;  // ids with count > c*
      bool found = false;
      for (int c0 = L; c0 >= 1 && !found; c0 -= kWave) {
        const int c = c0 - (int)lane;
        const uint32_t h = c >= 1 ? s.hist[c] : 0;
        const uint32_t inc = wave_incl_scan(h);
        const uint64_t hit = __ballot(above + inc >= (uint32_t)a.k);
        if (hit) {
          const int f = __ffsll((unsigned long long)hit) - 1;
          cstar = (uint32_t)(c0 - f);
          above += __shfl(inc - h, f, kWave);
          found = true;
        } else {
          above += __shfl(inc, kWave - 1, kWave);
        }
      }
      const uint32_t need = (uint32_t)a.k - above;
      const uint32_t ties = s.hist[cstar];
      __syncthreads();
      if (ties > need) {
        uint32_t prefix = 0, rem = need;  // rem-th smallest tied id (1-based)
        for (int sh = a.top_shift; sh >= 0; sh -= 8) {
          for (uint32_t i = lane; i < 256; i += kWave) s.hist[i] = 0;
          __syncthreads();
          for (uint32_t i = lane; i < nd; i += kWave) {
            const uint32_t vv = s.tab[s.used[i]];
            const uint32_t id = vv >> a.cbits;
            if ((vv & cmask) == cstar && (((uint64_t)(id ^ prefix)) >> (sh + 8)) == 0)
              atomicAdd(&s.hist[(id >> sh) & 255u], 1u);
          }
          __syncthreads();
          const uint32_t h0 = s.hist[4 * lane], h1 = s.hist[4 * lane + 1], h2 = s.hist[4 * lane + 2],
                         h3 = s.hist[4 * lane + 3];
          const uint32_t sum4 = h0 + h1 + h2 + h3;
          const uint32_t inc = wave_incl_scan(sum4);
          const uint64_t hit = __ballot(inc >= rem);
          const int f = __ffsll((unsigned long long)hit) - 1;
          uint32_t cum = __shfl(inc - sum4, f, kWave);
          const uint32_t g0 = __shfl(h0, f, kWave), g1 = __shfl(h1, f, kWave),
                         g2 = __shfl(h2, f, kWave);
          uint32_t d = 4 * (uint32_t)f;
          if (cum + g0 >= rem) {
          } else if (cum + g0 + g1 >= rem) {
            d += 1;
            cum += g0;
          } else if (cum + g0 + g1 + g2 >= rem) {
            d += 2;
            cum += g0 + g1;
          } else {
            d += 3;
            cum += g0 + g1 + g2;
          }
          prefix |= d << sh;
          rem -= cum;
          __syncthreads();
        }
        thr_id = prefix;
      }
    }

    // 4. survivors, sorted by (count desc, id asc)
    for (uint32_t i = lane; i < nd; i += kWave) {
      const uint32_t vv = s.tab[s.used[i]];
      const uint32_t c = vv & cmask, id = vv >> a.cbits;
      if (c > cstar || (c == cstar && id <= thr_id)) {
        const uint32_t pos = atomicAdd(&s.scal[1], 1u);
        if (pos < a.ks) s.outk[pos] = ((uint64_t)(uint32_t)(L - (int)c) << 32) | id;
      }
    }
    __syncthreads();
    const uint32_t m = s.scal[1] < a.ks ? s.scal[1] : a.ks;
    const uint32_t P = pow2_ceil(m);
    for (uint32_t i = m + lane; i < P; i += kWave) s.outk[i] = ~0ull;
    __syncthreads();
    block64_bitonic_sort(s.outk, P);
    for (uint32_t j = lane; j < (uint32_t)a.k; j += kWave) {
      const uint64_t o = q * (uint64_t)a.k + j;
      if (j < m) {
        const uint64_t v = s.outk[j];
        a.out_ids[o] = (int32_t)(uint32_t)v;
        a.out_counts[o] = L - (int32_t)(v >> 32);
      } else {
        a.out_ids[o] = -1;
        a.out_counts[o] = 0;
      }
    }
    // 5. leave the table empty for the next query
    for (uint32_t i = lane; i < nd; i += kWave) s.tab[s.used[i]] = kEmpty;
    __syncthreads();
  }
}

template <int CAP>
hipError_t launch_cap(const QueryArgs& a, int grid, hipStream_t st) {
  const size_t lds = smem_bytes(CAP, a.L, a.ks);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&count_topk_kernel<CAP>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(count_topk_kernel<CAP>, dim3(grid), dim3(64), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_any(int cap, const QueryArgs& a, int grid, hipStream_t st) {
  switch (cap) {
    case 512: return launch_cap<512>(a, grid, st);
    case 1024: return launch_cap<1024>(a, grid, st);
    case 2048: return launch_cap<2048>(a, grid, st);
    case 4096: return launch_cap<4096>(a, grid, st);
    case 8192: return launch_cap<8192>(a, grid, st);
    case 16384: return launch_cap<16384>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v && *v ? atoi(v) : dflt;
}

}  // namespace

size_t query_ws_bytes(const Cfg&, int64_t n_queries) {
  return align256(4 * (uint64_t)(n_queries > 0 ? n_queries : 1)) + align256(4);
}

QueryWs query_ws_carve(const Cfg&, int64_t n_queries, void* ws) {
  QueryWs w;
  w.ovf_list = (uint32_t*)ws;
  w.ovf_len = (uint32_t*)((char*)ws + align256(4 * (uint64_t)(n_queries > 0 ? n_queries : 1)));
  return w;
}

hipError_t launch_query(const Cfg& c, const uint32_t* counts, const int32_t* ids,
                        int64_t n_indexed, int64_t n_queries, const uint32_t* qkeys,
                        const int32_t* self_ids, int self_mode, int32_t k, int32_t* out_ids,
                        int32_t* out_counts, const QueryWs& w, hipStream_t st) {
  if (n_queries <= 0) return hipSuccess;
  QueryArgs a = {};
  a.counts = counts;
  a.ids = ids;
  a.qkeys = qkeys;
  a.self_ids = self_ids;
  a.out_ids = out_ids;
  a.out_counts = out_counts;
  a.n_queries = n_queries;
  a.M = c.M;
  a.L = c.L;
  a.R = c.R;
  a.k = k;
  a.self_mode = self_mode;
  a.cbits = 32 - __builtin_clz((unsigned)c.L + 1u);
  const uint64_t maxid = n_indexed > 1 ? (uint64_t)(n_indexed - 1) : 1;
  const int idbits = 64 - __builtin_clzll(maxid);
  a.top_shift = ((idbits + 7) / 8) * 8 - 8;
  a.ks = 1;
  while (a.ks < (uint32_t)k) a.ks <<= 1;

  const uint32_t full = 2u * (uint32_t)c.L * (uint32_t)c.R;  // table size that never overflows
  uint32_t big = 512;
  while (big < full) big <<= 1;
  int cap = env_int("FLASH_QUERY_CAP", 2048);
  if ((uint32_t)cap > big) cap = (int)big;
  const int cus = device_info().cus;
  const int per_cu = env_int("FLASH_QUERY_BLOCKS_PER_CU", 16);
  const int64_t want = (int64_t)cus * per_cu;
  const int grid = (int)(n_queries < want ? n_queries : want);
  hipError_t e;
  if ((uint32_t)cap >= big) {
    return launch_any(cap, a, grid, st);
  }
  a.ovf_list = w.ovf_list;
  a.ovf_len = w.ovf_len;
  if ((e = launch_fill_u32(w.ovf_len, 1, 0u, st)) != hipSuccess) return e;
  if ((e = launch_any(cap, a, grid, st)) != hipSuccess) return e;
  QueryArgs b = a;
  b.qlist = w.ovf_list;
  b.qlist_len = w.ovf_len;
  b.ovf_list = nullptr;
  b.ovf_len = nullptr;
  return launch_any((int)big, b, cus * 2, st);
}

}  // namespace flashk
