// Densified one-permutation minwise hashing (paper Sec. 2.3) and the table
// keys of Sec. 2.2 ("MapKHashesToAddress"), one wavefront per CSR row.
//
// Per row the wave
//   1. reads the row's column ids (one per lane for rows of at most 256,
//      else 16-byte loads with the unaligned ends one per lane), hashes each
//      id with the permutation pi(i) = fmix32(i ^ s_h), and keeps the minimum
//      per bin with an LDS atomic min; bins are the B equal slices of the
//      permuted range;
//   2. builds the occupancy bitmask with ballots (one 64-bit ballot per 64
//      bins) and, when B <= 256, an occupancy byte per bin;
//   3. fills every empty bin from an originally occupied one: up to A probes
//      at bins given by fmix32(((j << 16) | a) ^ s_d), then the nearest
//      occupied bin to the right (cyclic).  The probe bins depend only on the
//      bin and the seed, so when B <= 256 each lane keeps its bins' first
//      eight as bytes in registers and tests them all at once;
//   4. writes the L keys (K low-b-bit fields each) and, if asked, the B codes.
// HBM traffic per row: 4 B per nonzero + 16 B of row_ptr + 4 L B of keys
// (+ 4 B bytes of codes).
#include "launch.hpp"

namespace flashk {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct HashArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  uint32_t* keys;
  uint32_t* codes;
  int64_t n_rows;
  int64_t nnz;
  uint32_t s_h, s_d;
  int B, K, L, b, A;
  uint32_t mask;
  int shift;  // 32 - log2(B) when B is a power of two
  uint32_t* tile_ctr;  // dynamic schedule's work counter (null: static)
  int64_t tile_rows;
};

template <bool POW2>
__device__ __forceinline__ void add_column(const HashArgs& a, uint32_t col, uint32_t* mins,
                                           uint32_t* top_bin) {
  const uint32_t h = fmix32(col ^ a.s_h);
  const uint32_t bin = POW2 ? (a.shift >= 32 ? 0u : (h >> a.shift)) : __umulhi(h, (uint32_t)a.B);
  // exactly one column id maps to 0xFFFFFFFF; its bin is remembered so that
  // occupancy never relies on a sentinel value
  if (h == kEmpty) *top_bin = bin;
  atomicMin(&mins[bin], h);
}

__device__ __forceinline__ bool occupied(const uint32_t* occw, uint32_t j) {
  return (occw[j >> 5] >> (j & 31)) & 1u;
}

// Densification probe t (1-based) of bin j: a bin given by fmix32 of (j, t).
__device__ __forceinline__ uint32_t probe_bin(const HashArgs& a, uint32_t j, uint32_t t) {
  return __umulhi(fmix32(((j << 16) | t) ^ a.s_d), (uint32_t)a.B);
}

// Source bin of empty bin j from probe t_first on: probes t_first..A, then
// the nearest occupied bin to the right (cyclically).  The row has at least
// one occupied bin.
__device__ __forceinline__ uint32_t probe_from(const HashArgs& a, const uint32_t* occw, uint32_t j,
                                               int t_first) {
  for (int t = t_first; t <= a.A; ++t) {
    const uint32_t p = probe_bin(a, j, (uint32_t)t);
    if (occupied(occw, p)) return p;
  }
  const uint32_t nwords = ((uint32_t)a.B + 31) >> 5;
  const uint32_t s0 = j + 1 == (uint32_t)a.B ? 0u : j + 1;
  uint32_t w = s0 >> 5;
  uint32_t bits = occw[w] & (0xFFFFFFFFu << (s0 & 31));
  while (bits == 0) {
    w = w + 1 == nwords ? 0 : w + 1;
    bits = occw[w];
  }
  return w * 32 + (uint32_t)(__ffs(bits) - 1);
}

// Bins of at most kPreBins (PRE): each lane owns bins lane + 64 r, r < 4,
// and holds their first kPreProbes probe bins as bytes in registers, worked
// out once per wave; they depend on the bin and the seed only.
constexpr int kPreRounds = 4;
constexpr int kPreProbes = 8;
constexpr int kPreBins = kPreRounds * kWave;  // 256: a bin fits a byte
struct ProbeTable {
  uint32_t w[kPreRounds][kPreProbes / 4];
};

__device__ __forceinline__ ProbeTable make_probe_table(const HashArgs& a) {
  ProbeTable pt;
  const uint32_t lane = threadIdx.x;
#pragma unroll
  for (int r = 0; r < kPreRounds; ++r) {
    const uint32_t j = (uint32_t)r * kWave + lane;
#pragma unroll
    for (int q = 0; q < kPreProbes / 4; ++q) {
      uint32_t w = 0;
      if (j < (uint32_t)a.B)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int t = q * 4 + i + 1;
          if (t <= a.A) w |= probe_bin(a, j, (uint32_t)t) << (8 * i);
        }
      pt.w[r][q] = w;
    }
  }
  return pt;
}

// Hashes one row with the whole wave.  LDS: mins[B] bin minima, occw[B/32]
// occupancy bits; with PRE also occ8[256], one occupancy byte per bin.
// row_ptr[next] and row_ptr[next + 1] (next >= 0), one per lane 0 and 1: a
// vector load, so that waiting for the row's columns waits for it too.
__device__ __forceinline__ int64_t load_row_bounds(const HashArgs& a, int64_t next) {
  return next >= 0 ? a.row_ptr[next + (threadIdx.x & 1)] : 0;
}

// Lane l's value of a 64-bit register.
__device__ __forceinline__ int64_t lane64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Hashes row `row`.  PF: its bounds (beg, end) were loaded a row ahead, and
// the bounds of row `next` (-1: none) are loaded into `bounds` before the
// row's columns; else the row loads its own bounds first.
template <bool POW2, bool PRE, bool PF>
__device__ __forceinline__ void hash_row(const HashArgs& a, int64_t row, int64_t beg, int64_t end, int64_t next,
                                         int64_t& bounds, uint32_t* mins, uint32_t* occw, uint8_t* occ8,
                                         const ProbeTable& pt, uint32_t& top_bin) {
  const uint32_t lane = threadIdx.x;
  const int B = a.B;
  const int nwords = (B + 31) >> 5;
  if (PF) {
    bounds = load_row_bounds(a, next);
  } else {
    beg = a.row_ptr[row];
    end = a.row_ptr[row + 1];
  }
  beg = beg < 0 ? 0 : (beg > a.nnz ? a.nnz : beg);
  end = end < beg ? beg : (end > a.nnz ? a.nnz : end);

  for (int j = lane; j < B; j += kWave) mins[j] = kEmpty;
  if (lane == 0) top_bin = kEmpty;
  __syncthreads();

  if (beg == end) {  // empty row: all keys and codes are the empty marker
    for (int t = lane; t < a.L; t += kWave) a.keys[row * a.L + t] = kEmpty;
    if (a.codes)
      for (int j = lane; j < B; j += kWave) a.codes[row * B + j] = kEmpty;
    __syncthreads();
    return;
  }

  // 1. bin minima
  if (end - beg <= 4 * kWave) {
    // short row: one column id per lane and round, up to four rounds in flight
    const int32_t* rp = a.col_idx + beg;
    const uint32_t nn = (uint32_t)(end - beg);
    uint32_t x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (lane + kWave * u < nn) x[u] = (uint32_t)__builtin_nontemporal_load(rp + lane + kWave * u);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (lane + kWave * u < nn) add_column<POW2>(a, x[u], mins, &top_bin);
  } else {
    // long row: 16-byte loads between the first and last aligned element
    // positions a0, a1; the unaligned ends one element per lane
    const uintptr_t mis = ((uintptr_t)a.col_idx >> 2) & 3;  // element misalignment vs 16 B
    int64_t a0 = beg + (int64_t)((4 - ((uint64_t)(beg + mis) & 3)) & 3);
    int64_t a1 = end - (int64_t)((uint64_t)(end + mis) & 3);
    if (a0 >= a1) {
      a0 = end;
      a1 = end;
    }
    {
      const int64_t e = beg + lane;
      if (e < a0) add_column<POW2>(a, (uint32_t)a.col_idx[e], mins, &top_bin);
      const int64_t f = a1 + lane;
      if (f < end) add_column<POW2>(a, (uint32_t)a.col_idx[f], mins, &top_bin);
    }
    const int64_t nvec = (a1 - a0) >> 2;
    const u32x4* vp = reinterpret_cast<const u32x4*>(a.col_idx + a0);
    constexpr int U = 8;
    for (int64_t v = lane; v < nvec; v += (int64_t)kWave * U) {
      u32x4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t idx = v + (int64_t)kWave * u;
        if (idx < nvec) x[u] = __builtin_nontemporal_load(vp + idx);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t idx = v + (int64_t)kWave * u;
        if (idx < nvec) {
          add_column<POW2>(a, x[u].x, mins, &top_bin);
          add_column<POW2>(a, x[u].y, mins, &top_bin);
          add_column<POW2>(a, x[u].z, mins, &top_bin);
          add_column<POW2>(a, x[u].w, mins, &top_bin);
        }
      }
    }
  }
  __syncthreads();

  // 2. occupancy: bits (ballots) and, with PRE, bytes; own bins' in `own`
  const uint32_t tb = top_bin;
  uint32_t own = 0;
  for (int j0 = 0; j0 < B; j0 += kWave) {
    const uint32_t j = (uint32_t)j0 + lane;
    const bool o = j < (uint32_t)B && (mins[j] != kEmpty || j == tb);
    const uint64_t m = __ballot(o);
    if (PRE) {
      if (j < (uint32_t)B) occ8[j] = (uint8_t)o;
      own |= (uint32_t)o << (j0 / kWave);
    }
    if (lane == 0) {
      occw[j0 >> 5] = (uint32_t)m;
      if ((j0 >> 5) + 1 < nwords) occw[(j0 >> 5) + 1] = (uint32_t)(m >> 32);
    }
  }
  __syncthreads();

  // 3. densification: only empty bins are written and only occupied bins
  // are read, so bins can be filled in place.
  if (PRE) {
    // the first kPreProbes probes of a bin are read all at once; the first
    // occupied one is the source, else the probes go on from kPreProbes + 1
    const uint32_t tmask = a.A >= kPreProbes ? (1u << kPreProbes) - 1u : (1u << a.A) - 1u;
    const int rounds = (B + kWave - 1) / kWave;
#pragma unroll 1
    for (int r = 0; r < rounds; ++r) {
      const uint32_t j = (uint32_t)r * kWave + lane;
      // the table words of bins r * 64 + lane (r is the same in every lane)
      const uint32_t w0 = r == 0 ? pt.w[0][0] : r == 1 ? pt.w[1][0] : r == 2 ? pt.w[2][0] : pt.w[3][0];
      const uint32_t w1 = r == 0 ? pt.w[0][1] : r == 1 ? pt.w[1][1] : r == 2 ? pt.w[2][1] : pt.w[3][1];
      if (j < (uint32_t)B && !((own >> r) & 1u)) {
        uint32_t hits = 0;
#pragma unroll
        for (int t = 0; t < kPreProbes; ++t)
          hits |= (uint32_t)occ8[__builtin_amdgcn_ubfe(t < 4 ? w0 : w1, (t & 3) * 8, 8)] << t;
        hits &= tmask;
        uint32_t src;
        if (hits) {
          const uint32_t t = (uint32_t)(__ffs(hits) - 1);
          src = __builtin_amdgcn_ubfe(t < 4 ? w0 : w1, (t & 3) * 8, 8);
        } else {
          src = probe_from(a, occw, j, kPreProbes + 1);
        }
        mins[j] = mins[src];
      }
    }
  } else {
    for (int j = lane; j < B; j += kWave) {
      if (occupied(occw, (uint32_t)j)) continue;
      mins[j] = mins[probe_from(a, occw, (uint32_t)j, 1)];
    }
  }
  __syncthreads();

  // 4. keys (and codes)
  for (int t = lane; t < a.L; t += kWave) {
    uint32_t key = 0;
    for (int j = 0; j < a.K; ++j) key |= (mins[t * a.K + j] & a.mask) << (a.b * j);
    a.keys[row * a.L + t] = key;
  }
  if (a.codes)
    for (int j = lane; j < B; j += kWave) a.codes[row * B + j] = mins[j];
  __syncthreads();
}

// Static schedule: wave w hashes rows w, w + grid, ...  Dynamic schedule
// (for batches of very uneven rows): each wave takes tiles of tile_rows
// consecutive rows from a work counter until the tiles run out.  Launch
// bounds for six waves per SIMD (at most 80 VGPRs).  PF: row bounds loaded a
// row ahead, which pays on long rows (their wait is not hidden by other work
// of the row) and costs a few instructions per row on short ones.
template <bool POW2, bool PRE, bool PF>
__global__ __launch_bounds__(64, 6) void doph_hash_kernel(HashArgs a) {
  extern __shared__ uint32_t lds[];
  uint8_t* occ8 = reinterpret_cast<uint8_t*>(lds);  // [256] (PRE)
  uint32_t* mins = lds + (PRE ? kPreBins / 4 : 0);  // [B]
  uint32_t* occw = mins + a.B;                       // [ceil(B / 32)]
  __shared__ uint32_t top_bin;
  ProbeTable pt = {};
  if (PRE) pt = make_probe_table(a);
  if (a.tile_ctr) {
    for (;;) {
      uint32_t t = 0;
      if (threadIdx.x == 0) t = atomicAdd(a.tile_ctr, 1u);
      t = (uint32_t)__builtin_amdgcn_readlane((int)t, 0);
      const int64_t r0 = (int64_t)t * a.tile_rows;
      if (r0 >= a.n_rows) break;
      const int64_t r1 = r0 + a.tile_rows < a.n_rows ? r0 + a.tile_rows : a.n_rows;
      int64_t bounds = PF ? load_row_bounds(a, r0) : 0;
      for (int64_t row = r0; row < r1; ++row) {
        const int64_t beg = PF ? lane64(bounds, 0) : 0, end = PF ? lane64(bounds, 1) : 0;
        hash_row<POW2, PRE, PF>(a, row, beg, end, row + 1 < r1 ? row + 1 : -1, bounds, mins, occw, occ8, pt,
                                top_bin);
      }
    }
  } else {
    int64_t bounds = PF ? load_row_bounds(a, blockIdx.x < a.n_rows ? (int64_t)blockIdx.x : -1) : 0;
    for (int64_t row = blockIdx.x; row < a.n_rows; row += gridDim.x) {
      const int64_t beg = PF ? lane64(bounds, 0) : 0, end = PF ? lane64(bounds, 1) : 0;
      const int64_t next = row + gridDim.x < a.n_rows ? row + gridDim.x : -1;
      hash_row<POW2, PRE, PF>(a, row, beg, end, next, bounds, mins, occw, occ8, pt, top_bin);
    }
  }
}

}  // namespace

hipError_t launch_doph_hash(const Cfg& c, int64_t n_rows, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col_idx, uint32_t* keys, uint32_t* codes,
                            uint32_t* tile_ctr, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  HashArgs a;
  a.row_ptr = row_ptr;
  a.col_idx = col_idx;
  a.keys = keys;
  a.codes = codes;
  a.n_rows = n_rows;
  a.nnz = nnz;
  a.s_h = c.seeds.s_h;
  a.s_d = c.seeds.s_d;
  a.B = c.B;
  a.K = c.K;
  a.L = c.L;
  a.b = c.b;
  a.A = c.A;
  a.mask = c.mask;
  const bool pow2 = (c.B & (c.B - 1)) == 0;
  a.shift = pow2 ? 32 - (31 - __builtin_clz((unsigned)c.B)) : 0;
  const bool pre = c.B <= kPreBins;
  const size_t lds = sizeof(uint32_t) * ((size_t)c.B + (size_t)((c.B + 31) / 32)) + (pre ? kPreBins : 0);
  // row bounds a row ahead when the rows average at least 256 ids
  const bool pf = nnz >= 256 * n_rows;
  const void* const kernels[8] = {
      (const void*)doph_hash_kernel<false, false, false>, (const void*)doph_hash_kernel<false, false, true>,
      (const void*)doph_hash_kernel<false, true, false>,  (const void*)doph_hash_kernel<false, true, true>,
      (const void*)doph_hash_kernel<true, false, false>,  (const void*)doph_hash_kernel<true, false, true>,
      (const void*)doph_hash_kernel<true, true, false>,   (const void*)doph_hash_kernel<true, true, true>};
  const void* kern = kernels[(pow2 ? 4 : 0) + (pre ? 2 : 0) + (pf ? 1 : 0)];
  // as many one-wave blocks as fit the chip at once: with the static stride
  // every block then starts at launch and no block runs behind the rest
  const int64_t want = (int64_t)device_info().cus * resident_blocks(kern, lds);
  const int grid = (int)(n_rows < want ? n_rows : want);
  const int tile = tuning().hash_tile_rows;
  a.tile_ctr = tile > 0 ? tile_ctr : nullptr;
  a.tile_rows = tile > 0 ? tile : 1;
  if (a.tile_ctr) {
    const hipError_t e = launch_fill_u32(a.tile_ctr, 1, 0u, s);
    if (e != hipSuccess) return e;
  }
  void* args[] = {&a};
  const hipError_t e = hipLaunchKernel(kern, dim3(grid), dim3(64), args, lds, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace flashk
