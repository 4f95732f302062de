// Exact re-rank of candidate lists: the paper's accuracy gold standard
// (Sec. 4.3), cosine similarity of binary rows (Eq. 3) or Jaccard (Eq. 2's
// right-hand side), used after the count-based top-k to order its candidates
// by their true similarity.
//
// One workgroup of four waves per query:
//   1. the query's columns go into an LDS hash set, kChunk at a time (longer
//      rows take several rounds, each adding to the intersections);
//   2. the waves take the candidates in turn, stream each candidate's
//      columns with coalesced loads and probe the set; the wave's matches
//      are the candidate's intersection with the chunk;
//   3. the block sorts (id, intersection, size) with a bitonic network in
//      LDS whose comparator compares similarities exactly (cross-multiplied
//      integers) and breaks ties by the smaller id; the first k are written.
#include "launch.hpp"

namespace flashk {

namespace {

constexpr int kRerankThreads = 256;
constexpr uint32_t kSet = 8192;             // LDS hash set slots
constexpr uint32_t kChunk = kSet / 2;        // query columns per round (load <= 1/2)
constexpr uint32_t kMaxCand = 1024;

struct RerankArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const int64_t* q_row_ptr;
  const int32_t* q_col_idx;
  const int32_t* cand;
  int32_t* out_ids;
  int32_t* out_inter;
  int64_t n_indexed, nnz, n_queries, q_nnz;
  int measure, n_cand, k;
};

// Row bounds clamped to [0, nnz].
__device__ __forceinline__ void row_bounds(const int64_t* rp, int64_t nnz, int64_t r, int64_t* b, int64_t* e) {
  int64_t x = rp[r], y = rp[r + 1];
  x = x < 0 ? 0 : (x > nnz ? nnz : x);
  y = y < x ? x : (y > nnz ? nnz : y);
  *b = x;
  *e = y;
}

__device__ __forceinline__ uint32_t set_slot(uint32_t col) {
  return (col * 0x9E3779B1u) >> (32 - __builtin_ctz(kSet));
}

// Entry a ranks before entry b: larger similarity, then smaller id; entries
// without a candidate (id < 0) last.  Similarities are compared exactly:
// Jaccard i / (nq + x - i) by cross-multiplication, cosine i / sqrt(nq x)
// through its square i^2 / (nq x) (nq cancels); no common column means 0.
__device__ __forceinline__ bool before(int measure, uint64_t nq, int32_t ida, uint32_t ia, uint32_t xa,
                                       int32_t idb, uint32_t ib, uint32_t xb) {
  if (ida < 0 || idb < 0) return ida >= 0 && idb < 0;
  bool gt = false, lt = false;
  if (ia == 0 || ib == 0) {
    gt = ia > 0 && ib == 0;
    lt = ib > 0 && ia == 0;
  } else if (measure == 1) {
    const unsigned __int128 l = (unsigned __int128)ia * (nq + xb - ib);
    const unsigned __int128 r = (unsigned __int128)ib * (nq + xa - ia);
    gt = l > r;
    lt = l < r;
  } else {
    const unsigned __int128 l = (unsigned __int128)((uint64_t)ia * ia) * xb;
    const unsigned __int128 r = (unsigned __int128)((uint64_t)ib * ib) * xa;
    gt = l > r;
    lt = l < r;
  }
  return gt || (!lt && ida < idb);
}

__global__ __launch_bounds__(kRerankThreads) void rerank_kernel(RerankArgs a) {
  __shared__ uint32_t set[kSet];
  __shared__ int32_t e_id[kMaxCand];
  __shared__ uint32_t e_in[kMaxCand];
  __shared__ uint32_t e_sz[kMaxCand];
  __shared__ uint32_t has_top;  // the query holds column 0xFFFFFFFF (the empty marker)
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr uint32_t NW = kRerankThreads / 64;
  const uint32_t nc = (uint32_t)a.n_cand;
  uint32_t P = 1;
  while (P < nc) P <<= 1;

  for (int64_t q = blockIdx.x; q < a.n_queries; q += gridDim.x) {
    int64_t qb, qe;
    row_bounds(a.q_row_ptr, a.q_nnz, q, &qb, &qe);
    const uint64_t nq = (uint64_t)(qe - qb);
    for (uint32_t c = tid; c < P; c += kRerankThreads) {
      int32_t id = -1;
      uint32_t sz = 0;
      if (c < nc) {
        id = a.cand[q * (int64_t)nc + c];
        if (id >= 0 && (int64_t)id < a.n_indexed) {
          int64_t b, e;
          row_bounds(a.row_ptr, a.nnz, id, &b, &e);
          sz = (uint32_t)(e - b);
        } else {
          id = -1;
        }
      }
      e_id[c] = id;
      e_in[c] = 0;
      e_sz[c] = sz;
    }
    // 1-2. rounds of up to kChunk query columns
    for (int64_t c0 = qb; c0 < qe || c0 == qb; c0 += kChunk) {
      const int64_t c1 = c0 + kChunk < qe ? c0 + kChunk : qe;
      for (uint32_t i = tid; i < kSet; i += kRerankThreads) set[i] = kEmpty;
      if (tid == 0) has_top = 0;
      __syncthreads();
      for (int64_t i = c0 + tid; i < c1; i += kRerankThreads) {
        const uint32_t col = (uint32_t)a.q_col_idx[i];
        if (col == kEmpty) {
          has_top = 1;
          continue;
        }
        uint32_t s = set_slot(col);
        for (;;) {
          const uint32_t old = atomicCAS(&set[s], kEmpty, col);
          if (old == kEmpty || old == col) break;
          s = (s + 1) & (kSet - 1);
        }
      }
      __syncthreads();
      const bool top = has_top != 0;
      for (uint32_t c = wv; c < nc; c += NW) {
        const int32_t id = e_id[c];
        if (id < 0) continue;
        int64_t b, e;
        row_bounds(a.row_ptr, a.nnz, id, &b, &e);
        uint32_t hit = 0;
        for (int64_t i = b + lane; i < e; i += 64) {
          const uint32_t col = (uint32_t)a.col_idx[i];
          if (col == kEmpty) {
            hit += top;
            continue;
          }
          uint32_t s = set_slot(col);
          for (;;) {
            const uint32_t v = set[s];
            if (v == col) {
              ++hit;
              break;
            }
            if (v == kEmpty) break;
            s = (s + 1) & (kSet - 1);
          }
        }
        hit = wave_sum(hit);
        if (lane == 0) e_in[c] += hit;
      }
      __syncthreads();
      if (c1 >= qe) break;
    }
    // 3. bitonic sort of the P entries by the exact comparator
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
      for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
        for (uint32_t i = tid; i < P; i += kRerankThreads) {
          const uint32_t ixj = i ^ j;
          if (ixj > i) {
            const bool up = (i & kk) == 0;
            const bool swap = up ? before(a.measure, nq, e_id[ixj], e_in[ixj], e_sz[ixj], e_id[i], e_in[i], e_sz[i])
                                 : before(a.measure, nq, e_id[i], e_in[i], e_sz[i], e_id[ixj], e_in[ixj], e_sz[ixj]);
            if (swap) {
              const int32_t ti = e_id[i];
              const uint32_t tn = e_in[i], ts = e_sz[i];
              e_id[i] = e_id[ixj];
              e_in[i] = e_in[ixj];
              e_sz[i] = e_sz[ixj];
              e_id[ixj] = ti;
              e_in[ixj] = tn;
              e_sz[ixj] = ts;
            }
          }
        }
        __syncthreads();
      }
    }
    for (uint32_t j = tid; j < (uint32_t)a.k; j += kRerankThreads) {
      const int32_t id = e_id[j];
      a.out_ids[q * (int64_t)a.k + j] = id;
      a.out_inter[q * (int64_t)a.k + j] = id >= 0 ? (int32_t)e_in[j] : 0;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_rerank(int measure, int64_t n_indexed, int64_t nnz, const int64_t* row_ptr,
                         const int32_t* col_idx, int64_t n_queries, int64_t q_nnz, const int64_t* q_row_ptr,
                         const int32_t* q_col_idx, const int32_t* cand, int32_t n_cand, int32_t k,
                         int32_t* out_ids, int32_t* out_inter, hipStream_t s) {
  if (n_queries <= 0) return hipSuccess;
  RerankArgs a;
  a.row_ptr = row_ptr;
  a.col_idx = col_idx;
  a.q_row_ptr = q_row_ptr;
  a.q_col_idx = q_col_idx;
  a.cand = cand;
  a.out_ids = out_ids;
  a.out_inter = out_inter;
  a.n_indexed = n_indexed;
  a.nnz = nnz;
  a.n_queries = n_queries;
  a.q_nnz = q_nnz;
  a.measure = measure;
  a.n_cand = n_cand;
  a.k = k;
  const int64_t want = (int64_t)device_info().cus * 3;
  const int grid = (int)(n_queries < want ? n_queries : want);
  hipLaunchKernelGGL(rerank_kernel, dim3(grid), dim3(kRerankThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace flashk
