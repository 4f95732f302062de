// Internal launch interface between the kernel files and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flash_device.hpp"

namespace flashk {

// Derived, validated parameters shared by all launches.
struct Cfg {
  int K, L, b, R, B, A;
  uint32_t M;      // buckets per table, 2^(K*b)
  uint32_t mask;   // 2^b - 1
  Seeds seeds;
  bool shared;     // reservoirs shared through a seeded map (Sec. 3.5)
  uint32_t s_r;    // seed of that map
  uint64_t P;      // reservoirs: L * M, or the shared pool
  uint32_t S;      // words per reservoir in the index: header + R slots, rounded up to 128 bytes
};

// Reservoir layout in the index: word 0 holds the arrival count, words 1..3
// are reserved, slot i is word kSlot0 + i; reservoirs are S words apart.
constexpr uint32_t kSlot0 = 4;
inline uint32_t reservoir_words(int R) { return ((uint32_t)R + kSlot0 + 31u) & ~31u; }

// Reservoir of bucket m of table t (see flash.h, flash_params).
__host__ __device__ __forceinline__ uint64_t reservoir_of(bool shared, uint32_t s_r, uint64_t P, uint32_t M,
                                                          uint32_t t, uint32_t m) {
  if (!shared) return (uint64_t)t * M + m;
  return ((uint64_t)fmix32_hd(((uint32_t)t * M + m) ^ s_r) * P) >> 32;
}

struct Device {
  int cus = 256;   // compute units of the current device
};
const Device& device_info();

// Launch-shape choices; none of them changes any result.  Process-wide.
struct Tuning {
  int query_cap1 = 2048;          // first query stage's table entries (0: no such stage)
  int query_cap2 = 4096;          // second stage's (0: none)
  int query_blocks_per_cu = 512;  // first-stage blocks per CU
  int query_big_waves = 8;        // waves per workgroup in a last stage of >= 8192 entries (1: one wave)
  int hash_tile_rows = 0;         // 0: static row stride; else rows per tile taken from a work counter
  int query_skip_full = 1;        // leave out stages too small for L * R candidates when buckets are full
  int query_filter = 1;           // run the filter stage (ids of count 1 told apart without a counting table) first
};
Tuning tuning();

// ---- hash (doph_hash.hip)
// tile_ctr: a device word for the dynamic schedule (may be null: static stride)
hipError_t launch_doph_hash(const Cfg& c, int64_t n_rows, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col_idx, uint32_t* keys, uint32_t* codes,
                            uint32_t* tile_ctr, hipStream_t s);

// ---- insert (reservoir_insert.hip)
struct InsertWs {
  uint32_t* keys_t;     // [L][np]        table-major keys (rows padded to 64)
  int32_t* staged;      // [n_rows * L]   row ids grouped by bucket
  uint32_t* part;       // [L * M * S]    arrivals per (bucket, row slice)       (one-level partition)
  uint32_t* partoff;    // [L * M * S]    exclusive prefix of part
  uint32_t* ent;        // [L][tiles][8192] tile entries sorted by chunk           (two-level partition)
  uint32_t* tile_off;   // [L][tiles][chunks + 1] chunk offsets in each tile
  uint32_t* chunk_tot;  // [L * chunks]   arrivals per chunk
  uint32_t* chunk_base; // [L * chunks]   their first staged slot
  uint32_t* seg;        // [L * M]        first staged slot of each bucket
  uint32_t* newcnt;     // [L * M]        the batch's arrivals per bucket
  uint4* work;          // [L * M]        {bucket, start, size} of the large buckets
  uint32_t* tile_sums;  // [tiles + 1]    scan carries
  uint32_t* wl_len;     // [2]
};
size_t insert_ws_bytes(const Cfg& c, int64_t n_rows);
InsertWs insert_ws_carve(const Cfg& c, int64_t n_rows, void* ws);
// Rows of this batch get ids id_base + row.  append: merge into the
// reservoirs and counts already in ids/counts (else they are replaced).
hipError_t launch_insert(const Cfg& c, int64_t n_rows, const uint32_t* keys, uint32_t id_base, bool append,
                         int32_t* index, const InsertWs& w, hipStream_t s);

// ---- query (count_topk.hip)
struct QueryWs {
  uint32_t* ovf_list[2];  // [n_queries] each: queries handed on to the next (larger) table
  uint32_t* ovf_len;      // [4]
};
size_t query_ws_bytes(const Cfg& c, int64_t n_queries);
QueryWs query_ws_carve(const Cfg& c, int64_t n_queries, void* ws);
// self_mode: 0 = none, 1 = self_ids array, 2 = query index is its own id
hipError_t launch_query(const Cfg& c, const int32_t* index,
                        int64_t n_indexed, int64_t n_queries, const uint32_t* qkeys,
                        const int32_t* self_ids, int self_mode, int32_t k, const int32_t* k_per_query,
                        int32_t* out_ids, int32_t* out_counts, const QueryWs& w, hipStream_t s);

// ---- exact re-rank (rerank.hip); measure 0 = cosine, 1 = Jaccard
hipError_t launch_rerank(int measure, int64_t n_indexed, int64_t nnz, const int64_t* row_ptr,
                         const int32_t* col_idx, int64_t n_queries, int64_t q_nnz, const int64_t* q_row_ptr,
                         const int32_t* q_col_idx, const int32_t* cand, int32_t n_cand, int32_t k,
                         int32_t* out_ids, int32_t* out_inter, hipStream_t s);

// ---- CSR validation (validate.hip): clears *flags, then ORs the
// FLASH_CSR_* bits of what it finds
hipError_t launch_validate_csr(int64_t n_rows, int64_t nnz, int64_t n_cols, const int64_t* row_ptr,
                               const int32_t* col_idx, uint32_t* flags, hipStream_t s);

// ---- misc
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// p[i * stride] = v for i < n
hipError_t launch_fill_strided_u32(uint32_t* p, uint64_t n, uint32_t stride, uint32_t v, hipStream_t s);

// Lets `kernel` launch with `bytes` of dynamic LDS (above the 64 KiB
// default).  The attribute is set once per kernel and size, not on every
// launch, so launches inside a stream capture issue no such call after the
// first eager one.
hipError_t allow_lds(const void* kernel, size_t bytes);

// One-wave (64-thread) blocks of `kernel` with `lds_bytes` of dynamic LDS
// that one CU holds at once.
int resident_blocks(const void* kernel, size_t lds_bytes);

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace flashk
