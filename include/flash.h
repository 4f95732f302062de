/*
 * flash.h — C ABI of the FLASH hot path for AMD Instinct MI355X (gfx950).
 *
 * FLASH (Wang, Shrivastava, Wang & Ryu, arXiv 1709.01190) answers k-nearest-
 * neighbour queries over ultra-sparse binary rows with three data-parallel
 * steps: densified one-permutation minwise hashing (paper Sec. 2.3), L hash
 * tables of fixed-size reservoirs (Sec. 2.4, Sec. 3.2 item 2, Alg. 1-2) and
 * count-based top-k selection over the L buckets a query hits (Sec. 3.2
 * item 3, Alg. 3).
 *
 * Conventions for every entry point:
 *  - All array pointers are DEVICE pointers (hipMalloc'd or torch CUDA
 *    tensors) unless a comment says "host".  The caller owns every buffer;
 *    the library never allocates device memory.  Scratch space is a
 *    caller-provided workspace of at least flash_workspace_bytes() bytes,
 *    256-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls only enqueue work and return; outputs are valid once the stream
 *    has been synchronised.  Calls that share a workspace must be ordered on
 *    one stream.
 *  - Return value: FLASH_OK (0) or a negative FLASH_E* code.  On error nothing
 *    has been enqueued (argument errors) or the HIP error is reported
 *    (FLASH_EHIP); flash_last_error() gives a message for the calling thread.
 *  - CSR input: row_ptr int64[n_rows + 1] and col_idx int32[nnz] with
 *    nnz = row_ptr[n_rows] passed explicitly.  Columns are read as unsigned
 *    32-bit ids; order inside a row is free and duplicates count once (binary
 *    set semantics, Sec. 2.1); float values are not taken.  Row bounds are
 *    clamped to [0, nnz] on the device, so a malformed row_ptr cannot read
 *    outside col_idx (such a row is hashed as whatever lies in its clamped
 *    range, possibly empty).
 *  - Index layout (Sec. 3.5: memory O(L * R * Range)): one device array
 *    `index`, int32[P][S], 16-byte aligned, holding the P = L * M reservoirs
 *    (M = 2^(K * bits_per_hash); reservoir t * M + m is bucket m of table t)
 *    S words apart, S = R + 4 rounded up to a multiple of 32 (128 bytes;
 *    flash_index_layout gives P and S).  Word 0 of a reservoir is its
 *    header: the number of rows whose key in table t is m (an unsigned
 *    32-bit count stored in the int32 word).  Words 1..3 are reserved and
 *    never read.  Words 4 .. 4 + min(count, R) - 1 hold the kept row ids in
 *    ascending reservoir priority; later words are not part of the index
 *    and hold anything.  The header and the first 28 slots share one
 *    128-byte line, so a query's visit to a small bucket reads one line.
 *    With shared reservoirs (flash_params.share_permille) P is the pool.
 *    Every call that takes `index` refuses a pointer that is not 16-byte
 *    aligned (FLASH_EINVAL).  FLASH_INDEX_LAYOUT names this layout; layout
 *    1 (separate counts uint32[P] and ids int32[P][R] arrays) is gone.
 */
#ifndef FLASH_H
#define FLASH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define FLASH_API __attribute__((visibility("default")))
#else
#define FLASH_API
#endif

#define FLASH_OK 0
#define FLASH_EINVAL (-1)   /* invalid argument or parameter */
#define FLASH_ENOSPC (-2)   /* workspace (or an output) too small */
#define FLASH_EHIP (-3)     /* HIP runtime / launch error */
#define FLASH_ENOTIMPL (-4) /* parameters outside what the kernels support */
#define FLASH_ERANGE (-5)   /* a column id outside [0, n_cols) (flash_validate_csr) */

/* Version of the index layout described above. */
#define FLASH_INDEX_LAYOUT 2

/* Key of an empty row or query in every table (never inserted). */
#define FLASH_EMPTY_KEY 0xFFFFFFFFu

/* Method parameters (Sec. 2.2, Sec. 4.4.1, Sec. 3.5).  Limits checked by
 * every call: 1 <= K, 1 <= L <= 256, 1 <= bits_per_hash, K * bits_per_hash
 * <= 30, K * L <= 4096 (DOPH bins), 1 <= R <= 1024, L * R <= 8192,
 * L * 2^(K * b) < 2^32, 0 <= densify_attempts <= 65535,
 * 0 <= share_permille <= 1000.
 *
 * Reservoir sharing (Sec. 3.5: F is the ratio of the reservoirs allocated to
 * the bucket range they serve): with 0 < share_permille < 1000,
 * F = share_permille / 1000 and the index has P = ceil(F * L * M)
 * reservoirs (at least one); bucket m of table t uses reservoir
 * floor(fmix32((t * M + m) ^ s_r) * P / 2^32), a seeded random map (s_r:
 * the fourth splitmix64 output of `seed`), so buckets of any tables may share
 * one.  A reservoir keeps its R lowest-priority arrivals, with priorities
 * keyed by the reservoir instead of the table; a query aggregates the
 * reservoirs of its L buckets and counts occurrences.  0 or 1000: no
 * sharing, P = L * M and reservoir t * M + m. */
typedef struct flash_params {
    int32_t K;                /* minhashes per table key (meta-hash width)      */
    int32_t L;                /* number of hash tables                          */
    int32_t bits_per_hash;    /* b: low bits of each minhash kept in a key      */
    int32_t R;                /* reservoir capacity per bucket                  */
    uint64_t seed;            /* expands to the permutation, densification and
                                 reservoir-priority seeds                       */
    int32_t densify_attempts; /* random probes per empty DOPH bin (default 64)  */
    int32_t share_permille;   /* reservoir sharing F in thousandths; 0: none    */
} flash_params;

/* Workspace users, for flash_workspace_bytes(). */
#define FLASH_OP_HASH 0       /* flash_hash: needs none                          */
#define FLASH_OP_INSERT 1     /* flash_insert_keys                               */
#define FLASH_OP_BUILD 2      /* flash_build_index                               */
#define FLASH_OP_QUERY_KEYS 3 /* flash_query_keys                                */
#define FLASH_OP_QUERY 4      /* flash_query_batch                               */
#define FLASH_OP_KNN_GRAPH 5  /* flash_knn_graph                                 */

/* Host only.  0 if *p is within the limits above, else FLASH_EINVAL or
 * FLASH_ENOTIMPL with a message in flash_last_error(). */
FLASH_API int flash_check_params(const flash_params *p);

/* Host only.  Shape of the index array: *reservoirs = P (L * M without
 * reservoir sharing), *stride_words = S (words per reservoir) and
 * *words = P * S, its length in int32 elements.  Any output may be NULL. */
FLASH_API int flash_index_layout(const flash_params *p, uint64_t *reservoirs, uint32_t *stride_words,
                                 uint64_t *words);

/* Host only.  Workspace bytes needed by operation `op` for n_rows indexed rows
 * (insert/build/graph) or n_queries queries (query ops) and k results per
 * query.  Unused sizes may be 0. */
FLASH_API int flash_workspace_bytes(int op, const flash_params *p, int64_t n_rows,
                                    int64_t n_queries, int32_t k, size_t *bytes);

/* Optional validation pass over a CSR batch.  The rows are subsets of
 * {0, ..., D-1} (Sec. 2.1, D = n_cols); the hot-path calls neither check
 * that nor need it (any int32 id is hashed, row pointers are clamped into
 * [0, nnz]), so this pass is for callers that cannot vouch for their input.
 * Clears the caller-owned device word *flags (uint32), then ORs into it
 *   FLASH_CSR_BAD_COLUMN   a column id < 0 or >= n_cols;
 *   FLASH_CSR_BAD_ROW_PTR  row_ptr[0] != 0, row_ptr[n_rows] != nnz, a row
 *                          pointer outside [0, nnz], or one that decreases.
 * Asynchronous on `stream` (no memset node: the clear is a fill kernel).
 * Read *flags after the stream has synchronised and pass it to
 * flash_csr_status.  row_ptr int64[n_rows + 1], col_idx int32[nnz], both
 * device pointers; n_cols >= 1.  FLASH_EINVAL for bad sizes or NULL arrays. */
#define FLASH_CSR_BAD_COLUMN 1u
#define FLASH_CSR_BAD_ROW_PTR 2u
FLASH_API int flash_validate_csr(int64_t n_rows, int64_t nnz, int64_t n_cols, const int64_t *row_ptr,
                                 const int32_t *col_idx, uint32_t *flags, void *stream);

/* Host only.  The status of a flags word written by flash_validate_csr:
 * FLASH_EINVAL if the row pointers are malformed, else FLASH_ERANGE if a
 * column is out of range, else FLASH_OK. */
FLASH_API int flash_csr_status(uint32_t flags);

/* Sec. 2.3 (DOPH) + Sec. 2.2 / Alg. 2 line 5 (MapKHashesToAddress).
 * For each CSR row i: the K*L densified one-permutation minhashes and the L
 * table keys keys[i][t] (uint32[n_rows][L], FLASH_EMPTY_KEY for an empty row).
 * codes (uint32[n_rows][K*L]) is written only if not NULL. */
FLASH_API int flash_hash(const flash_params *p, int64_t n_rows, int64_t nnz,
                         const int64_t *row_ptr, const int32_t *col_idx, uint32_t *keys,
                         uint32_t *codes, void *stream);

/* Alg. 2 (adding phase) with Alg. 1's reservoir read as bottom-R priority
 * sampling.  Clears the index, then adds row i (id i, 0 <= i < n_rows) to bucket
 * keys[i][t] of every table t.  Keys that are FLASH_EMPTY_KEY or >= M are
 * skipped.  Requires n_rows * L < 2^32 and n_rows < 2^31.  The tables are
 * bit-identical for any launch order or configuration. */
FLASH_API int flash_insert_keys(const flash_params *p, int64_t n_rows, const uint32_t *keys,
                                int32_t *index, void *workspace,
                                size_t workspace_bytes, void *stream);

/* Alg. 2 (adding phase) from CSR: flash_hash, then flash_insert_keys.  The keys are
 * written to keys_out (uint32[n_rows][L]) if it is not NULL, else kept in the
 * workspace. */
FLASH_API int flash_build_index(const flash_params *p, int64_t n_rows, int64_t nnz,
                                const int64_t *row_ptr, const int32_t *col_idx,
                                int32_t *index, uint32_t *keys_out,
                                void *workspace, size_t workspace_bytes, void *stream);

/* Incremental insertion into a resident index (Sec. 3.2 item 2; Sec. 3.4:
 * rows are added independently).  Adds n_rows rows, given by their keys
 * (device uint32[n_rows][L], as flash_hash writes them), with ids id_base ..
 * id_base + n_rows - 1 to `index`, which already holds rows with other ids
 * (a fresh index: every header zero).  A reservoir keeps the R
 * lowest priorities of its arrivals, so after any sequence of calls the
 * index is bit-identical (headers and occupied slots) to one
 * flash_insert_keys over all rows added, whatever the batching and order.
 * Ids must not repeat across calls (not checked).  0 <= id_base and
 * id_base + n_rows <= 2^32 / 2^ceil(log2(L+2)) (the largest index the
 * query accepts; FLASH_ENOTIMPL otherwise) and < 2^31.  Workspace:
 * FLASH_OP_INSERT for n_rows.  Calls on one index must be ordered on one
 * stream; n_rows = 0 enqueues nothing. */
FLASH_API int flash_insert_keys_append(const flash_params *p, int64_t n_rows, const uint32_t *keys,
                                       int64_t id_base, int32_t *index,
                                       void *workspace, size_t workspace_bytes, void *stream);

/* flash_insert_keys_append from CSR rows: flash_hash into the workspace, then
 * the append.  Workspace: FLASH_OP_BUILD for n_rows. */
FLASH_API int flash_build_index_append(const flash_params *p, int64_t n_rows, int64_t nnz,
                                       const int64_t *row_ptr, const int32_t *col_idx,
                                       int64_t id_base, int32_t *index,
                                       void *workspace, size_t workspace_bytes, void *stream);

/* Alg. 3 (querying phase) from precomputed keys qkeys uint32[n_queries][L].
 * cnt(x) = number of tables whose bucket qkeys[q][t] keeps id x; ids equal to
 * self_ids[q] (if self_ids is not NULL and the entry is >= 0) are left out.
 * out_ids / out_counts (int32[n_queries][k]) get the first k ids by (cnt
 * descending, id ascending), padded with id -1, count 0.  Requires
 * 1 <= k <= 1024, n_queries < 2^31 and
 * n_indexed <= 2^32 / 2^ceil(log2(L+2)) (FLASH_ENOTIMPL otherwise; ids and
 * counts share one 32-bit word in the query's table).  Every id stored in
 * the index must be < n_indexed (not checked: a larger id may be dropped or
 * corrupted in the lists). */
FLASH_API int flash_query_keys(const flash_params *p, const int32_t *index,
                               int64_t n_indexed, int64_t n_queries, const uint32_t *qkeys,
                               const int32_t *self_ids, int32_t k, int32_t *out_ids,
                               int32_t *out_counts, void *workspace, size_t workspace_bytes,
                               void *stream);

/* Alg. 3 (querying phase) from CSR queries: flash_hash of the queries into the
 * workspace, then flash_query_keys. */
FLASH_API int flash_query_batch(const flash_params *p, const int32_t *index,
                                int64_t n_indexed, int64_t n_queries, int64_t nnz,
                                const int64_t *q_row_ptr, const int32_t *q_col_idx,
                                const int32_t *self_ids, int32_t k, int32_t *out_ids,
                                int32_t *out_counts, void *workspace, size_t workspace_bytes,
                                void *stream);

/* For callers that cannot allocate device memory at all (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation and arguments as flash_query_batch, without the workspace.  Its
 * scratch (the query keys, stage lists and counters) lives in a fixed area
 * owned by the library, flash_noalloc_scratch_bytes() bytes (32 MiB) on each
 * device it runs on, held until the process ends; nothing is allocated by
 * this call.  A batch whose flash_workspace_bytes(FLASH_OP_QUERY) exceeds
 * that size is refused with FLASH_ENOSPC before anything is enqueued (about
 * 246,000 queries at L = 32, 127,000 at L = 64).  Every call on one device
 * shares that device's area: calls that overlap on one device (other
 * streams, other threads) race and give wrong results, so order them on one
 * stream.  The area's first use on a device looks its address up once. */
FLASH_API int flash_query_batch_noalloc(const flash_params *p, const int32_t *index,
                                        int64_t n_indexed, int64_t n_queries,
                                        int64_t nnz, const int64_t *q_row_ptr,
                                        const int32_t *q_col_idx, const int32_t *self_ids, int32_t k,
                                        int32_t *out_ids, int32_t *out_counts, void *stream);

/* Host only.  Size of the fixed scratch area of flash_query_batch_noalloc. */
FLASH_API size_t flash_noalloc_scratch_bytes(void);

/* Alg. 3 for a batch whose queries want different k (batched uneven
 * queries).  As flash_query_keys, except that query q returns its first
 * k_per_query[q] ids (device int32[n_queries]; values are clamped to
 * [1, k_max]) and its output row, of stride k_max, is padded with (-1, 0)
 * after them.  1 <= k_max <= 1024.  Workspace: FLASH_OP_QUERY_KEYS. */
FLASH_API int flash_query_keys_mixed(const flash_params *p, const int32_t *index,
                                     int64_t n_indexed, int64_t n_queries,
                                     const uint32_t *qkeys, const int32_t *self_ids,
                                     const int32_t *k_per_query, int32_t k_max, int32_t *out_ids,
                                     int32_t *out_counts, void *workspace, size_t workspace_bytes,
                                     void *stream);

/* flash_query_batch with a k per query: CSR queries are hashed into the
 * workspace, then answered as flash_query_keys_mixed.  Workspace:
 * FLASH_OP_QUERY. */
FLASH_API int flash_query_batch_mixed(const flash_params *p, const int32_t *index,
                                      int64_t n_indexed, int64_t n_queries,
                                      int64_t nnz, const int64_t *q_row_ptr,
                                      const int32_t *q_col_idx, const int32_t *self_ids,
                                      const int32_t *k_per_query, int32_t k_max, int32_t *out_ids,
                                      int32_t *out_counts, void *workspace, size_t workspace_bytes,
                                      void *stream);

/* Sec. 1 / Sec. 4.3: approximate k-NN graph.  Builds the index of all rows
 * into `index`, then queries every row with its own keys, leaving the row
 * itself out. */
FLASH_API int flash_knn_graph(const flash_params *p, int64_t n_rows, int64_t nnz,
                              const int64_t *row_ptr, const int32_t *col_idx, int32_t k,
                              int32_t *index, int32_t *out_ids,
                              int32_t *out_counts, void *workspace, size_t workspace_bytes,
                              void *stream);

#define FLASH_SIM_COSINE 0  /* Eq. 3: |x ∩ y| / sqrt(|x| |y|) */
#define FLASH_SIM_JACCARD 1 /* Eq. 2's right-hand side: |x ∩ y| / |x ∪ y| */

/* Exact re-rank (Sec. 4.3: the exact similarity is the accuracy gold
 * standard; S@k averages it over the top k).  For each query row q of the
 * CSR q_row_ptr / q_col_idx (n_queries rows, q_nnz columns) and its
 * candidates cand_ids[q][0..n_cand) (ids of rows of the indexed CSR
 * row_ptr / col_idx, n_indexed rows, nnz columns; ids < 0 or >= n_indexed
 * are no candidate): the intersection |q ∩ x| is counted exactly, the
 * candidates are ordered by `measure` (FLASH_SIM_*) descending, compared
 * exactly in integers, ties by the smaller id, and the first k are written:
 * out_ids[q][0..k) and out_inter[q][0..k) (int32), padded with (-1, 0).
 * The similarity follows from the intersection and the two row lengths.
 * Rows must hold distinct column ids (duplicates would be counted twice);
 * order inside a row is free.  1 <= k <= n_cand <= 1024.  Needs no
 * workspace. */
FLASH_API int flash_rerank_exact(int measure, int64_t n_indexed, int64_t nnz, const int64_t *row_ptr,
                                 const int32_t *col_idx, int64_t n_queries, int64_t q_nnz,
                                 const int64_t *q_row_ptr, const int32_t *q_col_idx,
                                 const int32_t *cand_ids, int32_t n_cand, int32_t k, int32_t *out_ids,
                                 int32_t *out_inter, void *stream);

/* Launch shapes (process-wide).  No field changes any result: they only
 * move the same work between launches, workgroups and waves.  A value of
 * 0 in a field marked "0 = ..." has that meaning; reserved must be 0. */
typedef struct flash_tuning {
    int32_t query_cap1;          /* LDS table entries of the first query stage (queries with at
                                    most 3/4 of it in candidates); 0 = no such stage, else
                                    1024..16384, rounded down to a power of two.  Default 2048 */
    int32_t query_cap2;          /* the same for the second stage; default 4096 */
    int32_t query_blocks_per_cu; /* one-wave workgroups per CU in the first stage, 1..1024;
                                    default 512 */
    int32_t query_big_waves;     /* waves per workgroup that share one query in the last stage
                                    when its table has >= 8192 entries: 1, 4, 8 or 16; default 8 */
    int32_t hash_tile_rows;      /* flash_query_batch*: 0 = static row stride; else each wave
                                    takes tiles of this many rows from a work counter,
                                    1..65536; default 0 */
    int32_t query_skip_full;     /* 1 = when the index averages at least R arrivals per bucket
                                    (n_indexed >= R * M, or R * P / L when shared), leave out
                                    the stages whose table holds fewer than L * R candidates;
                                    0 = always run the stages above; default 1 */
    int32_t query_filter;        /* 1 = first run every query through the filter stage: one wave
                                    keeps its <= 2048 candidates in registers, a 32K-bit LDS
                                    filter finds the ids that may repeat, only those are counted
                                    exactly, and the smallest ids of count 1 are picked by a radix
                                    select; queries it cannot finish (more candidates, more than
                                    128 suspected repeats, or k ids of count >= 2) go on to the
                                    counting-table stages.  It is left out when full buckets give
                                    every query more than 2048 candidates.  0 = counting-table
                                    stages only; default 1 */
    int32_t reserved;
} flash_tuning;

/* Current tuning (host struct). */
FLASH_API int flash_get_tuning(flash_tuning *out);

/* Replaces the tuning (host struct; NULL restores the defaults).  Values are
 * checked as documented above (FLASH_EINVAL).  Launches already enqueued
 * keep the shape they were enqueued with. */
FLASH_API int flash_set_tuning(const flash_tuning *t);

/* Autotuner for a batch of (uneven) CSR queries: runs the batch as
 * flash_query_batch_mixed (k_per_query may be NULL: k_max for all) under a
 * fixed list of candidate tunings, one field at a time (coordinate descent),
 * timing each run with HIP events on `stream`, keeps the fastest (the least
 * of `reps` runs, 1..20), installs it with flash_set_tuning and copies it to
 * *best (host) and its time to *best_ms (host, may be NULL).  Unlike every
 * other entry point it blocks: it synchronises `stream` after each run.
 * The outputs hold the batch's result (the same for every candidate).
 * Arguments as flash_query_batch_mixed; workspace FLASH_OP_QUERY.  On error
 * the previous tuning is restored. */
FLASH_API int flash_autotune_query_batch(const flash_params *p, const int32_t *index,
                                         int64_t n_indexed, int64_t n_queries,
                                         int64_t nnz, const int64_t *q_row_ptr,
                                         const int32_t *q_col_idx, const int32_t *self_ids,
                                         const int32_t *k_per_query, int32_t k_max,
                                         int32_t *out_ids, int32_t *out_counts, void *workspace,
                                         size_t workspace_bytes, int32_t reps, void *stream,
                                         flash_tuning *best, float *best_ms);

/* Text for a FLASH_* code (static storage). */
FLASH_API const char *flash_strerror(int code);

/* Detail of the last error on the calling thread ("" if none). */
FLASH_API const char *flash_last_error(void);

/* Library version string. */
FLASH_API const char *flash_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FLASH_H */
