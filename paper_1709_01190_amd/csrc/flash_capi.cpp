// C ABI of the FLASH hot path: argument checks, workspace carving and kernel
// launches on the caller's stream.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "flash.h"
#include "launch.hpp"

namespace flashk {

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(FLASH_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

int make_cfg(const flash_params* p, Cfg* c) {
  if (!p) return fail(FLASH_EINVAL, "params is NULL");
  if (p->share_permille < 0 || p->share_permille > 1000)
    return fail(FLASH_EINVAL, "share_permille must be in [0, 1000]");
  if (p->K < 1 || p->L < 1 || p->bits_per_hash < 1 || p->R < 1)
    return fail(FLASH_EINVAL, "K, L, bits_per_hash and R must be >= 1");
  if (p->L > 256) return fail(FLASH_ENOTIMPL, "L > 256 is not supported");
  if ((int64_t)p->K * p->bits_per_hash > 30)
    return fail(FLASH_EINVAL, "K * bits_per_hash must be <= 30");
  if ((int64_t)p->K * p->L > 4096) return fail(FLASH_ENOTIMPL, "K * L > 4096 bins is not supported");
  if (p->R > 1024) return fail(FLASH_ENOTIMPL, "R > 1024 is not supported");
  if ((int64_t)p->L * p->R > 8192) return fail(FLASH_ENOTIMPL, "L * R > 8192 is not supported");
  if (((uint64_t)p->L << (p->K * p->bits_per_hash)) > 0xFFFFFFFFull)
    return fail(FLASH_ENOTIMPL, "L * 2^(K * bits_per_hash) buckets must be < 2^32");
  if (p->densify_attempts < 0 || p->densify_attempts > 65535)
    return fail(FLASH_EINVAL, "densify_attempts must be in [0, 65535]");
  c->K = p->K;
  c->L = p->L;
  c->b = p->bits_per_hash;
  c->R = p->R;
  c->S = reservoir_words(p->R);
  c->B = p->K * p->L;
  c->A = p->densify_attempts;
  c->M = 1u << (p->K * p->bits_per_hash);
  c->mask = (1u << p->bits_per_hash) - 1u;
  c->seeds = expand_seed(p->seed);
  c->s_r = c->seeds.s_r;
  const uint64_t LM = (uint64_t)c->L * c->M;
  c->shared = p->share_permille > 0 && p->share_permille < 1000;
  c->P = LM;
  if (c->shared) {
    // Sec. 3.5: F = allocated / served reservoirs, so the pool serving all
    // L * M buckets holds ceil(F * L * M) of them (at least one)
    const uint64_t P = (LM * (uint64_t)p->share_permille + 999) / 1000;
    c->P = P < 1 ? 1 : P;
  }
  return FLASH_OK;
}

int check_rows(const Cfg& c, int64_t n_rows, bool for_insert) {
  if (n_rows < 0) return fail(FLASH_EINVAL, "n_rows must be >= 0");
  if (for_insert) {
    if (n_rows >= (int64_t)1 << 31) return fail(FLASH_EINVAL, "n_rows must be < 2^31");
    if ((uint64_t)n_rows * (uint64_t)c.L >= (uint64_t)1 << 32)
      return fail(FLASH_EINVAL, "n_rows * L must be < 2^32");
  }
  return FLASH_OK;
}

int check_csr(int64_t n_rows, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx) {
  if (nnz < 0) return fail(FLASH_EINVAL, "nnz must be >= 0");
  if (n_rows > 0 && !row_ptr) return fail(FLASH_EINVAL, "row_ptr is NULL");
  if (nnz > 0 && !col_idx) return fail(FLASH_EINVAL, "col_idx is NULL");
  return FLASH_OK;
}

int check_query(const Cfg& c, int64_t n_indexed, int64_t n_queries, int32_t k) {
  if (n_queries < 0 || n_indexed < 0) return fail(FLASH_EINVAL, "sizes must be >= 0");
  if (n_queries >= ((int64_t)1 << 31)) return fail(FLASH_ENOTIMPL, "n_queries must be < 2^31");
  if (k < 1 || k > 1024) return fail(FLASH_EINVAL, "k must be in [1, 1024]");
  const int cbits = 32 - __builtin_clz((unsigned)c.L + 1u);
  if (n_indexed > ((int64_t)1 << (32 - cbits)))
    return fail(FLASH_ENOTIMPL, "too many indexed rows for the packed (id, count) query table");
  return FLASH_OK;
}

size_t keys_bytes(const Cfg& c, int64_t n) { return align256(4 * (uint64_t)n * (uint64_t)c.L); }

int check_index(const int32_t* index) {
  if (!index) return fail(FLASH_EINVAL, "index is NULL");
  if (((uintptr_t)index & 15) != 0) return fail(FLASH_EINVAL, "index must be 16-byte aligned");
  return FLASH_OK;
}

}  // namespace

const Device& device_info() {
  static Device infos[64];
  static bool have[64] = {};
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  if (!have[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      infos[dev].cus = cus;
    have[dev] = true;
  }
  return infos[dev];
}

int resident_blocks(const void* kernel, size_t lds_bytes) {
  // cached per (kernel, LDS bytes, device); past 64 triples it is asked again
  static std::mutex mu;
  static const void* kern[64];
  static size_t size[64];
  static int devs[64], val[64];
  static int n = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < n; ++i)
      if (kern[i] == kernel && size[i] == lds_bytes && devs[i] == dev) return val[i];
  }
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, 64, lds_bytes) != hipSuccess || blocks < 1)
    blocks = 8;
  std::lock_guard<std::mutex> lock(mu);
  if (n < 64) {
    kern[n] = kernel;
    size[n] = lds_bytes;
    devs[n] = dev;
    val[n] = blocks;
    ++n;
  }
  return blocks;
}

hipError_t allow_lds(const void* kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  // the attribute is per (kernel, device); past 64 pairs it is simply set again
  static std::mutex mu;
  static const void* kern[64];
  static int devs[64];
  static size_t size[64];
  static int n = 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < n; ++i)
    if (kern[i] == kernel && devs[i] == dev && size[i] >= bytes) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i)
    if (kern[i] == kernel && devs[i] == dev) {
      size[i] = bytes;
      return hipSuccess;
    }
  if (n < 64) {
    kern[n] = kernel;
    devs[n] = dev;
    size[n] = bytes;
    ++n;
  }
  return hipSuccess;
}

std::mutex g_tuning_mu;
Tuning g_tuning;

Tuning tuning() {
  std::lock_guard<std::mutex> lock(g_tuning_mu);
  return g_tuning;
}

}  // namespace flashk

using namespace flashk;

namespace {

int tuning_from_c(const flash_tuning* t, Tuning* out) {
  if (!t) {
    *out = Tuning();
    return FLASH_OK;
  }
  if (t->reserved)
    return fail(FLASH_EINVAL, "tuning.reserved must be 0");
  for (int v : {t->query_cap1, t->query_cap2})
    if (v != 0 && (v < 1024 || v > 16384)) return fail(FLASH_EINVAL, "query caps must be 0 or in [1024, 16384]");
  if (t->query_blocks_per_cu < 1 || t->query_blocks_per_cu > 1024)
    return fail(FLASH_EINVAL, "query_blocks_per_cu must be in [1, 1024]");
  const int w = t->query_big_waves;
  if (w != 1 && w != 4 && w != 8 && w != 16) return fail(FLASH_EINVAL, "query_big_waves must be 1, 4, 8 or 16");
  if (t->hash_tile_rows < 0 || t->hash_tile_rows > 65536)
    return fail(FLASH_EINVAL, "hash_tile_rows must be in [0, 65536]");
  if (t->query_skip_full != 0 && t->query_skip_full != 1) return fail(FLASH_EINVAL, "query_skip_full must be 0 or 1");
  if (t->query_filter != 0 && t->query_filter != 1) return fail(FLASH_EINVAL, "query_filter must be 0 or 1");
  out->query_cap1 = t->query_cap1;
  out->query_cap2 = t->query_cap2;
  out->query_blocks_per_cu = t->query_blocks_per_cu;
  out->query_big_waves = t->query_big_waves;
  out->hash_tile_rows = t->hash_tile_rows;
  out->query_skip_full = t->query_skip_full;
  out->query_filter = t->query_filter;
  return FLASH_OK;
}

flash_tuning tuning_to_c(const Tuning& t) {
  flash_tuning o = {};
  o.query_cap1 = t.query_cap1;
  o.query_cap2 = t.query_cap2;
  o.query_blocks_per_cu = t.query_blocks_per_cu;
  o.query_big_waves = t.query_big_waves;
  o.hash_tile_rows = t.hash_tile_rows;
  o.query_skip_full = t.query_skip_full;
  o.query_filter = t.query_filter;
  return o;
}

void install_tuning(const Tuning& t) {
  std::lock_guard<std::mutex> lock(g_tuning_mu);
  g_tuning = t;
}

}  // namespace

extern "C" {

FLASH_API int flash_check_params(const flash_params* p) {
  Cfg c;
  return make_cfg(p, &c);
}

FLASH_API int flash_index_layout(const flash_params* p, uint64_t* reservoirs, uint32_t* stride_words,
                                 uint64_t* words) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if (reservoirs) *reservoirs = c.P;
  if (stride_words) *stride_words = c.S;
  if (words) *words = c.P * (uint64_t)c.S;
  return FLASH_OK;
}

FLASH_API int flash_workspace_bytes(int op, const flash_params* p, int64_t n_rows, int64_t n_queries,
                                    int32_t k, size_t* bytes) {
  (void)k;
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if (!bytes) return fail(FLASH_EINVAL, "bytes is NULL");
  if (n_rows < 0 || n_queries < 0) return fail(FLASH_EINVAL, "sizes must be >= 0");
  size_t b = 0;
  switch (op) {
    case FLASH_OP_HASH: b = 0; break;
    case FLASH_OP_INSERT: b = insert_ws_bytes(c, n_rows); break;
    case FLASH_OP_BUILD: b = keys_bytes(c, n_rows) + insert_ws_bytes(c, n_rows); break;
    case FLASH_OP_QUERY_KEYS: b = query_ws_bytes(c, n_queries); break;
    case FLASH_OP_QUERY: b = keys_bytes(c, n_queries) + query_ws_bytes(c, n_queries); break;
    case FLASH_OP_KNN_GRAPH: {
      const size_t ins = insert_ws_bytes(c, n_rows), qry = query_ws_bytes(c, n_rows);
      b = keys_bytes(c, n_rows) + (ins > qry ? ins : qry);
      break;
    }
    default: return fail(FLASH_EINVAL, "unknown op");
  }
  *bytes = b;
  return FLASH_OK;
}

FLASH_API int flash_validate_csr(int64_t n_rows, int64_t nnz, int64_t n_cols, const int64_t* row_ptr,
                                 const int32_t* col_idx, uint32_t* flags, void* stream) {
  if (n_rows < 0) return fail(FLASH_EINVAL, "n_rows must be >= 0");
  if (n_cols < 1) return fail(FLASH_EINVAL, "n_cols must be >= 1");
  if (!row_ptr) return fail(FLASH_EINVAL, "row_ptr is NULL");
  int r = check_csr(n_rows, nnz, row_ptr, col_idx);
  if (r) return r;
  if (!flags) return fail(FLASH_EINVAL, "flags is NULL");
  hipError_t e = launch_validate_csr(n_rows, nnz, n_cols, row_ptr, col_idx, flags, (hipStream_t)stream);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "validate_csr");
}

FLASH_API int flash_csr_status(uint32_t flags) {
  if (flags & FLASH_CSR_BAD_ROW_PTR) return fail(FLASH_EINVAL, "malformed row pointers");
  if (flags & FLASH_CSR_BAD_COLUMN) return fail(FLASH_ERANGE, "a column id is outside [0, n_cols)");
  return FLASH_OK;
}

FLASH_API int flash_hash(const flash_params* p, int64_t n_rows, int64_t nnz, const int64_t* row_ptr,
                         const int32_t* col_idx, uint32_t* keys, uint32_t* codes, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_rows(c, n_rows, false))) return r;
  if ((r = check_csr(n_rows, nnz, row_ptr, col_idx))) return r;
  if (n_rows > 0 && !keys) return fail(FLASH_EINVAL, "keys is NULL");
  hipError_t e = launch_doph_hash(c, n_rows, nnz, row_ptr, col_idx, keys, codes, nullptr, (hipStream_t)stream);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "doph_hash");
}

FLASH_API int flash_insert_keys(const flash_params* p, int64_t n_rows, const uint32_t* keys,
                                int32_t* index, void* workspace,
                                size_t workspace_bytes, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_rows(c, n_rows, true))) return r;
  if ((r = check_index(index))) return r;
  if (n_rows > 0 && !keys) return fail(FLASH_EINVAL, "NULL array");
  const size_t need = insert_ws_bytes(c, n_rows);
  if (!workspace || workspace_bytes < need)
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_INSERT)");
  const InsertWs w = insert_ws_carve(c, n_rows, workspace);
  hipError_t e = launch_insert(c, n_rows, keys, 0u, false, index, w, (hipStream_t)stream);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "reservoir_insert");
}

namespace {

int check_append(const Cfg& c, int64_t n_rows, int64_t id_base) {
  if (id_base < 0) return fail(FLASH_EINVAL, "id_base must be >= 0");
  if (n_rows < 0) return fail(FLASH_EINVAL, "n_rows must be >= 0");
  if (id_base + n_rows > ((int64_t)1 << 31) - 1) return fail(FLASH_EINVAL, "id_base + n_rows must be < 2^31");
  const int cbits = 32 - __builtin_clz((unsigned)c.L + 1u);
  if (id_base + n_rows > ((int64_t)1 << (32 - cbits)))
    return fail(FLASH_ENOTIMPL, "ids beyond what the query's packed (id, count) table holds");
  if ((uint64_t)n_rows * (uint64_t)c.L >= (uint64_t)1 << 32)
    return fail(FLASH_EINVAL, "n_rows * L must be < 2^32");
  return FLASH_OK;
}

}  // namespace

FLASH_API int flash_insert_keys_append(const flash_params* p, int64_t n_rows, const uint32_t* keys,
                                       int64_t id_base, int32_t* index, void* workspace,
                                       size_t workspace_bytes, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_append(c, n_rows, id_base))) return r;
  if ((r = check_index(index))) return r;
  if (n_rows > 0 && !keys) return fail(FLASH_EINVAL, "NULL array");
  const size_t need = insert_ws_bytes(c, n_rows);
  if (n_rows > 0 && (!workspace || workspace_bytes < need))
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_INSERT)");
  if (n_rows == 0) return FLASH_OK;
  const InsertWs w = insert_ws_carve(c, n_rows, workspace);
  hipError_t e = launch_insert(c, n_rows, keys, (uint32_t)id_base, true, index, w, (hipStream_t)stream);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "reservoir_insert");
}

FLASH_API int flash_build_index_append(const flash_params* p, int64_t n_rows, int64_t nnz,
                                       const int64_t* row_ptr, const int32_t* col_idx, int64_t id_base,
                                       int32_t* index, void* workspace,
                                       size_t workspace_bytes, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_append(c, n_rows, id_base))) return r;
  if ((r = check_csr(n_rows, nnz, row_ptr, col_idx))) return r;
  if ((r = check_index(index))) return r;
  const size_t kb = keys_bytes(c, n_rows);
  const size_t need = kb + insert_ws_bytes(c, n_rows);
  if (n_rows > 0 && (!workspace || workspace_bytes < need))
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_BUILD)");
  if (n_rows == 0) return FLASH_OK;
  hipStream_t s = (hipStream_t)stream;
  uint32_t* keys = (uint32_t*)workspace;
  hipError_t e = launch_doph_hash(c, n_rows, nnz, row_ptr, col_idx, keys, nullptr, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "doph_hash");
  e = launch_insert(c, n_rows, keys, (uint32_t)id_base, true, index, insert_ws_carve(c, n_rows, (char*)workspace + kb),
                    s);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "reservoir_insert");
}

FLASH_API int flash_build_index(const flash_params* p, int64_t n_rows, int64_t nnz,
                                const int64_t* row_ptr, const int32_t* col_idx, int32_t* index,
                                uint32_t* keys_out, void* workspace,
                                size_t workspace_bytes, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_rows(c, n_rows, true))) return r;
  if ((r = check_csr(n_rows, nnz, row_ptr, col_idx))) return r;
  if ((r = check_index(index))) return r;
  const size_t kb = keys_bytes(c, n_rows);
  const size_t need = kb + insert_ws_bytes(c, n_rows);
  if (!workspace || workspace_bytes < need)
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_BUILD)");
  uint32_t* keys = keys_out ? keys_out : (uint32_t*)workspace;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_doph_hash(c, n_rows, nnz, row_ptr, col_idx, keys, nullptr, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "doph_hash");
  const InsertWs w = insert_ws_carve(c, n_rows, (char*)workspace + kb);
  e = launch_insert(c, n_rows, keys, 0u, false, index, w, s);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "reservoir_insert");
}

FLASH_API int flash_query_keys(const flash_params* p, const int32_t* index,
                               int64_t n_indexed, int64_t n_queries, const uint32_t* qkeys,
                               const int32_t* self_ids, int32_t k, int32_t* out_ids,
                               int32_t* out_counts, void* workspace, size_t workspace_bytes,
                               void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_query(c, n_indexed, n_queries, k))) return r;
  if (n_queries > 0 && (r = check_index(index))) return r;
  if (n_queries > 0 && (!qkeys || !out_ids || !out_counts))
    return fail(FLASH_EINVAL, "NULL array");
  const size_t need = query_ws_bytes(c, n_queries);
  if (!workspace || workspace_bytes < need)
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_QUERY_KEYS)");
  const QueryWs w = query_ws_carve(c, n_queries, workspace);
  hipError_t e = launch_query(c, index, n_indexed, n_queries, qkeys, self_ids, self_ids ? 1 : 0,
                              k, nullptr, out_ids, out_counts, w, (hipStream_t)stream);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "count_topk");
}

FLASH_API int flash_query_batch(const flash_params* p, const int32_t* index,
                                int64_t n_indexed, int64_t n_queries, int64_t nnz,
                                const int64_t* q_row_ptr, const int32_t* q_col_idx,
                                const int32_t* self_ids, int32_t k, int32_t* out_ids,
                                int32_t* out_counts, void* workspace, size_t workspace_bytes,
                                void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_query(c, n_indexed, n_queries, k))) return r;
  if ((r = check_csr(n_queries, nnz, q_row_ptr, q_col_idx))) return r;
  if (n_queries > 0 && (r = check_index(index))) return r;
  if (n_queries > 0 && (!out_ids || !out_counts))
    return fail(FLASH_EINVAL, "NULL array");
  const size_t kb = keys_bytes(c, n_queries);
  const size_t need = kb + query_ws_bytes(c, n_queries);
  if (!workspace || workspace_bytes < need)
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_QUERY)");
  hipStream_t s = (hipStream_t)stream;
  uint32_t* qkeys = (uint32_t*)workspace;
  // the query workspace's spare word 2 counts the hash tiles (dynamic schedule)
  const QueryWs w = query_ws_carve(c, n_queries, (char*)workspace + kb);
  hipError_t e = launch_doph_hash(c, n_queries, nnz, q_row_ptr, q_col_idx, qkeys, nullptr, w.ovf_len + 2, s);
  if (e != hipSuccess) return hip_fail(e, "doph_hash");
  e = launch_query(c, index, n_indexed, n_queries, qkeys, self_ids, self_ids ? 1 : 0, k,
                   nullptr, out_ids, out_counts, w, s);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "count_topk");
}

}  // extern "C"

namespace {

// Library-owned scratch of flash_query_batch_noalloc: query keys, the stage
// lists and their counters, carved exactly as that call's workspace.  Every
// device holds its own copy; host code reaches it only through the address
// hipGetSymbolAddress reports for the current device.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on the current device (looked up once per
// device), or null with *err set.
void* scratch_address(hipError_t* err) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  if (dev < 0 || dev >= 64) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    addr[dev] = p;
  }
  return addr[dev];
}

}  // namespace

extern "C" {

FLASH_API size_t flash_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

FLASH_API int flash_query_batch_noalloc(const flash_params* p, const int32_t* index,
                                        int64_t n_indexed, int64_t n_queries, int64_t nnz,
                                        const int64_t* q_row_ptr, const int32_t* q_col_idx,
                                        const int32_t* self_ids, int32_t k, int32_t* out_ids,
                                        int32_t* out_counts, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_query(c, n_indexed, n_queries, k))) return r;
  if ((r = check_csr(n_queries, nnz, q_row_ptr, q_col_idx))) return r;
  if (n_queries > 0 && (r = check_index(index))) return r;
  if (n_queries > 0 && (!out_ids || !out_counts))
    return fail(FLASH_EINVAL, "NULL array");
  const size_t kb = keys_bytes(c, n_queries);
  const size_t need = kb + query_ws_bytes(c, n_queries);
  if (need > kNoAllocScratchBytes)
    return fail(FLASH_ENOSPC, "batch needs " + std::to_string(need) + " bytes of scratch; the library's fixed area holds " +
                                  std::to_string(kNoAllocScratchBytes) + " (use flash_query_batch with a workspace)");
  if (n_queries == 0) return FLASH_OK;
  hipError_t e = hipSuccess;
  char* ws = (char*)scratch_address(&e);
  if (!ws) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  hipStream_t s = (hipStream_t)stream;
  uint32_t* qkeys = (uint32_t*)ws;
  const QueryWs w = query_ws_carve(c, n_queries, ws + kb);
  e = launch_doph_hash(c, n_queries, nnz, q_row_ptr, q_col_idx, qkeys, nullptr, w.ovf_len + 2, s);
  if (e != hipSuccess) return hip_fail(e, "doph_hash");
  e = launch_query(c, index, n_indexed, n_queries, qkeys, self_ids, self_ids ? 1 : 0, k, nullptr, out_ids,
                   out_counts, w, s);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "count_topk");
}

FLASH_API int flash_query_keys_mixed(const flash_params* p, const int32_t* index,
                                     int64_t n_indexed, int64_t n_queries, const uint32_t* qkeys,
                                     const int32_t* self_ids, const int32_t* k_per_query, int32_t k_max,
                                     int32_t* out_ids, int32_t* out_counts, void* workspace,
                                     size_t workspace_bytes, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_query(c, n_indexed, n_queries, k_max))) return r;
  if (n_queries > 0 && (r = check_index(index))) return r;
  if (n_queries > 0 && (!qkeys || !out_ids || !out_counts || !k_per_query))
    return fail(FLASH_EINVAL, "NULL array");
  const size_t need = query_ws_bytes(c, n_queries);
  if (!workspace || workspace_bytes < need)
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_QUERY_KEYS)");
  const QueryWs w = query_ws_carve(c, n_queries, workspace);
  hipError_t e = launch_query(c, index, n_indexed, n_queries, qkeys, self_ids, self_ids ? 1 : 0,
                              k_max, k_per_query, out_ids, out_counts, w, (hipStream_t)stream);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "count_topk");
}

FLASH_API int flash_query_batch_mixed(const flash_params* p, const int32_t* index,
                                      int64_t n_indexed, int64_t n_queries, int64_t nnz,
                                      const int64_t* q_row_ptr, const int32_t* q_col_idx,
                                      const int32_t* self_ids, const int32_t* k_per_query,
                                      int32_t k_max, int32_t* out_ids, int32_t* out_counts,
                                      void* workspace, size_t workspace_bytes, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_query(c, n_indexed, n_queries, k_max))) return r;
  if ((r = check_csr(n_queries, nnz, q_row_ptr, q_col_idx))) return r;
  if (n_queries > 0 && (r = check_index(index))) return r;
  if (n_queries > 0 && (!out_ids || !out_counts || !k_per_query))
    return fail(FLASH_EINVAL, "NULL array");
  const size_t kb = keys_bytes(c, n_queries);
  const size_t need = kb + query_ws_bytes(c, n_queries);
  if (!workspace || workspace_bytes < need)
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_QUERY)");
  hipStream_t s = (hipStream_t)stream;
  uint32_t* qkeys = (uint32_t*)workspace;
  // the query workspace's spare word 2 counts the hash tiles (dynamic schedule)
  const QueryWs w = query_ws_carve(c, n_queries, (char*)workspace + kb);
  hipError_t e = launch_doph_hash(c, n_queries, nnz, q_row_ptr, q_col_idx, qkeys, nullptr, w.ovf_len + 2, s);
  if (e != hipSuccess) return hip_fail(e, "doph_hash");
  e = launch_query(c, index, n_indexed, n_queries, qkeys, self_ids, self_ids ? 1 : 0, k_max,
                   k_per_query, out_ids, out_counts, w, s);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "count_topk");
}

FLASH_API int flash_knn_graph(const flash_params* p, int64_t n_rows, int64_t nnz,
                              const int64_t* row_ptr, const int32_t* col_idx, int32_t k,
                              int32_t* index, int32_t* out_ids, int32_t* out_counts,
                              void* workspace, size_t workspace_bytes, void* stream) {
  Cfg c;
  int r = make_cfg(p, &c);
  if (r) return r;
  if ((r = check_rows(c, n_rows, true))) return r;
  if ((r = check_csr(n_rows, nnz, row_ptr, col_idx))) return r;
  if ((r = check_query(c, n_rows, n_rows, k))) return r;
  if ((r = check_index(index))) return r;
  if (n_rows > 0 && (!out_ids || !out_counts))
    return fail(FLASH_EINVAL, "NULL array");
  const size_t kb = keys_bytes(c, n_rows);
  const size_t ins = insert_ws_bytes(c, n_rows), qry = query_ws_bytes(c, n_rows);
  const size_t need = kb + (ins > qry ? ins : qry);
  if (!workspace || workspace_bytes < need)
    return fail(FLASH_ENOSPC, "workspace smaller than flash_workspace_bytes(FLASH_OP_KNN_GRAPH)");
  hipStream_t s = (hipStream_t)stream;
  uint32_t* keys = (uint32_t*)workspace;
  char* rest = (char*)workspace + kb;
  hipError_t e = launch_doph_hash(c, n_rows, nnz, row_ptr, col_idx, keys, nullptr, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "doph_hash");
  e = launch_insert(c, n_rows, keys, 0u, false, index, insert_ws_carve(c, n_rows, rest), s);
  if (e != hipSuccess) return hip_fail(e, "reservoir_insert");
  e = launch_query(c, index, n_rows, n_rows, keys, nullptr, 2, k, nullptr, out_ids, out_counts,
                   query_ws_carve(c, n_rows, rest), s);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "count_topk");
}

FLASH_API int flash_rerank_exact(int measure, int64_t n_indexed, int64_t nnz, const int64_t* row_ptr,
                                 const int32_t* col_idx, int64_t n_queries, int64_t q_nnz,
                                 const int64_t* q_row_ptr, const int32_t* q_col_idx, const int32_t* cand_ids,
                                 int32_t n_cand, int32_t k, int32_t* out_ids, int32_t* out_inter, void* stream) {
  if (measure != FLASH_SIM_COSINE && measure != FLASH_SIM_JACCARD)
    return fail(FLASH_EINVAL, "measure must be FLASH_SIM_COSINE or FLASH_SIM_JACCARD");
  if (n_indexed < 0 || n_queries < 0) return fail(FLASH_EINVAL, "sizes must be >= 0");
  if (n_cand < 1 || n_cand > 1024) return fail(FLASH_EINVAL, "n_cand must be in [1, 1024]");
  if (k < 1 || k > n_cand) return fail(FLASH_EINVAL, "k must be in [1, n_cand]");
  int r;
  if ((r = check_csr(n_indexed, nnz, row_ptr, col_idx))) return r;
  if ((r = check_csr(n_queries, q_nnz, q_row_ptr, q_col_idx))) return r;
  if (n_queries > 0 && (!cand_ids || !out_ids || !out_inter)) return fail(FLASH_EINVAL, "NULL array");
  hipError_t e = launch_rerank(measure, n_indexed, nnz, row_ptr, col_idx, n_queries, q_nnz, q_row_ptr, q_col_idx,
                               cand_ids, n_cand, k, out_ids, out_inter, (hipStream_t)stream);
  return e == hipSuccess ? FLASH_OK : hip_fail(e, "rerank");
}

FLASH_API int flash_get_tuning(flash_tuning* out) {
  if (!out) return fail(FLASH_EINVAL, "out is NULL");
  *out = tuning_to_c(tuning());
  return FLASH_OK;
}

FLASH_API int flash_set_tuning(const flash_tuning* t) {
  Tuning v;
  const int r = tuning_from_c(t, &v);
  if (r) return r;
  install_tuning(v);
  return FLASH_OK;
}

FLASH_API int flash_autotune_query_batch(const flash_params* p, const int32_t* index,
                                         int64_t n_indexed, int64_t n_queries, int64_t nnz,
                                         const int64_t* q_row_ptr, const int32_t* q_col_idx,
                                         const int32_t* self_ids, const int32_t* k_per_query,
                                         int32_t k_max, int32_t* out_ids, int32_t* out_counts,
                                         void* workspace, size_t workspace_bytes, int32_t reps,
                                         void* stream, flash_tuning* best, float* best_ms) {
  if (reps < 1 || reps > 20) return fail(FLASH_EINVAL, "reps must be in [1, 20]");
  if (!best) return fail(FLASH_EINVAL, "best is NULL");
  const Tuning before = tuning();
  hipStream_t s = (hipStream_t)stream;
  auto run_once = [&]() {
    return k_per_query
               ? flash_query_batch_mixed(p, index, n_indexed, n_queries, nnz, q_row_ptr, q_col_idx,
                                         self_ids, k_per_query, k_max, out_ids, out_counts, workspace,
                                         workspace_bytes, stream)
               : flash_query_batch(p, index, n_indexed, n_queries, nnz, q_row_ptr, q_col_idx, self_ids,
                                   k_max, out_ids, out_counts, workspace, workspace_bytes, stream);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(FLASH_EHIP, "hipEventCreate failed");
  }
  int rc = FLASH_OK;
  // time of one candidate: the least of reps runs (ms), or a negative code
  auto measure = [&](const Tuning& t, float* ms) -> int {
    install_tuning(t);
    float bestt = 3.4e38f;
    for (int i = 0; i < reps; ++i) {
      hipError_t he = hipEventRecord(e0, s);
      if (he != hipSuccess) return hip_fail(he, "hipEventRecord");
      const int r = run_once();
      if (r) return r;
      if ((he = hipEventRecord(e1, s)) != hipSuccess) return hip_fail(he, "hipEventRecord");
      if ((he = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(he, "hipEventSynchronize");
      float v = 0.f;
      if ((he = hipEventElapsedTime(&v, e0, e1)) != hipSuccess) return hip_fail(he, "hipEventElapsedTime");
      if (v < bestt) bestt = v;
    }
    *ms = bestt;
    return FLASH_OK;
  };
  Tuning cur = before;
  float cur_ms = 0.f;
  rc = measure(cur, &cur_ms);  // also warms up
  if (!rc) rc = measure(cur, &cur_ms);
  // candidate values, one field at a time
  const int waves[] = {1, 4, 8, 16};
  const int stages[][2] = {{2048, 4096}, {2048, 0}, {1024, 4096}, {4096, 0}, {1024, 0}, {0, 0}};
  const int per_cu[] = {64, 128, 256, 512};
  const int tiles[] = {0, 4, 16, 64};
  // the full-bucket stage skip first: it decides whether the stage layouts differ
  for (int field = 0; field < 6 && !rc; ++field) {
    const int n = (field == 0 || field == 5) ? 2 : (field == 2 ? 6 : 4);
    for (int i = 0; i < n && !rc; ++i) {
      Tuning t = cur;
      if (field == 5) t.query_filter = 1 - i;
      if (field == 0) t.query_skip_full = 1 - i;
      if (field == 1) t.query_big_waves = waves[i];
      if (field == 2) {
        t.query_cap1 = stages[i][0];
        t.query_cap2 = stages[i][1];
      }
      if (field == 3) t.query_blocks_per_cu = per_cu[i];
      if (field == 4) t.hash_tile_rows = tiles[i];
      float ms = 0.f;
      rc = measure(t, &ms);
      if (!rc && ms < cur_ms) {
        cur = t;
        cur_ms = ms;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    install_tuning(before);
    return rc;
  }
  install_tuning(cur);
  *best = tuning_to_c(cur);
  if (best_ms) *best_ms = cur_ms;
  return FLASH_OK;
}

FLASH_API const char* flash_strerror(int code) {
  switch (code) {
    case FLASH_OK: return "ok";
    case FLASH_EINVAL: return "invalid argument";
    case FLASH_ENOSPC: return "workspace or output too small";
    case FLASH_EHIP: return "HIP runtime error";
    case FLASH_ENOTIMPL: return "parameters outside the supported range";
    case FLASH_ERANGE: return "column id out of range";
    default: return "unknown error";
  }
}

FLASH_API const char* flash_last_error(void) { return g_last_error.c_str(); }

FLASH_API const char* flash_version(void) { return "flash-mi355x 0.1 (gfx950)"; }

}  // extern "C"
