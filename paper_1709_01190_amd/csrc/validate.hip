// Optional validation pass over a CSR batch: column ids in [0, n_cols) and
// well-formed row pointers.  Streams col_idx once (16-byte loads when it is
// aligned); each wave ORs its findings into the flags word with one atomic.
#include "flash.h"
#include "launch.hpp"

namespace flashk {

namespace {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bad_col(int32_t c, int64_t n_cols) {
  return (c < 0 || (int64_t)c >= n_cols) ? FLASH_CSR_BAD_COLUMN : 0u;
}

__global__ __launch_bounds__(256) void validate_csr_kernel(int64_t n_rows, int64_t nnz, int64_t n_cols,
                                                           const int64_t* row_ptr, const int32_t* col_idx,
                                                           uint32_t* flags) {
  uint32_t f = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // columns: 16-byte loads over the aligned body, one id per thread for the
  // unaligned head and the tail
  const int64_t head = (int64_t)((4 - (((uintptr_t)col_idx >> 2) & 3)) & 3);
  const int64_t h = head < nnz ? head : nnz;
  const int64_t nvec = (nnz - h) >> 2;
  if (tid < h) f |= bad_col(col_idx[tid], n_cols);
  const i32x4* vp = reinterpret_cast<const i32x4*>(col_idx + h);
  for (int64_t v = tid; v < nvec; v += stride) {
    const i32x4 x = __builtin_nontemporal_load(vp + v);
    f |= bad_col(x.x, n_cols) | bad_col(x.y, n_cols) | bad_col(x.z, n_cols) | bad_col(x.w, n_cols);
  }
  const int64_t t0 = h + 4 * nvec;
  if (t0 + tid < nnz) f |= bad_col(col_idx[t0 + tid], n_cols);
  // row pointers
  for (int64_t i = tid; i <= n_rows; i += stride) {
    const int64_t v = row_ptr[i];
    bool bad = v < 0 || v > nnz;
    if (i == 0) bad = bad || v != 0;
    if (i == n_rows) bad = bad || v != nnz;
    else bad = bad || row_ptr[i + 1] < v;
    if (bad) f |= FLASH_CSR_BAD_ROW_PTR;
  }
  const uint64_t mc = __ballot((f & FLASH_CSR_BAD_COLUMN) != 0);
  const uint64_t mr = __ballot((f & FLASH_CSR_BAD_ROW_PTR) != 0);
  if ((threadIdx.x & (kWave - 1)) == 0 && (mc | mr))
    atomicOr(flags, (mc ? FLASH_CSR_BAD_COLUMN : 0u) | (mr ? FLASH_CSR_BAD_ROW_PTR : 0u));
}

}  // namespace

hipError_t launch_validate_csr(int64_t n_rows, int64_t nnz, int64_t n_cols, const int64_t* row_ptr,
                               const int32_t* col_idx, uint32_t* flags, hipStream_t s) {
  hipError_t e = launch_fill_u32(flags, 1, 0u, s);
  if (e != hipSuccess) return e;
  const int64_t work = (nnz / 4 > n_rows + 1 ? nnz / 4 : n_rows + 1);
  const int64_t want = (int64_t)device_info().cus * 8;
  const int64_t need = (work + 255) / 256;
  const int grid = (int)(need < 1 ? 1 : (need < want ? need : want));
  hipLaunchKernelGGL(validate_csr_kernel, dim3(grid), dim3(256), 0, s, n_rows, nnz, n_cols, row_ptr, col_idx,
                     flags);
  return hipGetLastError();
}

}  // namespace flashk
