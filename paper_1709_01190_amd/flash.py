"""Python binding of the FLASH C ABI (include/flash.h): argument marshalling only.

Every function has the name of the C entry point it calls and takes torch
tensors that live on the GPU (their data pointers are passed through).  32-bit
unsigned arrays (keys, codes, counts) are carried in int32 tensors, bit for bit.
There is no CPU path: if ``libflash.so`` has not been built, loading fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflash.so")

FLASH_OK = 0
FLASH_EINVAL = -1
FLASH_ENOSPC = -2
FLASH_EHIP = -3
FLASH_ENOTIMPL = -4
FLASH_ERANGE = -5
FLASH_CSR_BAD_COLUMN = 1
FLASH_CSR_BAD_ROW_PTR = 2
EMPTY_KEY = 0xFFFFFFFF

OP_HASH, OP_INSERT, OP_BUILD, OP_QUERY_KEYS, OP_QUERY, OP_KNN_GRAPH = range(6)


class FlashError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class flash_params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("L", ctypes.c_int32),
                ("bits_per_hash", ctypes.c_int32), ("R", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("densify_attempts", ctypes.c_int32),
                ("share_permille", ctypes.c_int32)]

    @classmethod
    def make(cls, K, L, bits_per_hash, R, seed=1, densify_attempts=64, share_permille=0):
        return cls(K, L, bits_per_hash, R, seed, densify_attempts, share_permille)

    @property
    def M(self) -> int:
        return 1 << (self.K * self.bits_per_hash)


class flash_tuning(ctypes.Structure):
    _fields_ = [("query_cap1", ctypes.c_int32), ("query_cap2", ctypes.c_int32),
                ("query_blocks_per_cu", ctypes.c_int32), ("query_big_waves", ctypes.c_int32),
                ("hash_tile_rows", ctypes.c_int32), ("query_skip_full", ctypes.c_int32),
                ("query_filter", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_ if f != "reserved"}


_lib = None
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64


def lib():
    """Load libflash.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FlashError(FLASH_EHIP, f"{LIB_PATH} is not built; run "
                         "`python -m paper_1709_01190_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(flash_params)
    sig = {
        "flash_check_params": [P],
        "flash_index_layout": [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32),
                               ctypes.POINTER(ctypes.c_uint64)],
        "flash_workspace_bytes": [ctypes.c_int, P, _I64, _I64, ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_size_t)],
        "flash_hash": [P, _I64, _I64, _VP, _VP, _VP, _VP, _VP],
        "flash_validate_csr": [_I64, _I64, _I64, _VP, _VP, _VP, _VP],
        "flash_csr_status": [ctypes.c_uint32],
        "flash_insert_keys": [P, _I64, _VP, _VP, _VP, ctypes.c_size_t, _VP],
        "flash_build_index": [P, _I64, _I64, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP],
        "flash_query_keys": [P, _VP, _I64, _I64, _VP, _VP, ctypes.c_int32, _VP, _VP, _VP,
                             ctypes.c_size_t, _VP],
        "flash_query_batch": [P, _VP, _I64, _I64, _I64, _VP, _VP, _VP, ctypes.c_int32, _VP,
                              _VP, _VP, ctypes.c_size_t, _VP],
        "flash_query_batch_noalloc": [P, _VP, _I64, _I64, _I64, _VP, _VP, _VP, ctypes.c_int32,
                                      _VP, _VP, _VP],
        "flash_query_keys_mixed": [P, _VP, _I64, _I64, _VP, _VP, _VP, ctypes.c_int32, _VP, _VP,
                                   _VP, ctypes.c_size_t, _VP],
        "flash_query_batch_mixed": [P, _VP, _I64, _I64, _I64, _VP, _VP, _VP, _VP, ctypes.c_int32,
                                    _VP, _VP, _VP, ctypes.c_size_t, _VP],
        "flash_knn_graph": [P, _I64, _I64, _VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP,
                            ctypes.c_size_t, _VP],
        "flash_insert_keys_append": [P, _I64, _VP, _I64, _VP, _VP, ctypes.c_size_t, _VP],
        "flash_build_index_append": [P, _I64, _I64, _VP, _VP, _I64, _VP, _VP, ctypes.c_size_t, _VP],
        "flash_rerank_exact": [ctypes.c_int, _I64, _I64, _VP, _VP, _I64, _I64, _VP, _VP, _VP, ctypes.c_int32,
                               ctypes.c_int32, _VP, _VP, _VP],
        "flash_get_tuning": [ctypes.POINTER(flash_tuning)],
        "flash_set_tuning": [ctypes.POINTER(flash_tuning)],
        "flash_autotune_query_batch": [P, _VP, _I64, _I64, _I64, _VP, _VP, _VP, _VP,
                                       ctypes.c_int32, _VP, _VP, _VP, ctypes.c_size_t,
                                       ctypes.c_int32, _VP, ctypes.POINTER(flash_tuning),
                                       ctypes.POINTER(ctypes.c_float)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.flash_noalloc_scratch_bytes.argtypes = []
    L.flash_noalloc_scratch_bytes.restype = ctypes.c_size_t
    for name in ("flash_strerror",):
        getattr(L, name).argtypes = [ctypes.c_int]
        getattr(L, name).restype = ctypes.c_char_p
    for name in ("flash_last_error", "flash_version"):
        getattr(L, name).argtypes = []
        getattr(L, name).restype = ctypes.c_char_p
    _lib = L
    return L


def _check(code: int):
    if code != FLASH_OK:
        L = lib()
        raise FlashError(code, f"{L.flash_strerror(code).decode()}: {L.flash_last_error().decode()}")


def _p(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("FLASH arrays must be GPU tensors")
    if not t.is_contiguous():
        raise ValueError("FLASH arrays must be contiguous")
    return _VP(t.data_ptr())


def _s(stream) -> _VP:
    if stream is None:
        stream = torch.cuda.current_stream()
    return _VP(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _need(t, numel, dtype, name):
    if t is None:
        return
    if t.dtype not in dtype:
        raise TypeError(f"{name}: dtype {t.dtype} not in {dtype}")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, need {numel}")


_U32 = (torch.int32, getattr(torch, "uint32", torch.int32))


# ------------------------------------------------------------------ host-only calls

def flash_check_params(p: flash_params) -> None:
    _check(lib().flash_check_params(ctypes.byref(p)))


def flash_index_layout(p: flash_params) -> Tuple[int, int, int]:
    """(P reservoirs, S words per reservoir, P * S words) of the index array."""
    a, b, c = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint64()
    _check(lib().flash_index_layout(ctypes.byref(p), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


SLOT0 = 4  # word of a reservoir that holds its first slot (word 0: the arrival count)


def _need_index(p, index):
    _need(index, flash_index_layout(p)[2], (torch.int32,), "index")


def flash_workspace_bytes(op: int, p: flash_params, n_rows: int = 0, n_queries: int = 0,
                          k: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(lib().flash_workspace_bytes(op, ctypes.byref(p), n_rows, n_queries, k, ctypes.byref(out)))
    return out.value


def flash_version() -> str:
    return lib().flash_version().decode()


# ------------------------------------------------------------------ device calls

def flash_validate_csr(row_ptr, col_idx, n_cols, flags=None, stream=None) -> int:
    """Runs the optional validation pass, waits for the device, and returns
    FLASH_OK, FLASH_ERANGE (a column outside [0, n_cols)) or FLASH_EINVAL
    (malformed row pointers).  flags: a one-element int32 device tensor to
    use (else one is allocated)."""
    n = row_ptr.numel() - 1
    _need(row_ptr, n + 1, (torch.int64,), "row_ptr")
    _need(col_idx, 0, (torch.int32,), "col_idx")
    if flags is None:
        flags = torch.empty(1, dtype=torch.int32, device=row_ptr.device)
    _need(flags, 1, _U32, "flags")
    _check(lib().flash_validate_csr(n, col_idx.numel(), int(n_cols), _p(row_ptr), _p(col_idx),
                                    _p(flags), _s(stream)))
    torch.cuda.synchronize(row_ptr.device)
    return int(lib().flash_csr_status(int(flags.view(torch.int32).item()) & 0xFFFFFFFF))


def flash_hash(p, row_ptr, col_idx, keys, codes=None, stream=None):
    n = row_ptr.numel() - 1
    _need(row_ptr, n + 1, (torch.int64,), "row_ptr")
    _need(col_idx, 0, (torch.int32,), "col_idx")
    _need(keys, n * p.L, _U32, "keys")
    _need(codes, n * p.K * p.L, _U32, "codes")
    _check(lib().flash_hash(ctypes.byref(p), n, col_idx.numel(), _p(row_ptr), _p(col_idx),
                            _p(keys), _p(codes), _s(stream)))


def flash_insert_keys(p, keys, index, workspace, stream=None):
    n = keys.numel() // p.L
    _need_index(p, index)
    _check(lib().flash_insert_keys(ctypes.byref(p), n, _p(keys), _p(index),
                                   _p(workspace), workspace.numel() * workspace.element_size(),
                                   _s(stream)))


def flash_build_index(p, row_ptr, col_idx, index, workspace, keys_out=None, stream=None):
    n = row_ptr.numel() - 1
    _need_index(p, index)
    _need(keys_out, n * p.L, _U32, "keys_out")
    _check(lib().flash_build_index(ctypes.byref(p), n, col_idx.numel(), _p(row_ptr), _p(col_idx),
                                   _p(index), _p(keys_out), _p(workspace),
                                   workspace.numel() * workspace.element_size(), _s(stream)))


def flash_insert_keys_append(p, keys, id_base, index, workspace, stream=None):
    n = keys.numel() // p.L
    _need_index(p, index)
    _check(lib().flash_insert_keys_append(ctypes.byref(p), n, _p(keys) if n else None, id_base,
                                          _p(index), _p(workspace) if workspace is not None else None,
                                          workspace.numel() * workspace.element_size() if workspace is not None else 0,
                                          _s(stream)))


def flash_build_index_append(p, row_ptr, col_idx, id_base, index, workspace, stream=None):
    n = row_ptr.numel() - 1
    _need_index(p, index)
    _check(lib().flash_build_index_append(ctypes.byref(p), n, col_idx.numel(), _p(row_ptr) if n else None,
                                          _p(col_idx) if col_idx.numel() else None, id_base, _p(index),
                                          _p(workspace) if workspace is not None else None,
                                          workspace.numel() * workspace.element_size() if workspace is not None else 0,
                                          _s(stream)))


def flash_query_keys(p, index, n_indexed, qkeys, k, out_ids, out_counts, workspace,
                     self_ids=None, stream=None):
    q = qkeys.numel() // p.L
    _need(out_ids, q * k, (torch.int32,), "out_ids")
    _need(out_counts, q * k, (torch.int32,), "out_counts")
    _need(self_ids, q, (torch.int32,), "self_ids")
    _check(lib().flash_query_keys(ctypes.byref(p), _p(index), n_indexed, q, _p(qkeys),
                                  _p(self_ids), k, _p(out_ids), _p(out_counts), _p(workspace),
                                  workspace.numel() * workspace.element_size(), _s(stream)))


def flash_query_batch(p, index, n_indexed, q_row_ptr, q_col_idx, k, out_ids, out_counts,
                      workspace, self_ids=None, stream=None):
    q = q_row_ptr.numel() - 1
    _need(out_ids, q * k, (torch.int32,), "out_ids")
    _need(out_counts, q * k, (torch.int32,), "out_counts")
    _need(self_ids, q, (torch.int32,), "self_ids")
    _check(lib().flash_query_batch(ctypes.byref(p), _p(index), n_indexed, q,
                                   q_col_idx.numel(), _p(q_row_ptr), _p(q_col_idx), _p(self_ids),
                                   k, _p(out_ids), _p(out_counts), _p(workspace),
                                   workspace.numel() * workspace.element_size(), _s(stream)))


def flash_query_batch_noalloc(p, index, n_indexed, q_row_ptr, q_col_idx, k, out_ids, out_counts,
                              self_ids=None, stream=None):
    q = q_row_ptr.numel() - 1
    _need(out_ids, q * k, (torch.int32,), "out_ids")
    _need(out_counts, q * k, (torch.int32,), "out_counts")
    _need(self_ids, q, (torch.int32,), "self_ids")
    _check(lib().flash_query_batch_noalloc(ctypes.byref(p), _p(index), n_indexed, q,
                                           q_col_idx.numel(), _p(q_row_ptr), _p(q_col_idx),
                                           _p(self_ids), k, _p(out_ids), _p(out_counts), _s(stream)))


def flash_noalloc_scratch_bytes() -> int:
    return int(lib().flash_noalloc_scratch_bytes())


def flash_query_keys_mixed(p, index, n_indexed, qkeys, k_per_query, k_max, out_ids,
                           out_counts, workspace, self_ids=None, stream=None):
    q = qkeys.numel() // p.L
    _need(k_per_query, q, (torch.int32,), "k_per_query")
    _need(out_ids, q * k_max, (torch.int32,), "out_ids")
    _need(out_counts, q * k_max, (torch.int32,), "out_counts")
    _need(self_ids, q, (torch.int32,), "self_ids")
    _check(lib().flash_query_keys_mixed(ctypes.byref(p), _p(index), n_indexed, q, _p(qkeys),
                                        _p(self_ids), _p(k_per_query), k_max, _p(out_ids),
                                        _p(out_counts), _p(workspace),
                                        workspace.numel() * workspace.element_size(), _s(stream)))


def flash_query_batch_mixed(p, index, n_indexed, q_row_ptr, q_col_idx, k_per_query, k_max,
                            out_ids, out_counts, workspace, self_ids=None, stream=None):
    q = q_row_ptr.numel() - 1
    _need(k_per_query, q, (torch.int32,), "k_per_query")
    _need(out_ids, q * k_max, (torch.int32,), "out_ids")
    _need(out_counts, q * k_max, (torch.int32,), "out_counts")
    _need(self_ids, q, (torch.int32,), "self_ids")
    _check(lib().flash_query_batch_mixed(ctypes.byref(p), _p(index), n_indexed, q,
                                         q_col_idx.numel(), _p(q_row_ptr), _p(q_col_idx),
                                         _p(self_ids), _p(k_per_query), k_max, _p(out_ids),
                                         _p(out_counts), _p(workspace),
                                         workspace.numel() * workspace.element_size(), _s(stream)))


SIM_COSINE, SIM_JACCARD = 0, 1


def flash_rerank_exact(measure, row_ptr, col_idx, q_row_ptr, q_col_idx, cand_ids, k, out_ids, out_inter,
                       stream=None):
    """cand_ids: int32 [n_queries, n_cand]; out_ids / out_inter: int32 [n_queries * k]."""
    n = row_ptr.numel() - 1
    q = q_row_ptr.numel() - 1
    nc = cand_ids.shape[-1] if cand_ids.dim() > 1 else cand_ids.numel() // max(q, 1)
    _need(cand_ids, q * nc, (torch.int32,), "cand_ids")
    _need(out_ids, q * k, (torch.int32,), "out_ids")
    _need(out_inter, q * k, (torch.int32,), "out_inter")
    _check(lib().flash_rerank_exact(int(measure), n, col_idx.numel(), _p(row_ptr), _p(col_idx) if col_idx.numel() else None,
                                    q, q_col_idx.numel(), _p(q_row_ptr), _p(q_col_idx) if q_col_idx.numel() else None,
                                    _p(cand_ids), nc, k, _p(out_ids), _p(out_inter), _s(stream)))


def flash_get_tuning() -> flash_tuning:
    t = flash_tuning()
    _check(lib().flash_get_tuning(ctypes.byref(t)))
    return t


def flash_set_tuning(t: Optional[flash_tuning] = None, **fields) -> None:
    """Installs `t` (None: the defaults); keyword fields modify the current tuning."""
    if fields:
        t = flash_get_tuning() if t is None else t
        for k, v in fields.items():
            setattr(t, k, int(v))
    _check(lib().flash_set_tuning(ctypes.byref(t) if t is not None else None))


def flash_autotune_query_batch(p, index, n_indexed, q_row_ptr, q_col_idx, k_per_query, k_max,
                               out_ids, out_counts, workspace, self_ids=None, reps=3, stream=None):
    """Returns (best flash_tuning, its time in ms); the best is installed."""
    q = q_row_ptr.numel() - 1
    _need(k_per_query, q, (torch.int32,), "k_per_query")
    _need(out_ids, q * k_max, (torch.int32,), "out_ids")
    _need(out_counts, q * k_max, (torch.int32,), "out_counts")
    _need(self_ids, q, (torch.int32,), "self_ids")
    best, ms = flash_tuning(), ctypes.c_float(0.0)
    _check(lib().flash_autotune_query_batch(ctypes.byref(p), _p(index), n_indexed, q,
                                            q_col_idx.numel(), _p(q_row_ptr), _p(q_col_idx),
                                            _p(self_ids), _p(k_per_query), k_max, _p(out_ids),
                                            _p(out_counts), _p(workspace),
                                            workspace.numel() * workspace.element_size(), reps,
                                            _s(stream), ctypes.byref(best), ctypes.byref(ms)))
    return best, float(ms.value)


def flash_knn_graph(p, row_ptr, col_idx, k, index, out_ids, out_counts, workspace,
                    stream=None):
    n = row_ptr.numel() - 1
    _need_index(p, index)
    _need(out_ids, n * k, (torch.int32,), "out_ids")
    _need(out_counts, n * k, (torch.int32,), "out_counts")
    _check(lib().flash_knn_graph(ctypes.byref(p), n, col_idx.numel(), _p(row_ptr), _p(col_idx), k,
                                 _p(index), _p(out_ids), _p(out_counts), _p(workspace),
                                 workspace.numel() * workspace.element_size(), _s(stream)))


# ------------------------------------------------------------------ allocation helpers

def alloc_index(p: flash_params, device="cuda"):
    """The index array, int32[P * S], uninitialised (the build writes every header)."""
    return torch.empty(flash_index_layout(p)[2], dtype=torch.int32, device=device)


def index_parts(p: flash_params, index: torch.Tensor):
    """Views of an index array: (arrival counts int32[P], slots int32[P][R]).  Slot j of
    reservoir b is meaningful for j < min(count, R)."""
    P, S, _ = flash_index_layout(p)
    res = index.view(P, S)
    return res[:, 0], res[:, SLOT0:SLOT0 + p.R]


def alloc_workspace(op: int, p: flash_params, n_rows=0, n_queries=0, k=0, device="cuda"):
    nbytes = flash_workspace_bytes(op, p, n_rows, n_queries, k)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
