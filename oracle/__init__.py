"""ctypes wrapper around the plain C oracle of the FLASH hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the library under ``paper_1709_01190_amd`` never
does.  Every function takes and returns numpy arrays on the host.

What each function follows (arXiv 1709.01190):
  doph            Sec. 2.3 (DOPH) and Sec. 2.2 (K hashes -> one table key)
  build           Sec. 2.4 / Alg. 1-2 (fixed-size reservoirs, bottom-R reading)
  query           Alg. 3 (gather L reservoirs, KSELECT by count)
  jaccard_knn     Eq. 2 right-hand side (exact Jaccard), for recall
  rerank          Sec. 4.3 gold standard: exact cosine (Eq. 3) or Jaccard
                  ordering of candidate lists
  pool_size,      Sec. 3.5 reservoir sharing (a seeded random map of buckets
  reservoir       to a pool of ceil(F * L * M) reservoirs)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flash_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
EMPTY = 0xFFFFFFFF


class Params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("L", ctypes.c_int32),
                ("bits_per_hash", ctypes.c_int32), ("R", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("densify_attempts", ctypes.c_int32),
                ("share_permille", ctypes.c_int32)]


# gcc flags of the checker build (portable: the same .so runs on any x86-64
# host) and of the timing build, which targets the host it is compiled on
CHECK_FLAGS = ["-O2"]
NATIVE_FLAGS = ["-O3", "-march=native"]


def build(force: bool = True, out: str = _LIB, opt=None) -> str:
    """Compile the oracle with gcc (OpenMP; CHECK_FLAGS unless `opt` names
    others) into `out` (default oracle/liboracle.so)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + list(opt or CHECK_FLAGS) +
                              ["-std=gnu99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp])
        os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        # FLASH_ORACLE_LIB names another build of this source (the mutation
        # tests load deliberately broken copies through it)
        path = os.environ.get("FLASH_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.orc_mix64.restype = ctypes.c_uint64
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_fmix32.restype = ctypes.c_uint32
        L.orc_fmix32.argtypes = [ctypes.c_uint32]
        L.orc_priority.restype = ctypes.c_uint64
        L.orc_priority.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int32]
        L.orc_seeds.restype = None
        L.orc_seeds.argtypes = [ctypes.c_uint64, P, P, P]
        L.orc_doph.restype = None
        L.orc_doph.argtypes = [P, ctypes.c_int64, P, P, P, P]
        L.orc_build.restype = None
        L.orc_build.argtypes = [P, ctypes.c_int64, P, P, P]
        L.orc_query.restype = None
        L.orc_query.argtypes = [P, P, P, ctypes.c_int64, P, P, ctypes.c_int32, P, P]
        L.orc_jaccard_pairs.restype = None
        L.orc_jaccard_pairs.argtypes = [P, P, ctypes.c_int64, P, P, P, P]
        L.orc_jaccard_knn.restype = None
        L.orc_jaccard_knn.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                      P, ctypes.c_int32, P, P, P]
        L.orc_pool_size.restype = ctypes.c_uint64
        L.orc_pool_size.argtypes = [P]
        L.orc_reservoir.restype = ctypes.c_uint64
        L.orc_reservoir.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_share_seed.restype = ctypes.c_uint32
        L.orc_share_seed.argtypes = [ctypes.c_uint64]
        L.orc_rerank.restype = None
        L.orc_rerank.argtypes = [ctypes.c_int, P, P, ctypes.c_int64, P, P, P, ctypes.c_int32,
                                 ctypes.c_int32, P, P]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def params(K, L, bits_per_hash, R, seed=1, densify_attempts=64, share_permille=0) -> Params:
    return Params(K, L, bits_per_hash, R, seed, densify_attempts, share_permille)


def pool_size(p: Params) -> int:
    """Reservoirs in the index: L * M, or about F * L * M when shared (Sec. 3.5)."""
    return lib().orc_pool_size(ctypes.byref(p))


def reservoir(p: Params, t: int, m: int) -> int:
    """Reservoir of bucket m of table t."""
    return lib().orc_reservoir(ctypes.byref(p), t, m)


def share_seed(seed: int) -> int:
    return lib().orc_share_seed(seed)


def seeds(seed: int):
    sh, sd, sp = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
    lib().orc_seeds(seed, ctypes.byref(sh), ctypes.byref(sd), ctypes.byref(sp))
    return sh.value, sd.value, sp.value


def mix64(z: int) -> int:
    return lib().orc_mix64(z)


def fmix32(x: int) -> int:
    return lib().orc_fmix32(x)


def priority(s_p: int, t: int, i: int) -> int:
    return lib().orc_priority(s_p, t, i)


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return lib().orc_num_threads()


def _csr(row_ptr, col_idx):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(col_idx, dtype=np.int32))


def doph(p: Params, row_ptr, col_idx, want_codes=False):
    """Returns keys uint32 [n][L] (and codes uint32 [n][K*L] if asked)."""
    row_ptr, col_idx = _csr(row_ptr, col_idx)
    n = row_ptr.shape[0] - 1
    keys = np.empty((n, p.L), dtype=np.uint32)
    codes = np.empty((n, p.K * p.L), dtype=np.uint32) if want_codes else None
    lib().orc_doph(ctypes.byref(p), n, _ptr(row_ptr), _ptr(col_idx), _ptr(keys), _ptr(codes))
    return (keys, codes) if want_codes else keys


def build_tables(p: Params, keys):
    """Returns counts uint32 [L][M] and ids int32 [L][M][R] (-1 past
    occupancy); with shared reservoirs counts [P] and ids [P][R]."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    n = keys.shape[0]
    M = 1 << (p.K * p.bits_per_hash)
    if 0 < p.share_permille < 1000:
        P = pool_size(p)
        counts = np.empty(P, dtype=np.uint32)
        ids = np.empty((P, p.R), dtype=np.int32)
    else:
        counts = np.empty((p.L, M), dtype=np.uint32)
        ids = np.empty((p.L, M, p.R), dtype=np.int32)
    lib().orc_build(ctypes.byref(p), n, _ptr(keys), _ptr(counts), _ptr(ids))
    return counts, ids


def query(p: Params, counts, ids, qkeys, k, self_ids=None):
    """Returns out_ids int32 [Q][k] and out_counts int32 [Q][k]."""
    qkeys = np.ascontiguousarray(qkeys, dtype=np.uint32)
    q = qkeys.shape[0]
    if self_ids is not None:
        self_ids = np.ascontiguousarray(self_ids, dtype=np.int32)
    oi = np.empty((q, k), dtype=np.int32)
    oc = np.empty((q, k), dtype=np.int32)
    lib().orc_query(ctypes.byref(p), _ptr(np.ascontiguousarray(counts, dtype=np.uint32)),
                    _ptr(np.ascontiguousarray(ids, dtype=np.int32)), q, _ptr(qkeys),
                    _ptr(self_ids), k, _ptr(oi), _ptr(oc))
    return oi, oc


def knn_graph(p: Params, row_ptr, col_idx, k):
    """Hash, build and query every row against the others (self left out)."""
    keys = doph(p, row_ptr, col_idx)
    counts, ids = build_tables(p, keys)
    n = keys.shape[0]
    oi, oc = query(p, counts, ids, keys, k, self_ids=np.arange(n, dtype=np.int32))
    return keys, counts, ids, oi, oc


def jaccard_pairs(row_ptr, col_idx, xs, ys):
    row_ptr, col_idx = _csr(row_ptr, col_idx)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    inter = np.empty(xs.shape[0], dtype=np.int64)
    uni = np.empty(xs.shape[0], dtype=np.int64)
    lib().orc_jaccard_pairs(_ptr(row_ptr), _ptr(col_idx), xs.shape[0], _ptr(xs), _ptr(ys),
                            _ptr(inter), _ptr(uni))
    return inter, uni


def jaccard_knn(row_ptr, col_idx, n_cols, queries, k):
    """Exact Jaccard top-k (J desc, id asc) of the given rows over all others."""
    row_ptr, col_idx = _csr(row_ptr, col_idx)
    queries = np.ascontiguousarray(queries, dtype=np.int64)
    q = queries.shape[0]
    oi = np.empty((q, k), dtype=np.int32)
    inter = np.empty((q, k), dtype=np.int64)
    uni = np.empty((q, k), dtype=np.int64)
    lib().orc_jaccard_knn(_ptr(row_ptr), _ptr(col_idx), row_ptr.shape[0] - 1, n_cols, q,
                          _ptr(queries), k, _ptr(oi), _ptr(inter), _ptr(uni))
    return oi, inter, uni


SIM_COSINE, SIM_JACCARD = 0, 1


def rerank(measure, row_ptr, col_idx, q_row_ptr, q_col_idx, cand, k):
    """Candidates cand[q][:] (ids of rows of row_ptr/col_idx, -1 = none)
    ordered by exact similarity to query row q (cosine, Eq. 3, or Jaccard)
    descending, ties by smaller id; first k as (ids int32, intersections
    int64), padded with (-1, 0)."""
    row_ptr, col_idx = _csr(row_ptr, col_idx)
    q_row_ptr, q_col_idx = _csr(q_row_ptr, q_col_idx)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    q, nc = cand.shape
    oi = np.empty((q, k), dtype=np.int32)
    inter = np.empty((q, k), dtype=np.int64)
    lib().orc_rerank(int(measure), _ptr(row_ptr), _ptr(col_idx), q, _ptr(q_row_ptr), _ptr(q_col_idx),
                     _ptr(cand), nc, k, _ptr(oi), _ptr(inter))
    return oi, inter


def recall_at_k(row_ptr, col_idx, n_cols, queries, found_ids):
    """R@k with Jaccard as the gold standard: a query is a hit when one of its
    returned ids ties the best exact Jaccard of any other row.  Queries with
    no other row sharing a column are left out.  Returns (R@k, n_scored)."""
    best, bi, bu = jaccard_knn(row_ptr, col_idx, n_cols, queries, 1)
    found_ids = np.asarray(found_ids)
    q, k = found_ids.shape
    xs = np.repeat(np.asarray(queries, dtype=np.int64), k)
    ys = found_ids.reshape(-1).astype(np.int64)
    valid = ys >= 0
    inter = np.zeros(q * k, dtype=np.int64)
    uni = np.ones(q * k, dtype=np.int64)
    if valid.any():
        i2, u2 = jaccard_pairs(row_ptr, col_idx, xs[valid], ys[valid])
        inter[valid], uni[valid] = i2, u2
    inter = inter.reshape(q, k)
    uni = uni.reshape(q, k)
    scored = best[:, 0] >= 0
    hit = (inter * bu[:, :1] == bi[:, :1] * uni) & (inter > 0)
    hits = hit.any(axis=1) & scored
    n = int(scored.sum())
    return (float(hits.sum()) / n if n else float("nan")), n
