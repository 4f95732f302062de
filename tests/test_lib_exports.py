"""The C-ABI library loads and exports every entry point include/flash.h declares
(CPU only: no kernel is launched; only host-side argument checks run)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flash.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"FLASH_API\s+[\w\s\*]*?\b(flash_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def fl():
    from paper_1709_01190_amd import flash
    return flash


def test_header_declares_the_four_hot_path_calls():
    names = declared_functions()
    for n in ("flash_hash", "flash_build_index", "flash_query_batch", "flash_knn_graph"):
        assert n in names


def test_library_exports_every_declared_symbol(fl):
    L = fl.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_library_exports_nothing_undeclared(fl):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", fl.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted({l.split()[-1] for l in out.splitlines() if " T " in l and "flash_" in l})
    assert exported == declared_functions()


def test_param_checks_run_on_the_host(fl):
    P = fl.flash_params.make
    fl.flash_check_params(P(4, 64, 4, 128))
    fl.flash_check_params(P(5, 32, 3, 64))
    for bad, code in [(P(0, 4, 4, 8), fl.FLASH_EINVAL), (P(4, 4, 8, 8), fl.FLASH_EINVAL),
                      (P(4, 300, 1, 8), fl.FLASH_ENOTIMPL), (P(4, 64, 4, 2048), fl.FLASH_ENOTIMPL),
                      (P(4, 64, 4, 256), fl.FLASH_ENOTIMPL)]:
        with pytest.raises(fl.FlashError) as e:
            fl.flash_check_params(bad)
        assert e.value.code == code
    p = P(4, 16, 4, 32)
    for v in (-1, 1001):
        bad = P(4, 16, 4, 32)
        bad.share_permille = v
        with pytest.raises(fl.FlashError):
            fl.flash_check_params(bad)


def test_index_and_workspace_sizes(fl):
    p = fl.flash_params.make(4, 64, 4, 128)
    P, S, words = fl.flash_index_layout(p)
    # header (count + 3 reserved words) and 128 slots, rounded up to 128 bytes
    assert P == 64 * 65536 and S == 160 and words == P * S
    for R, want in ((1, 32), (28, 32), (29, 64), (32, 64), (64, 96), (256, 288), (1024, 1056)):
        assert fl.flash_index_layout(fl.flash_params.make(1, 8, 2, R))[1] == want, R
    n = 350_000
    ins = fl.flash_workspace_bytes(fl.OP_INSERT, p, n_rows=n)
    assert ins >= 8 * n * 64 + 8 * 64 * 65536
    g = fl.flash_workspace_bytes(fl.OP_KNN_GRAPH, p, n_rows=n, k=128)
    assert g >= ins + 4 * n * 64
    assert fl.flash_workspace_bytes(fl.OP_HASH, p, n_rows=n) == 0
    with pytest.raises(fl.FlashError):
        fl.flash_workspace_bytes(99, p)


def test_device_calls_reject_bad_arguments_before_launch(fl):
    # argument errors return before anything touches the GPU
    L = fl.lib()
    p = fl.flash_params.make(4, 16, 4, 32)
    rc = L.flash_hash(ctypes.byref(p), 10, 100, None, None, None, None, None)
    assert rc == fl.FLASH_EINVAL
    rc = L.flash_insert_keys(ctypes.byref(p), 10, ctypes.c_void_p(16), ctypes.c_void_p(16), None, 0, None)
    assert rc == fl.FLASH_ENOSPC
    # the index array must be 16-byte aligned (every task is one 16-byte load)
    rc = L.flash_insert_keys(ctypes.byref(p), 10, ctypes.c_void_p(16), ctypes.c_void_p(20), None, 0, None)
    assert rc == fl.FLASH_EINVAL and b"aligned" in L.flash_last_error()
    rc = L.flash_query_keys(ctypes.byref(p), ctypes.c_void_p(24), 10, 10, ctypes.c_void_p(16), None, 8,
                            ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 1 << 20, None)
    assert rc == fl.FLASH_EINVAL and b"aligned" in L.flash_last_error()
    rc = L.flash_query_keys(ctypes.byref(p), ctypes.c_void_p(16), 10, 10,
                            ctypes.c_void_p(16), None, 0, ctypes.c_void_p(16), ctypes.c_void_p(16),
                            ctypes.c_void_p(16), 1 << 20, None)
    assert rc == fl.FLASH_EINVAL
    assert b"k must be" in L.flash_last_error()
    # query ids travel between table-size stages as 32-bit words
    rc = L.flash_query_keys(ctypes.byref(p), ctypes.c_void_p(16), 10, 1 << 31,
                            ctypes.c_void_p(16), None, 10, ctypes.c_void_p(16), ctypes.c_void_p(16),
                            ctypes.c_void_p(16), 1 << 20, None)
    assert rc == fl.FLASH_ENOTIMPL
    assert b"n_queries" in L.flash_last_error()


def test_csr_validation_status_and_host_checks(fl):
    L = fl.lib()
    # the status of a flags word: malformed row pointers first, then columns
    assert L.flash_csr_status(0) == fl.FLASH_OK
    assert L.flash_csr_status(fl.FLASH_CSR_BAD_COLUMN) == fl.FLASH_ERANGE
    assert b"column" in L.flash_last_error()
    assert L.flash_csr_status(fl.FLASH_CSR_BAD_ROW_PTR) == fl.FLASH_EINVAL
    assert L.flash_csr_status(fl.FLASH_CSR_BAD_ROW_PTR | fl.FLASH_CSR_BAD_COLUMN) == fl.FLASH_EINVAL
    assert L.flash_strerror(fl.FLASH_ERANGE) == b"column id out of range"
    # argument errors return before anything touches the GPU
    v = ctypes.c_void_p(16)
    assert L.flash_validate_csr(10, 100, 0, v, v, v, None) == fl.FLASH_EINVAL      # n_cols < 1
    assert b"n_cols" in L.flash_last_error()
    assert L.flash_validate_csr(-1, 100, 5, v, v, v, None) == fl.FLASH_EINVAL      # n_rows < 0
    assert L.flash_validate_csr(10, -1, 5, v, v, v, None) == fl.FLASH_EINVAL       # nnz < 0
    assert L.flash_validate_csr(10, 100, 5, None, v, v, None) == fl.FLASH_EINVAL   # no row_ptr
    assert L.flash_validate_csr(10, 100, 5, v, None, v, None) == fl.FLASH_EINVAL   # no col_idx
    assert L.flash_validate_csr(10, 100, 5, v, v, None, None) == fl.FLASH_EINVAL   # no flags
    assert b"flags" in L.flash_last_error()


def test_binding_refuses_cpu_tensors(fl):
    import torch
    p = fl.flash_params.make(4, 16, 4, 32)
    rp = torch.zeros(3, dtype=torch.int64)
    ci = torch.zeros(0, dtype=torch.int32)
    keys = torch.zeros(2 * 16, dtype=torch.int32)
    with pytest.raises(ValueError):
        fl.flash_hash(p, rp, ci, keys)


def test_tuning_is_checked_and_restorable(fl):
    fl.flash_set_tuning(None)
    d = fl.flash_get_tuning().as_dict()
    assert d == {"query_cap1": 2048, "query_cap2": 4096, "query_blocks_per_cu": 512,
                 "query_big_waves": 8, "hash_tile_rows": 0, "query_skip_full": 1, "query_filter": 1}
    fl.flash_set_tuning(query_big_waves=16, hash_tile_rows=32, query_cap2=0)
    d2 = fl.flash_get_tuning().as_dict()
    assert d2["query_big_waves"] == 16 and d2["hash_tile_rows"] == 32 and d2["query_cap2"] == 0
    for bad in (dict(query_big_waves=3), dict(query_cap1=512), dict(query_cap2=32768),
                dict(query_blocks_per_cu=0), dict(hash_tile_rows=-1), dict(query_skip_full=2),
                dict(query_filter=3)):
        with pytest.raises(fl.FlashError) as e:
            fl.flash_set_tuning(**bad)
        assert e.value.code == fl.FLASH_EINVAL
        assert fl.flash_get_tuning().as_dict() == d2       # a rejected tuning changes nothing
    t = fl.flash_get_tuning()
    t.reserved = 7
    with pytest.raises(fl.FlashError):
        fl.flash_set_tuning(t)
    fl.flash_set_tuning(None)
    assert fl.flash_get_tuning().as_dict() == d


def test_append_arguments_are_checked_on_the_host(fl):
    import torch
    p = fl.flash_params.make(4, 16, 4, 32)
    L = fl.lib()
    for n, base in ((10, -1), (10, (1 << 31) - 5)):
        r = L.flash_insert_keys_append(ctypes.byref(p), n, ctypes.c_void_p(16), base, ctypes.c_void_p(16),
                                       ctypes.c_void_p(16), 1 << 30, None)
        assert r == fl.FLASH_EINVAL
    # ids past what a query can hold in its packed (id, count) words: L = 16
    # leaves 27 id bits
    r = L.flash_insert_keys_append(ctypes.byref(p), 10, ctypes.c_void_p(16), (1 << 27) - 5, ctypes.c_void_p(16),
                                   ctypes.c_void_p(16), 1 << 30, None)
    assert r == fl.FLASH_ENOTIMPL
    # too small a workspace
    r = L.flash_insert_keys_append(ctypes.byref(p), 1000, ctypes.c_void_p(16), 0, ctypes.c_void_p(16),
                                   ctypes.c_void_p(16), 8, None)
    assert r == fl.FLASH_ENOSPC
    # nothing to add: nothing enqueued, no workspace needed
    assert L.flash_insert_keys_append(ctypes.byref(p), 0, None, 5, ctypes.c_void_p(16),
                                      None, 0, None) == fl.FLASH_OK


def test_rerank_arguments_are_checked_on_the_host(fl):
    L = fl.lib()
    vp = ctypes.c_void_p(16)
    for measure, nc, k in ((2, 10, 5), (0, 0, 1), (0, 1025, 5), (1, 10, 11), (1, 10, 0)):
        r = L.flash_rerank_exact(measure, 10, 100, vp, vp, 5, 50, vp, vp, vp, nc, k, vp, vp, None)
        assert r == fl.FLASH_EINVAL, (measure, nc, k)


def test_shared_pool_size_matches_the_oracle(fl, orc):
    # the library's pool arithmetic against the oracle's (both read Sec. 3.5)
    for K, L, b, R, permille in ((4, 64, 4, 128, 200), (5, 32, 3, 64, 500), (2, 3, 3, 4, 1),
                                 (1, 2, 2, 8, 500), (4, 16, 4, 32, 999), (4, 16, 4, 32, 1000), (4, 16, 4, 32, 0)):
        ce, S, words = fl.flash_index_layout(fl.flash_params.make(K, L, b, R, share_permille=permille))
        P = orc.pool_size(orc.params(K, L, b, R, share_permille=permille))
        assert ce == P and words == P * S, (K, L, b, permille)


def test_noalloc_query_checks_its_fixed_scratch_on_the_host(fl):
    # the batch is refused before anything touches the GPU when its keys and
    # stage lists do not fit the library's 32 MiB area
    L = fl.lib()
    vp = ctypes.c_void_p(16)
    assert fl.flash_noalloc_scratch_bytes() == 32 << 20
    p = fl.flash_params.make(4, 64, 4, 128)
    need = fl.flash_workspace_bytes(fl.OP_QUERY, p, n_queries=200_000, k=8)
    assert need > 32 << 20
    r = L.flash_query_batch_noalloc(ctypes.byref(p), vp, 10, 200_000, 100, vp, vp, None, 8, vp, vp, None)
    assert r == fl.FLASH_ENOSPC
    assert b"scratch" in L.flash_last_error()
    r = L.flash_query_batch_noalloc(ctypes.byref(p), vp, 10, 10, 100, vp, vp, None, 0, vp, vp, None)
    assert r == fl.FLASH_EINVAL
    # nothing to answer: nothing enqueued
    assert L.flash_query_batch_noalloc(ctypes.byref(p), vp, 10, 0, 0, vp, None, None, 8, vp, vp,
                                       None) == fl.FLASH_OK
