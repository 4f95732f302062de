"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer work, so every comparison is bit-exact: keys, codes, bucket counts,
the occupied reservoir slots and the (id, count) k-NN lists.  Slots past a
bucket's occupancy are not part of the index and are not compared.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EMPTY = 0xFFFFFFFF


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_01190_amd import flash
    flash.lib()
    return flash


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def i32(t):
    return t.detach().cpu().numpy().view(np.int32)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.view(dtype)
    return t.cuda()


def csr_from_rows(rows):
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate([np.asarray(r, dtype=np.int64).astype(np.int32) for r in rows]) if rows \
        else np.zeros(0, np.int32)
    return rp, ci


def fmix32_inverse(h):
    h = np.asarray([h], dtype=np.uint32)

    def unxorshift(v, s):
        r = v.copy()
        for _ in range(32 // s + 1):
            r = v ^ (r >> np.uint32(s))
        return r
    h = unxorshift(h, 16)
    h = h * np.uint32(pow(0xC2B2AE35, -1, 1 << 32))
    h = unxorshift(h, 13)
    h = h * np.uint32(pow(0x85EBCA6B, -1, 1 << 32))
    h = unxorshift(h, 16)
    return int(h[0])


def host_index(fl, p, index):
    """(arrival counts uint32[P], slots int32[P * R]) of a device index array."""
    cnt, slots = fl.index_parts(p, index)
    return u32(cnt.contiguous()), i32(slots.contiguous()).reshape(-1)


def occupied_equal(counts_a, ids_a, counts_b, ids_b, L, M, R):
    """counts equal and the occupied slots of every bucket equal."""
    ca = counts_a.reshape(L, M)
    cb = counts_b.reshape(L, M)
    assert np.array_equal(ca, cb), "bucket counts differ"
    ia = ids_a.reshape(L, M, R)
    ib = ids_b.reshape(L, M, R)
    occ = np.minimum(ca, R)
    slot = np.arange(R)[None, None, :]
    mask = slot < occ[:, :, None]
    assert np.array_equal(ia[mask], ib[mask]), "reservoir contents differ"


def gpu_hash(fl, p, rp, ci, codes=True, offset=0):
    import torch
    n = rp.shape[0] - 1
    buf = torch.zeros(ci.shape[0] + 8, dtype=torch.int32, device="cuda")
    buf[offset:offset + ci.shape[0]] = dev(ci)
    ci_d = buf[offset:offset + ci.shape[0]]
    keys = torch.empty(n * p.L, dtype=torch.int32, device="cuda")
    cod = torch.empty(n * p.K * p.L, dtype=torch.int32, device="cuda") if codes else None
    fl.flash_hash(p, dev(rp), ci_d, keys, cod)
    torch.cuda.synchronize()
    return u32(keys).reshape(n, p.L), (u32(cod).reshape(n, p.K * p.L) if codes else None)


def gpu_insert(fl, p, keys_np):
    import torch
    n = keys_np.shape[0]
    index = fl.alloc_index(p)
    ws = fl.alloc_workspace(fl.OP_INSERT, p, n_rows=n)
    fl.flash_insert_keys(p, dev(keys_np.astype(np.uint32), torch.int32), index, ws)
    torch.cuda.synchronize()
    return index


def gpu_query(fl, p, index, n_indexed, qkeys_np, k, self_ids=None):
    import torch
    q = qkeys_np.shape[0]
    oi = torch.empty(q * k, dtype=torch.int32, device="cuda")
    oc = torch.empty(q * k, dtype=torch.int32, device="cuda")
    ws = fl.alloc_workspace(fl.OP_QUERY_KEYS, p, n_queries=q, k=k)
    sd = dev(self_ids.astype(np.int32)) if self_ids is not None else None
    fl.flash_query_keys(p, index, n_indexed, dev(qkeys_np.astype(np.uint32), torch.int32), k,
                        oi, oc, ws, self_ids=sd)
    torch.cuda.synchronize()
    return i32(oi).reshape(q, k), i32(oc).reshape(q, k)


# ------------------------------------------------------------------ hash

def test_hash_tiny_workload(fl, orc):
    from paper_1709_01190_amd import datagen
    say("hash tiny 10k rows K4 L16 b4")
    rp, ci = (a.numpy() for a in datagen.make_rows(datagen.TINY, 1))
    p = fl.flash_params.make(4, 16, 4, 32, seed=1)
    keys, codes = gpu_hash(fl, p, rp, ci)
    okeys, ocodes = orc.doph(orc.params(4, 16, 4, 32, seed=1), rp, ci, want_codes=True)
    assert np.array_equal(codes, ocodes)
    assert np.array_equal(keys, okeys)


@pytest.mark.parametrize("K,L,b,A", [(4, 16, 4, 64), (5, 32, 3, 64), (1, 1, 16, 64), (16, 256, 1, 64),
                                     (3, 3, 5, 0), (4, 64, 4, 2), (2, 70, 7, 64), (5, 32, 3, 12),
                                     (3, 40, 4, 8)])
def test_hash_edge_rows(fl, orc, K, L, b, A):
    say("hash edge rows", K, L, b, A)
    rng = np.random.default_rng(K * 1000 + L)
    seed = 77
    s_h = orc.seeds(seed)[0]
    top_col = fmix32_inverse(0xFFFFFFFF) ^ s_h  # the one column whose pi is 0xFFFFFFFF
    top_col = top_col - (1 << 32) if top_col >= (1 << 31) else top_col
    rows = [[], [5], [1, 2], list(range(63)), list(range(64)), list(range(65)),
            rng.integers(-(1 << 31), (1 << 31) - 1, size=1000).tolist(),
            [7, 7, 7, 3, 3, 9], rng.permutation(300).tolist(), [top_col], [top_col, 11, 12],
            rng.integers(0, 1 << 20, size=5000).tolist(), [], [0],
            # either side of the one-id-per-lane path for short rows
            rng.integers(0, 1 << 20, size=256).tolist(), rng.integers(0, 1 << 20, size=257).tolist(),
            rng.integers(0, 1 << 20, size=129).tolist()]
    rp, ci = csr_from_rows(rows)
    p = fl.flash_params.make(K, L, b, 8, seed=seed, densify_attempts=A)
    okeys, ocodes = orc.doph(orc.params(K, L, b, 8, seed=seed, densify_attempts=A), rp, ci,
                             want_codes=True)
    for off in range(4):  # every 16-byte misalignment of the column array
        keys, codes = gpu_hash(fl, p, rp, ci, offset=off)
        assert np.array_equal(codes, ocodes), off
        assert np.array_equal(keys, okeys), off


def test_hash_malformed_row_pointers_stay_in_bounds(fl, orc):
    say("hash malformed row_ptr")
    import torch
    ci = np.arange(100, dtype=np.int32)
    rp = np.array([0, 10, 5, 200, -3, 100], dtype=np.int64)  # decreasing, past nnz, negative
    p = fl.flash_params.make(4, 16, 4, 8)
    keys = torch.empty(5 * 16, dtype=torch.int32, device="cuda")
    fl.flash_hash(p, dev(rp), dev(ci), keys)
    torch.cuda.synchronize()
    k = u32(keys).reshape(5, 16)
    # clamped rows: [0,10), [10,10) empty, [5,100), [100,100) empty, [0,100)
    want_rows = [ci[0:10], ci[0:0], ci[5:100], ci[0:0], ci[0:100]]
    wrp, wci = csr_from_rows(want_rows)
    assert np.array_equal(k, orc.doph(orc.params(4, 16, 4, 8), wrp, wci))


def csr_status_by_definition(fl, rp, ci, n_cols):
    """The code flash_validate_csr must give, from the definitions (numpy)."""
    nnz = ci.size
    bad_rp = (rp.size == 0 or rp[0] != 0 or rp[-1] != nnz or bool((rp < 0).any()) or bool((rp > nnz).any())
              or bool((np.diff(rp) < 0).any()))
    bad_col = bool(((ci.astype(np.int64) < 0) | (ci.astype(np.int64) >= n_cols)).any())
    return fl.FLASH_EINVAL if bad_rp else (fl.FLASH_ERANGE if bad_col else fl.FLASH_OK)


def test_validate_csr(fl):
    import torch
    rng = np.random.default_rng(3)
    n_cols = 1000
    rows = [rng.integers(0, n_cols, size=int(s)).tolist() for s in rng.integers(0, 300, size=500)]
    rp, ci = csr_from_rows(rows)
    flags = torch.empty(1, dtype=torch.int32, device="cuda")

    def check(rp, ci, n_cols, what):
        want = csr_status_by_definition(fl, rp, ci, n_cols)
        for off in range(4):   # the 16-byte body, the unaligned head and the tail all see every id
            say("validate csr", what, "offset", off)
            buf = torch.zeros(ci.size + 4, dtype=torch.int32, device="cuda")
            if ci.size:
                buf[off:off + ci.size] = torch.from_numpy(ci).cuda()
            got = fl.flash_validate_csr(dev(rp), buf[off:off + ci.size], n_cols, flags=flags)
            assert got == want, (what, off, got, want)
        return want

    assert check(rp, ci, n_cols, "valid") == fl.FLASH_OK
    nnz = ci.size
    for pos in (0, 1, 2, 3, nnz // 2, nnz - 4, nnz - 3, nnz - 2, nnz - 1):
        for bad in (n_cols, -1, 1 << 30):
            c2 = ci.copy()
            c2[pos] = bad
            assert check(rp, c2, n_cols, f"column {bad} at {pos}") == fl.FLASH_ERANGE
    assert check(rp, ci, int(ci.max()), "n_cols = the largest id") == fl.FLASH_ERANGE
    assert check(rp, ci, int(ci.max()) + 1, "n_cols = the largest id + 1") == fl.FLASH_OK
    r2 = rp.copy()
    r2[250] = r2[251] + 1   # decreases
    assert check(r2, ci, n_cols, "decreasing row_ptr") == fl.FLASH_EINVAL
    r3 = rp.copy()
    r3[-1] -= 1             # does not end at nnz
    assert check(r3, ci, n_cols, "row_ptr not ending at nnz") == fl.FLASH_EINVAL
    r4 = rp.copy()
    r4[0] = 1               # does not start at 0
    assert check(r4, ci, n_cols, "row_ptr not starting at 0") == fl.FLASH_EINVAL
    # both wrong: the row pointers decide
    c5 = ci.copy()
    c5[7] = -5
    assert check(r2, c5, n_cols, "both") == fl.FLASH_EINVAL
    # no rows, no columns
    assert check(np.zeros(1, np.int64), np.zeros(0, np.int32), 5, "empty") == fl.FLASH_OK
    # a large batch with one bad id far inside (many grid strides)
    big = rng.integers(0, 1 << 20, size=6_000_003).astype(np.int32)
    brp = np.array([0, 1_000_000, 6_000_003], dtype=np.int64)
    assert check(brp, big, 1 << 20, "large valid") == fl.FLASH_OK
    big[5_123_457] = 1 << 20
    assert check(brp, big, 1 << 20, "large, one bad id") == fl.FLASH_ERANGE
    # the hot path itself still takes any id: validation is optional
    p = fl.flash_params.make(4, 16, 4, 32)
    keys = torch.empty(2 * 16, dtype=torch.int32, device="cuda")
    fl.flash_hash(p, dev(brp), dev(big), keys)
    torch.cuda.synchronize()


# ------------------------------------------------------------------ insert

def test_insert_tiny_workload(fl, orc):
    from paper_1709_01190_amd import datagen
    say("insert tiny")
    rp, ci = (a.numpy() for a in datagen.make_rows(datagen.TINY, 1))
    op = orc.params(4, 16, 4, 32, seed=1)
    keys = orc.doph(op, rp, ci)
    ocounts, oids = orc.build_tables(op, keys)
    p = fl.flash_params.make(4, 16, 4, 32, seed=1)
    index = gpu_insert(fl, p, keys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), 16, 1 << 16, 32)


@pytest.mark.parametrize("R", [1, 4, 32, 256, 1024])
def test_insert_heavy_buckets(fl, orc, R):
    # bucket sizes around every path switch: one thread (<= 8), a wave
    # sorting all arrivals, and the priority-threshold select
    say("insert heavy buckets R", R)
    rng = np.random.default_rng(R)
    K, L, b = 2, 3, 5
    M = 1 << (K * b)
    sizes = [0, 1, 7, 8, 9, 63, 64, 65, R - 1, R, R + 1, 2 * R, 2 * R + 1, 3 * R, 2047, 2049, 5000,
             40000, 120000]
    sizes = [s for s in sizes if s >= 0]
    keys = []
    for t in range(L):
        col = np.concatenate([np.full(s, (i * 7 + t) % M, dtype=np.uint32) for i, s in enumerate(sizes)])
        rng.shuffle(col)
        keys.append(col)
    n = max(len(c) for c in keys)
    km = np.full((n, L), EMPTY, dtype=np.uint32)
    for t in range(L):
        km[:len(keys[t]), t] = keys[t]
    km[rng.random((n, L)) < 0.01] = M + 5  # out-of-range keys are skipped like empty ones
    op = orc.params(K, L, b, R, seed=R + 3)
    ocounts, oids = orc.build_tables(op, km)
    p = fl.flash_params.make(K, L, b, R, seed=R + 3)
    index = gpu_insert(fl, p, km)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, M, R)


@pytest.mark.parametrize("R", [8, 128])
def test_insert_sparse_buckets_with_a_hot_chunk(fl, orc, R):
    # The two-level partition (few arrivals per bucket on average: 65,536
    # buckets, ~2 arrivals each) with one chunk of buckets far above its
    # LDS copy (the chunk's ids stored straight to the staged array), buckets
    # of every select size (1..8, 9..64, 65..256, above) and appends on top.
    import torch
    say("insert sparse buckets with a hot chunk R", R)
    rng = np.random.default_rng(40 + R)
    K, L, b = 4, 2, 4
    M = 1 << (K * b)
    n = 150_000
    keys = rng.integers(0, M, size=(n, L), dtype=np.int64).astype(np.uint32)
    # rows 0..29,999 of table 0 land in buckets 0..99 (one chunk, ~300 each);
    # a few single buckets get 20, 90, 300 and 3,000 arrivals
    keys[:30_000, 0] = rng.integers(0, 100, size=30_000).astype(np.uint32)
    for bkt, cnt, lo in ((40_000, 20, 40_000), (41_000, 90, 41_000), (42_000, 300, 42_000), (43_000, 3000, 43_000)):
        keys[lo:lo + cnt, 1] = bkt
    keys[rng.random((n, L)) < 0.01] = EMPTY
    op = orc.params(K, L, b, R, seed=3)
    ocounts, oids = orc.build_tables(op, keys)
    p = fl.flash_params.make(K, L, b, R, seed=3)
    index = gpu_insert(fl, p, keys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, M, R)
    index2 = _append_batches(fl, p, keys, [0, 20_000, 70_000, n], [1, 0, 2])
    occupied_equal(*host_index(fl, p, index2), ocounts.reshape(-1), oids.reshape(-1), L, M, R)


def test_insert_is_deterministic(fl):
    import torch
    say("insert determinism")
    rng = np.random.default_rng(5)
    K, L, b, R = 3, 8, 3, 16
    M = 1 << (K * b)
    keys = (rng.zipf(1.3, size=(200000, L)) % M).astype(np.uint32)
    p = fl.flash_params.make(K, L, b, R, seed=9)
    index1 = gpu_insert(fl, p, keys)
    index2 = gpu_insert(fl, p, keys)
    occupied_equal(*host_index(fl, p, index1), *host_index(fl, p, index2), L, M, R)


# ------------------------------------------------------------------ query

@pytest.fixture(scope="module")
def tiny_index(fl, orc):
    from paper_1709_01190_amd import datagen
    rp, ci = (a.numpy() for a in datagen.make_rows(datagen.TINY, 1))
    op = orc.params(4, 16, 4, 32, seed=1)
    keys = orc.doph(op, rp, ci)
    ocounts, oids = orc.build_tables(op, keys)
    p = fl.flash_params.make(4, 16, 4, 32, seed=1)
    index = gpu_insert(fl, p, keys)
    return p, op, rp, ci, keys, index, ocounts, oids


@pytest.mark.parametrize("k", [1, 16, 100, 1024])
def test_query_tiny_graph_mode(fl, orc, tiny_index, k):
    say("query tiny graph k", k)
    p, op, rp, ci, keys, index, ocounts, oids = tiny_index
    n = keys.shape[0]
    self_ids = np.arange(n, dtype=np.int32)
    oi, oc = gpu_query(fl, p, index, n, keys, k, self_ids)
    wi, wc = orc.query(op, ocounts, oids, keys, k, self_ids=self_ids)
    assert np.array_equal(oi, wi) and np.array_equal(oc, wc)


def test_query_mixed_keys_and_self(fl, orc, tiny_index):
    say("query mixed keys")
    p, op, rp, ci, keys, index, ocounts, oids = tiny_index
    rng = np.random.default_rng(8)
    q = 3000
    qk = keys[rng.integers(0, keys.shape[0], size=q)].copy()
    mask = rng.random(qk.shape) < 0.2
    qk[mask] = rng.integers(0, 1 << 16, size=int(mask.sum()))
    qk[::17] = EMPTY
    qk[5, 3] = (1 << 16) + 9  # out of range: ignored
    self_ids = rng.integers(-1, keys.shape[0], size=q).astype(np.int32)
    for sids in (None, self_ids):
        oi, oc = gpu_query(fl, p, index, keys.shape[0], qk, 40, sids)
        wi, wc = orc.query(op, ocounts, oids, qk, 40, self_ids=sids)
        assert np.array_equal(oi, wi) and np.array_equal(oc, wc)


@pytest.fixture
def tuned(fl):
    """Lets a test change the launch tuning; restores the defaults after it."""
    fl.flash_set_tuning(None)
    yield fl.flash_set_tuning
    fl.flash_set_tuning(None)


# launch shapes of the query stages: first/second table sizes (0: no such
# stage) and the waves per workgroup of a large last stage
# (query_skip_full=0 keeps the small stages even where the buckets are full;
# the defaults, with the skip, come first)
# (query_filter=0 sends every query to the counting-table stages; with the
# filter stage on they see only the queries it hands on)
STAGE_SHAPES = [dict(), dict(query_filter=0)] + [
    dict(query_cap1=c1, query_cap2=c2, query_big_waves=w, query_skip_full=0, query_filter=f)
    for (c1, c2) in ((1024, 4096), (2048, 0), (0, 0), (16384, 0)) for w in (1, 4, 8, 16) for f in (0, 1)]


def test_query_overflow_table(fl, orc, tuned):
    # buckets far fuller than the first-pass table: every query takes the
    # large-table launch; a second run with a table that fits checks both
    say("query overflow")
    rng = np.random.default_rng(9)
    K, L, b, R = 1, 32, 2, 256
    n = 6000
    keys = rng.integers(0, 1 << (K * b), size=(n, L)).astype(np.uint32)
    keys[:50] = rng.integers(0, 1 << (K * b), size=(50, L))
    op = orc.params(K, L, b, R, seed=4)
    ocounts, oids = orc.build_tables(op, keys)
    p = fl.flash_params.make(K, L, b, R, seed=4)
    index = gpu_insert(fl, p, keys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, 1 << (K * b), R)
    qk = keys[:700].copy()
    qk[100:400, 4:] = EMPTY     # small queries stay in the first pass
    wi, wc = orc.query(op, ocounts, oids, qk, 300, self_ids=np.arange(700, dtype=np.int32))
    for shape in STAGE_SHAPES:
        tuned(None)
        tuned(**shape)
        oi, oc = gpu_query(fl, p, index, n, qk, 300, np.arange(700, dtype=np.int32))
        assert np.array_equal(oi, wi) and np.array_equal(oc, wc), shape


@pytest.mark.parametrize("k", [113, 120, 128])
def test_query_top_k_among_thousands_of_ties(fl, orc, k):
    # every query has ~2,000 candidates, most seen once or twice, so the tie
    # cut leaves k .. k + 16 survivors (k <= 128: 129-144 of them at most)
    say("query top-k among ties", k)
    rng = np.random.default_rng(21)
    K, L, b, R = 1, 32, 3, 64
    n = 4000
    keys = rng.integers(0, 1 << (K * b), size=(n, L)).astype(np.uint32)
    op = orc.params(K, L, b, R, seed=8)
    ocounts, oids = orc.build_tables(op, keys)
    p = fl.flash_params.make(K, L, b, R, seed=8)
    index = gpu_insert(fl, p, keys)
    wi, wc = orc.query(op, ocounts, oids, keys[:600], k, self_ids=np.arange(600, dtype=np.int32))
    oi, oc = gpu_query(fl, p, index, n, keys[:600], k, np.arange(600, dtype=np.int32))
    assert np.array_equal(oi, wi) and np.array_equal(oc, wc)


def test_query_many_tables(fl, orc):
    say("query L=200")
    rng = np.random.default_rng(10)
    K, L, b, R = 2, 200, 4, 40
    n = 3000
    keys = rng.integers(0, 1 << (K * b), size=(n, L)).astype(np.uint32)
    keys[1000:1100] = keys[0]  # one heavy cluster
    op = orc.params(K, L, b, R, seed=6)
    ocounts, oids = orc.build_tables(op, keys)
    p = fl.flash_params.make(K, L, b, R, seed=6)
    index = gpu_insert(fl, p, keys)
    wi, wc = orc.query(op, ocounts, oids, keys[:500], 64, self_ids=np.arange(500, dtype=np.int32))
    oi, oc = gpu_query(fl, p, index, n, keys[:500], 64, np.arange(500, dtype=np.int32))
    assert np.array_equal(oi, wi) and np.array_equal(oc, wc)


@pytest.mark.parametrize("case", ["repeats", "crowded", "high_ids", "k_edges"])
def test_filter_stage_edges(fl, orc, tuned, case):
    # the filter stage's limits, with the stage on and off, against the oracle:
    # repeats: 1000 identical rows, so queries bring ~1000 repeated ids (more
    #   suspects than the stage holds, or k ids of count >= 2: handed on);
    # crowded: n_indexed far above every stored id, so the first radix level
    #   puts all ids in one bin and the select refines it;
    # high_ids: the queries meet only the last 1000 rows, far above the
    #   expected cut, so the cut falls in the first level's overflow bin;
    # k_edges: k = 1 and k = 1024 (all candidates survive).
    say("filter stage", case)
    rng = np.random.default_rng(31)
    K, L, b, R = 1, 32, 3, 64
    n = 20000
    nq = 500
    keys = rng.integers(0, 1 << (K * b), size=(n, L)).astype(np.uint32)
    n_indexed = n
    ks = [64]
    if case == "repeats":
        keys[500:1500] = keys[0]
    elif case == "crowded":
        n_indexed = 1 << 26   # the largest the packed query table takes at L = 32
    elif case == "high_ids":
        K, b = 1, 6
        keys = rng.integers(0, 32, size=(n, L)).astype(np.uint32)
        keys[n - 1000:] = rng.integers(32, 64, size=(1000, L))
    else:
        ks = [1, 1024]
    op = orc.params(K, L, b, R, seed=12)
    ocounts, oids = orc.build_tables(op, keys)
    p = fl.flash_params.make(K, L, b, R, seed=12)
    index = gpu_insert(fl, p, keys)
    qk = keys[n - nq:] if case == "high_ids" else keys[:nq]
    sid = np.arange(n - nq, n, dtype=np.int32) if case == "high_ids" else np.arange(nq, dtype=np.int32)
    for k in ks:
        wi, wc = orc.query(op, ocounts, oids, qk, k, self_ids=sid)
        for filt in (1, 0):
            tuned(None)
            tuned(query_filter=filt)
            oi, oc = gpu_query(fl, p, index, n_indexed, qk, k, sid)
            assert np.array_equal(oi, wi) and np.array_equal(oc, wc), (case, k, filt)


def test_query_launch_shape_does_not_change_results(fl, orc, tiny_index, tuned):
    say("query launch shapes")
    p, op, rp, ci, keys, index, ocounts, oids = tiny_index
    n = keys.shape[0]
    ref = None
    for per_cu, filt in ((1, 1), (4, 0), (32, 1), (32, 0)):
        tuned(query_blocks_per_cu=per_cu, query_filter=filt)
        out = gpu_query(fl, p, index, n, keys, 16, np.arange(n, dtype=np.int32))
        if ref is None:
            ref = out
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])


def test_empty_batches_and_empty_rows(fl, orc):
    # zero-row and zero-query calls enqueue nothing (a build of zero rows
    # still clears the counts); rows and queries without columns take part
    # in no bucket, so their lists are all padding
    import torch
    say("empty batches and empty rows")
    p = fl.flash_params.make(4, 16, 4, 32, seed=1)
    op = orc.params(4, 16, 4, 32, seed=1)
    rp0 = torch.zeros(1, dtype=torch.int64, device="cuda")
    ci0 = torch.zeros(0, dtype=torch.int32, device="cuda")
    index = fl.alloc_index(p)
    index.fill_(9)
    fl.index_parts(p, index)[0].fill_(5)
    ws = fl.alloc_workspace(fl.OP_BUILD, p, n_rows=0)
    keys0 = torch.zeros(0, dtype=torch.int32, device="cuda")
    fl.flash_hash(p, rp0, ci0, keys0)
    fl.flash_insert_keys_append(p, keys0, 0, index, ws)
    fl.flash_build_index_append(p, rp0, ci0, 0, index, ws)
    torch.cuda.synchronize()
    hc, hs = host_index(fl, p, index)
    assert (hc == 5).all() and (hs == 9).all()
    fl.flash_build_index(p, rp0, ci0, index, ws)
    torch.cuda.synchronize()
    assert (host_index(fl, p, index)[0] == 0).all()
    # a real index, then empty query batches and a batch of empty queries
    from paper_1709_01190_amd import datagen
    spec = datagen.scaled(datagen.TINY, 2000)
    rp, ci = datagen.make_rows(spec, 1)
    ws = fl.alloc_workspace(fl.OP_BUILD, p, n_rows=spec.n_rows)
    fl.flash_build_index(p, rp.cuda(), ci.cuda(), index, ws)
    torch.cuda.synchronize()
    snap = i32(index).copy()
    k = 8
    sentinel = torch.full((4 * k,), 77, dtype=torch.int32, device="cuda")
    oi, oc = sentinel.clone(), sentinel.clone()
    qws = fl.alloc_workspace(fl.OP_QUERY, p, n_queries=0, k=k)
    fl.flash_query_keys(p, index, spec.n_rows, keys0, k, oi, oc, qws)
    fl.flash_query_batch(p, index, spec.n_rows, rp0, ci0, k, oi, oc, qws)
    fl.flash_query_batch_mixed(p, index, spec.n_rows, rp0, ci0,
                               torch.zeros(0, dtype=torch.int32, device="cuda"), k, oi, oc, qws)
    gws = fl.alloc_workspace(fl.OP_KNN_GRAPH, p, n_rows=0, k=k)
    index2 = fl.alloc_index(p)
    fl.flash_knn_graph(p, rp0, ci0, k, index2, oi, oc, gws)
    fl.flash_rerank_exact(fl.SIM_COSINE, rp.cuda(), ci.cuda(), rp0, ci0,
                          torch.zeros((0, k), dtype=torch.int32, device="cuda"), k, oi, oc)
    torch.cuda.synchronize()
    assert (i32(oi) == 77).all() and (i32(oc) == 77).all()
    assert (host_index(fl, p, index2)[0] == 0).all()
    q = 4
    qrp = torch.zeros(q + 1, dtype=torch.int64, device="cuda")   # four rows without columns
    qws = fl.alloc_workspace(fl.OP_QUERY, p, n_queries=q, k=k)
    fl.flash_query_batch(p, index, spec.n_rows, qrp, ci0, k, oi, oc, qws)
    torch.cuda.synchronize()
    wi, wc = orc.query(op, *orc.build_tables(op, orc.doph(op, rp.numpy(), ci.numpy())),
                       orc.doph(op, qrp.cpu().numpy(), np.zeros(0, np.int32)), k)
    assert (wi == -1).all() and (wc == 0).all()
    assert np.array_equal(i32(oi).reshape(q, k), wi.reshape(q, k))
    assert np.array_equal(i32(oc).reshape(q, k), wc.reshape(q, k))
    assert np.array_equal(i32(index), snap)
    # an index of rows without columns holds nothing
    rpe = torch.zeros(101, dtype=torch.int64, device="cuda")
    ws = fl.alloc_workspace(fl.OP_BUILD, p, n_rows=100)
    fl.flash_build_index(p, rpe, ci0, index, ws)
    torch.cuda.synchronize()
    assert (host_index(fl, p, index)[0] == 0).all()


# ------------------------------------------------------------------ whole path

def _gpu_graph(fl, p, rp, ci, k):
    import torch
    n = rp.shape[0] - 1
    index = fl.alloc_index(p)
    ws = fl.alloc_workspace(fl.OP_KNN_GRAPH, p, n_rows=n, k=k)
    oi = torch.empty(n * k, dtype=torch.int32, device="cuda")
    oc = torch.empty(n * k, dtype=torch.int32, device="cuda")
    rp_d = rp if hasattr(rp, "is_cuda") else dev(rp)
    ci_d = ci if hasattr(ci, "is_cuda") else dev(ci)
    fl.flash_knn_graph(p, rp_d, ci_d, k, index, oi, oc, ws)
    torch.cuda.synchronize()
    return index, oi.view(n, k), oc.view(n, k)


def test_knn_graph_tiny_end_to_end(fl, orc):
    from paper_1709_01190_amd import datagen
    say("knn graph tiny")
    rp, ci = (a.numpy() for a in datagen.make_rows(datagen.TINY, 1))
    p = fl.flash_params.make(4, 16, 4, 32, seed=1)
    index, oi, oc = _gpu_graph(fl, p, rp, ci, 16)
    okeys, ocounts, oids, wi, wc = orc.knn_graph(orc.params(4, 16, 4, 32, seed=1), rp, ci, 16)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), 16, 1 << 16, 32)
    assert np.array_equal(i32(oi), wi) and np.array_equal(i32(oc), wc)
    r, nq = orc.recall_at_k(rp, ci, datagen.TINY.n_cols, np.arange(rp.shape[0] - 1), i32(oi))
    say(f"tiny R@16 (Jaccard gold standard) = {r:.4f} over {nq} queries")


def test_query_batch_from_csr(fl, orc):
    import torch
    from paper_1709_01190_amd import datagen
    say("query batch csr")
    rp, ci = (a.numpy() for a in datagen.make_rows(datagen.TINY, 1))
    spec = datagen.scaled(datagen.TINY, 2000)
    qrp, qci = (a.numpy() for a in datagen.make_rows(spec, 2))
    op = orc.params(4, 16, 4, 32, seed=1)
    okeys = orc.doph(op, rp, ci)
    ocounts, oids = orc.build_tables(op, okeys)
    wi, wc = orc.query(op, ocounts, oids, orc.doph(op, qrp, qci), 25)
    p = fl.flash_params.make(4, 16, 4, 32, seed=1)
    index = fl.alloc_index(p)
    n = rp.shape[0] - 1
    ws = fl.alloc_workspace(fl.OP_BUILD, p, n_rows=n)
    fl.flash_build_index(p, dev(rp), dev(ci), index, ws)
    q = qrp.shape[0] - 1
    oi = torch.empty(q * 25, dtype=torch.int32, device="cuda")
    oc = torch.empty(q * 25, dtype=torch.int32, device="cuda")
    qws = fl.alloc_workspace(fl.OP_QUERY, p, n_queries=q, k=25)
    fl.flash_query_batch(p, index, n, dev(qrp), dev(qci), 25, oi, oc, qws)
    torch.cuda.synchronize()
    assert np.array_equal(i32(oi).reshape(q, 25), wi) and np.array_equal(i32(oc).reshape(q, 25), wc)


def test_url_full_size_graph(fl, orc):
    # The URL-shaped graph at full size: 2.4M rows, B = 160 (not a power of
    # two), 73 arrivals per bucket against R = 64, so most buckets are full
    # and the query runs its full-bucket stage layout.  Keys, tables and all
    # 2.4M k-NN lists against the oracle.
    import torch
    from paper_1709_01190_amd import datagen
    say("url-shaped full size graph")
    spec = datagen.URL
    rp_d, ci_d = datagen.make_rows(spec, 1, device="cuda")
    n = spec.n_rows
    K, L, b, R, k = 5, 32, 3, 64, 64
    p = fl.flash_params.make(K, L, b, R, seed=1)
    index, oi, oc = _gpu_graph(fl, p, rp_d, ci_d, k)
    gkeys = torch.empty(n * L, dtype=torch.int32, device="cuda")
    fl.flash_hash(p, rp_d, ci_d, gkeys)
    torch.cuda.synchronize()
    rp, ci = rp_d.cpu().numpy(), ci_d.cpu().numpy()
    del rp_d, ci_d
    okeys, ocounts, oids, wi, wc = orc.knn_graph(orc.params(K, L, b, R, seed=1), rp, ci, k)
    assert np.array_equal(u32(gkeys).reshape(n, L), okeys)
    occ = np.minimum(ocounts, R)
    assert occ.mean() > 0.6 * R, "the full-bucket regime is not reached"
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, 1 << 15, R)
    assert np.array_equal(i32(oi).reshape(n, k), wi) and np.array_equal(i32(oc).reshape(n, k), wc)


def test_webspam_full_size_graph(fl, orc):
    # The benchmark's workload and launch shape: 350,000 rows, ~1.3G nonzeros.
    # Keys, tables and all 350,000 k-NN lists against the oracle.
    import torch
    from paper_1709_01190_amd import datagen
    say("webspam-shaped full size graph")
    spec = datagen.WEBSPAM
    rp_d, ci_d = datagen.make_rows(spec, 1, device="cuda")
    n = spec.n_rows
    K, L, b, R, k = 4, 64, 4, 128, 128
    p = fl.flash_params.make(K, L, b, R, seed=1)
    index, oi, oc = _gpu_graph(fl, p, rp_d, ci_d, k)
    gkeys = torch.empty(n * L, dtype=torch.int32, device="cuda")
    fl.flash_hash(p, rp_d, ci_d, gkeys)
    torch.cuda.synchronize()
    rp, ci = rp_d.cpu().numpy(), ci_d.cpu().numpy()
    del rp_d, ci_d
    op = orc.params(K, L, b, R, seed=1)
    okeys = orc.doph(op, rp, ci)
    assert np.array_equal(u32(gkeys).reshape(n, L), okeys)
    ocounts, oids = orc.build_tables(op, okeys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, 1 << 16, R)
    wi, wc = orc.query(op, ocounts, oids, okeys, k, self_ids=np.arange(n, dtype=np.int32))
    assert np.array_equal(i32(oi).reshape(n, k), wi) and np.array_equal(i32(oc).reshape(n, k), wc)


def test_query_mixed_k(fl, orc, tiny_index):
    # one launch, a k per query: each row equals the fixed-k answer for its k,
    # padded past it
    import torch
    say("query mixed k")
    p, op, rp, ci, keys, index, ocounts, oids = tiny_index
    rng = np.random.default_rng(12)
    q = 2500
    qk = keys[rng.integers(0, keys.shape[0], size=q)]
    kq = rng.choice([1, 10, 37, 100], size=q).astype(np.int32)
    kq[7] = 0        # clamped to 1
    kq[8] = 500      # clamped to k_max
    k_max = 100
    oi = torch.empty(q * k_max, dtype=torch.int32, device="cuda")
    oc = torch.empty(q * k_max, dtype=torch.int32, device="cuda")
    ws = fl.alloc_workspace(fl.OP_QUERY_KEYS, p, n_queries=q, k=k_max)
    fl.flash_query_keys_mixed(p, index, keys.shape[0], dev(qk.astype(np.uint32), torch.int32),
                              dev(kq), k_max, oi, oc, ws)
    torch.cuda.synchronize()
    gi, gc = i32(oi).reshape(q, k_max), i32(oc).reshape(q, k_max)
    wi, wc = orc.query(op, ocounts, oids, qk, k_max)
    for j in range(q):
        kk = min(max(int(kq[j]), 1), k_max)
        assert np.array_equal(gi[j, :kk], wi[j, :kk]) and np.array_equal(gc[j, :kk], wc[j, :kk])
        assert np.all(gi[j, kk:] == -1) and np.all(gc[j, kk:] == 0)


# ------------------------------------------------------------------ uneven batches

def _uneven_queries(spec, n_queries, device="cuda"):
    """Heavy-tailed query rows (Pareto sizes clip(floor(5 U^-1), 5, 50000))
    from the clusters of `spec`'s rows (seed 1), drawn with seed 2, and a k
    per query from {10, 100} by a fair seeded coin."""
    import dataclasses
    import torch
    from paper_1709_01190_amd import datagen
    sizes = datagen.heavy_tail_sizes(n_queries, 5, 50_000, 1.0, seed=2, device=device)
    qrp, qci = datagen.make_rows(dataclasses.replace(spec, n_rows=n_queries), 1, device=device,
                                 row_seed=2, sizes=sizes)
    g = torch.Generator(device="cpu")
    g.manual_seed(2)
    kq = torch.where(torch.rand(n_queries, generator=g) < 0.5, 10, 100).to(torch.int32)
    return qrp, qci, kq


def _mixed_expected(orc, op, ocounts, oids, okeys_q, kq, k_max, self_ids=None):
    """Row q: the first kq[q] entries of the k_max answer (the ranking is a
    total order, so a shorter answer is its prefix), then (-1, 0)."""
    wi, wc = orc.query(op, ocounts, oids, okeys_q, k_max, self_ids=self_ids)
    wi, wc = wi.copy(), wc.copy()
    for j, kk in enumerate(np.minimum(np.maximum(kq, 1), k_max)):
        wi[j, kk:] = -1
        wc[j, kk:] = 0
    return wi, wc


def _gpu_batch_mixed(fl, p, index, n_indexed, qrp_d, qci_d, kq, k_max):
    import torch
    q = qrp_d.numel() - 1
    oi = torch.empty(q * k_max, dtype=torch.int32, device="cuda")
    oc = torch.empty(q * k_max, dtype=torch.int32, device="cuda")
    ws = fl.alloc_workspace(fl.OP_QUERY, p, n_queries=q, k=k_max)
    fl.flash_query_batch_mixed(p, index, n_indexed, qrp_d, qci_d, dev(kq.numpy()), k_max, oi, oc, ws)
    torch.cuda.synchronize()
    return i32(oi).reshape(q, k_max), i32(oc).reshape(q, k_max)


@pytest.fixture(scope="module")
def saturated_index(fl, orc):
    """Click-log-shaped rows (mean 11 nonzeros) with K=2, b=4: 256 buckets per
    table, ~1,170 arrivals per bucket, so every reservoir of R=256 is full and
    a query meets up to L*R = 8,192 candidates (the large last stage)."""
    import dataclasses
    import torch
    from paper_1709_01190_amd import datagen
    spec = dataclasses.replace(datagen.CLICKLOG, n_rows=300_000, n_clusters=3_000)
    rp_d, ci_d = datagen.make_rows(spec, 1, device="cuda")
    K, L, b, R = 2, 32, 4, 256
    p = fl.flash_params.make(K, L, b, R, seed=1)
    index = fl.alloc_index(p)
    ws = fl.alloc_workspace(fl.OP_BUILD, p, n_rows=spec.n_rows)
    fl.flash_build_index(p, rp_d, ci_d, index, ws)
    torch.cuda.synchronize()
    op = orc.params(K, L, b, R, seed=1)
    okeys = orc.doph(op, rp_d.cpu().numpy(), ci_d.cpu().numpy())
    ocounts, oids = orc.build_tables(op, okeys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, 1 << (K * b), R)
    return spec, p, op, index, ocounts, oids


def test_uneven_batch_every_launch_shape(fl, orc, saturated_index, tuned):
    # heavy-tailed query sizes (5 .. 50,000 nonzeros) and mixed k in one
    # batch, under every stage layout, workgroup width and hash schedule
    spec, p, op, index, ocounts, oids = saturated_index
    qrp_d, qci_d, kq = _uneven_queries(spec, 3000)
    qrp, qci = qrp_d.cpu().numpy(), qci_d.cpu().numpy()
    assert int((qrp[1:] - qrp[:-1]).max()) > 5000          # the tail is present
    wi, wc = _mixed_expected(orc, op, ocounts, oids, orc.doph(op, qrp, qci), kq.numpy(), 100)
    for shape in STAGE_SHAPES + [dict(hash_tile_rows=t) for t in (1, 16, 4096)]:
        say("uneven batch", shape)
        tuned(None)
        tuned(**shape)
        gi, gc = _gpu_batch_mixed(fl, p, index, spec.n_rows, qrp_d, qci_d, kq, 100)
        assert np.array_equal(gi, wi) and np.array_equal(gc, wc), shape


def test_autotune_query_batch(fl, orc, saturated_index, tuned):
    import torch
    say("autotune")
    spec, p, op, index, ocounts, oids = saturated_index
    qrp_d, qci_d, kq = _uneven_queries(spec, 2000)
    q = 2000
    oi = torch.empty(q * 100, dtype=torch.int32, device="cuda")
    oc = torch.empty_like(oi)
    ws = fl.alloc_workspace(fl.OP_QUERY, p, n_queries=q, k=100)
    best, ms = fl.flash_autotune_query_batch(p, index, spec.n_rows, qrp_d, qci_d,
                                             dev(kq.numpy()), 100, oi, oc, ws, reps=2)
    torch.cuda.synchronize()
    assert ms > 0 and fl.flash_get_tuning().as_dict() == best.as_dict()
    wi, wc = _mixed_expected(orc, op, ocounts, oids, orc.doph(op, qrp_d.cpu().numpy(), qci_d.cpu().numpy()),
                             kq.numpy(), 100)
    assert np.array_equal(i32(oi).reshape(q, 100), wi) and np.array_equal(i32(oc).reshape(q, 100), wc)
    gi, gc = _gpu_batch_mixed(fl, p, index, spec.n_rows, qrp_d, qci_d, kq, 100)
    assert np.array_equal(gi, wi) and np.array_equal(gc, wc)


def test_clicklog_full_size_uneven(fl, orc):
    # The uneven-batch workload at full size: a 40M-row click-log-shaped
    # index (K=4, L=32, b=4, R=256; most reservoirs full) compared in full
    # with the oracle's, and 100,000 heavy-tailed queries with mixed k (every
    # one of them compared, the few hundred above 1,000 nonzeros included).
    import torch
    from paper_1709_01190_amd import datagen
    say("click-log full size index + uneven queries")
    spec = datagen.CLICKLOG
    rp_d, ci_d = datagen.make_rows(spec, 1, device="cuda")
    K, L, b, R = 4, 32, 4, 256
    p = fl.flash_params.make(K, L, b, R, seed=1)
    index = fl.alloc_index(p)
    ws = fl.alloc_workspace(fl.OP_BUILD, p, n_rows=spec.n_rows)
    fl.flash_build_index(p, rp_d, ci_d, index, ws)
    torch.cuda.synchronize()
    del ws
    nq = 100_000
    qrp_d, qci_d, kq = _uneven_queries(spec, nq)
    sizes = (qrp_d[1:] - qrp_d[:-1]).cpu().numpy()
    assert (sizes > 1000).sum() >= 100 and sizes.max() > 10_000   # the tail is present
    gi, gc = _gpu_batch_mixed(fl, p, index, spec.n_rows, qrp_d, qci_d, kq, 100)
    op = orc.params(K, L, b, R, seed=1)
    okeys = orc.doph(op, rp_d.cpu().numpy(), ci_d.cpu().numpy())
    del rp_d, ci_d
    ocounts, oids = orc.build_tables(op, okeys)
    del okeys
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, 1 << 16, R)
    wi, wc = _mixed_expected(orc, op, ocounts, oids, orc.doph(op, qrp_d.cpu().numpy(), qci_d.cpu().numpy()),
                             kq.numpy(), 100)
    assert np.array_equal(gi, wi) and np.array_equal(gc, wc)


# ------------------------------------------------------------------ incremental insertion

def _append_batches(fl, p, keys_np, cuts, order, first_fresh=False):
    """Index built by appending row ranges [cuts[i], cuts[i+1]) in the given
    order into a zeroed index (or, with first_fresh, the first range by
    flash_insert_keys, which numbers rows from 0, so that range must start at
    row 0, and the rest appended)."""
    import torch
    index = fl.alloc_index(p)
    index.fill_(-7)                        # slots past the occupancy are never read
    fl.index_parts(p, index)[0].zero_()
    for j, i in enumerate(order):
        lo, hi = cuts[i], cuts[i + 1]
        part = dev(np.ascontiguousarray(keys_np[lo:hi]).astype(np.uint32), torch.int32)
        ws = fl.alloc_workspace(fl.OP_INSERT, p, n_rows=hi - lo) if hi > lo else None
        if first_fresh and j == 0:
            assert lo == 0
            fl.flash_insert_keys(p, part, index, ws)
        else:
            fl.flash_insert_keys_append(p, part, lo, index, ws)
    torch.cuda.synchronize()
    return index


def test_append_batches_equal_one_build(fl, orc, tiny_index):
    # any batching and order of appends gives the one-shot build's tables
    say("append tiny")
    p, op, rp, ci, keys, index0, ocounts, oids = tiny_index
    n = keys.shape[0]
    cuts = [0, 3000, 3001, 3001, 7000, n]
    for order, fresh in (([0, 1, 2, 3, 4], False), ([3, 0, 4, 2, 1], False), ([0, 4, 2, 3, 1], True)):
        say("append order", order, "fresh first" if fresh else "")
        index = _append_batches(fl, p, keys, cuts, order, first_fresh=fresh)
        occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), p.L, p.M, p.R)


@pytest.mark.parametrize("R", [1, 4, 32, 256])
def test_append_into_full_reservoirs(fl, orc, R):
    # saturated buckets: every path of the select merges old slots with new
    # arrivals (thread, lane segments, wave sort, priority threshold)
    say("append heavy buckets R", R)
    rng = np.random.default_rng(100 + R)
    K, L, b = 2, 3, 5
    M = 1 << (K * b)
    sizes = [1, 5, 9, 20, 40, 63, 64, 65, R + 1, 2 * R + 1, 3000, 40000]
    cols = []
    for t in range(L):
        col = np.concatenate([np.full(s, (i * 5 + t) % M, dtype=np.uint32) for i, s in enumerate(sizes)])
        rng.shuffle(col)
        cols.append(col)
    n = max(len(c) for c in cols)
    km = np.full((n, L), EMPTY, dtype=np.uint32)
    for t in range(L):
        km[:len(cols[t]), t] = cols[t]
    op = orc.params(K, L, b, R, seed=R + 11)
    ocounts, oids = orc.build_tables(op, km)
    p = fl.flash_params.make(K, L, b, R, seed=R + 11)
    cuts = [0, 7, 500, 20000, n // 2, n]
    index = _append_batches(fl, p, km, cuts, [2, 0, 4, 1, 3])
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, M, R)


def test_append_csr_batches_then_query(fl, orc):
    # a URL-shaped index grown from CSR batches, then queried
    import torch
    from paper_1709_01190_amd import datagen
    say("append url csr")
    spec = datagen.scaled(datagen.URL, 120_000)
    rp_d, ci_d = datagen.make_rows(spec, 1, device="cuda")
    rp, ci = rp_d.cpu().numpy(), ci_d.cpu().numpy()
    K, L, b, R = 5, 32, 3, 64
    p = fl.flash_params.make(K, L, b, R, seed=1)
    op = orc.params(K, L, b, R, seed=1)
    okeys = orc.doph(op, rp, ci)
    ocounts, oids = orc.build_tables(op, okeys)
    index = fl.alloc_index(p)
    index.fill_(-7)
    fl.index_parts(p, index)[0].zero_()
    cuts = [0, 50_000, 50_001, 90_000, spec.n_rows]
    for lo, hi in zip(cuts, cuts[1:]):
        brp = dev((rp[lo:hi + 1] - rp[lo]).astype(np.int64))
        bci = dev(ci[rp[lo]:rp[hi]])
        ws = fl.alloc_workspace(fl.OP_BUILD, p, n_rows=hi - lo)
        fl.flash_build_index_append(p, brp, bci, lo, index, ws)
    torch.cuda.synchronize()
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), L, 1 << 15, R)
    sample = np.arange(0, spec.n_rows, 97)
    gi, gc = gpu_query(fl, p, index, spec.n_rows, okeys[sample], 20, sample.astype(np.int32))
    wi, wc = orc.query(op, ocounts, oids, okeys[sample], 20, self_ids=sample.astype(np.int32))
    assert np.array_equal(gi, wi) and np.array_equal(gc, wc)


# ------------------------------------------------------------------ exact re-rank

def _gpu_rerank(fl, measure, rp, ci, qrp, qci, cand, k):
    import torch
    q, nc = cand.shape
    oi = torch.empty(q * k, dtype=torch.int32, device="cuda")
    on = torch.empty(q * k, dtype=torch.int32, device="cuda")
    fl.flash_rerank_exact(measure, dev(rp), dev(ci), dev(qrp), dev(qci), dev(cand), k, oi, on)
    torch.cuda.synchronize()
    return i32(oi).reshape(q, k), i32(on).reshape(q, k)


def _random_rows(rng, n, max_len, n_cols):
    rows = [np.unique(rng.integers(0, n_cols, size=int(rng.integers(0, max_len + 1)))) for _ in range(n)]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32) if rp[-1] else np.zeros(0, np.int32)
    return rp, ci


@pytest.mark.parametrize("measure", [0, 1])
def test_rerank_random_rows(fl, orc, measure):
    say("rerank random measure", measure)
    rng = np.random.default_rng(50 + measure)
    rp, ci = _random_rows(rng, 2000, 60, 300)
    qrp, qci = _random_rows(rng, 700, 60, 300)
    for nc, k in ((1, 1), (37, 7), (200, 200), (1024, 16)):
        cand = rng.integers(-1, 2000, size=(700, nc)).astype(np.int32)
        for q in range(700):                   # distinct ids per list
            _, first = np.unique(cand[q], return_index=True)
            dup = np.ones(nc, bool)
            dup[first] = False
            cand[q, dup] = -1
        wi, wn = orc.rerank(measure, rp, ci, qrp, qci, cand, k)
        gi, gn = _gpu_rerank(fl, measure, rp, ci, qrp, qci, cand, k)
        assert np.array_equal(gi, wi) and np.array_equal(gn, wn), (nc, k)
        # ids past the index are no candidate
        bad = cand.copy()
        bad[:, 0] = 2000 + 5
        ref = cand.copy()
        ref[:, 0] = -1
        wi, wn = orc.rerank(measure, rp, ci, qrp, qci, ref, k)
        gi, gn = _gpu_rerank(fl, measure, rp, ci, qrp, qci, bad, k)
        assert np.array_equal(gi, wi) and np.array_equal(gn, wn), (nc, k, "out of range")


def test_rerank_long_rows_and_top_column(fl, orc):
    # queries longer than one LDS round (4,096 columns), and column 0xFFFFFFFF
    say("rerank long rows")
    rng = np.random.default_rng(60)
    rows = [np.unique(rng.integers(0, 30000, size=int(s))) for s in rng.integers(1000, 12000, size=300)]
    rows[5] = np.concatenate([rows[5], [-1]])          # read as column 0xFFFFFFFF
    qrows = [np.unique(np.concatenate([rows[i][: len(rows[i]) // 2], rng.integers(0, 30000, size=3000)]))
             for i in range(0, 300, 7)]
    qrows[0] = np.concatenate([qrows[0], [-1]])
    rp = np.zeros(301, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    nq = len(qrows)
    qrp = np.zeros(nq + 1, np.int64)
    qrp[1:] = np.cumsum([len(r) for r in qrows])
    qci = np.concatenate(qrows).astype(np.int32)
    cand = np.array([rng.permutation(300)[:64] for _ in range(nq)], dtype=np.int32)
    cand[0, 0] = 5
    cand[0, 1:] = np.where(cand[0, 1:] == 5, 6, cand[0, 1:])
    for measure in (0, 1):
        wi, wn = orc.rerank(measure, rp, ci, qrp, qci, cand, 20)
        gi, gn = _gpu_rerank(fl, measure, rp, ci, qrp, qci, cand, 20)
        assert np.array_equal(gi, wi) and np.array_equal(gn, wn), measure


def test_rerank_of_flash_candidates(fl, orc):
    # the use it is for: FLASH's count-ranked top-100 of URL-shaped queries
    # (the oracle's lists, so no input comes from the GPU) re-ranked by
    # exact cosine to a top-10
    import dataclasses
    from paper_1709_01190_amd import datagen
    say("rerank flash candidates")
    spec = datagen.scaled(datagen.URL, 60_000)
    rp, ci = (a.numpy() for a in datagen.make_rows(spec, 1))
    qrp, qci = (a.numpy() for a in datagen.make_rows(dataclasses.replace(spec, n_rows=1500), 1, row_seed=2))
    op = orc.params(5, 32, 3, 64, seed=1)
    counts, ids = orc.build_tables(op, orc.doph(op, rp, ci))
    cand, _ = orc.query(op, counts, ids, orc.doph(op, qrp, qci), 100)
    for measure in (0, 1):
        wi, wn = orc.rerank(measure, rp, ci, qrp, qci, cand, 10)
        gi, gn = _gpu_rerank(fl, measure, rp, ci, qrp, qci, cand, 10)
        assert np.array_equal(gi, wi) and np.array_equal(gn, wn), measure


# ------------------------------------------------------------------ reservoir sharing

def _shared_pair(fl, orc, K, L, b, R, seed, permille):
    p = fl.flash_params.make(K, L, b, R, seed=seed, share_permille=permille)
    op = orc.params(K, L, b, R, seed=seed, share_permille=permille)
    P = orc.pool_size(op)
    S = fl.flash_index_layout(p)[1]
    assert fl.flash_index_layout(p) == (P, S, P * S)
    return p, op, P


@pytest.mark.parametrize("permille", [1, 100, 600])
def test_shared_insert_tiny(fl, orc, tiny_index, permille):
    say("shared insert tiny", permille)
    _, _, rp, ci, keys, _, _, _ = tiny_index
    p, op, P = _shared_pair(fl, orc, 4, 16, 4, 32, 1, permille)
    ocounts, oids = orc.build_tables(op, keys)
    index = gpu_insert(fl, p, keys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), 1, P, 32)


@pytest.mark.parametrize("R", [4, 64, 300])
def test_shared_heavy_reservoirs(fl, orc, R):
    # a pool far smaller than the buckets: many rows arrive twice in one
    # reservoir, every select path merges arrivals of several tables
    say("shared heavy R", R)
    rng = np.random.default_rng(90 + R)
    K, L, b = 2, 8, 4
    n = 20000
    keys = rng.integers(0, 1 << (K * b), size=(n, L), dtype=np.int64).astype(np.uint32)
    keys[rng.random((n, L)) < 0.02] = EMPTY
    p, op, P = _shared_pair(fl, orc, K, L, b, R, 7, 5)
    ocounts, oids = orc.build_tables(op, keys)
    index = gpu_insert(fl, p, keys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), 1, P, R)
    q = 500
    wi, wc = orc.query(op, ocounts, oids, keys[:q], 40, self_ids=np.arange(q, dtype=np.int32))
    gi, gc = gpu_query(fl, p, index, n, keys[:q], 40, np.arange(q, dtype=np.int32))
    assert np.array_equal(gi, wi) and np.array_equal(gc, wc)


@pytest.mark.parametrize("K,L,b,R,permille", [(5, 32, 3, 64, 50), (5, 32, 3, 64, 999), (4, 64, 4, 128, 7),
                                               (1, 2, 2, 8, 1), (1, 2, 2, 8, 300), (2, 3, 3, 16, 17)])
def test_shared_pool_of_any_size(fl, orc, K, L, b, R, permille):
    # pools of exactly ceil(F * L * M) reservoirs: several partition chunks of
    # 16,384 and a short last one (52,429 = 3 * 16,384 + 3,277 for the
    # URL-shaped parameters at F = 0.05), one short chunk (F = 0.999), and
    # pools of 1, 3 and 4 reservoirs
    say("shared pool", K, L, b, R, permille)
    rng = np.random.default_rng(1000 + permille)
    n = 60_000
    keys = rng.integers(0, 1 << (K * b), size=(n, L), dtype=np.int64).astype(np.uint32)
    keys[rng.random((n, L)) < 0.01] = EMPTY
    p, op, P = _shared_pair(fl, orc, K, L, b, R, 3, permille)
    LM = L << (K * b)
    assert P == max(1, -(-LM * permille // 1000))
    ocounts, oids = orc.build_tables(op, keys)
    index = gpu_insert(fl, p, keys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), 1, P, R)
    q = 2000
    k = min(64, L * R)
    wi, wc = orc.query(op, ocounts, oids, keys[:q], k, self_ids=np.arange(q, dtype=np.int32))
    gi, gc = gpu_query(fl, p, index, n, keys[:q], k, np.arange(q, dtype=np.int32))
    assert np.array_equal(gi, wi) and np.array_equal(gc, wc)


def test_shared_url_graph_and_append(fl, orc):
    # a URL-shaped graph with F = 0.2: one-shot graph, then the same index
    # grown by appends, both against the oracle
    import torch
    from paper_1709_01190_amd import datagen
    say("shared url graph")
    spec = datagen.scaled(datagen.URL, 200_000)
    rp_d, ci_d = datagen.make_rows(spec, 1, device="cuda")
    rp, ci = rp_d.cpu().numpy(), ci_d.cpu().numpy()
    p, op, P = _shared_pair(fl, orc, 5, 32, 3, 64, 1, 200)
    index, oi, oc = _gpu_graph(fl, p, rp_d, ci_d, 32)
    okeys = orc.doph(op, rp, ci)
    ocounts, oids = orc.build_tables(op, okeys)
    occupied_equal(*host_index(fl, p, index), ocounts.reshape(-1), oids.reshape(-1), 1, P, 64)
    n = spec.n_rows
    sample = np.arange(0, n, 41)
    wi, wc = orc.query(op, ocounts, oids, okeys[sample], 32, self_ids=sample.astype(np.int32))
    assert np.array_equal(i32(oi)[sample], wi) and np.array_equal(i32(oc)[sample], wc)
    index2 = _append_batches(fl, p, okeys, [0, 70_000, 70_001, 150_000, n], [2, 0, 3, 1])
    occupied_equal(*host_index(fl, p, index2), ocounts.reshape(-1), oids.reshape(-1), 1, P, 64)
