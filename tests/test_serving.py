"""Serving loop scheduling (CPU: a fake executor answers with the oracle) and
the same loop on the GPU through the C ABI."""
import time

import numpy as np
import pytest

from paper_1709_01190_amd import serving


class FakeExecutor:
    """Answers a request with the CPU oracle and reports it done after a
    simulated device time; records how many requests overlap."""

    def __init__(self, orc, op, counts, ids, per_query_s=2e-5, base_s=1e-3):
        self.orc, self.op, self.counts, self.ids = orc, op, counts, ids
        self.per_query_s, self.base_s = per_query_s, base_s
        self.inflight = 0
        self.max_inflight = 0

    def bytes_for(self, n, nnz, k):
        return 8 * (n + 1) + 4 * nnz + 4 * n * self.op.L + 8 * n * k

    def new_slot(self):
        return {}

    def launch(self, slot, rp, ci, k):
        keys = self.orc.doph(self.op, rp, ci)
        slot["res"] = self.orc.query(self.op, self.counts, self.ids, keys, k)
        slot["ready"] = time.perf_counter() + self.base_s + self.per_query_s * (rp.shape[0] - 1)
        self.inflight += 1
        self.max_inflight = max(self.max_inflight, self.inflight)

    def done(self, slot):
        ok = time.perf_counter() >= slot["ready"]
        return ok

    def result(self, slot, n, k):
        self.inflight -= 1
        oi, oc = slot.pop("res")
        return oi.reshape(n, k), oc.reshape(n, k)


class FakeViewExecutor(FakeExecutor):
    """Hands completed lists out as flat views (as the GPU executor's pinned
    buffers), so the continuous server drains them in chunks."""

    def result_views(self, slot, n, k):
        self.inflight -= 1
        oi, oc = slot.pop("res")
        return oi.reshape(-1), oc.reshape(-1)


@pytest.fixture(scope="module")
def small_index(orc):
    from paper_1709_01190_amd import datagen
    spec = datagen.scaled(datagen.TINY, 3000)
    rp, ci = (a.numpy() for a in datagen.make_rows(spec, 1))
    op = orc.params(4, 16, 4, 32, seed=1)
    keys = orc.doph(op, rp, ci)
    counts, ids = orc.build_tables(op, keys)
    qspec = datagen.scaled(datagen.TINY, 50_000)

    def rows(n, seed):
        g_rp, g_ci = datagen.make_rows(datagen.scaled(qspec, n), seed)
        return g_rp.numpy(), g_ci.numpy()
    return op, counts, ids, rows


def alone(orc, op, counts, ids, r):
    keys = orc.doph(op, r.row_ptr, r.col_idx)
    return orc.query(op, counts, ids, keys, r.k)


def test_request_generator_shapes():
    rows = lambda n, s: (np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32))
    reqs = serving.make_requests(rows, 400, qps=1e5, seed=3, max_batch=64, ks=(10, 50))
    sizes = np.array([r.n for r in reqs])
    assert sizes.min() >= 1 and sizes.max() <= 64
    assert set(r.k for r in reqs) <= {10, 50}
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) >= 0) and arr[0] == 0
    # mean offered load close to the requested queries per second
    offered = sizes.sum() / arr[-1]
    assert 0.7e5 < offered < 1.4e5


def test_continuous_results_equal_alone_and_overlap(orc, small_index):
    op, counts, ids, rows = small_index
    reqs = serving.make_requests(rows, 40, qps=2e5, seed=5, max_batch=64)
    ex = FakeExecutor(orc, op, counts, ids)
    stats = serving.ContinuousServer(ex, budget_bytes=1 << 30, slots=4).run(reqs)
    assert stats["requests"] == 40 and stats["rejected"] == 0
    assert ex.max_inflight > 1          # requests overlapped
    for r in reqs:
        wi, wc = alone(orc, op, counts, ids, r)
        assert np.array_equal(r.out_ids, wi) and np.array_equal(r.out_counts, wc)
        assert r.done >= r.admitted >= r.arrival


def test_chunked_drain_gives_the_same_lists(orc, small_index):
    # lists handed out as views are copied out in chunks between admissions
    # (a chunk smaller than most lists, so most take several passes)
    op, counts, ids, rows = small_index
    reqs = serving.make_requests(rows, 40, qps=4e4, seed=12, max_batch=64)
    ex = FakeViewExecutor(orc, op, counts, ids)
    srv = serving.ContinuousServer(ex, budget_bytes=1 << 30, slots=4)
    srv.drain_chunk = 97
    stats = srv.run(reqs)
    assert stats["requests"] == 40 and stats["rejected"] == 0
    assert ex.inflight == 0
    for r in reqs:
        wi, wc = alone(orc, op, counts, ids, r)
        assert np.array_equal(r.out_ids, wi.reshape(r.n, r.k)) and np.array_equal(r.out_counts, wc.reshape(r.n, r.k))


def test_budget_rejects_and_serialises(orc, small_index):
    op, counts, ids, rows = small_index
    reqs = serving.make_requests(rows, 30, qps=5e5, seed=6, max_batch=64)
    ex = FakeExecutor(orc, op, counts, ids)
    biggest = max(ex.bytes_for(r.n, r.nnz, r.k) for r in reqs)
    smallest = min(ex.bytes_for(r.n, r.nnz, r.k) for r in reqs)
    # a budget below the largest request: those are rejected, never run
    budget = (biggest + smallest) // 2
    stats = serving.ContinuousServer(ex, budget_bytes=budget, slots=4).run(reqs)
    too_big = [r for r in reqs if ex.bytes_for(r.n, r.nnz, r.k) > budget]
    assert too_big and all(r.rejected and r.out_ids is None for r in too_big)
    assert stats["rejected"] == len(too_big)
    # a budget below twice the smallest request: at most one in flight, still correct
    reqs2 = serving.make_requests(rows, 20, qps=5e5, seed=7, max_batch=4, ks=(10,))
    ex2 = FakeExecutor(orc, op, counts, ids)
    budget2 = 2 * min(ex2.bytes_for(r.n, r.nnz, r.k) for r in reqs2) - 1
    serving.ContinuousServer(ex2, budget_bytes=budget2, slots=4).run(reqs2)
    assert ex2.max_inflight == 1
    ran = [r for r in reqs2 if not r.rejected]
    assert len(ran) >= 2
    assert all(ex2.bytes_for(r.n, r.nnz, r.k) > budget2 for r in reqs2 if r.rejected)
    order = sorted(ran, key=lambda r: r.admitted)
    for a, b in zip(order, order[1:]):
        assert b.admitted >= a.done - 1e-9
    for r in ran:
        wi, wc = alone(orc, op, counts, ids, r)
        assert np.array_equal(r.out_ids, wi) and np.array_equal(r.out_counts, wc)


def test_burst_and_batch_all_agree(orc, small_index):
    op, counts, ids, rows = small_index
    reqs = serving.make_requests(rows, 30, qps=1e5, seed=8, max_batch=32)
    for r in reqs[10:20]:
        r.arrival = reqs[10].arrival        # a burst of ten at one instant
    ex = FakeExecutor(orc, op, counts, ids)
    serving.ContinuousServer(ex, budget_bytes=1 << 30, slots=3).run(reqs)
    cont = [(r.out_ids.copy(), r.out_counts.copy()) for r in reqs]
    for r in reqs:
        r.out_ids = r.out_counts = None
    ex2 = FakeExecutor(orc, op, counts, ids)
    stats = serving.BatchAllServer(ex2, budget_bytes=1 << 30).run(reqs)
    assert stats["requests"] == 30
    for r, (ci_, cc_) in zip(reqs, cont):
        assert np.array_equal(r.out_ids, ci_) and np.array_equal(r.out_counts, cc_)


@pytest.mark.gpu
def test_gpu_continuous_serving_equals_alone(orc):
    # The serving workload's index: the full 2.4M-row URL-shaped index.  240
    # requests of 1..4,096 queries with k in {10, 50, 200} go through the
    # continuous server on several streams at once; each request's lists
    # must equal the same request run alone and the oracle's.
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_01190_amd import datagen, flash
    print("[case] gpu serving identity on the full URL-shaped index", flush=True)
    spec = datagen.URL
    rp_d, ci_d = datagen.make_rows(spec, 1, device="cuda")
    p = flash.flash_params.make(5, 32, 3, 64, seed=1)
    index = flash.alloc_index(p)
    ws = flash.alloc_workspace(flash.OP_BUILD, p, n_rows=spec.n_rows)
    flash.flash_build_index(p, rp_d, ci_d, index, ws)
    torch.cuda.synchronize()
    rp, ci = rp_d.cpu(), ci_d.cpu()
    del ws, rp_d, ci_d

    # query rows from the index's clusters (drawn with seed 2); a request
    # takes a random slice of the pool
    import dataclasses
    pool_n = 150_000
    qrp, qci = (a.cpu().numpy() for a in datagen.make_rows(dataclasses.replace(spec, n_rows=pool_n), 1,
                                                           device="cuda", row_seed=2))

    def rows(n, seed):
        st = np.random.default_rng(seed).integers(0, pool_n - n + 1)
        a, b = int(qrp[st]), int(qrp[st + n])
        return (qrp[st:st + n + 1] - a).astype(np.int64), qci[a:b].copy()
    reqs = serving.make_requests(rows, 240, qps=2e6, seed=11, max_batch=4096)
    assert {r.k for r in reqs} == {10, 50, 200}
    ex = serving.GpuExecutor(p, index, spec.n_rows)
    stats = serving.ContinuousServer(ex, budget_bytes=1 << 30, slots=8).run(reqs)
    assert stats["requests"] == 240 and stats["rejected"] == 0
    # each result is the same as the request run alone, and as the oracle
    op = orc.params(5, 32, 3, 64, seed=1)
    okeys = orc.doph(op, rp.numpy(), ci.numpy())
    ocounts, oids = orc.build_tables(op, okeys)
    del okeys
    slot = ex.new_slot()
    for r in reqs:
        ex.launch(slot, r.row_ptr, r.col_idx, r.k)
        torch.cuda.synchronize()
        ai, ac = ex.result(slot, r.n, r.k)
        assert np.array_equal(r.out_ids, ai) and np.array_equal(r.out_counts, ac)
        wi, wc = orc.query(op, ocounts, oids, orc.doph(op, r.row_ptr, r.col_idx), r.k)
        assert np.array_equal(r.out_ids, wi) and np.array_equal(r.out_counts, wc)
