"""The entry point that allocates nothing (flash_query_batch_noalloc) against
flash_query_batch with a workspace, bit for bit, on two calls in a row (the
second smaller, so stale scratch from the first would show), and against the
oracle.  Called through the C ABI."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def _lists(fl, p, index, n_indexed, rp, ci, k, self_ids, noalloc):
    import torch
    q = rp.numel() - 1
    oi = torch.full((q * k,), 7, dtype=torch.int32, device="cuda")
    oc = torch.full((q * k,), 7, dtype=torch.int32, device="cuda")
    if noalloc:
        fl.flash_query_batch_noalloc(p, index, n_indexed, rp, ci, k, oi, oc, self_ids=self_ids)
    else:
        ws = fl.alloc_workspace(fl.OP_QUERY, p, n_queries=q, k=k)
        fl.flash_query_batch(p, index, n_indexed, rp, ci, k, oi, oc, ws, self_ids=self_ids)
    torch.cuda.synchronize()
    return oi.cpu().numpy().reshape(q, k), oc.cpu().numpy().reshape(q, k)


@pytest.mark.parametrize("K,L,b,R,k", [(5, 32, 3, 64, 50), (4, 64, 4, 128, 128)])
def test_noalloc_equals_workspace_call_twice(fl, orc, K, L, b, R, k):
    import torch
    from paper_1709_01190_amd import datagen
    spec = datagen.scaled(datagen.URL, 200_000)
    say("noalloc", K, L, b, R, k, "index rows", spec.n_rows)
    rp, ci = datagen.make_rows(spec, 1, device="cuda")
    p = fl.flash_params.make(K, L, b, R, seed=1)
    index = fl.alloc_index(p)
    ws = fl.alloc_workspace(fl.OP_BUILD, p, n_rows=spec.n_rows)
    fl.flash_build_index(p, rp, ci, index, ws)
    torch.cuda.synchronize()
    assert fl.flash_noalloc_scratch_bytes() == 32 << 20
    # the first batch is large, the second small: its stage lists and keys
    # start where the first call left its own
    for nq, with_self in ((60_000, False), (777, True)):
        qspec = datagen.scaled(datagen.URL, nq)
        qrp, qci = datagen.make_rows(qspec, 1, device="cuda", row_seed=2)
        self_ids = torch.arange(nq, dtype=torch.int32, device="cuda") * 3 if with_self else None
        say("noalloc batch", nq, "self ids" if with_self else "no self")
        wi, wc = _lists(fl, p, index, spec.n_rows, qrp, qci, k, self_ids, noalloc=False)
        ni, nc = _lists(fl, p, index, spec.n_rows, qrp, qci, k, self_ids, noalloc=True)
        assert np.array_equal(ni, wi) and np.array_equal(nc, wc), "noalloc lists differ from the workspace call"
        if nq <= 1000:
            op = orc.params(K, L, b, R, seed=1)
            oc_, oi_ = orc.build_tables(op, orc.doph(op, rp.cpu().numpy(), ci.cpu().numpy()))
            qk = orc.doph(op, qrp.cpu().numpy(), qci.cpu().numpy())
            sid = self_ids.cpu().numpy() if with_self else None
            ri, rc = orc.query(op, oc_, oi_, qk, k, self_ids=sid)
            assert np.array_equal(ni, ri) and np.array_equal(nc, rc), "noalloc lists differ from the oracle"


def test_noalloc_refuses_a_batch_beyond_its_scratch(fl):
    import torch
    p = fl.flash_params.make(4, 64, 4, 128, seed=1)
    index = fl.alloc_index(p)
    fl.index_parts(p, index)[0].zero_()
    nq = 200_000   # 64 keys + two list entries per query: more than 32 MiB
    rp = torch.zeros(nq + 1, dtype=torch.int64, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    oi = torch.empty(nq * 8, dtype=torch.int32, device="cuda")
    oc = torch.empty(nq * 8, dtype=torch.int32, device="cuda")
    with pytest.raises(fl.FlashError) as e:
        fl.flash_query_batch_noalloc(p, index, 1, rp, ci, 8, oi, oc)
    assert e.value.code == fl.FLASH_ENOSPC
    # an empty batch is accepted and enqueues nothing
    fl.flash_query_batch_noalloc(p, index, 1, rp[:1], ci, 8, oi, oc)
    torch.cuda.synchronize()
