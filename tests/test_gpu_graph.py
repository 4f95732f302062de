"""The build and the query captured in a HIP graph: every replay (with eager
work and synchronisations between replays) must give the eager result."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_build_and_query_replay_in_a_hip_graph(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_01190_amd import datagen, flash
    print("[case] hip graph build + query", flush=True)
    spec = datagen.scaled(datagen.URL, 50_000)
    rp, ci = datagen.make_rows(spec, 1, device="cuda")
    K, L, b, R, k = 5, 32, 3, 64, 16
    p = flash.flash_params.make(K, L, b, R, seed=1)
    n = spec.n_rows
    index = flash.alloc_index(p)
    counts, ids = flash.index_parts(p, index)   # views of the index array
    keys = torch.empty(n * L, dtype=torch.int32, device="cuda")
    bws = flash.alloc_workspace(flash.OP_BUILD, p, n_rows=n)
    qws = flash.alloc_workspace(flash.OP_QUERY_KEYS, p, n_queries=n, k=k)
    sid = torch.arange(n, dtype=torch.int32, device="cuda")
    oi = torch.empty(n * k, dtype=torch.int32, device="cuda")
    oc = torch.empty_like(oi)
    s = torch.cuda.Stream()

    def step():
        flash.flash_build_index(p, rp, ci, index, bws, keys_out=keys, stream=s)
        flash.flash_query_keys(p, index, n, keys, k, oi, oc, qws, self_ids=sid, stream=s)

    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.synchronize()
    ref_i, ref_c, ref_n = oi.clone(), oc.clone(), counts.clone()
    occ = torch.clamp(ref_n.view(-1).long(), max=R)
    mask = torch.arange(R, device="cuda")[None, :] < occ[:, None]
    ref_ids = ids[mask].clone()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        oi.fill_(-7)
        oc.fill_(-7)
        index.fill_(-3)
        counts.fill_(12345)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(oi, ref_i) and torch.equal(oc, ref_c), rep
        assert torch.equal(counts, ref_n) and torch.equal(ids[mask], ref_ids), rep
    # the eager result itself against the oracle on sampled queries
    op = orc.params(K, L, b, R, seed=1)
    okeys = orc.doph(op, rp.cpu().numpy(), ci.cpu().numpy())
    ocounts, oids = orc.build_tables(op, okeys)
    sample = np.arange(0, n, 53)
    wi, wc = orc.query(op, ocounts, oids, okeys[sample], k, self_ids=sample.astype(np.int32))
    gi = ref_i.view(n, k).cpu().numpy()[sample]
    gc = ref_c.view(n, k).cpu().numpy()[sample]
    assert np.array_equal(gi, wi) and np.array_equal(gc, wc)
