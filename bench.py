#!/usr/bin/env python3
"""Benchmark of the FLASH hot path on one MI355X: the approximate k-NN graph
of a webspam-shaped synthetic set (350,000 rows, 16.6M columns, ~1.3G
nonzeros; K=4, L=64, b=4, R=128, k=128).

One step = the whole path over the batch, with the input already in HBM:
DOPH hashing of every row, reservoir insertion into the L tables, and the
count-based top-k query of every row against the index (itself left out).
The same kernels flash_knn_graph launches are called phase by phase so that
HIP events on the launch stream time each phase inside the timed region.

Prints one JSON line (rank 0).  Extra keys: "roofline" (dominant kernel vs
the 8 TB/s HBM peak), "cpu_baseline" (the CPU oracle on the host's cores),
"phases" (per-phase times and algorithmic bytes).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (row recipe, K, L, b, R, k)
    "webspam": ("WEBSPAM", 4, 64, 4, 128, 128),
    "tiny": ("TINY", 4, 16, 4, 32, 16),
    "url": ("URL", 5, 32, 3, 64, 64),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="webspam", choices=sorted(WORKLOADS) + ["serving", "uneven", "append", "rerank", "share"])
    ap.add_argument("--queries", type=int, default=1_000_000, help="uneven: queries in the batch")
    ap.add_argument("--batches", type=int, default=24, help="append: batches the index is grown in")
    ap.add_argument("--rates", default="5e4,2e5,5e5,1e6,2e6",
                    help="serving: offered queries per second, comma separated")
    ap.add_argument("--requests", type=int, default=20000, help="serving: requests per rate and repeat")
    ap.add_argument("--serving-warmup", type=int, default=2000, help="serving: untimed requests per rate")
    ap.add_argument("--serving-repeats", type=int, default=3, help="serving: timed runs per rate")
    ap.add_argument("--serving-leg", default="1e6,2e6",
                    help="graph workloads: offered rates of the short serving leg on the URL-shaped "
                         "index (6,000 requests each, after 1,000 untimed); empty skips it")
    ap.add_argument("--slots", type=int, default=8, help="serving: requests in flight at once (streams)")
    ap.add_argument("--recall-queries", type=int, default=None,
                    help="sampled queries (graph workloads: rows) scored against brute-force "
                         "exact Jaccard; 0 skips it")
    ap.add_argument("--rows", type=int, default=0, help="override the row count (parity/debug only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="uneven: keep the default tuning")
    ap.add_argument("--no-per-bucket", action="store_true", help="uneven: leave out the per-bucket baseline")
    ap.add_argument("--traffic-table", default=os.path.join(ROOT, "profiles", "hbm_traffic.txt"),
                    help="calibrated per-launch HBM bytes from rocprofv3 FETCH_SIZE/WRITE_SIZE runs")
    ap.add_argument("--copy-reps", type=int, default=1,
                    help="with --copy-mib: also time this many warm copies and read-only "
                         "sums (the practical HBM ceilings)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="instead of the benchmark, copy this many MiB device to device (a plain "
                         "copy kernel of known size that calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.recall_queries is None:   # the serving workload scores 10,000 sampled queries
        args.recall_queries = 10_000 if args.workload == "serving" else 1000
    if args.copy_mib:
        copy_calibration(args.copy_mib, args.copy_reps)
        return
    if args.workload in ("serving", "uneven", "append", "rerank", "share"):
        if args.gpus != 1:
            print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
            sys.exit(2)
        {"serving": serving_bench, "uneven": uneven_bench, "append": append_bench,
         "rerank": rerank_bench, "share": share_bench}[args.workload](args)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        log("multi-GPU runs are not part of this build (one GPU per box); rerun with --gpus 1")
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1709_01190_amd import datagen, flash

    torch.cuda.set_device(0)
    rec_name, K, L, b, R, k = WORKLOADS[args.workload]
    spec = getattr(datagen, rec_name)
    if args.rows:
        spec = datagen.scaled(spec, args.rows)
    n = spec.n_rows
    t0 = time.time()
    rp, ci = datagen.make_rows(spec, 1, device="cuda")
    torch.cuda.synchronize()
    nnz = int(ci.numel())
    log(f"generated {args.workload}: {n} rows, {nnz} nnz ({nnz / n:.1f}/row) in {time.time() - t0:.1f}s")

    p = flash.flash_params.make(K, L, b, R, seed=1)
    M = p.M
    index = flash.alloc_index(p)
    counts = flash.index_parts(p, index)[0]     # each reservoir's header word
    keys = torch.empty(n * L, dtype=torch.int32, device="cuda")
    ins_ws = flash.alloc_workspace(flash.OP_INSERT, p, n_rows=n)
    q_ws = flash.alloc_workspace(flash.OP_QUERY_KEYS, p, n_queries=n, k=k)
    self_ids = torch.arange(n, dtype=torch.int32, device="cuda")
    oi = torch.empty(n * k, dtype=torch.int32, device="cuda")
    oc = torch.empty(n * k, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev):
        ev[0].record(stream)
        flash.flash_hash(p, rp, ci, keys, stream=stream)
        ev[1].record(stream)
        flash.flash_insert_keys(p, keys, index, ins_ws, stream=stream)
        ev[2].record(stream)
        flash.flash_query_keys(p, index, n, keys, k, oi, oc, q_ws, self_ids=self_ids,
                               stream=stream)
        ev[3].record(stream)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    warm = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(args.warmup):
        step(warm)
    torch.cuda.synchronize()
    log("warmup done")
    w0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    # the same step captured once in a HIP graph and replayed (no launch overhead)
    gs = torch.cuda.Stream()

    def gstep():
        flash.flash_hash(p, rp, ci, keys, stream=gs)
        flash.flash_insert_keys(p, keys, index, ins_ws, stream=gs)
        flash.flash_query_keys(p, index, n, keys, k, oi, oc, q_ws, self_ids=self_ids, stream=gs)

    gs.wait_stream(stream)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        gstep()
    graph.replay()
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(args.steps):
        graph.replay()
    g1.record(stream)
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / args.steps
    log(f"graph replay: {graph_ms:.3f} ms/step")
    phase_ms = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in evs])
    step_ms = float(np.mean([e[0].elapsed_time(e[3]) for e in evs]))
    ph = phase_ms.mean(axis=0)
    log(f"steps done: {step_ms:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}); "
        f"hash {ph[0]:.3f} insert {ph[1]:.3f} query {ph[2]:.3f} ms")

    # algorithmic bytes per launch
    kq = keys.view(n, L).long() & 0xFFFFFFFF
    cnt = counts.reshape(L, M).long()
    occ = torch.clamp(cnt[torch.arange(L, device="cuda")[None, :], kq.clamp(0, M - 1)], max=R)
    occ = torch.where(kq < M, occ, torch.zeros_like(occ))   # empty rows' keys hit no bucket
    occ_sum = int(occ.sum().item())
    per_q = occ.sum(dim=1).float()
    qs = torch.quantile(per_q[:min(n, 1 << 20)], torch.tensor([0.5, 0.9, 0.99, 1.0], device="cuda"))
    log("occupied ids per query: mean %.1f p50 %.0f p90 %.0f p99 %.0f max %.0f; >1024: %.3f >2048: %.3f"
        % (per_q.mean().item(), *qs.tolist(), (per_q > 1024).float().mean().item(),
           (per_q > 2048).float().mean().item()))
    bytes_hash = 4 * nnz + 8 * (n + 1) + 4 * n * L
    # insert: read the keys (4 B per insertion), stage an (id, priority)
    # pair per insertion (12 B), write every reservoir's header (4 B) and the
    # kept ids (4 B per occupied slot)
    n_ins = int((kq < M).sum().item())
    nb = L * M
    bytes_insert = 4 * n * L + 12 * n_ins + 4 * nb + 4 * int(torch.clamp(cnt, max=R).sum().item())
    bytes_query = 4 * n * L * 2 + 4 * occ_sum + 8 * n * k + 4 * n
    phases = {
        "hash": {"ms": round(float(ph[0]), 4), "alg_bytes": bytes_hash,
                 "GBps": round(bytes_hash / (ph[0] * 1e6), 1)},
        "insert": {"ms": round(float(ph[1]), 4), "alg_bytes": bytes_insert,
                   "GBps": round(bytes_insert / (ph[1] * 1e6), 1)},
        "query": {"ms": round(float(ph[2]), 4), "alg_bytes": bytes_query,
                  "GBps": round(bytes_query / (ph[2] * 1e6), 1),
                  "occupied_ids_per_query": round(occ_sum / n, 1)},
    }
    dom = max(("hash", "query"), key=lambda x: phases[x]["ms"])
    kernel = {"hash": "doph_hash_kernel", "query": "count_topk"}[dom]
    achieved = phases[dom]["alg_bytes"] / (phases[dom]["ms"] * 1e6)
    traffic = _traffic(args.traffic_table, args.workload, kernel)
    roofline = {"bound": "hbm",
                "kernel": kernel + (" kernels (filter stage + counting-table stages)" if dom == "query" else ""),
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic}

    recall = None
    if args.recall_queries > 0:
        sel = np.sort(np.random.default_rng(3).choice(n, size=min(args.recall_queries, n), replace=False))
        sel_d = torch.from_numpy(sel).cuda()
        t1 = time.time()
        recall = recall_exact_jaccard(rp, ci, spec.n_cols, rp, ci, oi.view(n, k)[sel_d], self_ids=sel,
                                      q_rows=sel)
        log(f"R@{k} over {len(sel)} sampled rows: {recall} ({time.time() - t1:.1f}s)")

    serving_leg = None
    if args.serving_leg and args.workload == "webspam":
        env = _url_serving_setup()
        rates = [float(x) for x in args.serving_leg.split(",")]
        table = _serving_rates(env, rates, 6000, 1000, 1, args.slots, 4 << 30)
        serving_leg = {"workload": "url-shaped serving (2.4M-row index; batches of 1..4096 queries, "
                                   "k in {10, 50, 200}, Poisson arrivals)",
                       "requests_per_rate": 6000, "warmup_requests": 1000, "slots": args.slots,
                       "rates": [{"offered_qps": r["offered_qps"],
                                  "continuous": {x: r["continuous"][x] for x in ("p50_ms", "p99_ms", "qps")},
                                  "batch_all": {x: r["batch_all"][x] for x in ("p50_ms", "p99_ms", "qps")},
                                  "identical_lists": r["identical_lists"],
                                  "buffer_grows_timed": r["repeats"][0]["buffer_grows_timed"]}
                                 for r in table]}
        del env
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(rp, ci, K, L, b, R, k, n)

    out = {
        "metric": f"k-NN graph build time + queries/s ({args.workload}-shape)",
        "value": round(n / (step_ms / 1e3), 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}-shaped k-NN graph", "rows": n, "nnz": nnz,
                   "K": K, "L": L, "bits_per_hash": b, "R": R, "k": k, "seed": 1},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases": phases,
        "graph_ms_per_step": round(graph_ms, 4),
        "recall": recall,
        "serving": serving_leg,
    }
    print(json.dumps(out), flush=True)


def _url_serving_setup(rows_override=0, pool_n=400_000):
    """The serving workload's resident index (URL-shaped, 2.4M rows; K=5 L=32
    b=3 R=64) and a pool of query rows from its clusters (rows drawn with seed
    2); a request of n queries takes a random slice of n pool rows."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1709_01190_amd import datagen, flash

    spec = datagen.URL
    if rows_override:
        spec = datagen.scaled(spec, rows_override)
    t0 = time.time()
    rp, ci = datagen.make_rows(spec, 1, device="cuda")
    p = flash.flash_params.make(5, 32, 3, 64, seed=1)
    index = flash.alloc_index(p)
    ws = flash.alloc_workspace(flash.OP_BUILD, p, n_rows=spec.n_rows)
    flash.flash_build_index(p, rp, ci, index, ws)
    torch.cuda.synchronize()
    del ws
    log(f"url-shaped index: {spec.n_rows} rows, {int(ci.numel())} nnz, built in {time.time() - t0:.1f}s")
    qrp_d, qci_d = datagen.make_rows(dataclasses.replace(spec, n_rows=pool_n), 1, device="cuda", row_seed=2)
    qrp, qci = qrp_d.cpu().numpy(), qci_d.cpu().numpy()
    del qrp_d, qci_d

    def rows(n, seed):
        st = np.random.default_rng(seed).integers(0, pool_n - n + 1)
        a, b = int(qrp[st]), int(qrp[st + n])
        return (qrp[st:st + n + 1] - a).astype(np.int64), qci[a:b].copy()

    return {"spec": spec, "p": p, "index": index, "rp": rp, "ci": ci,
            "rows": rows, "qrp": qrp, "qci": qci, "pool_n": pool_n}


def _serving_rates(env, rates, n_requests, warmup, repeats, slots, budget):
    """Continuous batching against batch-all at each offered rate: `warmup`
    untimed requests at that rate through both servers, then `repeats` timed
    runs of `n_requests` each (fresh arrivals per repeat, the same for both
    servers).  Every continuous slot is sized beforehand for the largest
    request and batch-all's slot for 64K queries, so that no timed request
    allocates; the number of buffer growths inside the timed runs is
    reported (0 expected)."""
    import numpy as np
    import torch

    from paper_1709_01190_amd import serving

    rows = env["rows"]
    ex = serving.GpuExecutor(env["p"], env["index"], env["spec"].n_rows)
    cont = serving.ContinuousServer(ex, budget_bytes=budget, slots=slots)
    batch = serving.BatchAllServer(ex, budget_bytes=budget)
    max_batch = 4096
    cont.reserve([serving.Request(0, 0.0, np.zeros(max_batch + 1, np.int64), np.zeros(max_batch * 2000, np.int32),
                                  200)])
    batch.reserve(65536, 65536 * 200, 200)
    table = []
    for rate in rates:
        seed0 = int(rate) % 100_003
        if warmup:
            cont.run(serving.make_requests(rows, warmup, qps=rate, seed=seed0 + 7919))
            batch.run(serving.make_requests(rows, warmup, qps=rate, seed=seed0 + 7919))
            torch.cuda.synchronize()
        reps = []
        for rep in range(repeats):
            g0 = ex.grows
            reqs = serving.make_requests(rows, n_requests, qps=rate, seed=seed0 + 104_729 * rep)
            c = cont.run(reqs)
            c_lists = [(r.out_ids, r.out_counts) for r in reqs]
            reqs2 = serving.make_requests(rows, n_requests, qps=rate, seed=seed0 + 104_729 * rep)
            b = batch.run(reqs2)
            same = all(np.array_equal(x[0], r.out_ids) and np.array_equal(x[1], r.out_counts)
                       for x, r in zip(c_lists, reqs2) if not r.rejected)
            reps.append({"continuous": {k2: round(v, 3) for k2, v in c.items()},
                         "batch_all": {k2: round(v, 3) for k2, v in b.items()},
                         "identical_lists": bool(same), "buffer_grows_timed": ex.grows - g0})
            log(json.dumps({"offered_qps": rate, "repeat": rep, **reps[-1]}))
        row = {"offered_qps": rate, "repeats": reps}
        for side in ("continuous", "batch_all"):
            for key in ("p50_ms", "p99_ms", "qps"):
                vals = [r[side][key] for r in reps]
                row.setdefault(side, {})[key] = round(float(np.median(vals)), 3)
                row[side][key + "_range"] = [round(min(vals), 3), round(max(vals), 3)]
        row["continuous_p99_wins"] = sum(r["continuous"]["p99_ms"] <= r["batch_all"]["p99_ms"] for r in reps)
        row["identical_lists"] = all(r["identical_lists"] for r in reps)
        table.append(row)
    return table


def serving_bench(args):
    """p50/p99 latency and throughput of the continuous-batching server against
    plain batch-all, on a resident URL-shaped index (2.4M rows; K=5 L=32 b=3
    R=64), with Poisson arrivals of batches of 1..4096 URL-shaped queries and
    k in {10, 50, 200}; R@50 of sampled queries against brute-force Jaccard."""
    import numpy as np
    import torch

    from paper_1709_01190_amd import flash

    torch.cuda.set_device(0)
    env = _url_serving_setup(args.rows)
    spec, p, index = env["spec"], env["p"], env["index"]
    budget = 4 << 30
    rates = [float(x) for x in args.rates.split(",")]
    table = _serving_rates(env, rates, args.requests, args.serving_warmup, args.serving_repeats,
                           args.slots, budget)
    recall = None
    if args.recall_queries > 0:
        qrp, qci, pool_n = env["qrp"], env["qci"], env["pool_n"]
        rng = np.random.default_rng(3)
        sel = np.sort(rng.choice(pool_n, size=min(args.recall_queries, pool_n), replace=False))
        k = 50
        srp = np.concatenate([[0], np.cumsum(qrp[sel + 1] - qrp[sel])]).astype(np.int64)
        sci = np.concatenate([qci[qrp[i]:qrp[i + 1]] for i in sel]).astype(np.int32)
        srp_d, sci_d = torch.from_numpy(srp).cuda(), torch.from_numpy(sci).cuda()
        oi = torch.empty(len(sel) * k, dtype=torch.int32, device="cuda")
        oc = torch.empty_like(oi)
        qws = flash.alloc_workspace(flash.OP_QUERY, p, n_queries=len(sel), k=k)
        flash.flash_query_batch(p, index, spec.n_rows, srp_d, sci_d, k, oi, oc, qws)
        torch.cuda.synchronize()
        t1 = time.time()
        recall = recall_exact_jaccard(env["rp"], env["ci"], spec.n_cols, srp_d, sci_d, oi.view(len(sel), k))
        log(f"R@{k} over {len(sel)} sampled queries: {recall} ({time.time() - t1:.1f}s)")
    top = max(table, key=lambda r: r["offered_qps"]) if table else None
    out = {
        "metric": "serving p99 latency (url-shape index, continuous batching)",
        "value": top["continuous"]["p99_ms"] if top else None,
        "unit": "ms",
        "n_gpus": 1,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "url-shaped serving", "index_rows": spec.n_rows, "K": 5, "L": 32,
                   "bits_per_hash": 3, "R": 64, "k": [10, 50, 200], "batch": [1, 4096],
                   "requests_per_rate": args.requests, "warmup_requests": args.serving_warmup,
                   "repeats": args.serving_repeats, "hbm_budget_bytes": budget, "slots": args.slots},
        "rates": table,
        "recall": recall,
    }
    print(json.dumps(out), flush=True)


def uneven_bench(args):
    """Batched uneven queries against a resident 40M-row click-log-shaped index
    (K=4, L=32, b=4, R=256): 1M queries whose sizes are Pareto,
    clip(floor(5 U^-1), 5, 50000), drawn from the index's clusters, with k in
    {10, 100} by a fair coin.  One persistent flash_query_batch_mixed launch
    sequence (autotuned on the first 128K queries) against one
    flash_query_batch call per (power-of-two size class, k) bucket; the
    buckets' CSR gathers happen before the timed region."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1709_01190_amd import datagen, flash

    torch.cuda.set_device(0)
    spec = datagen.CLICKLOG
    if args.rows:
        spec = datagen.scaled(spec, args.rows)
    K, L, b, R = 4, 32, 4, 256
    t0 = time.time()
    rp, ci = datagen.make_rows(spec, 1, device="cuda")
    torch.cuda.synchronize()
    log(f"click-log-shaped index rows: {spec.n_rows} rows, {int(ci.numel())} nnz in {time.time() - t0:.1f}s")
    p = flash.flash_params.make(K, L, b, R, seed=1)
    index = flash.alloc_index(p)
    ws = flash.alloc_workspace(flash.OP_BUILD, p, n_rows=spec.n_rows)
    stream = torch.cuda.current_stream()
    build_ms = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        flash.flash_build_index(p, rp, ci, index, ws, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        build_ms.append(e0.elapsed_time(e1))
    del ws
    log(f"index build (hash + insert of {spec.n_rows} rows): {build_ms} ms")

    nq = args.queries
    sizes = datagen.heavy_tail_sizes(nq, 5, 50_000, 1.0, seed=2, device="cuda")
    qrp, qci = datagen.make_rows(dataclasses.replace(spec, n_rows=nq), 1, device="cuda", row_seed=2,
                                 sizes=sizes)
    g = torch.Generator(device="cpu")
    g.manual_seed(2)
    kq_h = torch.where(torch.rand(nq, generator=g) < 0.5, 10, 100).to(torch.int32)
    kq = kq_h.cuda()
    lens = (qrp[1:] - qrp[:-1])
    torch.cuda.synchronize()
    log(f"queries: {nq}, {int(qci.numel())} nnz, median {int(lens.median())}, max {int(lens.max())}")
    kmax = 100
    oi = torch.empty(nq * kmax, dtype=torch.int32, device="cuda")
    oc = torch.empty_like(oi)
    qws = flash.alloc_workspace(flash.OP_QUERY, p, n_queries=nq, k=kmax)

    def timed(fn, reps):
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return out

    def persistent():
        flash.flash_query_batch_mixed(p, index, spec.n_rows, qrp, qci, kq, kmax, oi, oc, qws,
                                      stream=stream)

    flash.flash_set_tuning(None)
    timed(persistent, args.warmup)
    default_ms = timed(persistent, args.steps)
    if args.no_autotune:
        best = flash.flash_get_tuning()
    else:
        # autotune on the first 128K queries
        ns = min(nq, 131072)
        srp, sci = qrp[:ns + 1], qci[: int(qrp[ns])]
        soi = torch.empty(ns * kmax, dtype=torch.int32, device="cuda")
        soc = torch.empty_like(soi)
        sws = flash.alloc_workspace(flash.OP_QUERY, p, n_queries=ns, k=kmax)
        best, best_ms = flash.flash_autotune_query_batch(p, index, spec.n_rows, srp, sci, kq[:ns].contiguous(),
                                                         kmax, soi, soc, sws, reps=2, stream=stream)
        log(f"autotuned on {ns} queries: {best.as_dict()} ({best_ms:.3f} ms)")
    timed(persistent, args.warmup)
    tuned_ms = timed(persistent, args.steps)
    torch.cuda.synchronize()

    # the query kernels alone, on the batch's precomputed keys (the same
    # tuning): their time, and their algorithmic bytes per query = 4L (keys)
    # + 4L (reservoir headers) + 4 per occupied slot + 8k (outputs)
    qkeys = torch.empty(nq * L, dtype=torch.int32, device="cuda")
    flash.flash_hash(p, qrp, qci, qkeys, stream=stream)
    qoi, qoc = torch.empty_like(oi), torch.empty_like(oc)
    kws = flash.alloc_workspace(flash.OP_QUERY_KEYS, p, n_queries=nq, k=kmax)

    def query_only():
        flash.flash_query_keys_mixed(p, index, spec.n_rows, qkeys, kq, kmax, qoi, qoc, kws, stream=stream)

    timed(query_only, args.warmup)
    query_ms = timed(query_only, args.steps)
    M = p.M
    counts = flash.index_parts(p, index)[0].reshape(L, M).long()
    kk = qkeys.view(nq, L).long() & 0xFFFFFFFF
    occ = torch.clamp(counts[torch.arange(L, device="cuda")[None, :], kk.clamp(0, M - 1)], max=R)
    occ_sum = int(torch.where(kk < M, occ, torch.zeros_like(occ)).sum().item())
    q_alg = nq * 8 * L + 4 * occ_sum + 8 * int(kq.long().sum().item())
    same_query_only = bool(torch.equal(qoi, oi) and torch.equal(qoc, oc))

    # baseline: one launch per (size class, k) bucket, default tuning
    flash.flash_set_tuning(None)
    cls = torch.ceil(torch.log2(lens.double())).to(torch.int64)
    bucket_key = (cls * 1000 + kq.to(torch.int64)).cpu().numpy()
    buckets = []
    for key in (np.unique(bucket_key) if not args.no_per_bucket else []):
        sel = torch.from_numpy(np.nonzero(bucket_key == key)[0]).cuda()
        blen = lens[sel]
        brp = torch.zeros(sel.numel() + 1, dtype=torch.int64, device="cuda")
        brp[1:] = torch.cumsum(blen, 0)
        starts = torch.repeat_interleave(qrp[:-1][sel] - brp[:-1], blen)
        bci = qci[starts + torch.arange(int(brp[-1]), device="cuda")]
        bk = int(key % 1000)
        boi = torch.empty(sel.numel() * bk, dtype=torch.int32, device="cuda")
        boc = torch.empty_like(boi)
        bws = flash.alloc_workspace(flash.OP_QUERY, p, n_queries=sel.numel(), k=bk)
        buckets.append((sel, brp, bci, bk, boi, boc, bws))
    log(f"per-bucket baseline: {len(buckets)} (size class, k) buckets")

    def per_bucket():
        for sel, brp, bci, bk, boi, boc, bws in buckets:
            flash.flash_query_batch(p, index, spec.n_rows, brp, bci, bk, boi, boc, bws, stream=stream)

    same = same_query_only
    bucket_ms = [math.nan]
    if not args.no_per_bucket:
        timed(per_bucket, args.warmup)
        bucket_ms = timed(per_bucket, args.steps)
        # identical lists: scatter the buckets back into query order
        got_i = torch.full((nq, kmax), -1, dtype=torch.int32, device="cuda")
        got_c = torch.zeros((nq, kmax), dtype=torch.int32, device="cuda")
        for sel, brp, bci, bk, boi, boc, bws in buckets:
            got_i[sel, :bk] = boi.view(-1, bk)
            got_c[sel, :bk] = boc.view(-1, bk)
        same = same and bool(torch.equal(got_i.view(-1), oi) and torch.equal(got_c.view(-1), oc))
    med = lambda v: float(np.median(v))
    t_p, t_b = med(tuned_ms), med(bucket_ms)
    t_q = med(query_ms)
    achieved = q_alg / (t_q * 1e6)
    out = {
        "metric": "uneven batch queries per second (40M-row click-log-shape index)",
        "value": round(nq / (t_p / 1e3), 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_p, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "click-log-shaped uneven batch", "index_rows": spec.n_rows,
                   "index_nnz": int(ci.numel()), "queries": nq, "query_nnz": int(qci.numel()),
                   "K": K, "L": L, "bits_per_hash": b, "R": R, "k": [10, 100]},
        "persistent_autotuned_ms": round(t_p, 3),
        "persistent_default_ms": round(med(default_ms), 3),
        "per_bucket_ms": round(t_b, 3) if not args.no_per_bucket else None,
        "per_bucket_launches": len(buckets),
        "speedup_vs_per_bucket": round(t_b / t_p, 3) if not args.no_per_bucket else None,
        "roofline": {"bound": "hbm", "kernel": "count_topk kernels (the query on precomputed keys)",
                     "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(achieved / 8000.0, 4),
                     "traffic": _traffic(args.traffic_table, "uneven", "count_topk")},
        "query_only_ms": round(t_q, 3),
        "query_alg_bytes": q_alg,
        "occupied_ids_per_query": round(occ_sum / nq, 1),
        "tuning": best.as_dict(),
        "index_build_ms": round(med(build_ms), 3),
        "identical_lists": same,
    }
    print(json.dumps(out), flush=True)


def append_bench(args):
    """Incremental insertion: the URL-shaped index (2.4M rows; K=5 L=32 b=3
    R=64) grown by flash_build_index_append in equal batches, against one
    flash_build_index over all rows; the tables must be identical."""
    import numpy as np
    import torch

    from paper_1709_01190_amd import datagen, flash

    torch.cuda.set_device(0)
    spec = datagen.URL
    if args.rows:
        spec = datagen.scaled(spec, args.rows)
    n = spec.n_rows
    rp, ci = datagen.make_rows(spec, 1, device="cuda")
    p = flash.flash_params.make(5, 32, 3, 64, seed=1)
    stream = torch.cuda.current_stream()
    index1 = flash.alloc_index(p)
    ws = flash.alloc_workspace(flash.OP_BUILD, p, n_rows=n)

    def timed(fn, reps):
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return out

    one = timed(lambda: flash.flash_build_index(p, rp, ci, index1, ws, stream=stream), args.warmup + args.steps)
    del ws
    cuts = [round(n * j / args.batches) for j in range(args.batches + 1)]
    batches = []
    for lo, hi in zip(cuts, cuts[1:]):
        a, b = int(rp[lo]), int(rp[hi])
        batches.append((lo, (rp[lo:hi + 1] - a).contiguous(), ci[a:b]))
    bws = flash.alloc_workspace(flash.OP_BUILD, p, n_rows=max(hi - lo for lo, hi in zip(cuts, cuts[1:])))
    index2 = flash.alloc_index(p)
    c2, i2 = flash.index_parts(p, index2)

    def grow():
        c2.zero_()
        for lo, brp, bci in batches:
            flash.flash_build_index_append(p, brp, bci, lo, index2, bws, stream=stream)

    grown = timed(grow, args.warmup + args.steps)
    L, M, R = p.L, p.M, p.R
    c1, i1 = flash.index_parts(p, index1)
    same_counts = bool(torch.equal(c1, c2))
    occ = torch.clamp(c1.reshape(L, M).long(), max=R)
    mask = torch.arange(R, device="cuda")[None, None, :] < occ[:, :, None]
    same_ids = bool(torch.equal(i1.reshape(L, M, R)[mask], i2.reshape(L, M, R)[mask]))
    t_one = float(np.median(one[args.warmup:]))
    t_grow = float(np.median(grown[args.warmup:]))
    out = {
        "metric": "incremental insertion rows per second (url-shape index grown in batches)",
        "value": round(n / (t_grow / 1e3), 1),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_grow, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "url-shaped incremental build", "rows": n, "nnz": int(ci.numel()),
                   "K": 5, "L": 32, "bits_per_hash": 3, "R": 64, "batches": args.batches},
        "one_shot_build_ms": round(t_one, 3),
        "grown_build_ms": round(t_grow, 3),
        "identical_tables": same_counts and same_ids,
    }
    print(json.dumps(out), flush=True)


def rerank_bench(args):
    """Count-ranked candidates re-ranked by exact similarity: 100K URL-shaped
    queries (from the index's clusters) against the resident URL-shaped
    index; FLASH's top-200 by count, then flash_rerank_exact by cosine to a
    top-10.  Reports both times and S@10 (mean cosine of the top 10, Sec. 4.3)
    of FLASH's own top-10 and of the re-ranked one."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1709_01190_amd import datagen, flash

    torch.cuda.set_device(0)
    spec = datagen.URL
    if args.rows:
        spec = datagen.scaled(spec, args.rows)
    rp, ci = datagen.make_rows(spec, 1, device="cuda")
    p = flash.flash_params.make(5, 32, 3, 64, seed=1)
    index = flash.alloc_index(p)
    ws = flash.alloc_workspace(flash.OP_BUILD, p, n_rows=spec.n_rows)
    flash.flash_build_index(p, rp, ci, index, ws)
    del ws
    nq = min(args.queries, 100_000)
    qrp, qci = datagen.make_rows(dataclasses.replace(spec, n_rows=nq), 1, device="cuda", row_seed=2)
    kc, k = 200, 10
    stream = torch.cuda.current_stream()
    cand = torch.empty(nq * kc, dtype=torch.int32, device="cuda")
    cc = torch.empty_like(cand)
    qws = flash.alloc_workspace(flash.OP_QUERY, p, n_queries=nq, k=kc)
    oi = torch.empty(nq * k, dtype=torch.int32, device="cuda")
    on = torch.empty_like(oi)

    def timed(fn, reps):
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return out

    q_ms = timed(lambda: flash.flash_query_batch(p, index, spec.n_rows, qrp, qci, kc, cand, cc, qws,
                                                 stream=stream), args.warmup + args.steps)
    c2 = cand.view(nq, kc)
    r_ms = timed(lambda: flash.flash_rerank_exact(flash.SIM_COSINE, rp, ci, qrp, qci, c2, k, oi, on,
                                                  stream=stream), args.warmup + args.steps)
    # S@10 of FLASH's count-ranked top-10 (its intersections via the same kernel)
    top10 = c2[:, :k].contiguous()
    fi = torch.empty_like(oi)
    fn_ = torch.empty_like(oi)
    flash.flash_rerank_exact(flash.SIM_COSINE, rp, ci, qrp, qci, top10, k, fi, fn_, stream=stream)
    torch.cuda.synchronize()
    rowlen = (rp[1:] - rp[:-1]).double()
    qlen = (qrp[1:] - qrp[:-1]).double()

    def s_at(ids_, inter):
        ids_ = ids_.view(nq, k).long()
        inter = inter.view(nq, k).double()
        valid = ids_ >= 0
        sz = torch.where(valid, rowlen[ids_.clamp(min=0)], torch.ones_like(inter))
        cos = torch.where(valid & (inter > 0), inter / torch.sqrt(qlen[:, None] * sz), torch.zeros_like(inter))
        return float(cos.sum(dim=1).div(k).mean().item())

    t_q = float(np.median(q_ms[args.warmup:]))
    t_r = float(np.median(r_ms[args.warmup:]))
    out = {
        "metric": "re-ranked queries per second (url-shape index, count top-200 -> exact cosine top-10)",
        "value": round(nq / ((t_q + t_r) / 1e3), 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_q + t_r, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "url-shaped exact re-rank", "index_rows": spec.n_rows, "queries": nq,
                   "K": 5, "L": 32, "bits_per_hash": 3, "R": 64, "candidates": kc, "k": k, "measure": "cosine"},
        "query_ms": round(t_q, 3),
        "rerank_ms": round(t_r, 3),
        "S_at_10_count_ranked": round(s_at(fi, fn_), 4),
        "S_at_10_reranked": round(s_at(oi, on), 4),
    }
    print(json.dumps(out), flush=True)


def share_bench(args):
    """Reservoir sharing (Sec. 3.5): the URL-shaped index at F = 1, 0.5, 0.2,
    0.1 and 0.05; index bytes, build and query times, and S@10 (mean exact
    cosine of the top 10) of 20K queries drawn from the index's clusters."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1709_01190_amd import datagen, flash

    torch.cuda.set_device(0)
    spec = datagen.URL
    if args.rows:
        spec = datagen.scaled(spec, args.rows)
    rp, ci = datagen.make_rows(spec, 1, device="cuda")
    nq, k = 20_000, 10
    qrp, qci = datagen.make_rows(dataclasses.replace(spec, n_rows=nq), 1, device="cuda", row_seed=2)
    stream = torch.cuda.current_stream()
    rowlen = (rp[1:] - rp[:-1]).double()
    qlen = (qrp[1:] - qrp[:-1]).double()

    def timed(fn, reps):
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out[1:])) if len(out) > 1 else out[0]

    rows = []
    for permille in (1000, 500, 200, 100, 50):
        p = flash.flash_params.make(5, 32, 3, 64, seed=1, share_permille=permille)
        index = flash.alloc_index(p)
        ws = flash.alloc_workspace(flash.OP_BUILD, p, n_rows=spec.n_rows)
        t_build = timed(lambda: flash.flash_build_index(p, rp, ci, index, ws, stream=stream), 3)
        del ws
        oi = torch.empty(nq * k, dtype=torch.int32, device="cuda")
        oc = torch.empty_like(oi)
        qws = flash.alloc_workspace(flash.OP_QUERY, p, n_queries=nq, k=k)
        t_query = timed(lambda: flash.flash_query_batch(p, index, spec.n_rows, qrp, qci, k, oi, oc, qws,
                                                        stream=stream), 3)
        ri = torch.empty_like(oi)
        rn = torch.empty_like(oi)
        flash.flash_rerank_exact(flash.SIM_COSINE, rp, ci, qrp, qci, oi.view(nq, k), k, ri, rn, stream=stream)
        torch.cuda.synchronize()
        idv = ri.view(nq, k).long()
        valid = idv >= 0
        sz = torch.where(valid, rowlen[idv.clamp(min=0)], torch.ones(1, device="cuda", dtype=torch.float64))
        cos = torch.where(valid & (rn.view(nq, k) > 0), rn.view(nq, k).double() / torch.sqrt(qlen[:, None] * sz),
                          torch.zeros(1, device="cuda", dtype=torch.float64))
        n_res, _, words = flash.flash_index_layout(p)
        row = {"F": permille / 1000, "reservoirs": int(n_res),
               "index_bytes": int(words * 4),
               "build_ms": round(t_build, 3), "query_ms": round(t_query, 3),
               "S_at_10": round(float(cos.sum(dim=1).div(k).mean().item()), 4)}
        log(json.dumps(row))
        rows.append(row)
        del index, qws
        torch.cuda.empty_cache()
    base = rows[0]
    out = {
        "metric": "reservoir sharing: index bytes and S@10 versus F (url-shape index)",
        "value": rows[2]["S_at_10"],
        "unit": "S@10 at F=0.2",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "url-shaped reservoir sharing", "index_rows": spec.n_rows, "queries": nq,
                   "K": 5, "L": 32, "bits_per_hash": 3, "R": 64, "k": k},
        "sweep": rows,
        "S_at_10_F1": base["S_at_10"],
    }
    print(json.dumps(out), flush=True)


def recall_exact_jaccard(rp, ci, n_cols, q_rp, q_ci, found, self_ids=None, q_rows=None):
    """R@k of the lists `found` (device int32 [Q, k], -1 padded) against brute-force
    exact Jaccard over every indexed row (device CSR rp, ci), with plain torch
    ops on the GPU: a measurement of the method's output, not part of the library.
    For each query its columns are marked in a per-column table, the table is
    gathered at every nonzero and prefix-summed in float64 (exact for 0/1 terms),
    and the sum over a row's range is its intersection with the query.  A query
    hits when a listed id ties the best exact Jaccard of any other row (self_ids[q]
    is left out); queries that share no column with another row are not scored.
    Query q is row q of (q_rp, q_ci), or row q_rows[q] if q_rows is given."""
    import torch
    n = rp.numel() - 1
    lens = rp[1:] - rp[:-1]
    mark = torch.zeros(n_cols, dtype=torch.float64, device=ci.device)
    cs = torch.zeros(ci.numel() + 1, dtype=torch.float64, device=ci.device)
    qrp = q_rp.cpu().tolist()
    hits = scored = 0
    for q in range(found.shape[0]):
        r = q if q_rows is None else int(q_rows[q])
        cols = q_ci[qrp[r]:qrp[r + 1]].long()
        mark[cols] = 1.0
        torch.index_select(mark, 0, ci, out=cs[1:])
        mark[cols] = 0.0
        cs[1:].cumsum_(0)
        inter = (cs[rp[1:]] - cs[rp[:-1]]).round().long()
        union = lens + cols.numel() - inter
        score = inter.double() / union.clamp(min=1).double()
        if self_ids is not None:
            score[int(self_ids[q])] = -1.0
        best = int(torch.argmax(score).item())
        bi, bu = int(inter[best].item()), int(union[best].item())
        if bi == 0:
            continue
        scored += 1
        f = found[q].long()
        f = f[(f >= 0) & (f < n)]
        if f.numel():
            fi, fu = inter[f], union[f]
            hits += int(((fi * bu == fu * bi) & (fi > 0)).any().item())
    return {"R_at_k": round(hits / scored, 4) if scored else None, "k": int(found.shape[1]),
            "sampled_queries": int(found.shape[0]), "scored_queries": scored,
            "gold": "exact Jaccard, brute force over every indexed row"}


def copy_calibration(mib, reps=1):
    """One device-to-device copy of `mib` MiB (the counter calibration); with
    reps > 1 also the practical HBM ceilings: the best of `reps` warm copies
    (bytes read + written per second) and of `reps` warm float64 sums over the
    same bytes (a read-only stream)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()

    def timed(fn):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1])
    ms = timed(lambda: dst.copy_(src))
    out = {"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": round(ms, 4),
           "GBps": round(8 * n / (ms * 1e6), 1)}
    if reps > 1:
        cp = min(timed(lambda: dst.copy_(src)) for _ in range(reps))
        out["warm_copy_GBps"] = round(8 * n / (cp * 1e6), 1)
        rd = min(timed(lambda: src.view(torch.float64).sum()) for _ in range(reps))
        out["warm_read_GBps"] = round(4 * n / (rd * 1e6), 1)
    print(json.dumps(out), flush=True)


def _traffic(path, workload, kernel):
    """Calibrated HBM bytes per launch for this kernel, or None if the table is
    missing or was measured on different kernel sources."""
    try:
        with open(path) as f:
            for line in f:
                w = line.split()
                if len(w) == 4 and not line.startswith("#") and w[0] == workload and w[1] == kernel:
                    return int(w[3]) if w[2] == _kernel_source_sha() else None
    except OSError:
        pass
    return None


def _kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1709_01190_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rp, ci, K, L, b, R, k, n, reps=3):
    """The CPU oracle (plain C + OpenMP over rows, queries and tables), built
    here with gcc -O3 -march=native for this host, on the same arrays: the
    whole k-NN graph (hash, build and all n queries, self left out), the
    median of `reps` runs on all host threads.  Also the tiny 10,000-row
    graph on one thread.  Input copies to the host are outside the timing."""
    import tempfile

    import numpy as np

    import oracle
    from paper_1709_01190_amd import datagen

    so = os.path.join(tempfile.mkdtemp(prefix="flash_oracle_native_"), "liboracle_native.so")
    oracle.build(force=True, out=so, opt=oracle.NATIVE_FLAGS)
    os.environ["FLASH_ORACLE_LIB"] = so   # read by oracle.lib() on its first call
    rph, cih = rp.cpu().numpy(), ci.cpu().numpy()
    op = oracle.params(K, L, b, R, seed=1)
    runs = []
    for _ in range(reps):
        t0 = time.perf_counter()
        keys = oracle.doph(op, rph, cih)
        t1 = time.perf_counter()
        counts, ids = oracle.build_tables(op, keys)
        t2 = time.perf_counter()
        oracle.query(op, counts, ids, keys, k, self_ids=np.arange(n, dtype=np.int32))
        t3 = time.perf_counter()
        runs.append((t3 - t0, t1 - t0, t2 - t1, t3 - t2))
        del keys, counts, ids
    runs.sort()
    total, th, tb, tq = runs[len(runs) // 2]
    threads = oracle.num_threads()
    log(f"cpu oracle ({threads} threads, -O3 -march=native): hash {th:.2f}s build {tb:.2f}s "
        f"query {tq:.2f}s -> {total:.2f}s for the graph (median of {reps})")
    # one thread, the tiny graph (10,000 rows; K=4 L=16 b=4 R=32 k=16)
    trp, tci = (a.numpy() for a in datagen.make_rows(datagen.TINY, 1))
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.knn_graph(oracle.params(4, 16, 4, 32, seed=1), trp, tci, 16)
    t_tiny = time.perf_counter() - t0
    oracle.set_num_threads(threads)
    log(f"cpu oracle, one thread: tiny graph {t_tiny:.3f}s")
    return {"value": round(n / total, 1), "unit": "queries/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the whole graph (hash + build of all {n} rows, all {n} queries), median of {reps}",
            "seconds_graph": round(total, 3),
            "phases_s": {"hash": round(th, 3), "build": round(tb, 3), "query": round(tq, 3)},
            "build_flags": " ".join(oracle.NATIVE_FLAGS),
            "host_cpu": _host_cpu_model(),
            "one_thread_tiny_graph_s": round(t_tiny, 4)}


if __name__ == "__main__":
    main()
