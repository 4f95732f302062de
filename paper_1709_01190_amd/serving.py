"""Serving loop for the FLASH query path: continuous batching over a resident index.

The index array stays in HBM.  Requests are CSR batches of query rows
with their own k.  Two servers share one interface:

* ContinuousServer: a request is admitted as soon as it has arrived, a slot
  (one HIP stream) is free and its device memory fits the HBM budget; each
  admitted request runs flash_query_batch on its own stream, so requests that
  arrive while others are on the GPU start at once and overlap on the device.
  Completion is polled with events; latency = completion seen - arrival.  A
  completed request's lists are copied out of its slot's pinned buffers in
  chunks, one per pass of the loop, so that a large result does not hold up
  the admission of the requests behind it; the slot is free again once
  drained.
* BatchAllServer: the plain baseline.  While one batch runs, arrivals wait;
  when it ends, everything that has arrived (within the budget) is
  concatenated into one batch, queried with the largest k of the batch, and
  each request takes the prefix of its own k.  The top-k by (count desc, id
  asc) is a prefix of the top-k' for k' >= k, so both servers return the same
  lists, and recall is equal by construction.

A request larger than the whole budget is rejected (it never runs).  All
arithmetic is in the HIP library; this module moves buffers and schedules.
The device side sits behind a small executor interface so that the
scheduling logic can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                # seconds after the start of the run
    row_ptr: np.ndarray           # int64 [n + 1]
    col_idx: np.ndarray           # int32 [nnz]
    k: int
    out_ids: Optional[np.ndarray] = None
    out_counts: Optional[np.ndarray] = None
    admitted: float = math.nan
    done: float = math.nan
    rejected: bool = False

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_requests(row_source: Callable[[int, int], tuple], n_requests: int, qps: float, seed: int,
                  max_batch: int = 4096, ks: Sequence[int] = (10, 50, 200)) -> List[Request]:
    """Poisson request arrivals carrying `qps` queries per second on average;
    batch sizes log-uniform on [1, max_batch]; k uniform over ks.
    row_source(n, seed) returns (row_ptr, col_idx) numpy arrays for n rows."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(0.0, math.log(max_batch + 1), size=n_requests))).astype(np.int64)
    sizes = np.clip(sizes, 1, max_batch)
    rate = qps / float(sizes.mean())                   # requests per second
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    kk = rng.choice(np.asarray(ks), size=n_requests)
    return [Request(i, float(arrivals[i]), *row_source(int(sizes[i]), int(seed) * 1_000_003 + i),
                    int(kk[i])) for i in range(n_requests)]


# ---------------------------------------------------------------- executors

class GpuExecutor:
    """Runs requests through the C ABI on per-slot HIP streams.  Each slot keeps
    its pinned host and device buffers (as large as the largest request it has
    run), so a request in steady state only copies and launches; the admission
    budget bounds the memory of the requests in flight."""

    def __init__(self, p, index, n_indexed, device="cuda"):
        import torch
        from . import flash
        self._torch, self._flash = torch, flash
        self.p, self.index, self.n_indexed = p, index, n_indexed
        self.device = torch.device(device)
        self.grows = 0   # buffers allocated or grown so far (a timed run should add none)

    def bytes_for(self, n: int, nnz: int, k: int) -> int:
        """Device memory one request holds while in flight."""
        ws = self._flash.flash_workspace_bytes(self._flash.OP_QUERY, self.p, n_queries=n, k=k)
        return 8 * (n + 1) + 4 * nnz + ws + 8 * n * k

    def new_slot(self):
        torch = self._torch
        return {"stream": torch.cuda.Stream(device=self.device), "event": torch.cuda.Event(),
                "bufs": {}}

    def _buf(self, slot, name, numel, dtype, pinned):
        """The slot's buffer `name` with at least numel elements (grown by
        doubling, then reused), so that steady-state requests neither pin host
        memory nor allocate device memory.  A slot is reused only after its
        previous request has completed, so its buffers are free again."""
        torch = self._torch
        numel = max(int(numel), 1)
        t = slot["bufs"].get(name)
        if t is None or t.numel() < numel:
            cap = max(numel, 2 * (t.numel() if t is not None else 0))
            t = (torch.empty(cap, dtype=dtype, pin_memory=True) if pinned
                 else torch.empty(cap, dtype=dtype, device=self.device))
            slot["bufs"][name] = t
            self.grows += 1
        return t[:numel]

    def reserve(self, slot, n: int, nnz: int, k: int) -> None:
        """Grows the slot's buffers now to what a request of n queries, nnz
        columns and this k needs, so that no request up to that size
        allocates or pins memory while it is being timed."""
        torch, flash = self._torch, self._flash
        i64, i32, u8 = torch.int64, torch.int32, torch.uint8
        wsb = flash.flash_workspace_bytes(flash.OP_QUERY, self.p, n_queries=n, k=k)
        with torch.cuda.stream(slot["stream"]):   # device buffers belong to the slot's stream
            for name, numel, dtype, pinned in (("rp_h", n + 1, i64, True), ("ci_h", nnz, i32, True),
                                               ("rp_d", n + 1, i64, False), ("ci_d", nnz, i32, False),
                                               ("oi", n * k, i32, False), ("oc", n * k, i32, False),
                                               ("ws", wsb, u8, False), ("oi_h", n * k, i32, True),
                                               ("oc_h", n * k, i32, True)):
                self._buf(slot, name, numel, dtype, pinned)
        torch.cuda.synchronize(self.device)

    def launch(self, slot, row_ptr: np.ndarray, col_idx: np.ndarray, k: int) -> None:
        torch, flash = self._torch, self._flash
        n = row_ptr.shape[0] - 1
        nnz = col_idx.shape[0]
        s = slot["stream"]
        i64, i32, u8 = torch.int64, torch.int32, torch.uint8
        rp_h = self._buf(slot, "rp_h", n + 1, i64, True)
        ci_h = self._buf(slot, "ci_h", nnz, i32, True)
        rp_h.numpy()[:] = row_ptr
        if nnz:
            ci_h.numpy()[:nnz] = col_idx
        wsb = flash.flash_workspace_bytes(flash.OP_QUERY, self.p, n_queries=n, k=k)
        with torch.cuda.stream(s):
            rp_d = self._buf(slot, "rp_d", n + 1, i64, False)
            ci_d = self._buf(slot, "ci_d", nnz, i32, False)
            oi = self._buf(slot, "oi", n * k, i32, False)
            oc = self._buf(slot, "oc", n * k, i32, False)
            ws = self._buf(slot, "ws", wsb, u8, False)
            rp_d.copy_(rp_h, non_blocking=True)
            ci_d.copy_(ci_h, non_blocking=True)
            if n > 0:
                flash.flash_query_batch(self.p, self.index, self.n_indexed, rp_d,
                                        ci_d[:nnz], k, oi, oc, ws, stream=s)
            oi_h = self._buf(slot, "oi_h", n * k, i32, True)
            oc_h = self._buf(slot, "oc_h", n * k, i32, True)
            oi_h.copy_(oi, non_blocking=True)
            oc_h.copy_(oc, non_blocking=True)
            slot["event"].record(s)
        slot["out"] = (oi_h, oc_h)

    def done(self, slot) -> bool:
        return bool(slot["event"].query())

    def result(self, slot, n: int, k: int):
        oi_h, oc_h = slot.pop("out")
        return (oi_h.numpy()[: n * k].reshape(n, k).copy(), oc_h.numpy()[: n * k].reshape(n, k).copy())

    def result_views(self, slot, n: int, k: int):
        """The completed request's lists (flat, n * k each) as views of the
        slot's pinned buffers, valid until the slot is launched again."""
        oi_h, oc_h = slot.pop("out")
        return oi_h.numpy()[: n * k], oc_h.numpy()[: n * k]


# ---------------------------------------------------------------- servers

def _reserve(executor, slot, n: int, nnz: int, k: int) -> None:
    if hasattr(executor, "reserve"):
        executor.reserve(slot, n, nnz, k)


class ContinuousServer:
    """Continuous batching: admit by arrival, a free slot and the HBM budget."""

    drain_chunk = 1 << 16   # list entries copied out of a completed slot per loop pass

    def __init__(self, executor, budget_bytes: int = 4 << 30, slots: int = 8):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = [executor.new_slot() for _ in range(slots)]

    def reserve(self, requests: List[Request]) -> None:
        """Sizes every slot for the largest of these requests (queries,
        columns and outputs taken separately), so that none of them
        allocates while it is timed."""
        if not requests:
            return
        n = max(r.n for r in requests)
        nnz = max(r.nnz for r in requests)
        k = max(r.k for r in requests)
        for slot in self.slots:
            _reserve(self.ex, slot, n, nnz, k)

    def run(self, requests: List[Request], clock=time.perf_counter) -> Dict:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        free = list(range(len(self.slots)))
        busy: Dict[int, tuple] = {}
        draining: collections.deque = collections.deque()   # [slot, request, copied, views]
        views = hasattr(self.ex, "result_views")
        in_use = 0
        t0 = clock()
        while pending or busy or draining:
            now = clock() - t0
            progressed = False
            for si in list(busy):
                if self.ex.done(self.slots[si]):
                    seen = clock() - t0
                    r, nbytes = busy.pop(si)
                    r.done = seen
                    in_use -= nbytes          # the device memory is free; the pinned lists are not yet
                    if views:
                        r.out_ids = np.empty((r.n, r.k), np.int32)
                        r.out_counts = np.empty((r.n, r.k), np.int32)
                        draining.append([si, r, 0, self.ex.result_views(self.slots[si], r.n, r.k)])
                    else:
                        r.out_ids, r.out_counts = self.ex.result(self.slots[si], r.n, r.k)
                        free.append(si)
                    progressed = True
            if draining:
                d = draining[0]
                si, r, pos, (vi, vc) = d
                end = min(pos + self.drain_chunk, r.n * r.k)
                r.out_ids.reshape(-1)[pos:end] = vi[pos:end]
                r.out_counts.reshape(-1)[pos:end] = vc[pos:end]
                d[2] = end
                if end >= r.n * r.k:
                    draining.popleft()
                    free.append(si)
                progressed = True
            now = clock() - t0
            # one admission per pass, so completions are seen between launches
            if pending and pending[0].arrival <= now and free:
                r = pending[0]
                need = self.ex.bytes_for(r.n, r.nnz, r.k)
                if need > self.budget:
                    pending.popleft()
                    r.rejected = True
                    progressed = True
                elif in_use + need <= self.budget:          # else wait until memory frees up
                    pending.popleft()
                    si = free.pop()
                    in_use += need
                    r.admitted = now
                    self.ex.launch(self.slots[si], r.row_ptr, r.col_idx, r.k)
                    busy[si] = (r, need)
                    progressed = True
            if not progressed and not busy and not draining and pending:
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        return summarize(requests)


class BatchAllServer:
    """Baseline: one batch at a time; everything that has arrived goes in."""

    def __init__(self, executor, budget_bytes: int = 4 << 30):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slot = executor.new_slot()

    def reserve(self, n: int, nnz: int, k: int) -> None:
        """Sizes the one slot for a batch of n queries, nnz columns and k."""
        _reserve(self.ex, self.slot, n, nnz, k)

    def run(self, requests: List[Request], clock=time.perf_counter) -> Dict:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = clock()
        running: List[Request] = []
        kmax = 0
        while pending or running:
            now = clock() - t0
            if running:
                if self.ex.done(self.slot):
                    done = clock() - t0
                    total = sum(r.n for r in running)
                    oi, oc = self.ex.result(self.slot, total, kmax)
                    off = 0
                    for r in running:
                        r.out_ids = oi[off:off + r.n, : r.k].copy()
                        r.out_counts = oc[off:off + r.n, : r.k].copy()
                        r.done = done
                        off += r.n
                    running = []
                continue
            if pending and pending[0].arrival <= now:
                batch: List[Request] = []
                while pending and pending[0].arrival <= now:
                    r = pending[0]
                    if self.ex.bytes_for(r.n, r.nnz, r.k) > self.budget:
                        pending.popleft()
                        r.rejected = True
                        continue
                    k2 = max([x.k for x in batch] + [r.k])
                    n2 = sum(x.n for x in batch) + r.n
                    z2 = sum(x.nnz for x in batch) + r.nnz
                    if batch and self.ex.bytes_for(n2, z2, k2) > self.budget:
                        break
                    pending.popleft()
                    batch.append(r)
                if not batch:
                    continue
                kmax = max(r.k for r in batch)
                rps, base = [np.zeros(1, np.int64)], 0
                for r in batch:
                    rps.append(r.row_ptr[1:] + base)
                    base += int(r.row_ptr[-1])
                rp = np.concatenate(rps)
                ci = np.concatenate([r.col_idx for r in batch])
                for r in batch:
                    r.admitted = now
                self.ex.launch(self.slot, rp, ci, kmax)
                running = batch
                continue
            if pending:
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        return summarize(requests)


def summarize(requests: List[Request]) -> Dict:
    ok = [r for r in requests if not r.rejected]
    lat = np.array([r.latency for r in ok], dtype=np.float64)
    queries = sum(r.n for r in ok)
    span = max((r.done for r in ok), default=0.0) - min((r.arrival for r in ok), default=0.0)
    return {
        "requests": len(ok),
        "rejected": len(requests) - len(ok),
        "queries": int(queries),
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else math.nan,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else math.nan,
        "mean_ms": float(lat.mean() * 1e3) if lat.size else math.nan,
        "qps": float(queries / span) if span > 0 else math.nan,
    }
