"""Seeded synthetic sparse binary rows shaped like the paper's datasets.

This module only draws inputs.  It holds none of the similarity-search
arithmetic (no hashing, bucketing or counting), so both the CPU oracle and
the HIP path can be fed from it.

Recipe (one call of ``make_rows``):

* every row picks one of ``n_clusters`` planted clusters uniformly;
* every cluster has a core of ``core = round(mean_nnz)`` columns drawn
  uniformly from ``[0, n_cols)``;
* a row's target size ``n`` is lognormal with arithmetic mean ``mean_nnz``
  and shape ``sigma`` (``mu = ln(mean_nnz) - sigma^2 / 2``), rounded and
  clipped to ``[lo, hi]``;
* the row keeps each core column with probability ``keep`` (0.6), truncated
  to ``n`` columns;
* the remaining ``n - kept`` columns are power-law noise: rank
  ``r = floor(U ** (-1 / (zipf_s - 1)))`` (a discretised Pareto whose pmf
  falls like ``r ** -zipf_s``), ranks beyond ``n_cols`` are dropped, and rank
  ``r`` maps to column ``perm[r - 1]`` of one seeded permutation of the
  columns; noise is over-drawn and the first distinct new columns in draw
  order are kept, so a row ends with at most ``n`` distinct columns;
* columns are stored sorted and distinct (int32), row pointers are int64.

The same seed on the same device type gives the same arrays.  CPU and GPU
draws differ (different torch generators); a comparison always hands one
set of arrays to both sides.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import torch


@dataclasses.dataclass(frozen=True)
class RowSpec:
    n_rows: int
    n_cols: int
    mean_nnz: float
    sigma: float = 0.5
    lo: int = 1
    hi: Optional[int] = None
    n_clusters: int = 1
    keep: float = 0.6
    zipf_s: float = 1.1


def _chunk_rows(spec: RowSpec, row0: int, nr: int, cores: torch.Tensor,
                perm: torch.Tensor, g: torch.Generator,
                device, sizes: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Rows [row0, row0 + nr): returns (nnz per row int64, sorted cols int64)."""
    core = cores.shape[1]
    if sizes is None:
        hi = spec.hi if spec.hi is not None else spec.n_cols
        mu = math.log(spec.mean_nnz) - 0.5 * spec.sigma * spec.sigma
        z = torch.randn(nr, generator=g, device=device, dtype=torch.float64)
        n = torch.exp(mu + spec.sigma * z).round().clamp_(spec.lo, min(hi, spec.n_cols)).to(torch.int64)
    else:
        n = sizes.to(device=device, dtype=torch.int64).clamp(1, spec.n_cols)
    clus = torch.randint(0, cores.shape[0], (nr,), generator=g, device=device)

    # core part: Bernoulli(keep) mask over the cluster core, first n kept
    keepmask = torch.rand(nr, core, generator=g, device=device) < spec.keep
    kept_rank = torch.cumsum(keepmask.to(torch.int64), dim=1) - 1
    keepmask &= kept_rank < n[:, None]
    kept = keepmask.sum(dim=1)
    core_cols = cores[clus]                                     # nr x core
    c_row = torch.arange(nr, device=device)[:, None].expand(nr, core)[keepmask]
    c_col = core_cols[keepmask]
    c_pri = kept_rank[keepmask]                                 # 0 .. kept-1

    # noise part: over-draw 4*deficit + 16 power-law ranks per row
    deficit = n - kept
    draws = torch.where(deficit > 0, 4 * deficit + 16, torch.zeros_like(deficit))
    tot = int(draws.sum().item())
    n_row = torch.repeat_interleave(torch.arange(nr, device=device), draws)
    start = torch.cumsum(draws, 0) - draws
    n_pri = core + (torch.arange(tot, device=device) - start[n_row])
    u = torch.rand(tot, generator=g, device=device, dtype=torch.float64).clamp_min_(1e-300)
    rank = torch.floor(u.pow(-1.0 / (spec.zipf_s - 1.0)))
    ok = rank <= spec.n_cols
    n_row, n_pri = n_row[ok], n_pri[ok]
    n_col = perm[(rank[ok].to(torch.int64) - 1)]

    row = torch.cat([c_row, n_row])
    col = torch.cat([c_col, n_col])
    pri = torch.cat([c_pri, n_pri])
    # distinct (row, col), keeping the earliest draw of each
    o = torch.argsort(pri, stable=True)
    row, col, pri = row[o], col[o], pri[o]
    o = torch.argsort(row * spec.n_cols + col, stable=True)
    row, col, pri = row[o], col[o], pri[o]
    key = row * spec.n_cols + col
    first = torch.ones_like(key, dtype=torch.bool)
    first[1:] = key[1:] != key[:-1]
    row, col, pri = row[first], col[first], pri[first]
    # keep the n earliest-drawn distinct columns of each row
    o = torch.argsort(row * (1 << 40) + pri)
    row, col = row[o], col[o]
    cnt = torch.bincount(row, minlength=nr)
    rstart = torch.cumsum(cnt, 0) - cnt
    pos = torch.arange(row.numel(), device=device) - rstart[row]
    sel = pos < n[row]
    row, col = row[sel], col[sel]
    o = torch.argsort(row * spec.n_cols + col)
    row, col = row[o], col[o]
    cnt = torch.bincount(row, minlength=nr)
    return cnt, col


def make_rows(spec: RowSpec, seed: int, device="cpu", chunk_rows: int = 65536,
              row_seed: Optional[int] = None,
              sizes: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Returns (row_ptr int64 [n_rows + 1], col_idx int32 [nnz]) on ``device``.

    ``seed`` draws the clusters and the noise permutation.  With ``row_seed``
    the rows themselves are drawn from a generator of that seed, so rows of
    another draw (queries) come from the same clusters as the rows of
    ``seed`` alone (the indexed set).  ``sizes`` (int64 [n_rows]) replaces
    the lognormal target sizes."""
    device = torch.device(device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    core = max(1, int(round(spec.mean_nnz)))
    cores = torch.randint(0, spec.n_cols, (max(1, spec.n_clusters), core),
                          generator=g, device=device)
    perm = torch.randperm(spec.n_cols, generator=g, device=device)
    if row_seed is not None:
        g = torch.Generator(device=device)
        g.manual_seed(int(row_seed))
    if sizes is not None and sizes.numel() != spec.n_rows:
        raise ValueError("sizes must have n_rows entries")
    counts, cols = [], []
    for r0 in range(0, spec.n_rows, chunk_rows):
        nr = min(chunk_rows, spec.n_rows - r0)
        c, col = _chunk_rows(spec, r0, nr, cores, perm, g, device,
                             None if sizes is None else sizes[r0:r0 + nr])
        counts.append(c)
        cols.append(col.to(torch.int32))
    cnt = torch.cat(counts) if counts else torch.zeros(0, dtype=torch.int64, device=device)
    row_ptr = torch.zeros(spec.n_rows + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(cnt, 0)
    col_idx = torch.cat(cols) if cols else torch.zeros(0, dtype=torch.int32, device=device)
    return row_ptr, col_idx


def heavy_tail_sizes(n: int, lo: int, hi: int, alpha: float, seed: int,
                     device="cpu") -> torch.Tensor:
    """Pareto sizes clip(floor(lo * U ** (-1/alpha)), lo, hi), int64."""
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(int(seed))
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64).clamp_min_(1e-300)
    return torch.floor(lo * u.pow(-1.0 / alpha)).clamp_(lo, hi).to(torch.int64)


# The workloads the method is measured on, restated as row recipes.
TINY = RowSpec(n_rows=10_000, n_cols=1 << 20, mean_nnz=100, sigma=0.5, lo=10, hi=1000,
               n_clusters=500)
WEBSPAM = RowSpec(n_rows=350_000, n_cols=16_609_143, mean_nnz=3700, sigma=0.5, lo=1,
                  n_clusters=20_000)
URL = RowSpec(n_rows=2_400_000, n_cols=3_231_961, mean_nnz=116, sigma=0.5, lo=5, hi=2000,
              n_clusters=100_000)
CLICKLOG = RowSpec(n_rows=40_000_000, n_cols=54_686_452, mean_nnz=11, sigma=0.5, lo=1, hi=200,
                   n_clusters=400_000)


def scaled(spec: RowSpec, n_rows: int) -> RowSpec:
    """Same row recipe with fewer rows; clusters shrink in proportion (at least 1)."""
    frac = n_rows / spec.n_rows
    return dataclasses.replace(spec, n_rows=n_rows,
                               n_clusters=max(1, int(round(spec.n_clusters * frac))))
