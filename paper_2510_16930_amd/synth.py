"""Seeded synthetic inputs: sparse COO tensors and raw Gaussian start matrices.

This module draws random numbers and shapes them into inputs. It holds none of
the HOQRI arithmetic (no products with factors, no QR, no contractions), so both
the GPU path and the CPU checker may take their inputs from here.

Workload shapes follow the paper's experiments: 3/4/5-way cubes with
nnz = 10I or 100I and uniform coordinates (§6.1), and Zipf-skewed
real-data-like index distributions standing in for the tagging and rating
tensors of Table 3 (§6.2), which are not available. Values are N(0,1),
lognormal(0,1) or uniform(0,1); the paper does not state a distribution.

Coordinates are returned as int32 arrays of shape [N, nnz] (structure of arrays,
0-based) and values as float64 (numpy) or float32 (torch) arrays of length nnz.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

__all__ = [
    "coo_uniform",
    "coo_zipf",
    "gaussian_start",
    "zipf_cdf",
    "coo_zipf_torch",
    "coo_uniform_torch",
    "gaussian_start_torch",
    "serve_stream_params",
    "poisson_arrivals",
]


def _draw_values(rng: np.random.Generator, n: int, kind: str) -> np.ndarray:
    if kind == "normal":
        return rng.standard_normal(n)
    if kind == "lognormal":
        return rng.lognormal(0.0, 1.0, n)
    if kind == "uniform":
        return rng.random(n)
    raise ValueError(f"unknown value distribution {kind!r}")


def coo_uniform(dims: Sequence[int], nnz: int, seed: int, values: str = "normal"):
    """nnz distinct coordinates drawn uniformly without replacement.

    Returns (idx int32 [N, nnz], vals float64 [nnz]); the order is the draw order
    (unsorted), so the plan builder's sort is exercised.
    """
    dims = [int(d) for d in dims]
    total = math.prod(dims)
    if nnz > total:
        raise ValueError("nnz exceeds the number of cells")
    rng = np.random.default_rng(seed)
    if total <= 50_000_000:
        lin = rng.choice(total, size=nnz, replace=False)
    else:
        lin = np.empty(0, dtype=np.int64)
        while lin.size < nnz:
            cand = rng.integers(0, total, size=2 * (nnz - lin.size) + 16, dtype=np.int64)
            both = np.concatenate([lin, cand])
            _, first = np.unique(both, return_index=True)
            lin = both[np.sort(first)][:nnz]
    idx = np.stack(np.unravel_index(lin, dims)).astype(np.int32)
    vals = _draw_values(rng, nnz, values)
    return idx, vals


def zipf_cdf(size: int, alpha: float) -> np.ndarray:
    """Cumulative distribution of the bounded Zipf law P(k) ~ k^-alpha, k = 1..size."""
    w = np.arange(1, size + 1, dtype=np.float64) ** (-float(alpha))
    c = np.cumsum(w)
    return c / c[-1]


def coo_zipf(dims: Sequence[int], nnz: int, alpha: float, seed: int, values: str = "lognormal",
             batch: int | None = None):
    """Exactly nnz distinct coordinates with per-mode bounded-Zipf indices.

    Each mode draws ranks from Zipf(alpha) by inverse CDF, then maps rank -> index
    through a seeded permutation so hot rows are scattered. Duplicate coordinates
    are merged by keeping the first draw (and its value); batches are drawn until
    nnz distinct coordinates exist. Returns (idx int32 [N, nnz], vals float64).
    """
    dims = [int(d) for d in dims]
    rng = np.random.default_rng(seed)
    perms = [rng.permutation(d) for d in dims]
    cdfs = [zipf_cdf(d, alpha) for d in dims]
    keys = np.empty(0, dtype=np.int64)
    vals = np.empty(0, dtype=np.float64)
    batch = batch or max(2 * nnz, 1024)
    while keys.size < nnz:
        cols = []
        for d, p, c in zip(dims, perms, cdfs):
            r = np.searchsorted(c, rng.random(batch), side="right")
            np.minimum(r, d - 1, out=r)
            cols.append(p[r])
        key = np.ravel_multi_index(tuple(cols), dims).astype(np.int64)
        v = _draw_values(rng, batch, values)
        allk = np.concatenate([keys, key])
        allv = np.concatenate([vals, v])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys, vals = allk[first], allv[first]
    keys, vals = keys[:nnz], vals[:nnz]
    idx = np.stack(np.unravel_index(keys, dims)).astype(np.int32)
    return idx, vals


def gaussian_start(dims: Sequence[int], ranks: Sequence[int], seed: int):
    """Raw N(0,1) matrices of shape I_n x K_n (seed + n for mode n), float64.

    HOQRI starts from an orthonormal basis of a random matrix (Alg. 2,
    initialisation); each side orthonormalises these with its own QR.
    """
    return [np.random.default_rng(seed + n).standard_normal((int(d), int(k)))
            for n, (d, k) in enumerate(zip(dims, ranks))]


# ---------------------------------------------------------------------------
# Device-side generators for the large workloads (tens of millions of
# nonzeros), where numpy would take minutes. Same recipe, torch Philox stream.
# ---------------------------------------------------------------------------

def _torch_values(torch, g, n, kind, device):
    if kind == "normal":
        return torch.randn(n, generator=g, device=device, dtype=torch.float32)
    if kind == "lognormal":
        return torch.randn(n, generator=g, device=device, dtype=torch.float32).exp_()
    if kind == "uniform":
        return torch.rand(n, generator=g, device=device, dtype=torch.float32)
    raise ValueError(f"unknown value distribution {kind!r}")


def coo_zipf_torch(dims: Sequence[int], nnz: int, alpha: float, seed: int, values: str = "lognormal",
                   device: str = "cuda"):
    """Device version of coo_zipf: returns (idx int32 [N, nnz], vals float32 [nnz]) on `device`.

    Distinct coordinates are kept in first-draw order with their first value.
    """
    import torch

    dims = [int(d) for d in dims]
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    perms = [torch.randperm(d, generator=g, device=device) for d in dims]
    cdfs = [torch.from_numpy(zipf_cdf(d, alpha)).to(device) for d in dims]
    strides = [math.prod(dims[m + 1:]) for m in range(len(dims))]
    keys = torch.empty(0, dtype=torch.int64, device=device)
    vals = torch.empty(0, dtype=torch.float32, device=device)
    while keys.numel() < nnz:
        batch = max(int(1.3 * (nnz - keys.numel())) + 1024, 1 << 20)
        key = torch.zeros(batch, dtype=torch.int64, device=device)
        for d, p, c, s in zip(dims, perms, cdfs, strides):
            u = torch.rand(batch, generator=g, device=device, dtype=torch.float64)
            r = torch.searchsorted(c, u, right=True).clamp_(max=d - 1)
            key += p[r].to(torch.int64) * s
        v = _torch_values(torch, g, batch, values, device)
        allk = torch.cat([keys, key])
        allv = torch.cat([vals, v])
        uniq, inv = torch.unique(allk, return_inverse=True)
        pos = torch.arange(allk.numel(), device=device, dtype=torch.int64)
        first = torch.full((uniq.numel(),), allk.numel(), dtype=torch.int64, device=device)
        first.scatter_reduce_(0, inv, pos, reduce="amin")
        first, _ = torch.sort(first)
        keys, vals = allk[first], allv[first]
        del allk, allv, uniq, inv, pos, first
    keys, vals = keys[:nnz], vals[:nnz].contiguous()
    idx = torch.empty((len(dims), nnz), dtype=torch.int32, device=device)
    rem = keys
    for m in range(len(dims) - 1, -1, -1):
        idx[m] = (rem % dims[m]).to(torch.int32)
        rem = rem // dims[m]
    return idx, vals


def coo_uniform_torch(dims: Sequence[int], nnz: int, seed: int, values: str = "normal", device: str = "cuda"):
    """Device version of coo_uniform (distinct uniform coordinates, draw order)."""
    import torch

    dims = [int(d) for d in dims]
    total = math.prod(dims)
    if nnz > total:
        raise ValueError("nnz exceeds the number of cells")
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    keys = torch.empty(0, dtype=torch.int64, device=device)
    while keys.numel() < nnz:
        batch = 2 * (nnz - keys.numel()) + 1024
        cand = torch.randint(0, total, (batch,), generator=g, device=device, dtype=torch.int64)
        allk = torch.cat([keys, cand])
        uniq, inv = torch.unique(allk, return_inverse=True)
        pos = torch.arange(allk.numel(), device=device, dtype=torch.int64)
        first = torch.full((uniq.numel(),), allk.numel(), dtype=torch.int64, device=device)
        first.scatter_reduce_(0, inv, pos, reduce="amin")
        first, _ = torch.sort(first)
        keys = allk[first]
    keys = keys[:nnz]
    vals = _torch_values(torch, g, nnz, values, device)
    idx = torch.empty((len(dims), nnz), dtype=torch.int32, device=device)
    rem = keys
    for m in range(len(dims) - 1, -1, -1):
        idx[m] = (rem % dims[m]).to(torch.int32)
        rem = rem // dims[m]
    return idx, vals


def gaussian_start_torch(dims: Sequence[int], ranks: Sequence[int], seed: int, device: str = "cuda"):
    """Raw N(0,1) float32 matrices I_n x K_n on `device` (seed + n for mode n)."""
    import torch

    out = []
    for n, (d, k) in enumerate(zip(dims, ranks)):
        g = torch.Generator(device=device)
        g.manual_seed(int(seed) + n)
        out.append(torch.randn((int(d), int(k)), generator=g, device=device, dtype=torch.float32))
    return out


def serve_stream_params(n_requests: int, seed: int, dim_range=(1_000, 200_000), nnz_range=(10_000, 2_000_000),
                        ranks=(4, 8, 16)):
    """Parameters of a stream of 3-way requests: each mode's size and the nnz are
    log-uniform on their ranges (independently), one rank from `ranks` for all
    three modes; each request also gets a data seed and a start seed."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_requests):
        dims = tuple(int(round(math.exp(rng.uniform(math.log(dim_range[0]), math.log(dim_range[1])))))
                     for _ in range(3))
        nnz = int(round(math.exp(rng.uniform(math.log(nnz_range[0]), math.log(nnz_range[1])))))
        r = int(ranks[int(rng.integers(len(ranks)))])
        out.append(dict(dims=dims, nnz=nnz, ranks=(r, r, r), data_seed=int(seed) * 100_000 + i,
                        init_seed=int(seed) * 100_000 + 50_000 + i))
    return out


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
