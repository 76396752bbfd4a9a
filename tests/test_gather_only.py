"""The gather-only measurement aid (include/hoqri_gather.h): library exports,
argument checks without device work, the index streams it runs on, and (GPU)
that it reads exactly the rows of those streams."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

from paper_2510_16930_amd import gather_only as GO

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hoqri_gather.h")


def test_library_exports_the_declared_entry_point():
    text = open(HEADER).read()
    declared = sorted(set(re.findall(r"^int\s+(hoqri_\w+)\s*\(", text, re.M)))
    assert declared == ["hoqri_gather_only"]
    L = GO.load()
    for name in declared:
        assert hasattr(L, name)


@pytest.mark.parametrize("nnz,wide,grid,ptr", [(16, 0, 0, 1), (15, 0, 1, 1), (0, 0, 1, 1), (16, 2, 1, 1),
                                               (16, 0, 1, 0)])
def test_argument_errors_return_before_any_launch(nnz, wide, grid, ptr):
    L = GO.load()
    p = ctypes.c_void_p(64 if ptr else 0)
    assert L.hoqri_gather_only(p, p, p, p, nnz, wide, p, grid, None) == 1


def test_streams_follow_the_plan_order():
    # labels: slices by descending size, ties by index; stream of mode n:
    # slices in index order, inside a slice the other modes' labels in C order
    rng = np.random.default_rng(3)
    dims = (30, 20, 10)
    idx = torch.from_numpy(np.stack([rng.zipf(1.5, 4000) % d for d in dims]).astype(np.int32))
    labs = GO.degree_labels(idx, dims)
    for m, d in enumerate(dims):
        deg = np.bincount(idx[m].numpy(), minlength=d)
        order = sorted(range(d), key=lambda i: (-deg[i], i))
        want = np.empty(d, dtype=np.int64)
        want[order] = np.arange(d)
        assert np.array_equal(labs[m].numpy(), want[idx[m].numpy()])
    for n in range(3):
        i1, i2, o = GO.mode_stream(idx, labs, dims, n)
        rows = sorted(zip(idx[n].tolist(), labs[o[0]].tolist(), labs[o[1]].tolist()))
        assert i1.tolist() == [r[1] for r in rows] and i2.tolist() == [r[2] for r in rows]


@pytest.mark.gpu
@pytest.mark.parametrize("wide", [False, True])
def test_reads_the_rows_of_the_streams(wide):
    dev = "cuda:0"
    print(f"[gather-only] wide={wide}", flush=True)
    g = torch.Generator().manual_seed(5)
    U1 = torch.randn(1000, 16, generator=g, dtype=torch.float64)
    U2 = torch.randn(300, 16, generator=g, dtype=torch.float64)
    nnz = 16 * 1037  # ragged against the waves' ranges
    i1 = torch.randint(0, 1000, (nnz,), generator=g, dtype=torch.int32)
    i2 = torch.randint(0, 300, (nnz,), generator=g, dtype=torch.int32)
    grid = 7
    out = torch.full((grid * 256,), float("nan"), device=dev)
    U1f, U2f = U1.float(), U2.float()
    GO.gather_only(U1f.to(dev), U2f.to(dev), i1.to(dev), i2.to(dev), wide, out, grid)
    torch.cuda.synchronize()
    terms = (U1f.double()[i1.long()] * U2f.double()[i2.long()]).sum(1)
    got = out.cpu().double()
    assert torch.isfinite(got).all()
    # every thread's float32 sum over its terms; the total against the float64 one
    bound = 64 * 2.0 ** -24 * (U1f.double()[i1.long()].abs() * U2f.double()[i2.long()].abs()).sum()
    assert abs(float(got.sum() - terms.sum())) <= float(bound)
