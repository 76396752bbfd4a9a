"""The QR step's entry point that allocates nothing (hoqri_orth_noalloc),
against hoqri_orth with a caller workspace: the same kernels on the same
partition, so the factors, R and the status agree bitwise; two calls in a row,
the second with a smaller input, so the fixed scratch is reused."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2510_16930_amd import _lib as H

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def case(rows, cols, cond, seed):
    rng = np.random.default_rng(seed)
    Q0, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    V0, _ = np.linalg.qr(rng.standard_normal((cols, cols)))
    s = np.geomspace(1.0, 1.0 / cond, cols)
    return ((Q0 * s) @ V0.T * 2.0).astype(np.float32)


def test_noalloc_orth_matches_workspace_orth():
    L = H.load()
    assert L.hoqri_orth_noalloc_scratch_bytes() >= H.hoqri_orth_workspace_size(1 << 30, 32)
    for rows, cols, cond, seed in ((1_200_000, 32, 1e3, 1), (50_000, 12, 1e2, 2)):
        print(f"[noalloc] rows={rows} cols={cols}", flush=True)
        A = torch.from_numpy(case(rows, cols, cond, seed)).to(DEV)
        U_ws, st_ws = H.hoqri_orth(A, R=(R_ws := torch.zeros((cols, cols), dtype=torch.float64, device=DEV)))
        U_na = torch.full_like(A, float("nan"))
        st_na = torch.full((1,), 7, dtype=torch.int32, device=DEV)
        R_na = torch.zeros((cols, cols), dtype=torch.float64, device=DEV)
        H.hoqri_orth_noalloc(A, U_na, R=R_na, status=st_na)
        torch.cuda.synchronize()
        assert st_ws.item() == 0 and st_na.item() == 0
        assert torch.equal(U_na, U_ws) and torch.equal(R_na, R_ws)
        Qref, _ = O.qr_positive(A.cpu().numpy().astype(np.float64))
        assert np.abs(U_na.cpu().numpy() - Qref).max() < 1e-6
    # a rank-deficient input reports breakdown and leaves U untouched, as hoqri_orth does
    B = torch.from_numpy(case(1000, 6, 1.0, 3)).to(DEV)
    B[:, 4] = B[:, 0] - 2 * B[:, 1]
    U_b = torch.zeros_like(B)
    st_b = torch.zeros(1, dtype=torch.int32, device=DEV)
    H.hoqri_orth_noalloc(B, U_b, status=st_b)
    torch.cuda.synchronize()
    assert st_b.item() == -4 and torch.count_nonzero(U_b).item() == 0
    # argument errors are detected before any launch
    with pytest.raises(H.HoqriError):
        H.hoqri_orth_noalloc(B[:, :0], U_b[:, :0], status=st_b)
