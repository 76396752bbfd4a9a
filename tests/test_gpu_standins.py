"""Stand-ins with the shapes of the paper's workloads on the GPU, against the
FP64 oracle: Table 3's real-tensor shapes (dims and nnz; Zipf coordinates stand
in for the missing datasets) at the ranks of its convergence figures, and
Fig. 1's I x I x I random tensors with nnz = 10 I.

FP32 runs follow the FP64 trajectory closely: after 3 sweeps from the same
start the fit agrees within 1e-5 relative and the factors stay orthonormal.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2510_16930_amd import _lib as H
from paper_2510_16930_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


CASES = [
    ("movielens", (610, 49_961, 8_215), 84_159, (10, 10, 10), "zipf"),
    ("movielens", (610, 49_961, 8_215), 84_159, (15, 25, 15), "zipf"),
    ("last", (2_100, 18_744, 12_647), 186_479, (15, 15, 15), "zipf"),
    ("fig1", (10_000, 10_000, 10_000), 100_000, (10, 10, 10), "uniform"),
]


@pytest.mark.parametrize("name,dims,nnz,K,dist", CASES)
def test_standin_run_follows_oracle(name, dims, nnz, K, dist):
    print(f"[standin] {name} dims={dims} nnz={nnz} K={K}", flush=True)
    if dist == "zipf":
        idx, vals = synth.coo_zipf(dims, nnz, alpha=1.2, seed=16)
    else:
        idx, vals = synth.coo_uniform(dims, nnz, seed=17)
    vals = vals.astype(np.float32)
    U0 = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 116))]
    plan = H.hoqri_plan_create(dev(idx), dev(vals), dims, K)
    Us = [dev(u) for u in U0]
    sweeps = 3
    G, st = H.hoqri_run(plan, Us, max_sweeps=sweeps, keep_on_breakdown=True)
    torch.cuda.synchronize()
    Uo, Go, h = O.hoqri(idx, vals.astype(np.float64), dims, K, [u.astype(np.float64) for u in U0], sweeps=sweeps,
                        on_breakdown="keep")
    assert st.skipped_updates == h["skipped"]
    assert st.fit == pytest.approx(h["fit"][-1], rel=1e-5)
    assert st.orth_err_max < 1e-5
