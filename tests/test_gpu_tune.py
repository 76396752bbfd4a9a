"""The launch-shape autotuner (hoqri_autotune): chosen shapes stay inside the
plan's limits, the passes stay parity-green against the FP64 oracle and
bitwise deterministic under them, a cached choice is reused for the same shape
class, and invalid shapes are refused."""
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


def case(dims, K, nnz, seed, zipf=True):
    if zipf:
        idx, vals = synth.coo_zipf(dims, nnz, alpha=1.2, seed=seed)
    else:
        idx, vals = synth.coo_uniform(dims, nnz, seed=seed)
    vals32 = vals.astype(np.float32)
    U = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, seed + 100))]
    return idx, vals32, U


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_autotune_choice_is_valid_parity_green_and_cached(prec, tmp_path):
    dims, K = ((30000, 15000, 600), (16, 16, 16)) if prec == "fp32" else ((3000, 2000, 400), (32, 32, 32))
    print(f"[tune] prec={prec} dims={dims} K={K}", flush=True)
    idx, vals32, U = case(dims, K, 200_000 if prec == "fp32" else 60_000, seed=31, zipf=prec == "fp32")
    cache = str(tmp_path / "tune.txt")
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    default = H.hoqri_plan_get_tuning(plan)
    t, fc = H.hoqri_autotune(plan, prec, cache)
    assert not fc
    cap = H.hoqri_plan_max_ranges(plan)
    for n in range(3):
        assert 1 <= t["ranges"][n] <= cap and t["waves_per_group"][n] >= 0
    assert H.hoqri_plan_get_tuning(plan) == t
    print(f"[tune] default {default} chosen {t}", flush=True)
    # passes under the chosen shapes against the oracle (float32: 1e-5; bfloat16: its rounding bound)
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    U64 = [u.astype(np.float64) for u in U]
    Ud = [dev(u) for u in U]
    G = H.hoqri_core(plan, Ud)
    Gref = O.core_segment(ci, cv, U64)
    G32 = Gref.astype(np.float32)
    for n in range(3):
        A = H.hoqri_ttmctc(plan, n, Ud, dev(G32), prec=prec).cpu().numpy().astype(np.float64)
        Aref = O.ttmctc_segment(ci, cv, U64, n, G32.astype(np.float64))
        if prec == "fp32":
            assert np.linalg.norm(A - Aref) / np.linalg.norm(Aref) < 1e-5
        else:
            Aabs = O.ttmctc_segment(ci, np.abs(cv), [np.abs(u) for u in U64], n, np.abs(G32.astype(np.float64)))
            assert np.all(np.abs(A - Aref) <= (5 * 2.0 ** -8 + 2e-5) * Aabs + 1e-9 * Aabs.max())
    # whole runs under the tuned shapes: deterministic, and the fit of the FP32
    # form equals the oracle's
    runs = []
    for _ in range(2):
        Us = [dev(u) for u in U]
        Gr, st = H.hoqri_run(plan, Us, max_sweeps=3, prec=prec)
        torch.cuda.synchronize()
        runs.append((Gr.clone(), [u.clone() for u in Us], st))
    assert torch.equal(runs[0][0], runs[1][0]) and all(torch.equal(a, b) for a, b in zip(runs[0][1], runs[1][1]))
    if prec == "fp32":
        _, _, h = O.hoqri(idx, vals32.astype(np.float64), dims, K, U64, sweeps=3)
        assert runs[0][2].fit == pytest.approx(h["fit"][-1], rel=1e-5)
    # a second plan of the same shape class takes the cached choice without timing
    plan2 = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    t2, fc2 = H.hoqri_autotune(plan2, prec, cache)
    assert fc2 and t2 == t and H.hoqri_plan_get_tuning(plan2) == t
    with open(cache) as f:
        assert len(f.read().strip().splitlines()) == 1


def test_set_tuning_validates():
    dims, K = (2000, 1500, 300), (8, 8, 8)
    idx, vals32, U = case(dims, K, 50_000, seed=33)
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    cap = H.hoqri_plan_max_ranges(plan)
    t = H.hoqri_plan_get_tuning(plan)
    assert all(1 <= w <= cap for w in t["ranges"]) and t["waves_per_group"] == [0, 0, 0]
    for bad in ([0, 1, 1], [cap + 1, 1, 1]):
        with pytest.raises(H.HoqriError):
            H.hoqri_plan_set_tuning(plan, bad)
    assert H.hoqri_plan_get_tuning(plan) == t            # unchanged by the refused calls
    # an explicit shape: one range per mode (a wave walks every nonzero), still correct
    H.hoqri_plan_set_tuning(plan, [1, 1, 1], [1, 1, 1])
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    U64 = [u.astype(np.float64) for u in U]
    Ud = [dev(u) for u in U]
    G32 = O.core_segment(ci, cv, U64).astype(np.float32)
    A = H.hoqri_ttmctc(plan, 1, Ud, dev(G32)).cpu().numpy().astype(np.float64)
    Aref = O.ttmctc_segment(ci, cv, U64, 1, G32.astype(np.float64))
    assert np.linalg.norm(A - Aref) / np.linalg.norm(Aref) < 1e-5
