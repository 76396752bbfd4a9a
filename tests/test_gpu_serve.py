"""Request server on the GPU: continuous batching gives every request the same
result as running it alone.

A request's kernels use the same ranges and summation order in a batched
launch as in hoqri_run, so the comparison is bitwise: factors, core, f and the
number of sweeps. Admission is exercised with an arena that holds only a few
plans and a slot cap, and with requests arriving while others are running.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2510_16930_amd import _lib as H
from paper_2510_16930_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def make_requests(n, seed, orders=(3,), dim_range=(300, 3000), nnz_range=(5_000, 40_000)):
    params = synth.serve_stream_params(n, seed, dim_range=dim_range, nnz_range=nnz_range)
    reqs = []
    for i, p in enumerate(params):
        N = orders[i % len(orders)]
        if N <= 3:
            dims, ranks = p["dims"][:N], p["ranks"][:N]
        else:  # 4-way: keep every Kronecker block count within the compiled kernels
            r = min(p["ranks"][0], 8)
            dims, ranks = p["dims"][:2] + (60, 40), (r, r, 3, 3)
        nnz = min(p["nnz"], int(np.prod(dims)) // 4)
        idx, vals = synth.coo_uniform_torch(dims, nnz, p["data_seed"], device=DEV)
        U0 = [H.hoqri_orth(r)[0] for r in synth.gaussian_start_torch(dims, ranks, p["init_seed"], device=DEV)]
        reqs.append(dict(idx=idx, vals=vals, dims=dims, ranks=ranks, U0=U0))
    torch.cuda.synchronize()
    return reqs


def alone(q, max_sweeps, tol):
    plan = H.hoqri_plan_create(q["idx"], q["vals"], q["dims"], q["ranks"])
    Us = [u.clone() for u in q["U0"]]
    G, st = H.hoqri_run(plan, Us, max_sweeps=max_sweeps, tol=tol, check_every=1)
    torch.cuda.synchronize()
    return Us, G, st


def serve(reqs, arena_bytes, max_slots, max_sweeps, tol, waves=1, use_graphs=False):
    srv = H.Server(arena_bytes, max_slots=max_slots, max_sweeps=max_sweeps, tol=tol, report_orth_err=True,
                   use_graphs=use_graphs)
    outs = {}
    for i, q in enumerate(reqs):
        outs[i] = ([u.clone() for u in q["U0"]], torch.empty(q["ranks"], dtype=torch.float32, device=DEV))
    results = {}
    # requests arrive in `waves` groups while earlier ones are running
    per = (len(reqs) + waves - 1) // waves
    submitted = 0
    max_active = 0
    steps = 0
    while len(results) < len(reqs):
        if submitted < len(reqs) and (steps % 3 == 0):
            for i in range(submitted, min(submitted + per, len(reqs))):
                q = reqs[i]
                srv.submit(i, q["idx"], q["vals"], q["dims"], q["ranks"], outs[i][0], outs[i][1])
            submitted = min(submitted + per, len(reqs))
        for r in srv.step():
            results[r.id] = r
        steps += 1
        q_, a_, used = srv.info()
        max_active = max(max_active, a_)
        assert used <= arena_bytes
        assert steps < 100_000
    srv.close()
    return outs, results, max_active


@pytest.mark.parametrize("use_graphs", [False, True])
def test_batched_results_equal_alone_bitwise(use_graphs):
    # with use_graphs every step's launches are one replayed graph, updated in
    # place from step to step (eager work and synchronisations in between):
    # each replay must give the eager results bitwise
    reqs = make_requests(10, seed=3, orders=(3, 3, 3, 4, 2))
    sizes = [H.hoqri_plan_workspace_size(len(q["dims"]), q["dims"], q["ranks"], q["vals"].numel()) for q in reqs]
    arena = sum(sorted(sizes)[-3:]) + (8 << 20)  # about three plans at a time
    print(f"[serve] 10 requests, arena {arena >> 20} MiB, graphs {use_graphs}", flush=True)
    outs, results, max_active = serve(reqs, arena, max_slots=4, max_sweeps=6, tol=1e-6, waves=3,
                                      use_graphs=use_graphs)
    assert max_active >= 2  # requests really overlapped
    for i, q in enumerate(reqs):
        r = results[i]
        assert r.status == 0, (i, r.status)
        Us, G, st = alone(q, 6, 1e-6)
        assert r.sweeps == st.sweeps
        assert r.f == st.f
        assert torch.equal(outs[i][1], G), i
        for n in range(len(q["dims"])):
            assert torch.equal(outs[i][0][n], Us[n]), (i, n)
        assert r.orth_err_max < 1e-5


def test_stop_rule_and_oracle_fit():
    reqs = make_requests(4, seed=5)
    outs, results, _ = serve(reqs, 1 << 30, max_slots=8, max_sweeps=40, tol=1e-3)
    for i, q in enumerate(reqs):
        r = results[i]
        Us, G, st = alone(q, 40, 1e-3)
        assert r.sweeps == st.sweeps
        assert r.f == st.f
        assert r.rel_change <= 1e-3 or r.sweeps == 40
    # one request against the FP64 oracle after the same sweeps
    q, r = reqs[0], results[0]
    idx = q["idx"].cpu().numpy()
    vals = q["vals"].cpu().numpy().astype(np.float64)
    U0 = [u.cpu().numpy().astype(np.float64) for u in q["U0"]]
    Uo, Go, h = O.hoqri(idx, vals, q["dims"], q["ranks"], U0, sweeps=r.sweeps)
    assert r.fit == pytest.approx(h["fit"][-1], rel=1e-5)


def test_errors_do_not_disturb_other_requests():
    reqs = make_requests(3, seed=7)
    # a request whose plan cannot fit in the arena, and one with too few nonempty slices
    big = dict(reqs[0])
    bad_idx = reqs[1]["idx"].clone()
    bad_idx[0] = bad_idx[0] % 2  # two nonempty mode-0 slices < K_0
    bad = dict(reqs[1], idx=bad_idx)
    sizes = [H.hoqri_plan_workspace_size(3, q["dims"], q["ranks"], q["vals"].numel()) for q in reqs]
    srv = H.Server(max(sizes) + (16 << 20), max_slots=4, max_sweeps=3, tol=0.0)
    huge_dims = (2_000_000, 2_000_000, 2_000_000)
    G_big = torch.empty(big["ranks"], dtype=torch.float32, device=DEV)
    U_big = [torch.zeros((d, k), dtype=torch.float32, device=DEV) for d, k in zip((8, 8, 8), big["ranks"])]
    # dims far larger than the arena allows (the plan keeps per-index tables)
    srv.submit(100, big["idx"], big["vals"], huge_dims, big["ranks"], U_big, G_big)
    Gb = torch.empty(bad["ranks"], dtype=torch.float32, device=DEV)
    Ub = [u.clone() for u in bad["U0"]]
    srv.submit(101, bad["idx"], bad["vals"], bad["dims"], bad["ranks"], Ub, Gb)
    outs = {}
    for i in (0, 2):
        q = reqs[i]
        outs[i] = ([u.clone() for u in q["U0"]], torch.empty(q["ranks"], dtype=torch.float32, device=DEV))
        srv.submit(i, q["idx"], q["vals"], q["dims"], q["ranks"], outs[i][0], outs[i][1])
    results = {}
    while len(results) < 4:
        for r in srv.step():
            results[r.id] = r
    srv.close()
    assert results[100].status == -5
    assert results[101].status == -4
    for i in (0, 2):
        Us, G, st = alone(reqs[i], 3, 0.0)
        assert results[i].status == 0 and results[i].sweeps == 3
        assert torch.equal(outs[i][1], G)


def test_pass_timing_counts_the_ttmctc_work():
    # time_passes: HIP events around each step's batched TTMcTC launches; the
    # algorithmic bytes and flops are those of the passes that ran (one pass per
    # request and step), so per timed step they lie between one request's
    # smallest and all requests' largest pass
    reqs = make_requests(4, seed=11)
    srv = H.Server(1 << 30, max_slots=8, max_sweeps=3, tol=0.0, time_passes=True)
    outs = {}
    for i, q in enumerate(reqs):
        outs[i] = ([u.clone() for u in q["U0"]], torch.empty(q["ranks"], dtype=torch.float32, device=DEV))
        srv.submit(i, q["idx"], q["vals"], q["dims"], q["ranks"], outs[i][0], outs[i][1])
    done = 0
    while done < len(reqs):
        done += len(srv.step())
    steps, ms, byts, flops = srv.ttm_stats()
    srv.close()
    assert steps >= 3 and ms > 0.0
    one = min(q["vals"].numel() * 4 * 3 for q in reqs)
    assert byts / steps >= one
    assert flops > 0.0
    # with graph-captured steps nothing is timed
    srv = H.Server(1 << 30, max_slots=8, max_sweeps=2, tol=0.0, use_graphs=True, time_passes=True)
    q = reqs[0]
    srv.submit(0, q["idx"], q["vals"], q["dims"], q["ranks"], [u.clone() for u in q["U0"]],
               torch.empty(q["ranks"], dtype=torch.float32, device=DEV))
    while not srv.step():
        pass
    assert srv.ttm_stats()[0] == 0
    srv.close()
