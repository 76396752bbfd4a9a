"""Builds the launch-shape database of hoqri_autotune for the benchmark
workloads on the current GPU: for each workload and operand form, the input is
generated on the device, the plan built, and the autotuner run with the
database file as its cache (one line per shape class is appended).

    python -m paper_2510_16930_amd.tune_db OUT.txt [workload ...]

Workload names are bench.py's configs (default: the 3-way 50M-nonzero tensor
at ranks 16^3 and 32^3 and the 4-way 100M-nonzero tensor, every form bench.py
times). bench.py reads paper_2510_16930_amd/tuning/<device>.txt by default.
"""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEFAULT = ("c2", "c3", "c4")


def main(argv):
    if len(argv) < 2:
        print(__doc__)
        return 2
    out = os.path.abspath(argv[1])
    names = argv[2:] or list(DEFAULT)
    sys.path.insert(0, ROOT)
    import torch
    import bench
    from paper_2510_16930_amd import _lib as H
    dev = torch.device("cuda:0")
    for name in names:
        cfg = bench.CONFIGS[name]
        idx, vals = bench.make_input(cfg, dev)
        plan = H.hoqri_plan_create(idx, vals, cfg["dims"], cfg["ranks"])
        del idx, vals
        for prec in [cfg["prec"]] + ([cfg["compare"]] if cfg.get("compare") else []):
            shape, cached = H.hoqri_autotune(plan, prec, out)
            print(f"{name} {prec}: {shape}{' (cached)' if cached else ''}", flush=True)
        plan.destroy()
        torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
