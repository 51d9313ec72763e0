"""Tune the launch plans of the benchmark workloads on the current GPU and
write them to a plan table (JSON), e.g. the table shipped with the package:

    python -m paper_2406_03762_amd.tune --out paper_2406_03762_amd/tuned_plans.json

Each workload's candidate plans (plan kind, workgroups per compute unit,
block size, exchange window) are built and timed in closed loop; the fastest
is stored under the key of (network description, device).  Existing entries
of other workloads in the output table are kept.
"""
from __future__ import annotations

import argparse
import os
import sys


def main() -> None:
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import netspec
    import paper_2406_03762_amd as cx

    workloads = {
        "brunel_2m_bf16": (netspec.brunel_2m_bf16, 5, 2000, 2000),
        "brunel_112k_alpha": (netspec.brunel_112k_alpha, 2, 4000, 500),
        "microcircuit_77k": (netspec.microcircuit_77k, 3, 4000, 500),
        "batched_64": (netspec.batched_brunel, 4, 2000, 200),
    }
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(workloads), help="workloads: " + ", ".join(workloads))
    ap.add_argument("--out", default=cx.TUNE_CACHE)
    ap.add_argument("--budget-s", type=float, default=600.0, help="per workload")
    args = ap.parse_args()

    def log(msg):
        print(msg, flush=True)

    for name in args.names:
        make, seed, steps, warmup = workloads[name]
        log(f"[tune] {name}")
        best, timings = cx.autotune(make(), seed, steps=steps, warmup=warmup, budget_s=args.budget_s,
                                    cache=args.out, log=log)
        log(f"[tune] {name}: best {best}")


if __name__ == "__main__":
    main()
