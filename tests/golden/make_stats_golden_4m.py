"""Writes stats_dimers_4M_transient.json: the oracle's statistics of the
4M-particle workload over its transient window, under PROTOCOL_4M of
stats_protocol.py.  Calls only oracle/ (and the seeded input generators).
The seeds run one after another, each on all the oracle's OpenMP threads
(about 30 minutes per seed on 8 cores).  Run from the repository root:

    python tests/golden/make_stats_golden_4m.py
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from paper_1310_0998_amd import inputs  # noqa: E402
from stats_protocol import PROTOCOL_4M, WindowAccumulator, window_ensemble  # noqa: E402


def run_seed(seed: int, log) -> dict:
    P = PROTOCOL_4M
    cfg = dict(inputs.physics(inputs.WORKLOADS[P["workload"]]), seed=seed)
    x, v = inputs.initial_state(cfg)
    F = oracle.forces(cfg, x, v, 0)
    s = 0
    acc = WindowAccumulator(cfg["L"])
    t0 = time.time()
    for k in range(P["steps"] // P["every"]):
        x, v, F, s, _ = oracle.step(cfg, x, v, F, s, P["every"])
        u, _ = oracle.bin_velocity(cfg, x.astype("float32"), v.astype("float32"), P["M"], 0.0, 0)
        acc.add(u)
        if (k + 1) % 10 == 0:
            log(f"seed {seed}: step {s}, {time.time() - t0:.0f} s")
    return acc.result()


def main():
    log = lambda m: print(m, flush=True)
    per_seed = []
    for seed in PROTOCOL_4M["seeds"]:
        per_seed.append(run_seed(seed, log))
        log(f"seed {seed}: L_gv per window {['%.4f' % a for a in per_seed[-1]['L_gv']]}")
    out = dict(protocol=PROTOCOL_4M, per_seed=per_seed, **window_ensemble(per_seed),
               source="oracle (FP64), oracle.step / oracle.bin_velocity / oracle.analysis")
    with open(os.path.join(HERE, "stats_dimers_4M_transient.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
