"""Writes stats_dimers_1600.json: the oracle's long-run statistics under the
protocol of stats_protocol.py.  Calls only oracle/ (and the seeded input
generators).  The seeds run in parallel processes of one oracle thread each.
Run from the repository root:

    python tests/golden/make_stats_golden.py [--procs 8]
"""
from __future__ import annotations

import json
import multiprocessing
import os
import sys
import time

os.environ["OMP_NUM_THREADS"] = "1"  # one oracle thread per process

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from paper_1310_0998_amd import inputs  # noqa: E402
from stats_protocol import PROTOCOL, SeedAccumulator, ensemble  # noqa: E402


def run_seed(seed: int) -> dict:
    cfg = dict(inputs.physics(inputs.WORKLOADS[PROTOCOL["workload"]]), seed=seed)
    x, v = inputs.initial_state(cfg)
    F = oracle.forces(cfg, x, v, 0)
    x, v, F, s, _ = oracle.step(cfg, x, v, F, 0, PROTOCOL["warmup"])
    acc = SeedAccumulator(cfg["L"])
    for _ in range(PROTOCOL["steps"] // PROTOCOL["every"]):
        x, v, F, s, _ = oracle.step(cfg, x, v, F, s, PROTOCOL["every"])
        x32, v32 = x.astype("float32"), v.astype("float32")
        u, _ = oracle.bin_velocity(cfg, x32, v32, PROTOCOL["M"], 0.0, 0)
        acc.add(u, x32, v32)
    return acc.result()


def main():
    procs = int(sys.argv[sys.argv.index("--procs") + 1]) if "--procs" in sys.argv else 8
    t0 = time.time()
    per_seed = []
    with multiprocessing.Pool(procs) as pool:
        for k, res in enumerate(pool.imap(run_seed, PROTOCOL["seeds"])):
            per_seed.append(res)
            print(f"seed {PROTOCOL['seeds'][k]}: L_gv {res['L_gv']:.4f}  ({time.time() - t0:.0f} s)",
                  flush=True)
    out = dict(protocol=PROTOCOL, per_seed=per_seed, **ensemble(per_seed),
               source="oracle (FP64), oracle.step / oracle.bin_velocity / oracle.analysis")
    with open(os.path.join(HERE, "stats_dimers_1600.json"), "w") as f:
        json.dump(out, f, indent=1)
    e = ensemble(per_seed)
    print("bands", [f"{m:.4g}+-{s / m * 100:.2f}%" for m, s in zip(e["E_bands"], e["E_bands_sem"])])
    print(f"L_gv {e['L_gv']:.4f} +- {e['L_gv_sem'] / e['L_gv'] * 100:.2f}%")


if __name__ == "__main__":
    main()
