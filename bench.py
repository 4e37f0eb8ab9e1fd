"""Throughput of the DPD hot path on one MI355X.

One step = one velocity-Verlet step of the whole hot path (cell binning, fused
pair / agent / integrator kernel), with the FP64 momentum and kinetic-energy
reduction every 100 steps (and at least once per timed window) and the binned
256 x 256 velocity field every 20 steps, on the 4M-particle system (2M dimers
in a 2000 x 2000 periodic box, synthetic random initial state).  The first
--t0-steps steps from the random start are timed on their own; then a fixed,
untimed relaxation of --relax steps (default 2000) brings the system to its
steady state, whatever --warmup is; then --warmup more steps, then exactly
--steps timed steps.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--relax R] [--cpu-steps S]

With --workload sweep64 it instead times the batched parameter sweep: 64
replicas of uneven size advanced together, against the same systems run one
after another; with --workload closure it trains the learned closure on
DPD-generated fields and times its rollout against plain DPD (each prints one
JSON line of its own); --workload paper runs the paper's own parameter set,
--workload rollout times the closure's batched rollout alone and --workload
grid200k the 200k-particle gamma x zeta grid.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (FP32 pair kernel, % HBM roofline); closure speedup at ≤5% E(k) err"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pair_pass_bytes(n_particles: int, n_cells: int) -> int:
    """Algorithmic HBM bytes of one pair-force pass (Eqs. 2.2-2.4 over the
    sorted state): per particle the sorted x (8), u (8) and id (4) read and the
    force (8) written, plus cell_start (4 per cell, n_cells + 1 entries);
    32 B per particle at one particle per cell.  Halo re-reads are the
    implementation's, not the pass's."""
    return n_particles * (8 + 8 + 4 + 8) + 4 * (n_cells + 1)


def fused_kernel_bytes(n_particles: int, n_cells: int) -> int:
    """What the fused step kernel itself must move: reads slot->index (4),
    x (8), u (8), id (4) per particle and cell_start (4 per cell + 1); writes
    the next x (8), u (8), id (4), cell key (4) and rank (4); one 4-byte atomic
    read-modify-write of a cell counter (8); clears the counter its own binning
    consumed (4 per cell).  60 B per particle + 8 per cell."""
    return (n_particles * (4 + 8 + 8 + 4 + 8 + 8 + 4 + 4 + 4 + 8) + 4 * (n_cells + 1)
            + 4 * n_cells)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("device.h", "kernels.h", "engine.hip"):
        with open(os.path.join(ROOT, "paper_1310_0998_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_fields(name: str):
    """"key: value" lines of a committed profile summary, or None when the file
    is missing or was taken with other kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as f:
        for line in f:
            k, sep, val = line.partition(":")
            if sep:
                d[k.strip()] = val.strip()
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d


def measured_traffic():
    """HBM bytes per launch of the pair kernel from the committed rocprofv3
    counter summary, if it was taken with the current kernel sources."""
    d = _profile_fields("pair_kernel_dimers_4M_counters.txt")
    try:
        return None if d is None else float(d["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes per clock (a 64-lane
# instruction takes 4 clocks) at 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9


def measured_valu(avg_launch_us: float):
    """Issued VALU lane-ops of the pair kernel per second against the issue
    peak: the committed SQ counter summary's instructions per launch (if taken
    with the current sources) over the launch time measured in this run."""
    d = _profile_fields("pair_kernel_dimers_4M_valu_counters.txt")
    if d is None:
        return None
    try:
        ops = 64.0 * float(d["valu_insts_per_launch"])
        achieved = ops / (avg_launch_us * 1e-6)
        return {"achieved": achieved, "peak": VALU_PEAK_LANE_OPS, "unit": "lane-ops/s",
                "frac": achieved / VALU_PEAK_LANE_OPS, "issued_lane_ops_per_launch": ops,
                "valu_busy_pct": float(d["valu_busy_pct"]),
                "lane_util_pct": float(d["valu_lane_util_pct"]),
                "source": "profiles/pair_kernel_dimers_4M_valu_counters.txt"}
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def cpu_baseline(cfg, x, v, steps: int):
    import oracle
    t0 = time.perf_counter()
    F = oracle.forces(cfg, x, v, 0)
    t1 = time.perf_counter()
    oracle.step(cfg, x, v, F, 0, steps)
    t2 = time.perf_counter()
    n = len(x)
    cores = oracle.num_threads()
    # the same from the same state on one thread, for one step
    oracle.set_threads(1)
    try:
        t3 = time.perf_counter()
        oracle.step(cfg, x, v, F, 0, 1)
        t4 = time.perf_counter()
    finally:
        oracle.set_threads(cores)
    return {
        "value": n * steps / (t2 - t1),
        "unit": "particle-steps/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{steps} velocity-Verlet steps of the full {n}-particle system from the "
                  f"benchmark's initial state (FP64 oracle, OpenMP; initial force evaluation "
                  f"{t1 - t0:.2f} s not counted); one further step on one thread for value_1_thread",
        "value_1_thread": n / (t4 - t3),
    }


def run_sweep(args):
    """The batched parameter sweep: 64 replicas of uneven size (2k-64k dimers,
    log-uniform) over area fraction x (gamma / zeta), all advanced by one launch
    per step kernel, against the same 64 systems run one after another."""
    import numpy as np
    import torch

    from paper_1310_0998_amd import dpd, inputs

    dev = torch.device("cuda:0")
    cfgs = [inputs.physics(c) for c in inputs.sweep_replicas()]
    states = [inputs.initial_state(c) for c in cfgs]
    x = np.concatenate([s[0] for s in states])
    v = np.concatenate([s[1] for s in states])
    N = len(x)
    steps = args.sweep_steps
    K = args.graph_chunk
    red_every = 100 if steps % 100 == 0 and 100 % K == 0 else 0
    log(f"sweep: {len(cfgs)} replicas, N={N} particles, {steps} steps, graph chunk {K}")

    def to_dev(a):
        return torch.from_numpy(a).to(dev)

    # batched: every replica's default tile (or, with --tune, the schedule the
    # tuner picks from trials at the random start, which measured slower over
    # the whole run: the start is not the steady state), captured chunks, one call
    b = dpd.Sim(cfgs, device=dev)
    b.set_state(to_dev(x), to_dev(v), 0)
    tune = None
    if args.tune:
        tune = b.autotune(10)
        log(f"autotune: replica 0 tile {tune[0]} x {tune[1]}, order {tune[2]}, {tune[3]:.4f} ms/step")
    b.set_graph_chunk(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pk = b.step(steps, reduce_every=red_every) if red_every else b.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.sync()
    xb, vb, _, _ = b.get_state()
    xb, vb = xb.cpu().numpy(), vb.cpu().numpy()
    # pair-kernel time of the batch from a short eager run with events
    b.set_graph_chunk(0)
    b.set_profiling(True)
    b.step(200)
    pair_ms, launches = b.pair_kernel_time()
    b.set_profiling(False)
    n_cells = b.n_cells
    b.close()
    log(f"batched: {t_batch:.3f} s, {1e3 * t_batch / steps:.4f} ms/step")

    # the same systems one after another (step loops only are timed)
    seq = {}
    equal = True
    for mode in (() if args.no_sequential else ("eager", "graph")):
        total = 0.0
        for q, (c, (xs, vs)) in enumerate(zip(cfgs, states)):
            s = dpd.Sim(c, device=dev)
            s.set_state(to_dev(xs), to_dev(vs), 0)
            if mode == "graph":
                s.set_graph_chunk(K)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if red_every:
                s.step(steps, reduce_every=red_every)
            else:
                s.step(steps)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
            if mode == "eager":
                xq, vq, _, _ = s.get_state()
                o = sum(len(t[0]) for t in states[:q])
                equal &= bool((xq.cpu().numpy() == xb[o:o + len(xs)]).all()
                              and (vq.cpu().numpy() == vb[o:o + len(xs)]).all())
            s.close()
        seq[mode] = total
        log(f"sequential ({mode}): {total:.3f} s")

    avg_us = 1e3 * pair_ms / max(launches, 1)
    alg = pair_pass_bytes(N, n_cells)
    achieved = alg / (avg_us * 1e-6) / 1e9
    rate = N * steps / t_batch
    line = {
        "metric": "batched sweep: particle-steps/s over 64 replicas in one launch per step kernel",
        "value": rate,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": 1e3 * t_batch / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "sweep64: 64 replicas, dimer counts log-uniform in [2000, 64000] (seed 401), "
                        "area fraction {0.2,0.4,0.6,0.8} x gamma/zeta {0.1,1,10,100} (4 replicas "
                        "per point), gamma=4.5, L=sqrt(N_a/phi) r_c, a=25, kT=1, F_p=1, dt=0.005, "
                        f"{steps} steps each from random positions at rest",
            "n_particles": N,
            "cells": n_cells,
            "graph_chunk": K,
            "schedule": "default tile per replica (8 x 7 scaled by 1 / particles per cell), XCD bands"
                        if tune is None else {"tuned": True, "replica0_tile": [tune[0], tune[1]], "order": tune[2]},
            "fp64_reduction_every": red_every,
            "parallelism": "single-gpu",
        },
        "sequential": None if not seq else {
            "eager_s": seq["eager"], "graph_s": seq["graph"],
            "value_eager": N * steps / seq["eager"], "value_graph": N * steps / seq["graph"],
        },
        "speedup_vs_sequential": None if not seq else {
            "eager": seq["eager"] / t_batch, "graph": seq["graph"] / t_batch},
        "bitwise_equal_to_sequential": equal if seq else None,
        "roofline": {
            "kernel": "k_pair (batched)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": alg,
            "avg_launch_us": avg_us,
        },
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_grid200k(args):
    """The 200k-particle pair-friction x Stokes-friction grid: gamma in
    {1, 4.5, 20} x zeta in {0, 0.5, 5} (seeds 201-209), each point advanced
    from its random start for --grid-steps steps in captured 50-step chunks
    (FP64 totals every 100 steps), then 200 eager steps with the pair kernel
    bracketed by events for its launch time.  The working set (about 12 MB)
    stays in the caches, so the pair kernel's byte rate is a cache-level
    figure, not an HBM one."""
    import torch

    from paper_1310_0998_amd import dpd, inputs

    dev = torch.device("cuda:0")
    base = inputs.physics(inputs.WORKLOADS["dimers_200k"])
    steps = args.grid_steps
    K = 50
    red_every = 100 if steps % 100 == 0 else 0
    points = []
    finals = []
    t_total = 0.0
    n_total = 0
    for k, (g, z) in enumerate(inputs.GAMMA_ZETA_GRID_200K):
        cfg = dict(base, gamma=g, gamma_s=z, seed=201 + k)
        x, v = inputs.initial_state(cfg)
        N = len(x)
        sim = dpd.Sim(cfg, device=dev)
        sim.set_state(torch.from_numpy(x).to(dev), torch.from_numpy(v).to(dev), 0)
        sim.set_graph_chunk(K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if red_every:
            sim.step(steps, reduce_every=red_every)
        else:
            sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sim.sync()
        xs_, vs_, _, _ = sim.get_state()
        finals.append((xs_.cpu().numpy(), vs_.cpu().numpy()))
        sim.set_graph_chunk(0)
        sim.set_profiling(True)
        sim.step(200)
        pair_ms, launches = sim.pair_kernel_time()
        sim.set_profiling(False)
        n_cells = sim.n_cells
        sim.close()
        avg_us = 1e3 * pair_ms / max(launches, 1)
        alg = pair_pass_bytes(N, n_cells)
        p = {"gamma": g, "zeta": z, "seed": 201 + k, "ms_per_step": 1e3 * dt / steps,
             "particle_steps_per_s": N * steps / dt, "pair_kernel_us": avg_us,
             "pair_kernel_GBps_alg": alg / (avg_us * 1e-6) / 1e9}
        points.append(p)
        t_total += dt
        n_total += N * steps
        log(f"gamma={g} zeta={z}: {p['ms_per_step']:.4f} ms/step, pair kernel {avg_us:.2f} us, "
            f"{p['pair_kernel_GBps_alg']:.0f} GB/s (32 B/particle)")
    # the same nine points as the replicas of one batch: one launch per step
    # kernel for 1.8 M particles instead of nine launch-latency-bound systems;
    # every replica must end bitwise where its own run ended
    import numpy as np
    cfgs = [dict(base, gamma=g, gamma_s=z, seed=201 + k) for k, (g, z) in enumerate(inputs.GAMMA_ZETA_GRID_200K)]
    sts = [inputs.initial_state(c) for c in cfgs]
    xb = np.concatenate([st[0] for st in sts])
    vb = np.concatenate([st[1] for st in sts])
    bat = dpd.Sim(cfgs, device=dev)
    bat.set_state(torch.from_numpy(xb).to(dev), torch.from_numpy(vb).to(dev), 0)
    bat.set_graph_chunk(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if red_every:
        bat.step(steps, reduce_every=red_every)
    else:
        bat.step(steps)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    bat.sync()
    xe, ve, _, _ = bat.get_state()
    xe, ve = xe.cpu().numpy(), ve.cpu().numpy()
    bat.close()
    off = np.cumsum([0] + [len(st[0]) for st in sts])
    equal = all(np.array_equal(xe[off[q]:off[q + 1]], finals[q][0]) and np.array_equal(ve[off[q]:off[q + 1]], finals[q][1])
                for q in range(len(cfgs)))
    batched = {"ms_per_step": 1e3 * t_bat / steps, "particle_steps_per_s": len(xb) * steps / t_bat,
               "speedup_vs_points": t_total / t_bat, "bitwise_equal_to_points": bool(equal)}
    log(f"the nine points as one batch: {batched['ms_per_step']:.4f} ms/step, "
        f"{batched['particle_steps_per_s']:.3e} particle-steps/s, {batched['speedup_vs_points']:.2f}x, "
        f"bitwise equal: {equal}")
    line = {
        "metric": "200k grid: particle-steps/s over the gamma x zeta grid; pair kernel GB/s",
        "value": n_total / t_total,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": 1e3 * t_total / (steps * len(points)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "grid200k: 2-D periodic box L=447 r_c, 100000 dimers (200000 particles), "
                        "a=25, kT=1, F_p=1, dt=0.005, gamma {1,4.5,20} x zeta {0,0.5,5}, "
                        f"{steps} steps per point from random positions at rest",
            "graph_chunk": K,
            "fp64_reduction_every": red_every,
            "parallelism": "single-gpu",
        },
        "points": points,
        "batched": batched,
        "pair_kernel_GBps_alg_mean": sum(p["pair_kernel_GBps_alg"] for p in points) / len(points),
        "cache_note": "working set about 12 MB: L2 / Infinity-Cache resident, not an HBM figure",
        "cpu_baseline": None,
    }
    print(json.dumps(_finite(line)), flush=True)


def _finite(o):
    """o with non-finite floats replaced by None (JSON has no inf or NaN)."""
    if isinstance(o, float):
        return o if o == o and abs(o) != float("inf") else None
    if isinstance(o, dict):
        return {k: _finite(v) for k, v in o.items()}
    if isinstance(o, (list, tuple)):
        return [_finite(v) for v in o]
    return o


def run_closure(args):
    """The learned closure: DPD-generated training pairs (independent replicas
    of every condition), training on the GPU, noise calibrated against the
    evaluated condition's training fields, then an ensemble of closure rollouts
    against an independent ensemble of DPD runs, timed, with the
    energy-spectrum, correlation-length and mode-autocorrelation errors.  The
    zero network (persistence, u(t + 50) = u(t)) goes through the same
    calibration and evaluation as the control of what the network adds."""
    import torch

    from paper_1310_0998_amd import closure, closure_train as ct, inputs

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    runs = ct.generate(dev, log=log)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    train_idx, test_idx = ct.split(runs)
    E, T = args.closure_ensemble, args.closure_steps
    mk = lambda: closure.Closure(ct.M, c_in=4, width=32, layers=4, max_batch=max(32, E), device=dev)
    net = mk()
    net.set_weights(torch.from_numpy(inputs.closure_init(601, 4, 32, 4)).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, n_upd = ct.train(net, runs, train_idx, dev, epochs=args.closure_epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    zero = mk()
    zero.set_weights(torch.zeros(zero.n_params, dtype=torch.float32, device=dev))
    mse_net, mse_per, _ = ct.evaluate(net, runs, test_idx, dev)
    _, _, res = ct.evaluate(net, runs, train_idx, dev)
    log(f"held-out one-step MSE: network {mse_net:.5e}, persistence {mse_per:.5e}; "
        f"training residual rms {res[0]:.4f} {res[1]:.4f}")
    r_eval = 4  # zeta = 0.5, F_p = 1
    idx_r = [q for q in train_idx if runs[q[0]]["run"] == r_eval]
    cond = torch.tensor(ct.runs_cond(r_eval), dtype=torch.float32, device=dev)
    # calibration: rollouts from the evaluated condition's training fields, against
    # the spectrum of those fields (no DPD beyond the training data)
    target = ct.condition_fields(runs, r_eval)
    cstart = ct.training_starts(runs, r_eval, E)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    filters = {}
    for name, model in (("network", net), ("zero", zero)):
        h0, R0 = ct.residual_filter(model, runs, idx_r, dev)
        h, _, cal = ct.calibrate_filter(model, cstart, target, args.closure_cal_steps, cond, R0, dev, log=log)
        filters[name] = (h0, h, cal)
    torch.cuda.synchronize()
    t_cal = time.perf_counter() - t0
    jstart, jfields, t_dpd = ct.ensemble(r_eval, E, args.closure_warm, T, 2000, dev, log=log)
    models = {"calibrated": (net, (1.0, 1.0), filters["network"][1]),
              "residual": (net, (1.0, 1.0), filters["network"][0]),
              "white": (net, (float(res[0]), float(res[1])), None),
              "zero_calibrated": (zero, (1.0, 1.0), filters["zero"][1]),
              "zero_no_noise": (zero, (0.0, 0.0), None)}
    j = ct.evaluate_rollouts(models, r_eval, jstart, jfields, t_dpd, dev, log=log)
    del jfields
    jm = j["models"]["calibrated"]
    jz = j["models"]["zero_calibrated"]
    valid = jm["max_band_err"] <= 0.05
    speed = j["t_dpd"] / jm["t_closure"]
    one_time = t_gen + t_train + t_cal
    line = {
        "metric": "closure speedup at <=5% E(k) err",
        "value": speed,
        "unit": "x (plain DPD wall time / closure wall time, same span; one-time costs apart)",
        "n_gpus": 1,
        "steps": args.closure_steps,
        "warmup": 0,
        "ms_per_step": 1e3 * jm["t_closure"] / args.closure_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 matmul inputs, f32 accumulate",
        "data": "synthetic (generated by the DPD engine)",
        "valid": valid,
        "config": {
            "workload": "closure: 200k particles (100k dimers, L=447), gamma=4.5, zeta {0,0.5} x F_p "
                        f"{{0.5,1,2}}, {ct.REPLICAS} independent replicas per condition; 64x64 binned "
                        "velocity every 10 steps; pairs 50 steps apart; 4 conv layers, 32 channels, 3x3 "
                        f"periodic; evaluated at zeta=0.5, F_p=1: {E} independent DPD replicas (one batch, "
                        f"own seeds) x {T * ct.INTERVAL} steps against {E} batched closure rollouts x {T} "
                        "steps from the same fields; rollout noise filtered to the training residual's "
                        "spectrum, scaled per shell until a rollout reproduces the spectrum of the "
                        "evaluated condition's training fields",
            "pairs_train": len(train_idx),
            "pairs_test": len(test_idx),
            "epochs": args.closure_epochs,
            "adam_steps": n_upd,
            "parallelism": "single-gpu",
        },
        "timing_s": {"generate": t_gen, "train": t_train, "calibrate": t_cal,
                     "dpd_span": j["t_dpd"], "closure_span": jm["t_closure"]},
        "speedup_with_one_time_costs": j["t_dpd"] / (jm["t_closure"] + one_time),
        "one_step_mse": {"network": mse_net, "persistence": mse_per,
                         "gain_over_persistence": mse_per / mse_net},
        "E_band_err": jm["band_err"],
        "E_band_err_se": jm["band_err_se"],
        "E_band_ref_rel_se": j["band_ref_se"],
        "max_E_band_err": jm["max_band_err"],
        "L_gv": {"dpd": j["L_gv_ref"], "closure": jm["L_gv_closure"], "rel_err": jm["L_gv_err"]},
        "autocorrelation": {"lags_coarse_steps": j["ac_lags"], "dpd": j["ac_ref"], "closure": jm["ac"],
                            "max_abs_err": jm["max_ac_err"]},
        "calibration_max_shell_dev": filters["network"][2],
        "zero_network_control": {
            "calibrated_noise": {"E_band_err": jz["band_err"], "max_E_band_err": jz["max_band_err"],
                                 "L_gv_rel_err": jz["L_gv_err"], "autocorrelation": jz["ac"],
                                 "max_ac_err": jz["max_ac_err"],
                                 "calibration_max_shell_dev": filters["zero"][2]},
            "no_noise": {"E_band_err": j["models"]["zero_no_noise"]["band_err"],
                         "max_E_band_err": j["models"]["zero_no_noise"]["max_band_err"],
                         "max_ac_err": j["models"]["zero_no_noise"]["max_ac_err"]},
        },
        "residual_spectrum_noise": {"E_band_err": j["models"]["residual"]["band_err"],
                                    "L_gv_rel_err": j["models"]["residual"]["L_gv_err"],
                                    "max_ac_err": j["models"]["residual"]["max_ac_err"]},
        "white_noise": {"noise_std": [float(res[0]), float(res[1])],
                        "E_band_err": j["models"]["white"]["band_err"],
                        "L_gv_rel_err": j["models"]["white"]["L_gv_err"]},
        "final_training_loss": hist[-1],
    }
    print(json.dumps(_finite(line)), flush=True)
    net.close()
    zero.close()


def run_rollout(args):
    """The closure's batched rollout alone: B = 32 fields of 64 x 64 through the
    4-layer, 32-channel network for 200 steps, with white and with filtered
    noise (seeded random weights and fields; the timing does not depend on
    their values)."""
    import numpy as np
    import torch

    from paper_1310_0998_amd import closure, inputs

    dev = torch.device("cuda:0")
    M, B, steps = 64, 32, args.rollout_steps
    net = closure.Closure(M, c_in=4, width=32, layers=4, max_batch=B, device=dev)
    net.set_weights(torch.from_numpy(inputs.closure_init(601, 4, 32, 4)).to(dev))
    rng = np.random.Generator(np.random.PCG64(17))
    u0 = torch.from_numpy((0.1 * rng.standard_normal((B, M, M, 2))).astype(np.float32)).to(dev)
    cond = torch.full((B, 2), 0.5, dtype=torch.float32, device=dev)
    ii = np.arange(M)
    d = np.minimum(ii, M - ii).astype(np.float64)
    h = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / 4.5)
    h = torch.from_numpy((h / np.sqrt((h * h).sum())).astype(np.float32)).to(dev)
    res = {}
    for name, filt in (("white", None), ("filtered", h)):
        net.rollout(u0, cond, 5, (0.05, 0.05), seed=1, noise_filter=filt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.rollout(u0, cond, steps, (0.05, 0.05), seed=2, noise_filter=filt)
        torch.cuda.synchronize()
        res[name] = 1e6 * (time.perf_counter() - t0) / steps
        log(f"{name}: {res[name]:.1f} us per batched step")
    net.close()
    # multiply-adds per pixel of the four 3 x 3 convolutions (4 -> 32 -> 32 -> 32 -> 2)
    macs = 9 * (4 * 32 + 32 * 32 + 32 * 32 + 32 * 2)
    flops = 2.0 * macs * B * M * M
    line = {
        "metric": "closure rollout: us per batched step (B=32, 64x64, 4x32 conv)",
        "value": res["filtered"],
        "unit": "us/step",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 5,
        "higher_is_better": False,
        "dtype": "bf16 matmul inputs, f32 accumulate",
        "data": "synthetic (seeded random weights and fields)",
        "config": {"workload": "closure rollout, B=32 fields of 64x64, 4 periodic 3x3 convolutions "
                               "(4->32->32->32->2 channels), filtered noise (h = periodic Gaussian)",
                   "parallelism": "single-gpu"},
        "white_noise_us_per_step": res["white"],
        "conv_flops_per_step": flops,
        "step_tflops_white": flops / (res["white"] * 1e-6) / 1e12,
    }
    print(json.dumps(line), flush=True)


def run_paper(args):
    """The paper's own parameter set as one batch (Sec. 5.1), with the
    statistics of Sec. 5.3-5.4 computed on the GPU and the paper's qualitative
    findings checked."""
    import torch

    from paper_1310_0998_amd import paper_runs

    dev = torch.device("cuda:0")
    reps = paper_runs.REPLICAS
    if args.paper_subset:
        keep = [tuple(float(t) for t in part.split(",")) for part in args.paper_subset.split(";")]
        reps = [r for r in reps if (r[1], r[2]) in keep]
    t0 = time.perf_counter()
    res, r_grid, schedule = paper_runs.run(dev, args.paper_warm, args.paper_steps, args.paper_every,
                                           replicas=reps, log=log)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_particles = sum(2 * int(round(4.0e4 * r[0])) for r in reps)
    line = {
        "metric": "paper parameter set: E(k), g_v and L_gv statistics (Sec. 5.3-5.4) on the GPU",
        "value": wall,
        "unit": "s (whole run)",
        "n_gpus": 1,
        "steps": args.paper_warm + args.paper_steps,
        "warmup": args.paper_warm,
        "higher_is_better": False,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "paper set: Phi=1.5, r_c=0.5, kT=0.05, kappa=1e3, l=1, f_SP=1, dt=3e-3, L=100, "
                        f"N=4e4 phi agents ({n_particles} particles in all); {len(reps)} replicas "
                        "(phi, Gamma, Gamma_s); u_M on 128x128, eps = L sqrt(10/N); g_v in bins of r_c/4; "
                        f"a snapshot every {args.paper_every} steps after {args.paper_warm} steps of "
                        "relaxation",
            "parallelism": "single-gpu (one batch)",
            "schedule": schedule,
        },
        "replicas": [{k: v for k, v in r.items() if k not in ("E_over_E1", "g_v")} for r in res],
        "checks": paper_runs.checks(res) if reps == paper_runs.REPLICAS else None,
        "E_over_E1": {f"{r['phi']},{r['Gamma']},{r['Gamma_s']}": r["E_over_E1"] for r in res},
        "g_v": {"r": r_grid, **{f"{r['phi']},{r['Gamma']},{r['Gamma_s']}": r["g_v"] for r in res}},
    }
    print(json.dumps(_finite(line)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--relax", type=int, default=2000,
                    help="untimed steps from the random start before the warm-up")
    ap.add_argument("--t0-steps", type=int, default=20,
                    help="steps timed on their own from the random start")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="dimers_4M")
    ap.add_argument("--rng-kind", type=int, default=0)
    ap.add_argument("--noise-kind", type=int, default=0)
    ap.add_argument("--skin", type=float, default=0.0,
                    help="Verlet skin (0: cell list rebuilt every step)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run a plain copy kernel of this many MiB (counter calibration)")
    ap.add_argument("--sweep-steps", type=int, default=5000,
                    help="steps of each replica (workload sweep64)")
    ap.add_argument("--graph-chunk", type=int, default=50,
                    help="steps per captured graph chunk (workload sweep64)")
    ap.add_argument("--tune", action="store_true",
                    help="time the tuner's schedules at the start and keep the fastest (workload sweep64)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the one-after-another runs (workload sweep64)")
    ap.add_argument("--closure-epochs", type=int, default=40)
    ap.add_argument("--closure-ensemble", type=int, default=32,
                    help="independent replicas of the evaluated run (and of its calibration ensemble)")
    ap.add_argument("--closure-warm", type=int, default=4000,
                    help="DPD warm-up steps of each ensemble before its fields are taken")
    ap.add_argument("--closure-steps", type=int, default=2000,
                    help="closure steps of the evaluated rollout (x50 DPD steps)")
    ap.add_argument("--closure-cal-steps", type=int, default=1000,
                    help="closure steps of each calibration rollout")
    ap.add_argument("--rollout-steps", type=int, default=200,
                    help="batched closure steps (workload rollout)")
    ap.add_argument("--grid-steps", type=int, default=10000,
                    help="steps per grid point (workload grid200k)")
    ap.add_argument("--paper-warm", type=int, default=100000)
    ap.add_argument("--paper-steps", type=int, default=200000)
    ap.add_argument("--paper-every", type=int, default=20000)
    ap.add_argument("--paper-subset", default="",
                    help="only these (Gamma,Gamma_s) pairs, e.g. '8,0.5;8,0' (workload paper)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the engine has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "sweep64":
        run_sweep(args)
        return
    if args.workload == "closure":
        run_closure(args)
        return
    if args.workload == "paper":
        run_paper(args)
        return
    if args.workload == "rollout":
        run_rollout(args)
        return
    if args.workload == "grid200k":
        run_grid200k(args)
        return

    run_headline(args)


def run_headline(args):
    """The 4M-particle system: a timed window of K steps (velocity field after
    every 20, FP64 totals every 100 and at least once), preceded by a fixed,
    untimed relaxation from the random start and W further warm-up steps; the
    rate of the first steps from the random start is timed on its own."""
    import numpy as np
    import torch

    from paper_1310_0998_amd import dpd, inputs

    wl = inputs.WORKLOADS[args.workload]
    cfg = dict(inputs.physics(wl), rng_kind=args.rng_kind, noise_kind=args.noise_kind,
               skin=args.skin)
    bin_M = wl.get("bin_M", 256)
    bin_every = wl.get("bin_every", 20)
    reduce_every = wl.get("reduce_every", 100)
    steps = max(1, args.steps)
    warm = max(0, args.warmup)
    relax = max(0, args.relax)
    t0_steps = max(1, args.t0_steps)
    dev = torch.device("cuda:0")
    if args.calibrate_copy_mb > 0:
        nb = args.calibrate_copy_mb << 20
        a = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            dpd.copy_kernel(a, b)
        torch.cuda.synchronize()
        log(f"copy kernel calibration: 3 x {nb} bytes")
        del a, b
    x, v = inputs.initial_state(cfg)
    N = len(x)
    log(f"workload {args.workload}: N={N} L={cfg['L']} t0 window {t0_steps}, relaxation {relax}, "
        f"warm-up {warm}, timed {steps} steps")

    sim = dpd.Sim(dict(cfg, bin_M_max=bin_M), device=dev)
    sim.set_state(torch.from_numpy(x).to(dev), torch.from_numpy(v).to(dev), 0)
    out = (torch.empty((bin_M, bin_M, 2), dtype=torch.float32, device=dev),
           torch.empty((bin_M, bin_M), dtype=torch.int32, device=dev))
    pk = torch.zeros((steps // reduce_every + 2, 3), dtype=torch.float64, device=dev)

    def run(nsteps, record):
        """nsteps steps in chunks of bin_every, the velocity field after every
        full chunk; with record, the FP64 totals after every reduce_every steps
        and after the last chunk if none was taken.  Returns (bins, reductions)."""
        bins = reds = done = 0
        while done < nsteps:
            n = min(bin_every, nsteps - done)
            last = done + n == nsteps
            if record and ((done + n) % reduce_every == 0 or (last and reds == 0)):
                sim.step(n, reduce_every=n, pk=pk[reds:reds + 1])
                reds += 1
            else:
                sim.step(n)
            done += n
            if n == bin_every:
                sim.bin_velocity(bin_M, 0.0, 0, out=out)
                bins += 1
        return bins, reds

    # t = 0: the first steps from the random start (Poisson cell occupancy)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    sim.step(t0_steps)
    torch.cuda.synchronize()
    t0_time = time.perf_counter() - ta
    # relaxation to the steady state, untimed and of fixed length
    sim.step(relax)
    run(warm, False)
    sim.sync()
    torch.cuda.synchronize()
    reb0 = sim.rebuilds()
    sim.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_bins, n_red = run(steps, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.sync()
    pair_ms, launches = sim.pair_kernel_time()
    reb = sim.rebuilds() - reb0
    sim.set_profiling(False)
    elapsed = t1 - t0
    value = N * steps / elapsed
    ms_per_step = 1e3 * elapsed / steps
    avg_us = 1e3 * pair_ms / max(launches, 1)
    n_cells = sim.n_c * sim.n_c
    alg = pair_pass_bytes(N, n_cells)
    fused = fused_kernel_bytes(N, n_cells)
    achieved = alg / (avg_us * 1e-6) / 1e9
    traffic = measured_traffic()
    valu = measured_valu(avg_us)
    pkh = pk.cpu().numpy()
    step_t0 = t0_steps + relax + warm
    log(f"t=0: {1e3 * t0_time / t0_steps:.4f} ms/step; timed: {elapsed:.4f} s, {ms_per_step:.4f} ms/step, "
        f"pair kernel {avg_us:.1f} us avg over {launches} launches, {achieved:.0f} GB/s algorithmic "
        f"(32 B/particle); {n_bins} velocity fields, {n_red} FP64 reductions (last KE {pkh[n_red - 1, 2]:.1f})")

    cpu = None
    if not args.no_cpu and args.cpu_steps > 0:
        log(f"cpu baseline: oracle, {args.cpu_steps} steps ...")
        cpu = cpu_baseline(cfg, x, v, args.cpu_steps)
        log(f"cpu baseline {cpu['value']:.3e} particle-steps/s on {cpu['cores']} threads")

    hbm_frac = achieved / HBM_PEAK_GBS
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: 2-D periodic box L={cfg['L']:g} r_c, "
                        f"{cfg['n_agents']} dimers ({N} particles, density 1), a=25, "
                        f"gamma={cfg['gamma']}, kT=1, zeta={cfg['gamma_s']}, F_p=1, "
                        f"dt={cfg['dt']}; {bin_M}x{bin_M} velocity field every {bin_every} steps, "
                        f"FP64 momentum/KE every {reduce_every} steps and at least once per window",
            "n_particles": N,
            "cells": n_cells,
            "rng": ["philox4x32-10", "philox2x32-10"][cfg["rng_kind"]],
            "noise": ["gaussian", "uniform"][cfg["noise_kind"]],
            "state": "fp32 (fp64 wrap and reductions)",
            "cell_list": (f"Verlet skin {args.skin:g}: {reb} rebuilds in {steps} timed steps"
                          if args.skin > 0 else "rebuilt every step"),
            "timed_window": {"first_step": step_t0, "steps": steps, "velocity_fields": n_bins,
                             "fp64_reductions": n_red,
                             "untimed_before": {"t0_window": t0_steps, "relaxation": relax,
                                                "warmup": warm}},
            "parallelism": "single-gpu",
        },
        "t0": {"steps": t0_steps, "value": N * t0_steps / t0_time,
               "ms_per_step": 1e3 * t0_time / t0_steps,
               "note": "first steps from the random start, before relaxation"},
        "roofline": {
            "kernel": "k_pair (fused pair + agent + Verlet)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hbm_frac,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg,
            "algorithmic_bytes_rule": "32 B per particle: x 8 + u 8 + id 4 read, F 8 written, "
                                      "cell_start 4 per cell",
            "avg_launch_us": avg_us,
            "timed_launches": launches,
            "fused_kernel_bytes_per_launch": fused,
            "frac_fused_bytes": fused / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "valu": valu,
            "binding": None if valu is None else ("valu" if valu["frac"] > hbm_frac else "hbm"),
        },
        "cpu_baseline": cpu,
    }
    sim.close()
    print(json.dumps(_finite(line)), flush=True)


if __name__ == "__main__":
    main()
