"""Runs at the paper's own parameters (Sec. 5.1) as one batch of replicas, with
the statistics of Sec. 5.3-5.4 computed on the GPU.

Parameters: Phi = 1.5, r_c = 0.5, kT = 0.05 (Pe = 20), kappa = 1e3, l = 1,
f_SP = 1, m = 1, dt = 3e-3, L = 100; N = 4e4 phi agents; the pair friction
Gamma and the Stokes friction Gamma_s per replica.  The replicas cover the
panels of the paper's spectra, correlation lengths and slopes: phi in
{0.2, 0.4, 0.6, 0.8} for Gamma in {0, 4, 8} with Gamma_s in {0.5, 0.1}, and
Gamma in {1, 4, 8} with Gamma_s = 0 (pair friction only).

Protocol (Sec. 5): a relaxation from the random start, then snapshots every
2 x 10^4 steps.  After the first 2 x 10^4 relaxation steps the tile schedule
is tuned on the state reached (clusters have formed by then, and the tiles of
the dense replicas overflow the default capacities), and tuned again every
2 x 10^5 relaxation steps as the clusters grow; the trajectories are bitwise
independent of the schedule, so only the run time changes.  Per snapshot and replica:
  - u_M on a 128 x 128 grid with overlapping windows of width
    eps = L sqrt(N_f / N), N_f = 10 agents per window on average (Eq. 5.10),
    particle velocities, binned once per replica with its own eps;
  - the velocity correlation function g_v of the agent centres of mass
    (Eqs. 5.5-5.6) from pair sums on the GPU, bins of r_c / 4 out to L/2.
Per replica, averaged over the snapshots: E(k) in unit shells, E/E_1, its
low-wavenumber slope alpha (least squares over the first ten shells,
Eq. 5.13), the shell of its maximum, the high-wavenumber slope over shells
32-56, and the integral length L_gv of the averaged g_v (Eq. 5.7, trapezoid
rule to L/2).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import dpd, fieldstats, inputs

PHIS = (0.2, 0.4, 0.6, 0.8)
# (Gamma, Gamma_s): Stokes and pair friction, Stokes friction only, pair friction only
FRICTIONS = [(0.0, 0.5), (4.0, 0.5), (8.0, 0.5), (0.0, 0.1), (4.0, 0.1), (8.0, 0.1),
             (1.0, 0.0), (4.0, 0.0), (8.0, 0.0)]
REPLICAS = [(phi, g, gs) for (g, gs) in FRICTIONS for phi in PHIS]
M = 128
N_F = 10            # agents per window on average (Eq. 5.10)
HIGH_K = (32, 56)   # shells of the high-wavenumber slope


def replica_cfg(phi: float, gamma: float, gamma_s: float, seed: int):
    n_agents = int(round(4.0e4 * phi))
    return dict(inputs.PAPER_SET, n_agents=n_agents, gamma=gamma, gamma_s=gamma_s, seed=seed,
                bin_M_max=M)


def slope_fit(E: np.ndarray, n: int = 10):
    """Least-squares alpha and C of ln(E/E_1) = ln C + alpha ln k over k = 1..n."""
    k = np.arange(1, n + 1, dtype=np.float64)
    y = np.log(E[:n] / E[0])
    A = np.stack([np.ones_like(k), np.log(k)], axis=1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(coef[1]), float(math.exp(coef[0]))


def run(device, warm: int, steps: int, every: int, replicas=None, log=print, tune: bool = True):
    reps = REPLICAS if replicas is None else replicas
    cfgs = [replica_cfg(*r, seed=701 + i) for i, r in enumerate(reps)]
    states = [inputs.initial_state(c) for c in cfgs]
    x = np.concatenate([s[0] for s in states])
    v = np.concatenate([s[1] for s in states])
    sim = dpd.Sim(cfgs, device=device)
    sim.set_state(torch.from_numpy(x).to(device), torch.from_numpy(v).to(device), 0)
    sim.set_graph_chunk(100)
    t0 = time.perf_counter()
    schedule = []
    for w0 in range(0, warm, 20000):
        done = min(w0 + 20000, warm)
        sim.step(done - w0)
        sim.sync()
        log(f"relaxation: {done} of {warm} steps, {time.perf_counter() - t0:.1f} s")
        if tune and (w0 == 0 or done % 200000 == 0):
            tx, ty, order, ms = sim.autotune(50)
            schedule.append(dict(replica0_tile=[tx, ty], order=order, trial_ms_per_step=ms,
                                 after_steps=done))
            log(f"schedule tuned after {done} steps: replica 0 tile {tx} x {ty}, order {order}, "
                f"{ms:.4f} ms/step in the trials")
    R = len(cfgs)
    eps = [c["L"] * math.sqrt(N_F / c["n_agents"]) for c in cfgs]
    base = np.concatenate([[0], np.cumsum([2 * c["n_agents"] for c in cfgs])])
    dr = inputs.PAPER_SET["r_c"] / 4.0
    nsnap = steps // every
    P = [np.zeros((M, M)) for _ in range(R)]
    G = [None] * R
    counts = torch.empty((R, M, M), dtype=torch.int32, device=device)
    fields = torch.empty((R, M, M, 2), dtype=torch.float32, device=device)
    for s in range(nsnap):
        sim.step(every)
        sim.bin_velocity_reps(M, eps, 0, out=(fields, counts))
        xs, vs, _, _ = sim.get_state()
        for q in range(R):
            P[q] += fieldstats.power(fields[q:q + 1].contiguous())
            r, g, _ = fieldstats.agent_vcf(xs[base[q]:base[q + 1]], vs[base[q]:base[q + 1]],
                                           cfgs[q]["L"], dr)
            G[q] = g if G[q] is None else G[q] + g
        log(f"snapshot {s + 1} of {nsnap}, {time.perf_counter() - t0:.1f} s")
    sim.sync()
    sim.close()
    out = []
    for q, (phi, gm, gs) in enumerate(reps):
        E = fieldstats.shells(P[q], nsnap)
        alpha, _ = slope_fit(E)
        En = E / E[0]
        k_peak = int(np.argmax(En)) + 1
        kh = np.arange(HIGH_K[0], HIGH_K[1] + 1)
        ah = float(np.polyfit(np.log(kh), np.log(En[kh - 1]), 1)[0])
        g = G[q] / nsnap
        L = cfgs[q]["L"]
        L_gv = fieldstats.integral_length(r, g, L, to_first_zero=False)
        out.append(dict(phi=phi, Gamma=gm, Gamma_s=gs, alpha=alpha, k_peak=k_peak, alpha_high=ah,
                        L_gv=L_gv, E_over_E1=En.tolist(), g_v=g.tolist()))
        log(f"phi {phi} Gamma {gm} Gamma_s {gs}: alpha {alpha:+.3f}, peak at k = {k_peak}, "
            f"high-k slope {ah:+.2f}, L_gv {L_gv:.3f}")
    return out, r.tolist(), schedule


def checks(res):
    """The paper's qualitative findings (Sec. 5.3-5.4), each as a boolean."""
    def sel(**kw):
        return [x for x in res if all(x[k] == v for k, v in kw.items())]

    stokes = [x for x in res if x["Gamma_s"] > 0]
    pair = [x for x in res if x["Gamma_s"] == 0]
    out = {
        # with Stokes friction: positive low-k slope and a maximum at intermediate k
        "stokes_low_k_slope_positive": all(x["alpha"] > 0 for x in stokes),
        "stokes_peak_at_intermediate_k": all(x["k_peak"] > 1 for x in stokes),
        # ... whose wavenumber grows with the area fraction
        "stokes_peak_moves_to_larger_k_with_phi": all(
            sel(Gamma=g, Gamma_s=gs, phi=0.8)[0]["k_peak"] >= sel(Gamma=g, Gamma_s=gs, phi=0.2)[0]["k_peak"]
            for g, gs in {(x["Gamma"], x["Gamma_s"]) for x in stokes}),
        # pair friction only: the energy collects in the first shell
        "pair_only_peak_in_first_shell": all(x["k_peak"] == 1 for x in pair if x["phi"] >= 0.4),
        "pair_only_low_k_slope_negative_at_Gamma_8": all(x["alpha"] < 0 for x in sel(Gamma=8.0, Gamma_s=0.0)),
        # pair friction only: L_gv grows with Gamma at every area fraction
        "pair_only_L_gv_grows_with_Gamma": all(
            sel(Gamma=8.0, Gamma_s=0.0, phi=p)[0]["L_gv"] > sel(Gamma=1.0, Gamma_s=0.0, phi=p)[0]["L_gv"]
            for p in PHIS),
        "high_k_slope_negative": all(x["alpha_high"] < 0 for x in res),
    }
    return out
