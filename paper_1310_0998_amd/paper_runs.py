"""Runs at the paper's own parameters (Sec. 5.1) as one batch of replicas, and
the energy-spectrum statistics of Sec. 5.4 computed on the GPU.

Parameters: Phi = 1.5, r_c = 0.5, kT = 0.05 (Pe = 20), kappa = 1e3, l = 1,
f_SP = 1, m = 1, dt = 3e-3, L = 100; N = 4e4 phi agents; the pair friction
Gamma and the Stokes friction Gamma_s per replica.  Fields: u_M on a
128 x 128 grid with overlapping windows of width eps = L sqrt(N_f / N),
N_f = 10 agents per window on average (Eq. 5.10), particle velocities.
Statistics per replica, averaged over the snapshots: E(k) in unit shells, the
normalised spectrum E/E_1, its low-wavenumber slope alpha (least squares over
the first ten shells, Eq. 5.13) and the shell of its maximum.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import dpd, fieldstats, inputs

# (phi, Gamma, Gamma_s): Stokes and pair friction, and pair friction only
REPLICAS = [(0.2, 8.0, 0.5), (0.8, 8.0, 0.5), (0.2, 8.0, 0.0), (0.8, 8.0, 0.0)]
M = 128


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


def run(device, warm: int, steps: int, every: int, log=print):
    cfgs = [replica_cfg(*r, seed=701 + i) for i, r in enumerate(REPLICAS)]
    states = [inputs.initial_state(c) for c in cfgs]
    x = np.concatenate([s[0] for s in states])
    v = np.concatenate([s[1] for s in states])
    sim = dpd.Sim(cfgs, device=device)
    sim.set_state(torch.from_numpy(x).to(device), torch.from_numpy(v).to(device), 0)
    sim.set_graph_chunk(100)
    t0 = time.perf_counter()
    for w0 in range(0, warm, 20000):
        sim.step(min(20000, warm - w0))
        sim.sync()
        log(f"warm-up: {min(w0 + 20000, warm)} of {warm} steps, {time.perf_counter() - t0:.1f} s")
    R = len(cfgs)
    nsnap = steps // every
    fields = torch.empty((nsnap, R, M, M, 2), dtype=torch.float32, device=device)
    counts = torch.empty((R, M, M), dtype=torch.int32, device=device)
    for s in range(nsnap):
        sim.step(every)
        if (s + 1) % 20 == 0:
            sim.sync()
            log(f"snapshot {s + 1} of {nsnap}, {time.perf_counter() - t0:.1f} s")
        # windows of eps = L sqrt(10 / N) per replica: one call per replica's eps
        for q, c in enumerate(cfgs):
            eps = c["L"] * math.sqrt(10.0 / c["n_agents"])
            u, _ = sim.bin_velocity(M, eps, 0)
            fields[s, q].copy_(u[q])
    sim.sync()
    sim.close()
    out = []
    for q, (phi, g, gs) in enumerate(REPLICAS):
        f = fields[:, q].contiguous()
        E = fieldstats.shells(fieldstats.power(f), nsnap)
        alpha, _ = slope_fit(E)
        En = E / E[0]
        k_peak = int(np.argmax(En)) + 1
        # high-wavenumber slope over shells 32..56
        kh = np.arange(32, 57)
        ah = float(np.polyfit(np.log(kh), np.log(En[kh - 1]), 1)[0])
        out.append(dict(phi=phi, Gamma=g, Gamma_s=gs, alpha=alpha, k_peak=k_peak, alpha_high=ah,
                        E_over_E1=En.tolist()))
        log(f"phi {phi} Gamma {g} Gamma_s {gs}: alpha {alpha:+.3f}, peak at k = {k_peak}, "
            f"high-k slope {ah:+.2f}")
    return out
