"""Long-run statistics protocol for the statistical comparison of the engine
with the oracle (the energy spectrum and velocity correlation length of
Sec. 5.3-5.4).

Trajectories are chaotic and the noise differs between runs only through the
seed, so the engine and the oracle are compared by ensemble means: several
seeds, a warm-up from the random start, then snapshots at a fixed cadence.
For every snapshot:
  - the filtered, projected field u_M on an M x M grid with plain bins
    (Eqs. 5.8-5.10, window equal to the grid spacing, particle velocities) and
    its energy spectrum E(k) (Eqs. 5.11-5.12), summed over log-spaced bands of
    shells;
  - the velocity correlation function of the agent centre-of-mass velocities
    (Eqs. 5.5-5.6) in bins of r_c / 4.
Each seed gives the band energies averaged over its snapshots and the
integral length (Eq. 5.7) of its snapshot-averaged correlation function; the
ensemble mean and its standard error over seeds are compared.

This module holds the protocol and the statistics, both written with the
oracle's analysis routines; it generates no trajectories.
"""
from __future__ import annotations

import numpy as np

from oracle import analysis

PROTOCOL = dict(
    workload="dimers_1600",
    seeds=[101, 102, 103, 104, 105, 106, 107, 108],
    warmup=4000,        # steps from the random start (20 time units)
    steps=40000,        # measured steps per seed (200 time units)
    every=200,          # steps between snapshots
    M=20,               # grid side (spacing 2 r_c at L = 40)
    dr=0.25,            # correlation-function bin width (r_c / 4)
    bands=[(1, 1), (2, 2), (3, 4), (5, 7), (8, 10)],
)


def band_energies(E: np.ndarray) -> np.ndarray:
    return np.array([E[a - 1:b].sum() for a, b in PROTOCOL["bands"]])


class SeedAccumulator:
    """Running snapshot sums of one seed."""

    def __init__(self, L: float):
        self.L = L
        self.n = 0
        self.E = np.zeros(len(PROTOCOL["bands"]))
        self.g = None

    def add(self, u: np.ndarray, x: np.ndarray, v: np.ndarray):
        self.E += band_energies(analysis.energy_spectrum(np.asarray(u, np.float64)))
        com, V = analysis.agent_com(x, v, self.L)
        r, g, _ = analysis.vcf_bruteforce(com, V, self.L, PROTOCOL["dr"])
        self.r = r
        self.g = g if self.g is None else self.g + g
        self.n += 1

    def result(self):
        g = self.g / self.n
        return dict(E_bands=(self.E / self.n).tolist(),
                    L_gv=analysis.integral_length(self.r, g, self.L),
                    snapshots=self.n)


def ensemble(per_seed: list) -> dict:
    """Mean and standard error over seeds of the band energies and of L_gv."""
    E = np.array([s["E_bands"] for s in per_seed])
    Lg = np.array([s["L_gv"] for s in per_seed])
    k = len(per_seed)
    return dict(E_bands=E.mean(0).tolist(), E_bands_sem=(E.std(0, ddof=1) / np.sqrt(k)).tolist(),
                L_gv=float(Lg.mean()), L_gv_sem=float(Lg.std(ddof=1) / np.sqrt(k)), seeds=k)
