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
ensemble mean and its standard error over seeds are compared.  512 seeds
bring the standard error of every compared mean below 0.5 % (the lowest band,
with its 8 modes, has a spread of about 7 % between seeds).

The correlation function is computed by vcf_pairs, a vectorised form of the
oracle's pair loop (analysis.vcf_bruteforce) over the same pairs and bins; a
CPU test checks that the two agree.

This module holds the protocol and the statistics, both written with the
oracle's analysis routines; it generates no trajectories.
"""
from __future__ import annotations

import numpy as np

from oracle import analysis

PROTOCOL = dict(
    workload="dimers_1600",
    seeds=list(range(1001, 1001 + 512)),  # independent replicas
    warmup=4000,        # steps from the random start (20 time units)
    steps=40000,        # measured steps per seed (200 time units)
    every=200,          # steps between snapshots
    M=20,               # grid side (spacing 2 r_c at L = 40)
    dr=0.25,            # correlation-function bin width (r_c / 4)
    bands=[(1, 1), (2, 2), (3, 4), (5, 7), (8, 10)],
)


def vcf_pairs(pos: np.ndarray, V: np.ndarray, L: float, dr: float):
    """analysis.vcf_bruteforce over the same pairs k < l and bins, vectorised:
    (r_centres, g, counts) with g(0) := 1 prepended at r = 0."""
    pos = np.asarray(pos, np.float64)
    V = np.asarray(V, np.float64)
    n = len(pos)
    mean = V.mean(axis=0)
    mean2 = float(mean @ mean)
    var = float((V * V).sum(axis=1).mean()) - mean2
    nb = int(np.floor(0.5 * L / dr))
    i, j = np.triu_indices(n, 1)
    d = pos[j] - pos[i]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(axis=1))
    b = np.floor(r / dr).astype(np.int64)
    ok = b < nb
    dots = (V[j] * V[i]).sum(axis=1)
    num = np.bincount(b[ok], weights=dots[ok], minlength=nb)[:nb]
    cnt = np.bincount(b[ok], minlength=nb)[:nb]
    with np.errstate(invalid="ignore", divide="ignore"):
        g = (num / cnt - mean2) / var
    rc = (np.arange(nb) + 0.5) * dr
    return np.concatenate([[0.0], rc]), np.concatenate([[1.0], g]), np.concatenate([[0], cnt])


def band_energies_batch(u: np.ndarray) -> np.ndarray:
    """band_energies(analysis.energy_spectrum(u[f])) for a batch of fields
    u [F][M][M][2] at once: (F, bands)."""
    u = np.asarray(u, np.float64)
    M = u.shape[1]
    uh = np.fft.fft2(u, axes=(1, 2)) / float(M * M)
    e = 0.5 * (np.abs(uh[..., 0]) ** 2 + np.abs(uh[..., 1]) ** 2)
    shell = np.floor(analysis.wavenumber_magnitude(M) + 0.5).astype(np.int64)
    out = np.zeros((u.shape[0], len(PROTOCOL["bands"])))
    for q, (a, b) in enumerate(PROTOCOL["bands"]):
        m = (shell >= a) & (shell <= b)
        out[:, q] = e[:, m].sum(axis=1)
    return out


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
        r, g, _ = vcf_pairs(com, V, self.L, PROTOCOL["dr"])
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


# ---- the 4M-particle transient window ------------------------------------------
# The headline workload from its random start over t <= 10 (2000 steps), four
# seeds, a snapshot every 20 steps: u_M on 256 x 256 plain bins (particle
# velocities), its energy in log-spaced shell bands, and the correlation
# function of the gridded field (its autocorrelation by Wiener-Khinchin,
# averaged over angles in bins of one grid spacing; the agents' pair loop is
# out of reach for the oracle at 2 M agents).  The statistics change along
# the transient, so they are compared in matched time windows of 400 steps:
# per window and seed the mean band energies over its 20 snapshots and the
# integral length of its mean correlation function.

PROTOCOL_4M = dict(
    workload="dimers_4M",
    seeds=[301, 302, 303, 304],
    steps=2000,
    every=20,
    window=400,
    M=256,
    bands=[(1, 1), (2, 3), (4, 7), (8, 15), (16, 31), (32, 63), (64, 128)],
)


def band_energies_of(E: np.ndarray, bands) -> np.ndarray:
    return np.array([E[a - 1:b].sum() for a, b in bands])


class WindowAccumulator:
    """Snapshot sums of one seed over the matched time windows of PROTOCOL_4M."""

    def __init__(self, L: float):
        P = PROTOCOL_4M
        self.L = L
        self.dr = L / P["M"]
        self.per_window = P["window"] // P["every"]
        self.nw = P["steps"] // P["window"]
        self.E = np.zeros((self.nw, len(P["bands"])))
        self.g = [None] * self.nw
        self.n = 0

    def add(self, u: np.ndarray):
        w = self.n // self.per_window
        u = np.asarray(u, np.float64)
        self.E[w] += band_energies_of(analysis.energy_spectrum(u), PROTOCOL_4M["bands"])
        r, g = analysis.vcf_grid(u, self.L, self.dr)
        self.r = r
        self.g[w] = g if self.g[w] is None else self.g[w] + g
        self.n += 1

    def result(self):
        k = self.per_window
        return dict(E_bands=(self.E / k).tolist(),
                    L_gv=[analysis.integral_length(self.r, g / k, self.L) for g in self.g],
                    snapshots=self.n)


def window_ensemble(per_seed: list) -> dict:
    """Mean and standard error over seeds, per window, of the band energies and L_gv."""
    E = np.array([s["E_bands"] for s in per_seed])   # seeds x windows x bands
    Lg = np.array([s["L_gv"] for s in per_seed])     # seeds x windows
    k = len(per_seed)
    return dict(E_bands=E.mean(0).tolist(), E_bands_sem=(E.std(0, ddof=1) / np.sqrt(k)).tolist(),
                L_gv=Lg.mean(0).tolist(), L_gv_sem=(Lg.std(0, ddof=1) / np.sqrt(k)).tolist(), seeds=k)
