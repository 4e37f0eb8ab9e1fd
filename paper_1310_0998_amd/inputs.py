"""Seeded synthetic inputs shared by the engine's tests, the oracle's tests and
the benchmark.

This module holds only workload parameters and random initial states; it
contains none of the method's arithmetic.  Initial states follow Sec. 5 of the
paper: agents randomly distributed and randomly oriented in the periodic box,
zero initial velocities.  Particle 2k is the head and 2k+1 the tail of agent k.
"""
from __future__ import annotations

import math

import numpy as np

# Force-law parameters common to the plain-DPD workloads (Groot-Warren-style
# constants with the paper's force law, Eqs. 2.2-2.7).
_BASE = dict(
    r_c=1.0, A=25.0, gamma=4.5, kT=1.0, kappa=1000.0, bond_l=0.5, f_sp=1.0,
    gamma_s=0.5, mass=1.0, dt=0.005, noise_kind=0, rng_kind=0, sp_split=0,
)

WORKLOADS = {
    # 40 x 40 box, 800 dimers (1600 particles); parity-scale system.
    "dimers_1600": dict(_BASE, n_agents=800, L=40.0, seed=101, steps=1000),
    # 447 x 447 box, 100k dimers (200k particles, density ~1).
    "dimers_200k": dict(_BASE, n_agents=100_000, L=447.0, seed=201, steps=10_000),
    # 2000 x 2000 box, 2M dimers (4M particles, density 1); velocity field
    # binned on 256 x 256 every 20 steps.
    "dimers_4M": dict(_BASE, n_agents=2_000_000, L=2000.0, seed=301, steps=2000,
                      bin_M=256, bin_every=20, reduce_every=100),
}

# The pair-friction x Stokes-friction grid run at 200k particles.
GAMMA_ZETA_GRID_200K = [(g, z) for g in (1.0, 4.5, 20.0) for z in (0.0, 0.5, 5.0)]

# The paper's own nondimensional parameter set (Sec. 5.1): Phi = 1.5,
# Pe = 20 (kT = 0.05), kappa = 1e3, l = 1, r_c = 0.5, L = 100, dt = 3e-3.
PAPER_SET = dict(
    r_c=0.5, A=1.5, kT=0.05, kappa=1000.0, bond_l=1.0, f_sp=1.0, mass=1.0,
    dt=0.003, L=100.0, noise_kind=0, rng_kind=0, sp_split=0,
)


# Batched sweep: replicas over area fraction phi and the friction ratio
# gamma / zeta (the paper varies phi, Gamma and Gamma_s, Sec. 5 and 5.1).
SWEEP_PHI = (0.2, 0.4, 0.6, 0.8)
SWEEP_RATIO = (0.1, 1.0, 10.0, 100.0)


def sweep_replicas(n_rep: int = 64, seed: int = 401, n_min: int = 2000, n_max: int = 64000,
                   base: dict | None = None) -> list:
    """Workload mappings of a seeded sweep: agent counts log-uniform on
    [n_min, n_max]; replica r takes grid point r mod 16 of phi x (gamma/zeta)
    with gamma = 4.5 and zeta = 4.5 / ratio; box side L = r_c sqrt(N_a / phi)
    rounded to a multiple of 2^-8 (areal density 2 phi / r_c^2); noise seed
    4000 + r."""
    b = dict(_BASE if base is None else base)
    rng = np.random.Generator(np.random.PCG64(seed))
    na = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_rep))
    grid = [(phi, ratio) for phi in SWEEP_PHI for ratio in SWEEP_RATIO]
    out = []
    for r in range(n_rep):
        phi, ratio = grid[r % len(grid)]
        n_agents = int(round(float(na[r])))
        L = b["r_c"] * math.sqrt(n_agents / phi)
        L = math.floor(L * 256.0) / 256.0
        out.append(dict(b, n_agents=n_agents, L=L, gamma=4.5, gamma_s=4.5 / ratio,
                        seed=4000 + r, phi=phi, ratio=ratio))
    return out


def physics(cfg: dict) -> dict:
    """The model parameters of a workload (drops run-length keys)."""
    keep = ("n_agents", "L", "r_c", "A", "gamma", "kT", "kappa", "bond_l", "f_sp",
            "gamma_s", "mass", "dt", "seed", "noise_kind", "rng_kind", "sp_split")
    return {k: cfg[k] for k in keep if k in cfg}


def _to_box_f32(p: np.ndarray, L: float) -> np.ndarray:
    q = np.mod(p, L).astype(np.float32)
    q[q >= np.float32(L)] = 0.0
    q[q < 0] = 0.0
    return q


def random_dimers(seed: int, n_agents: int, L: float, bond_l: float) -> np.ndarray:
    """Uniform centres of mass in [0, L)^2, uniform axis angles in [0, 2 pi);
    head/tail at COM +- (l/2)(cos, sin).  Returns FP32 (2 n_agents, 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    com = rng.uniform(0.0, L, size=(n_agents, 2))
    th = rng.uniform(0.0, 2.0 * math.pi, size=n_agents)
    half = 0.5 * bond_l * np.stack([np.cos(th), np.sin(th)], axis=1)
    x = np.empty((2 * n_agents, 2), np.float64)
    x[0::2] = com + half
    x[1::2] = com - half
    return _to_box_f32(x, L)


def thermal_velocities(seed: int, n: int, kT: float, mass: float) -> np.ndarray:
    """Maxwell-Boltzmann velocities N(0, kT/m) per component, mean removed."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    v = rng.normal(0.0, math.sqrt(kT / mass), size=(n, 2))
    v -= v.mean(axis=0)
    return v.astype(np.float32)


def clustered_dimers(seed: int, n_agents: int, L: float, bond_l: float,
                     centre=(0.5, 0.5), radius: float = 3.0) -> np.ndarray:
    """Agents packed in a disc of the given radius (dense cells)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rr = radius * np.sqrt(rng.uniform(0.0, 1.0, n_agents))
    ph = rng.uniform(0.0, 2.0 * math.pi, n_agents)
    com = np.stack([centre[0] * L + rr * np.cos(ph), centre[1] * L + rr * np.sin(ph)], axis=1)
    th = rng.uniform(0.0, 2.0 * math.pi, size=n_agents)
    half = 0.5 * bond_l * np.stack([np.cos(th), np.sin(th)], axis=1)
    x = np.empty((2 * n_agents, 2), np.float64)
    x[0::2] = com + half
    x[1::2] = com - half
    return _to_box_f32(x, L)


def edge_dimers(seed: int, n_agents: int, L: float, bond_l: float, r_c: float) -> np.ndarray:
    """Adversarial layout: agents centred on cell edges and on the box faces,
    heads at exactly 0 and just below L, agents straddling the periodic
    boundary; the rest random."""
    x = random_dimers(seed, n_agents, L, bond_l).astype(np.float64)
    nc = int(math.floor(L / r_c))
    w = L / nc
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    k = 0
    below_L = float(np.nextafter(np.float32(L), np.float32(0)))
    specials = []
    for c in range(0, nc, max(1, nc // 8)):
        specials.append((c * w, rng.uniform(0, L)))          # on a vertical cell edge
        specials.append((rng.uniform(0, L), c * w))          # on a horizontal cell edge
    specials += [(0.0, 0.0), (below_L, below_L), (0.0, below_L), (below_L, 0.0)]
    for (cx, cy) in specials:
        if k >= n_agents:
            break
        th = rng.uniform(0, 2 * math.pi)
        x[2 * k] = (cx, cy)                                   # head exactly on the edge
        x[2 * k + 1] = (cx - bond_l * math.cos(th), cy - bond_l * math.sin(th))
        k += 1
    return _to_box_f32(x, L)


def initial_state(cfg: dict, kind: str = "random", thermal: bool = False):
    """(x, v) FP32 arrays of shape (N, 2) for a workload mapping."""
    n_agents, L, l = int(cfg["n_agents"]), float(cfg["L"]), float(cfg["bond_l"])
    seed = int(cfg.get("seed", 0))
    if kind == "random":
        x = random_dimers(seed, n_agents, L, l)
    elif kind == "clustered":
        x = clustered_dimers(seed, n_agents, L, l)
    elif kind == "edge":
        x = edge_dimers(seed, n_agents, L, l, float(cfg["r_c"]))
    else:
        raise ValueError(kind)
    if thermal:
        v = thermal_velocities(seed, 2 * n_agents, float(cfg["kT"]), float(cfg.get("mass", 1.0)))
    else:
        v = np.zeros_like(x)
    return x, v


# ---- learned closure -------------------------------------------------------------

def closure_shapes(c_in: int, width: int, layers: int):
    """(c_in, c_out) of every convolution of the closure network."""
    return [(c_in if l == 0 else width, 2 if l == layers - 1 else width) for l in range(layers)]


def closure_init(seed: int, c_in: int, width: int, layers: int, out_scale: float = 0.1):
    """Seeded initial parameters of the closure network in its flat layout
    (per layer W[9][c_in][c_out], then b[c_out]): He-normal weights, the last
    layer scaled by out_scale, zero biases.  FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    shp = closure_shapes(c_in, width, layers)
    for l, (ci, co) in enumerate(shp):
        std = math.sqrt(2.0 / (9 * ci)) * (out_scale if l == len(shp) - 1 else 1.0)
        parts.append(rng.normal(0.0, std, size=9 * ci * co))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
