"""Plain FP64 CPU reference ("oracle") for the self-propelled soft-core dumbbell
DPD model of Hinz, Panchenko, Kim & Fried (arXiv:1310.0998).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP engine: the arithmetic lives in ``oracle.c`` (FP64, built with
``-ffp-contract=off``), and this module only marshals numpy arrays through
ctypes.

Parameters are given as a plain mapping with the keys of ``FIELDS``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Mapping

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FIELDS = (
    ("n_agents", ctypes.c_int64),
    ("L", ctypes.c_double),
    ("r_c", ctypes.c_double),
    ("A", ctypes.c_double),
    ("gamma", ctypes.c_double),
    ("kT", ctypes.c_double),
    ("kappa", ctypes.c_double),
    ("bond_l", ctypes.c_double),
    ("f_sp", ctypes.c_double),
    ("gamma_s", ctypes.c_double),
    ("mass", ctypes.c_double),
    ("dt", ctypes.c_double),
    ("seed", ctypes.c_uint64),
    ("noise_kind", ctypes.c_int32),
    ("rng_kind", ctypes.c_int32),
    ("sp_split", ctypes.c_int32),
    ("pad_", ctypes.c_int32),
    ("w_exp", ctypes.c_double),
)


class OracleParams(ctypes.Structure):
    _fields_ = list(FIELDS)


def build(force: bool = False) -> str:
    """Compile liboracle.so (gcc, FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))
    ):
        tmp = _LIB + ".tmp"
        cmd = [
            "gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(OracleParams)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        sig = {
            "oracle_philox4x32_10": (None, [u32p, u32p, u32p]),
            "oracle_philox2x32_10": (None, [u32p, ctypes.c_uint32, u32p]),
            "oracle_pair_words": (None, [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, u32p]),
            "oracle_pair_alpha": (ctypes.c_double, [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]),
            "oracle_pair_force": (ctypes.c_int, [P, dp, dp, ctypes.c_double, dp, dp]),
            "oracle_pairs_brute": (ctypes.c_int64, [P, dp, i64p, ctypes.c_int64, i64p]),
            "oracle_pairs_cells": (ctypes.c_int64, [P, dp, i64p, ctypes.c_int64, i64p]),
            "oracle_forces": (ctypes.c_int, [P, dp, dp, ctypes.c_int64, dp, ctypes.c_int]),
            "oracle_forces_subset": (ctypes.c_int, [P, dp, dp, ctypes.c_int64, i64p, ctypes.c_int64, dp]),
            "oracle_force_parts": (ctypes.c_int, [P, dp, dp, ctypes.c_int64, dp, dp, ctypes.c_int]),
            "oracle_step": (ctypes.c_int, [P, dp, dp, dp, i64p, ctypes.c_int64, ctypes.c_int,
                                           ctypes.c_int64, dp]),
            "oracle_momentum_ke": (None, [P, dp, dp]),
            "oracle_bin": (ctypes.c_int64, [P, fp, i32p, i32p]),
            "oracle_n_cells_side": (ctypes.c_int64, [P]),
            "oracle_bin_velocity": (ctypes.c_int, [P, fp, fp, ctypes.c_int32, ctypes.c_double,
                                                   ctypes.c_int32, dp, i32p]),
            "oracle_minimg": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
            "oracle_wrap": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
            "oracle_num_threads": (ctypes.c_int, []),
            "oracle_set_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


DEFAULTS = dict(noise_kind=0, rng_kind=0, sp_split=0, seed=0, mass=1.0, w_exp=2.0)


def make_params(cfg: Mapping) -> OracleParams:
    """Build the C parameter struct from a mapping (missing optional keys take
    DEFAULTS; unknown keys are ignored)."""
    vals = dict(DEFAULTS)
    vals.update({k: cfg[k] for k in cfg})
    p = OracleParams()
    for name, ctype in FIELDS:
        if name == "pad_":
            continue
        v = vals[name]
        setattr(p, name, int(v) if ctype in (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64) else float(v))
    return p


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _u32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _vec64(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(n, 2)
    return a


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls."""
    lib().oracle_set_threads(int(n))


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_u32(c), _u32(k), _u32(out))
    return out


def philox2x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(2, np.uint32)
    lib().oracle_philox2x32_10(_u32(c), ctypes.c_uint32(int(key)), _u32(out))
    return out


def pair_words(cfg, i, j, step):
    p = make_params(cfg)
    out = np.zeros(4, np.uint32)
    lib().oracle_pair_words(ctypes.byref(p), int(i), int(j), int(step), _u32(out))
    return out


def pair_alpha(cfg, i, j, step) -> float:
    p = make_params(cfg)
    return float(lib().oracle_pair_alpha(ctypes.byref(p), int(i), int(j), int(step)))


def pair_force(cfg, d, dv, alpha):
    """Force on i from j for separation d = x_i - x_j and dv = v_i - v_j.
    Returns (f, parts(3,2), interacts)."""
    p = make_params(cfg)
    d = np.ascontiguousarray(d, dtype=np.float64)
    dv = np.ascontiguousarray(dv, dtype=np.float64)
    f = np.zeros(2)
    parts = np.zeros(6)
    hit = lib().oracle_pair_force(ctypes.byref(p), _d(d), _d(dv), float(alpha), _d(f), _d(parts))
    return f, parts.reshape(3, 2), bool(hit)


def pairs(cfg, x, method: str = "cells"):
    """Sorted interacting pairs (i < j) as an (n, 2) int64 array."""
    p = make_params(cfg)
    n = 2 * int(cfg["n_agents"])
    x = _vec64(x, n)
    fn = lib().oracle_pairs_cells if method == "cells" else lib().oracle_pairs_brute
    need = ctypes.c_int64(0)
    cap = max(16, 8 * n)
    while True:
        buf = np.zeros((cap, 2), np.int64)
        r = fn(ctypes.byref(p), _d(x), _i64(buf), cap, ctypes.byref(need))
        if r >= 0:
            return buf[:r].copy()
        if need.value <= cap:
            raise RuntimeError("oracle pair search failed")
        cap = int(need.value)


def forces(cfg, x, v, step, method: str = "cells"):
    p = make_params(cfg)
    n = 2 * int(cfg["n_agents"])
    x = _vec64(x, n)
    v = _vec64(v, n)
    F = np.zeros((n, 2))
    m = 1 if method == "cells" else 0
    if lib().oracle_forces(ctypes.byref(p), _d(x), _d(v), int(step), _d(F), m):
        raise RuntimeError("oracle_forces failed")
    return F


def forces_subset(cfg, x, v, step, idx):
    p = make_params(cfg)
    n = 2 * int(cfg["n_agents"])
    x = _vec64(x, n)
    v = _vec64(v, n)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    F = np.zeros((len(idx), 2))
    if lib().oracle_forces_subset(ctypes.byref(p), _d(x), _d(v), int(step), _i64(idx), len(idx), _d(F)):
        raise RuntimeError("oracle_forces_subset failed")
    return F


def force_parts(cfg, x, v, step, method: str = "cells"):
    """Per-particle sums of the conservative, dissipative and random pair
    forces, (N, 3, 2), and the per-particle force scale S_i, (N,)."""
    p = make_params(cfg)
    n = 2 * int(cfg["n_agents"])
    x = _vec64(x, n)
    v = _vec64(v, n)
    out = np.zeros((n, 6))
    scale = np.zeros(n)
    m = 1 if method == "cells" else 0
    if lib().oracle_force_parts(ctypes.byref(p), _d(x), _d(v), int(step), _d(out), _d(scale), m):
        raise RuntimeError("oracle_force_parts failed")
    return out.reshape(n, 3, 2), scale


def step(cfg, x, v, F, step0, n, method: str = "cells", every: int = 0):
    """Advance (x, v, F) by n velocity-Verlet steps.  Returns
    (x, v, F, step, pk) with pk an (n // every, 3) array of (Px, Py, KE)."""
    p = make_params(cfg)
    npart = 2 * int(cfg["n_agents"])
    x = _vec64(x, npart).copy()
    v = _vec64(v, npart).copy()
    F = _vec64(F, npart).copy()
    s = ctypes.c_int64(int(step0))
    nrec = (n // every) if every > 0 else 0
    pk = np.zeros((max(nrec, 1), 3))
    m = 1 if method == "cells" else 0
    if lib().oracle_step(ctypes.byref(p), _d(x), _d(v), _d(F), ctypes.byref(s), int(n), m,
                         int(every), _d(pk)):
        raise RuntimeError("oracle_step failed")
    return x, v, F, int(s.value), pk[:nrec]


def momentum_ke(cfg, v):
    p = make_params(cfg)
    n = 2 * int(cfg["n_agents"])
    v = _vec64(v, n)
    out = np.zeros(3)
    lib().oracle_momentum_ke(ctypes.byref(p), _d(v), _d(out))
    return out


def n_cells_side(cfg) -> int:
    p = make_params(cfg)
    return int(lib().oracle_n_cells_side(ctypes.byref(p)))


def bin_cells(cfg, x32):
    """(cell_start[n_c^2 + 1], ids[N]) for FP32 positions, ids in (cell, id) order."""
    p = make_params(cfg)
    n = 2 * int(cfg["n_agents"])
    x32 = np.ascontiguousarray(x32, dtype=np.float32).reshape(n, 2)
    nc = n_cells_side(cfg)
    cs = np.zeros(nc * nc + 1, np.int32)
    ids = np.zeros(max(n, 1), np.int32)
    r = lib().oracle_bin(ctypes.byref(p), _f(x32), _i32(cs), _i32(ids))
    if r < 0:
        raise RuntimeError("oracle_bin failed")
    return cs, ids[:n]


def bin_velocity(cfg, x32, v32, M, eps=0.0, mode=0):
    """Mean velocity (M, M, 2) [row j, column i] and counts (M, M) per grid window."""
    p = make_params(cfg)
    n = 2 * int(cfg["n_agents"])
    x32 = np.ascontiguousarray(x32, dtype=np.float32).reshape(n, 2)
    v32 = np.ascontiguousarray(v32, dtype=np.float32).reshape(n, 2)
    u = np.zeros((M * M, 2))
    cnt = np.zeros(M * M, np.int32)
    if lib().oracle_bin_velocity(ctypes.byref(p), _f(x32), _f(v32), int(M), float(eps), int(mode),
                                 _d(u), _i32(cnt)):
        raise RuntimeError("oracle_bin_velocity failed")
    return u.reshape(M, M, 2), cnt.reshape(M, M)


def minimg(d, L):
    return float(lib().oracle_minimg(float(d), float(L)))


def wrap(y, L):
    return float(lib().oracle_wrap(float(y), float(L)))
