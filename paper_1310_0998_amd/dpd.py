"""Python binding of the HIP DPD engine (libdpd.so, C ABI in include/dpd.h).

Argument marshalling only: every step of the hot path runs in the engine's
kernels.  PyTorch provides device memory (the workspace and the state
tensors) and the stream.  If libdpd.so is missing the import of the engine
fails loudly; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Mapping, Optional, Sequence, Union

import torch  # loaded first so that the engine binds to torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpd.so")

DPD_OK = 0
ERRORS = {
    -1: "DPD_EINVAL", -2: "DPD_EWORKSPACE", -3: "DPD_EHIP", -4: "DPD_ENONFINITE",
    -5: "DPD_ESTATE", -6: "DPD_EBOND", -7: "DPD_ERANGE",
}


class DPDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
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
        ("bin_M_max", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("skin", ctypes.c_float),
        ("w_exp", ctypes.c_float),
        ("reserved", ctypes.c_int32 * 1),
    ]


_INT_FIELDS = {"n_agents", "seed", "noise_kind", "rng_kind", "sp_split", "bin_M_max", "tile"}
_DEFAULTS = dict(mass=1.0, seed=0, noise_kind=0, rng_kind=0, sp_split=0, bin_M_max=0, tile=0,
                 skin=0.0, w_exp=0.0)


def make_params(cfg: Mapping) -> Params:
    vals = dict(_DEFAULTS)
    vals.update(cfg)
    p = Params()
    for name, _ in Params._fields_:
        if name == "reserved":
            continue
        v = vals[name]
        setattr(p, name, int(v) if name in _INT_FIELDS else float(v))
    return p


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER(Params)
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "dpd_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
            "dpd_create": (ctypes.c_int, [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
            "dpd_destroy": (None, [vp]),
            "dpd_last_error": (ctypes.c_char_p, [vp]),
            "dpd_set_state": (ctypes.c_int, [vp, vp, vp, i64, vp]),
            "dpd_get_state": (ctypes.c_int, [vp, vp, vp, vp, ctypes.POINTER(i64)]),
            "dpd_forces": (ctypes.c_int, [vp, vp]),
            "dpd_step": (ctypes.c_int, [vp, i32, i32, vp]),
            "dpd_bin_velocity": (ctypes.c_int, [vp, i32, f64, i32, vp, vp]),
            "dpd_sync": (ctypes.c_int, [vp]),
            "dpd_get_cells": (ctypes.c_int, [vp, vp, vp]),
            "dpd_cells_per_side": (i64, [P]),
            "dpd_rng_words": (ctypes.c_int, [P, vp, vp, i64, i32, vp, vp, vp]),
            "dpd_set_profiling": (ctypes.c_int, [vp, i32]),
            "dpd_pair_kernel_time": (ctypes.c_int, [vp, ctypes.POINTER(f64), ctypes.POINTER(i64)]),
            "dpd_cell_list_rebuilds": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
            "dpd_copy_kernel": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
            "dpd_forces_noalloc": (ctypes.c_int, [P, vp, vp, i64, vp, vp]),
            "dpd_bin_velocity_reps": (ctypes.c_int, [vp, i32, ctypes.POINTER(f64), i32, vp, vp]),
            "dpd_agent_vcf": (ctypes.c_int, [vp, vp, i64, f64, f64, i32, vp, vp, vp, vp]),
            "dpd_batch_workspace_bytes": (ctypes.c_int, [P, i32, ctypes.POINTER(ctypes.c_size_t)]),
            "dpd_create_batch": (ctypes.c_int, [P, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
            "dpd_set_graph_chunk": (ctypes.c_int, [vp, i32]),
            "dpd_set_schedule": (ctypes.c_int, [vp, i32, i32, i32]),
            "dpd_get_schedule": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                                ctypes.POINTER(i32)]),
            "dpd_autotune": (ctypes.c_int, [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                            ctypes.POINTER(i32), ctypes.POINTER(f64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, handle=None):
    if rc != DPD_OK:
        msg = lib().dpd_last_error(handle).decode()
        raise DPDError(rc, msg)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _vec(t: torch.Tensor, n: int, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == 2 * n):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of {n} x 2 values")
    return t


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def cells_per_side(cfg: Mapping) -> int:
    r = lib().dpd_cells_per_side(ctypes.byref(make_params(cfg)))
    if r < 0:
        _check(int(r))
    return int(r)


def _param_array(cfgs: Sequence[Mapping]):
    arr = (Params * len(cfgs))()
    for k, c in enumerate(cfgs):
        arr[k] = make_params(c)
    return arr


def workspace_bytes(cfg: Union[Mapping, Sequence[Mapping]]) -> int:
    cfgs = [cfg] if isinstance(cfg, Mapping) else list(cfg)
    n = ctypes.c_size_t(0)
    _check(lib().dpd_batch_workspace_bytes(_param_array(cfgs), len(cfgs), ctypes.byref(n)))
    return int(n.value)


class Sim:
    """One simulation, or a batch of independent replicas (cfg a list of
    configurations), bound to the current torch stream of `device`.  For a
    batch every state tensor is the replicas' (N_q, 2) blocks concatenated in
    replica order."""

    def __init__(self, cfg: Union[Mapping, Sequence[Mapping]], device="cuda"):
        self.batch = not isinstance(cfg, Mapping)
        cfgs = [dict(cfg)] if not self.batch else [dict(c) for c in cfg]
        self.cfgs = cfgs
        self.cfg = cfgs[0]
        self.R = len(cfgs)
        self.device = torch.device(device)
        self._params = _param_array(cfgs)
        self.params = self._params[0]
        self.sizes = [2 * int(c["n_agents"]) for c in cfgs]
        self.N = sum(self.sizes)
        nbytes = workspace_bytes(cfgs)
        # the allocator returns 512-byte aligned blocks; keep 256 spare anyway
        self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws_raw.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self._stream = _stream_handle(self.device)
        h = ctypes.c_void_p()
        _check(lib().dpd_create_batch(self._params, self.R, ctypes.c_void_p(self._ws_ptr),
                                      ctypes.c_size_t(nbytes), self._stream, ctypes.byref(h)))
        self._h = h
        ncs = [cells_per_side(c) for c in cfgs]
        self.n_c = ncs if self.batch else ncs[0]
        self.n_cells = sum(n * n for n in ncs)

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            lib().dpd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, rc):
        _check(rc, self._h)

    # -- state
    def set_state(self, x: torch.Tensor, v: torch.Tensor, step: int = 0,
                  F: Optional[torch.Tensor] = None):
        _vec(x, self.N, "x")
        _vec(v, self.N, "v")
        if F is not None:
            _vec(F, self.N, "F")
        self._c(lib().dpd_set_state(self._h, _ptr(x), _ptr(v), int(step), _ptr(F)))

    def get_state(self):
        x = torch.empty((self.N, 2), dtype=torch.float32, device=self.device)
        v = torch.empty_like(x)
        F = torch.empty_like(x)
        s = ctypes.c_int64(0)
        self._c(lib().dpd_get_state(self._h, _ptr(x), _ptr(v), _ptr(F), ctypes.byref(s)))
        return x, v, F, int(s.value)

    def forces(self) -> torch.Tensor:
        F = torch.empty((self.N, 2), dtype=torch.float32, device=self.device)
        self._c(lib().dpd_forces(self._h, _ptr(F)))
        return F

    def step(self, n: int, reduce_every: int = 0, pk: Optional[torch.Tensor] = None):
        """Advance n steps.  With reduce_every > 0 returns a (n // reduce_every, 3)
        float64 device tensor of (P_x, P_y, KE) records ((n // reduce_every, R, 3)
        for a batch)."""
        if reduce_every > 0 and pk is None:
            nrec = n // reduce_every
            shape = (max(nrec, 1), self.R, 3) if self.batch else (max(nrec, 1), 3)
            pk = torch.zeros(shape, dtype=torch.float64, device=self.device)
        self._c(lib().dpd_step(self._h, int(n), int(reduce_every), _ptr(pk)))
        if reduce_every > 0:
            return pk[: n // reduce_every]
        return None

    def sync(self):
        self._c(lib().dpd_sync(self._h))

    def bin_velocity(self, M: int, eps: float = 0.0, mode: int = 0, out=None):
        """Mean velocity (M, M, 2) [row j, column i] and counts (M, M) per grid
        window ((R, M, M, 2) and (R, M, M) for a batch); asynchronous on the
        stream (reading the tensors waits for it)."""
        if out is None:
            lead = (self.R,) if self.batch else ()
            u = torch.empty(lead + (M, M, 2), dtype=torch.float32, device=self.device)
            n = torch.empty(lead + (M, M), dtype=torch.int32, device=self.device)
        else:
            u, n = out
        self._c(lib().dpd_bin_velocity(self._h, int(M), float(eps), int(mode), _ptr(u), _ptr(n)))
        return u, n

    def bin_velocity_reps(self, M: int, eps, mode: int = 0, out=None):
        """bin_velocity with window width eps[r] for replica r of a batch."""
        if out is None:
            lead = (self.R,) if self.batch else ()
            u = torch.empty(lead + (M, M, 2), dtype=torch.float32, device=self.device)
            n = torch.empty(lead + (M, M), dtype=torch.int32, device=self.device)
        else:
            u, n = out
        e = (ctypes.c_double * self.R)(*[float(x) for x in eps])
        self._c(lib().dpd_bin_velocity_reps(self._h, int(M), e, int(mode), _ptr(u), _ptr(n)))
        return u, n

    def cells(self):
        cs = torch.empty(self.n_cells + 1, dtype=torch.int32, device=self.device)
        ids = torch.empty(self.N, dtype=torch.int32, device=self.device)
        self._c(lib().dpd_get_cells(self._h, _ptr(cs), _ptr(ids)))
        return cs, ids

    # -- profiling
    def set_profiling(self, on: bool):
        self._c(lib().dpd_set_profiling(self._h, 1 if on else 0))

    def pair_kernel_time(self):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        self._c(lib().dpd_pair_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def rebuilds(self) -> int:
        """Steps that rebuilt the cell list under a Verlet skin (0 without one)."""
        n = ctypes.c_int64(0)
        self._c(lib().dpd_cell_list_rebuilds(self._h, ctypes.byref(n)))
        return int(n.value)

    # -- captured chunks and schedules
    def set_graph_chunk(self, steps: int):
        """Replay dpd_step in captured chunks of `steps` launches (0: off)."""
        self._c(lib().dpd_set_graph_chunk(self._h, int(steps)))

    def set_schedule(self, tile_x: int, tile_y: int, tile_order: int = 0):
        self._c(lib().dpd_set_schedule(self._h, int(tile_x), int(tile_y), int(tile_order)))

    def schedule(self):
        tx, ty, o = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        self._c(lib().dpd_get_schedule(self._h, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(o)))
        return int(tx.value), int(ty.value), int(o.value)

    def autotune(self, trial_steps: int = 20):
        """Time the candidate schedules on the current state, keep the fastest
        (the state is left as it was).  Returns (tile_x, tile_y, order, ms/step)."""
        tx, ty, o = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        ms = ctypes.c_double(0.0)
        self._c(lib().dpd_autotune(self._h, int(trial_steps), ctypes.byref(tx), ctypes.byref(ty),
                                   ctypes.byref(o), ctypes.byref(ms)))
        return int(tx.value), int(ty.value), int(o.value), float(ms.value)


def rng_words(cfg: Mapping, i: torch.Tensor, j: torch.Tensor, step: int):
    """Generator words (n, 4) as int32 (bit pattern of uint32) and alpha (n,)."""
    n = i.numel()
    ii = i.int().contiguous()
    jj = j.int().contiguous()
    words = torch.empty((n, 4), dtype=torch.int32, device=i.device)
    alpha = torch.empty(n, dtype=torch.float32, device=i.device)
    _check(lib().dpd_rng_words(ctypes.byref(make_params(cfg)), _ptr(ii), _ptr(jj), int(step),
                               int(n), _ptr(words), _ptr(alpha), _stream_handle(i.device)))
    return words, alpha


def copy_kernel(src: torch.Tensor, dst: torch.Tensor):
    nbytes = src.numel() * src.element_size()
    _check(lib().dpd_copy_kernel(_ptr(src), _ptr(dst), ctypes.c_size_t(nbytes),
                                 _stream_handle(src.device)))


def forces_noalloc(cfg: Mapping, x: torch.Tensor, v: torch.Tensor, step: int = 0,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """F(x, v, step) of one system through dpd_forces_noalloc (the library's
    static device scratch, no workspace); out may be given to avoid any
    allocation here too."""
    n = 2 * int(cfg["n_agents"])
    _vec(x, n, "x")
    _vec(v, n, "v")
    F = torch.empty((n, 2), dtype=torch.float32, device=x.device) if out is None else _vec(out, n, "out")
    _check(lib().dpd_forces_noalloc(ctypes.byref(make_params(cfg)), _ptr(x), _ptr(v), int(step),
                                    _ptr(F), _stream_handle(x.device)))
    return F
