"""Python binding of the learned closure (C ABI in include/closure.h, built into
libdpd.so).  Argument marshalling only: the network's forward pass, gradients,
optimiser and rollout run in the library's kernels; PyTorch provides the
device memory and the stream."""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import dpd

_bound = False


class NNParams(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32),
        ("c_in", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("layers", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


def lib():
    global _bound
    L = dpd.lib()
    if not _bound:
        vp, P = ctypes.c_void_p, ctypes.POINTER(NNParams)
        i32, f32, f64 = ctypes.c_int32, ctypes.c_float, ctypes.c_double
        sig = {
            "dpd_nn_param_count": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64)]),
            "dpd_nn_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
            "dpd_nn_create": (ctypes.c_int, [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
            "dpd_nn_destroy": (None, [vp]),
            "dpd_nn_last_error": (ctypes.c_char_p, [vp]),
            "dpd_nn_set_weights": (ctypes.c_int, [vp, vp]),
            "dpd_nn_get_weights": (ctypes.c_int, [vp, vp]),
            "dpd_nn_forward": (ctypes.c_int, [vp, vp, vp, i32, vp]),
            "dpd_nn_gradient": (ctypes.c_int, [vp, vp, vp, vp, i32, vp, vp]),
            "dpd_nn_adam": (ctypes.c_int, [vp, vp, f32, f32, f32, f32]),
            "dpd_nn_train_step": (ctypes.c_int, [vp, vp, vp, vp, i32, f32, f32, f32, f32, vp]),
            "dpd_nn_rollout": (ctypes.c_int, [vp, vp, vp, i32, i32, ctypes.POINTER(f32), vp,
                                              ctypes.c_uint64, i32, vp]),
            "dpd_nn_sync": (ctypes.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _check(rc, h=None):
    if rc != 0:
        raise dpd.DPDError(rc, lib().dpd_nn_last_error(h).decode())


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _f32(t: torch.Tensor, shape, name):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape {tuple(shape)}")
    return t


def make_params(M: int, c_in: int = 4, width: int = 32, layers: int = 4, max_batch: int = 32):
    p = NNParams()
    p.M, p.c_in, p.width, p.layers, p.max_batch = M, c_in, width, layers, max_batch
    return p


def param_count(M: int, c_in: int = 4, width: int = 32, layers: int = 4) -> int:
    n = ctypes.c_int64(0)
    _check(lib().dpd_nn_param_count(ctypes.byref(make_params(M, c_in, width, layers, 1)), ctypes.byref(n)))
    return int(n.value)


class Closure:
    """The closure network bound to the current torch stream of `device`."""

    def __init__(self, M: int, c_in: int = 4, width: int = 32, layers: int = 4,
                 max_batch: int = 32, device="cuda"):
        self.M, self.c_in, self.width, self.layers, self.max_batch = M, c_in, width, layers, max_batch
        self.device = torch.device(device)
        self.params = make_params(M, c_in, width, layers, max_batch)
        n = ctypes.c_size_t(0)
        _check(lib().dpd_nn_workspace_bytes(ctypes.byref(self.params), ctypes.byref(n)))
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        _check(lib().dpd_nn_create(ctypes.byref(self.params), ctypes.c_void_p(ptr),
                                   ctypes.c_size_t(n.value),
                                   ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream),
                                   ctypes.byref(h)))
        self._h = h
        self.n_params = param_count(M, c_in, width, layers)
        self._loss = torch.zeros(1, dtype=torch.float64, device=self.device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            lib().dpd_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, rc):
        _check(rc, self._h)

    def set_weights(self, w: torch.Tensor):
        self._c(lib().dpd_nn_set_weights(self._h, _p(_f32(w, (self.n_params,), "w"))))

    def get_weights(self) -> torch.Tensor:
        w = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        self._c(lib().dpd_nn_get_weights(self._h, _p(w)))
        return w

    def _io(self, u, cond):
        B = u.shape[0]
        _f32(u, (B, self.M, self.M, 2), "u")
        _f32(cond, (B, self.c_in - 2), "cond")
        return B

    def forward(self, u: torch.Tensor, cond: torch.Tensor) -> torch.Tensor:
        B = self._io(u, cond)
        pred = torch.empty_like(u)
        self._c(lib().dpd_nn_forward(self._h, _p(u), _p(cond), B, _p(pred)))
        return pred

    def gradient(self, u, cond, target):
        B = self._io(u, cond)
        _f32(target, u.shape, "target")
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        self._c(lib().dpd_nn_gradient(self._h, _p(u), _p(cond), _p(target), B, _p(g), _p(self._loss)))
        return float(self._loss.item()), g

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._c(lib().dpd_nn_adam(self._h, _p(_f32(grad, (self.n_params,), "grad")), lr, beta1, beta2, eps))

    def train_step(self, u, cond, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   loss_out: Optional[torch.Tensor] = None):
        """One Adam step on the batch; the loss goes to loss_out (device float64,
        one value) if given, else to an internal tensor (read with last_loss)."""
        B = self._io(u, cond)
        out = self._loss if loss_out is None else loss_out
        self._c(lib().dpd_nn_train_step(self._h, _p(u), _p(cond), _p(target), B, lr, beta1, beta2,
                                        eps, _p(out)))

    def last_loss(self) -> float:
        return float(self._loss.item())

    def rollout(self, u0: torch.Tensor, cond: torch.Tensor, steps: int, noise_std=(0.0, 0.0),
                seed: int = 0, save_every: int = 1,
                noise_filter: Optional[torch.Tensor] = None) -> torch.Tensor:
        """steps applications of the network with noise after each: white
        noise_std[c] w, or noise_std[c] (h * w) with the periodic filter h
        ([M][M]) if given.  u0 is one field [M][M][2] with cond [c_in - 2]
        (returns [steps // save_every][M][M][2]) or a batch [B][M][M][2] with
        cond [B][c_in - 2] (returns [steps // save_every][B][M][M][2])."""
        single = u0.dim() == 3
        B = 1 if single else int(u0.shape[0])
        _f32(u0, ((self.M, self.M, 2) if single else (B, self.M, self.M, 2)), "u0")
        _f32(cond, ((self.c_in - 2,) if single else (B, self.c_in - 2)), "cond")
        if noise_filter is not None:
            _f32(noise_filter, (self.M, self.M), "noise_filter")
        nsave = steps // save_every
        traj = torch.empty((max(nsave, 1), B, self.M, self.M, 2), dtype=torch.float32, device=self.device)
        sd = (ctypes.c_float * 2)(float(noise_std[0]), float(noise_std[1]))
        self._c(lib().dpd_nn_rollout(self._h, _p(u0), _p(cond), B, int(steps), sd, _p(noise_filter),
                                     int(seed), int(save_every), _p(traj)))
        return traj[:nsave, 0] if single else traj[:nsave]

    def sync(self):
        self._c(lib().dpd_nn_sync(self._h))
