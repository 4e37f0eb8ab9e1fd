"""Statistics of binned velocity fields (Sec. 5.3-5.4): the power spectrum of
a set of fields on the GPU (dpd_field_power), and from it the energy spectrum
E(k) in unit shells (Eq. 5.12) and the velocity correlation function of the
gridded field with its integral length (the spectrum's inverse transform, by
Wiener-Khinchin).  The shell sums and the radial binning are host
post-processing of the M x M spectrum."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import dpd

_bound = False


def _lib():
    global _bound
    L = dpd.lib()
    if not _bound:
        vp = ctypes.c_void_p
        fn = L.dpd_field_power
        fn.restype = ctypes.c_int
        fn.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        fe = L.dpd_nn_last_error
        fe.restype = ctypes.c_char_p
        fe.argtypes = [vp]
        _bound = True
    return L


def power(fields: torch.Tensor) -> np.ndarray:
    """Sum over the fields [nf][M][M][2] (CUDA FP32) of |u^(l, k)|^2 for both
    components, u^ = DFT(u) / M^2; an (M, M) FP64 array indexed [l][k]."""
    if not (fields.is_cuda and fields.dtype == torch.float32 and fields.is_contiguous()
            and fields.dim() == 4 and fields.shape[1] == fields.shape[2] and fields.shape[3] == 2):
        raise ValueError("fields must be a contiguous CUDA float32 tensor [nf][M][M][2]")
    nf, M = int(fields.shape[0]), int(fields.shape[1])
    work = torch.empty(4 * nf * M * M, dtype=torch.float32, device=fields.device)
    P = torch.empty((M, M), dtype=torch.float64, device=fields.device)
    rc = _lib().dpd_field_power(ctypes.c_void_p(fields.data_ptr()), nf, M,
                                ctypes.c_void_p(work.data_ptr()), ctypes.c_void_p(P.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream(fields.device).cuda_stream))
    if rc != 0:
        raise dpd.DPDError(rc, _lib().dpd_nn_last_error(None).decode())
    return P.cpu().numpy()


def _kmag(M: int) -> np.ndarray:
    k = np.fft.fftfreq(M) * M
    ky, kx = np.meshgrid(k, k, indexing="ij")
    return np.sqrt(kx * kx + ky * ky)


def shells(P: np.ndarray, nf: int = 1) -> np.ndarray:
    """E(s) for s = 1..M/2, s - 1/2 <= |k| < s + 1/2, as the mean over nf
    fields of the sum of |u^|^2 / 2 (index 0 is shell 1)."""
    M = P.shape[0]
    s = np.floor(_kmag(M) + 0.5).astype(np.int64)
    E = np.zeros(M // 2)
    for k in range(1, M // 2 + 1):
        E[k - 1] = 0.5 * P[s == k].sum() / nf
    return E


def bands(E: np.ndarray):
    """Mean of E over the log-spaced shell bands 1, 2-3, 4-7, ... (up to M/2)."""
    out, lo = [], 1
    while lo <= len(E):
        hi = min(2 * lo - 1, len(E))
        out.append(float(E[lo - 1:hi].mean()))
        lo *= 2
    return np.array(out)


def correlation(P: np.ndarray, L: float, dr: float):
    """Velocity correlation g(r) of the gridded fields: the normalised circular
    autocorrelation without the mean (the k = 0 term), angularly averaged in
    bins of width dr out to L/2, g(0) = 1.  Returns (r, g)."""
    M = P.shape[0]
    Q = np.array(P, dtype=np.float64)
    Q[0, 0] = 0.0
    C = np.real(np.fft.ifft2(Q)) * M * M  # sum_k Q e^{i k r}
    dx = L / M
    off = np.fft.fftfreq(M) * M * dx
    oy, ox = np.meshgrid(off, off, indexing="ij")
    r = np.sqrt(ox * ox + oy * oy)
    nb = int(np.floor(0.5 * L / dr))
    b = np.floor(r / dr).astype(np.int64)
    g = np.full(nb, np.nan)
    for k in range(nb):
        m = (b == k) & (r > 0)
        if m.any():
            g[k] = C[m].mean() / C[0, 0]
    rc = (np.arange(nb) + 0.5) * dr
    return np.concatenate([[0.0], rc]), np.concatenate([[1.0], g])


def integral_length(r, g, L: float, to_first_zero: bool = True) -> float:
    """Trapezoid integral of g over [0, L/2], or up to its first zero crossing
    (linearly interpolated)."""
    r = np.asarray(r, np.float64)
    g = np.asarray(g, np.float64)
    ok = np.isfinite(g) & (r <= 0.5 * L)
    r, g = r[ok], g[ok]
    if to_first_zero:
        neg = np.nonzero(g <= 0)[0]
        if len(neg):
            i = int(neg[0])
            r0 = r[i - 1] + (r[i] - r[i - 1]) * g[i - 1] / (g[i - 1] - g[i])
            r = np.concatenate([r[:i], [r0]])
            g = np.concatenate([g[:i], [0.0]])
    return float(np.trapezoid(g, r))


def band_index(M: int) -> np.ndarray:
    """Band of every Fourier mode (l, k): 0 for shell 1, 1 for shells 2-3, 2 for
    4-7, ... (the bands of `bands`), -1 for k = 0 and shells beyond M/2."""
    s = np.floor(_kmag(M) + 0.5).astype(np.int64)
    b = np.full(s.shape, -1, np.int64)
    ok = (s >= 1) & (s <= M // 2)
    b[ok] = np.floor(np.log2(s[ok])).astype(np.int64)
    return b


def band_autocorrelation(fields: torch.Tensor, lags) -> np.ndarray:
    """Temporal autocorrelation of the Fourier modes of trajectories
    fields [T][B][M][M][2] (CUDA FP32), per shell band and lag tau (in field
    steps): C_b(tau) = sum Re(u^_t conj u^_{t+tau}) / sum (|u^_t|^2 + |u^_{t+tau}|^2) / 2
    over the modes of band b, both components, t and the B trajectories.
    The cross term comes from the power spectra of u_t + u_{t+tau} and
    u_t - u_{t+tau} (polarisation: 4 Re(a conj b) = |a + b|^2 - |a - b|^2),
    so only the GPU power kernel is used.  Returns [n_bands][len(lags)]."""
    T, B, M = int(fields.shape[0]), int(fields.shape[1]), int(fields.shape[2])
    bi = band_index(M)
    nb = int(bi.max()) + 1
    out = np.zeros((nb, len(lags)))
    for j, tau in enumerate(lags):
        num = np.zeros(nb)
        den = np.zeros(nb)
        for q in range(B):
            a = fields[:T - tau, q]
            b = fields[tau:, q]
            Pp = power((a + b).contiguous())
            Pm = power((a - b).contiguous())
            num += np.bincount(bi[bi >= 0], (Pp - Pm)[bi >= 0], nb)
            den += np.bincount(bi[bi >= 0], (Pp + Pm)[bi >= 0], nb)
        out[:, j] = num / np.maximum(den, 1e-300)
    return out


VCF_SCALE = 2.0 ** 20  # fixed-point scale of the pair sums of dpd_agent_vcf


def agent_vcf(x: torch.Tensor, v: torch.Tensor, L: float, dr: float):
    """Velocity correlation function of the agents (Sec. 5.3, Eqs. 5.5-5.6)
    from the state x, v (CUDA FP32 (N, 2), id order): pair sums by separation
    on the GPU (dpd_agent_vcf) in bins of width dr out to L/2, normalised with
    the mean and mean square of the agent velocities.  Returns
    (r_centres, g, counts) with g(0) := 1 and count 0 prepended at r = 0."""
    n = int(x.shape[0]) // 2
    nb = int(np.floor(0.5 * L / dr))
    dev = x.device
    work = torch.empty(4 * n + 1, dtype=torch.float64, device=dev)
    sums = torch.empty(nb, dtype=torch.int64, device=dev)
    counts = torch.empty(nb, dtype=torch.int64, device=dev)
    vp = ctypes.c_void_p
    rc = dpd.lib().dpd_agent_vcf(vp(x.data_ptr()), vp(v.data_ptr()), n, float(L), float(dr), nb,
                                 vp(work.data_ptr()), vp(sums.data_ptr()), vp(counts.data_ptr()),
                                 vp(torch.cuda.current_stream(dev).cuda_stream))
    if rc != 0:
        raise dpd.DPDError(rc, dpd.lib().dpd_last_error(None).decode())
    V = work[2 * n:4 * n].view(n, 2).cpu().numpy()
    mean = V.mean(axis=0)
    mean2 = float(mean @ mean)
    var = float((V * V).sum(axis=1).mean()) - mean2
    S = sums.cpu().numpy().astype(np.float64) / VCF_SCALE
    c = counts.cpu().numpy()
    with np.errstate(invalid="ignore", divide="ignore"):
        g = (S / c - mean2) / var
    rc_ = (np.arange(nb) + 0.5) * dr
    return np.concatenate([[0.0], rc_]), np.concatenate([[1.0], g]), np.concatenate([[0], c])
