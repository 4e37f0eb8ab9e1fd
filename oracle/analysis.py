"""Statistics of the filtered velocity field and of agent velocities
(Sec. 5.3 and Sec. 5.4 of the paper), written as plain numpy definitions.

TEST INFRASTRUCTURE ONLY (the reference for long-run statistics); the engine's hot
path ends at the binned field u_M.

Readings where the paper is silent or garbled:
  - Fourier coefficients u_hat = FFT2(u_M) / M^2, integer wavenumber index k;
    shell s collects s - 1/2 <= |k| < s + 1/2 for s = 1..M/2; the k = 0 mode and
    the corners |k| >= M/2 + 1/2 are dropped (Eqs. 5.11-5.12);
  - the low-k slope is the ordinary least-squares fit of ln(E/E_1) on ln k over
    the first ten shells (Eq. 5.13 and the fit range stated in Sec. 5.4);
  - the velocity correlation function uses agent centre-of-mass velocities at
    minimum-image midpoints, global means in the normalisation, and g(0) = 1
    (Eqs. 5.5-5.6);
  - the integral length scale integrates g from 0 to L/2 (trapezoid rule)
    because the box is periodic (Eq. 5.7).
"""
from __future__ import annotations

import numpy as np


def fourier_coefficients(u: np.ndarray) -> np.ndarray:
    """u: (M, M, 2) grid field [row j (y), column i (x), component].
    Returns u_hat (M, M, 2) with u = sum_k u_hat exp(i k . x)."""
    M = u.shape[0]
    return np.fft.fft2(u, axes=(0, 1)) / float(M * M)


def wavenumber_magnitude(M: int) -> np.ndarray:
    k = np.fft.fftfreq(M) * M
    ky, kx = np.meshgrid(k, k, indexing="ij")
    return np.sqrt(kx * kx + ky * ky)


def energy_spectrum(u: np.ndarray) -> np.ndarray:
    """E(s) for shells s = 1..M/2 (index 0 of the result is shell 1)."""
    M = u.shape[0]
    uh = fourier_coefficients(u)
    e = 0.5 * (np.abs(uh[..., 0]) ** 2 + np.abs(uh[..., 1]) ** 2)
    kmag = wavenumber_magnitude(M)
    shell = np.floor(kmag + 0.5).astype(np.int64)
    E = np.zeros(M // 2)
    for s in range(1, M // 2 + 1):
        E[s - 1] = e[shell == s].sum()
    return E


def slope_fit(E: np.ndarray, n_shells: int = 10):
    """Least-squares fit ln(E/E_1) = ln C + alpha ln k over k = 1..n_shells.
    Returns (alpha, C)."""
    k = np.arange(1, n_shells + 1, dtype=np.float64)
    y = np.log(E[:n_shells] / E[0])
    X = np.stack([np.ones_like(k), np.log(k)], axis=1)
    coef, *_ = np.linalg.lstsq(X, y, rcond=None)
    return float(coef[1]), float(np.exp(coef[0]))


def agent_com(x: np.ndarray, v: np.ndarray, L: float):
    """Agent centre-of-mass positions (minimum-image midpoint, wrapped) and
    velocities V_k = (v_2k + v_2k+1)/2."""
    x = np.asarray(x, np.float64)
    v = np.asarray(v, np.float64)
    h, t = x[0::2], x[1::2]
    d = h - t
    d -= L * np.round(d / L)
    com = np.mod(t + 0.5 * d, L)
    V = 0.5 * (v[0::2] + v[1::2])
    return com, V


def vcf_bruteforce(pos: np.ndarray, V: np.ndarray, L: float, dr: float):
    """g(r) over all pairs k != l, binned by minimum-image separation in bins of
    width dr out to L/2.  Returns (r_centres, g, counts) with g(0) := 1
    prepended at r = 0."""
    pos = np.asarray(pos, np.float64)
    V = np.asarray(V, np.float64)
    n = len(pos)
    mean = V.mean(axis=0)
    mean2 = float(mean @ mean)
    var = float((V * V).sum(axis=1).mean()) - mean2
    nb = int(np.floor(0.5 * L / dr))
    num = np.zeros(nb)
    cnt = np.zeros(nb, np.int64)
    for k in range(n - 1):
        d = pos[k + 1:] - pos[k]
        d -= L * np.round(d / L)
        r = np.sqrt((d * d).sum(axis=1))
        b = np.floor(r / dr).astype(np.int64)
        ok = b < nb
        dots = V[k + 1:] @ V[k]
        np.add.at(num, b[ok], dots[ok])
        np.add.at(cnt, b[ok], 1)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = (num / cnt - mean2) / var
    rc = (np.arange(nb) + 0.5) * dr
    return np.concatenate([[0.0], rc]), np.concatenate([[1.0], g]), np.concatenate([[0], cnt])


def grid_autocorrelation(u: np.ndarray) -> np.ndarray:
    """C(r) = mean over grid points x of u(x) . u(x + r) for every grid offset
    r, by the Wiener-Khinchin theorem.  Returns (M, M)."""
    M = u.shape[0]
    fh = np.fft.fft2(u, axes=(0, 1))
    p = (np.abs(fh) ** 2).sum(axis=2)
    return np.real(np.fft.ifft2(p)) / float(M * M)


def grid_autocorrelation_bruteforce(u: np.ndarray) -> np.ndarray:
    M = u.shape[0]
    C = np.zeros((M, M))
    for sy in range(M):
        for sx in range(M):
            sh = np.roll(np.roll(u, -sy, axis=0), -sx, axis=1)
            C[sy, sx] = (u * sh).sum(axis=2).mean()
    return C


def vcf_grid(u: np.ndarray, L: float, dr: float):
    """Angular average of the normalised grid autocorrelation; bins of width
    dr out to L/2, g(0) = 1.  Returns (r_centres, g)."""
    M = u.shape[0]
    dx = L / M
    mean = u.reshape(-1, 2).mean(axis=0)
    mean2 = float(mean @ mean)
    C = grid_autocorrelation(u)
    var = C[0, 0] - mean2
    off = np.fft.fftfreq(M) * M * dx
    oy, ox = np.meshgrid(off, off, indexing="ij")
    r = np.sqrt(ox * ox + oy * oy)
    nb = int(np.floor(0.5 * L / dr))
    b = np.floor(r / dr).astype(np.int64)
    g = np.full(nb, np.nan)
    for k in range(nb):
        m = (b == k) & (r > 0)
        if m.any():
            g[k] = (C[m].mean() - mean2) / var
    rc = (np.arange(nb) + 0.5) * dr
    return np.concatenate([[0.0], rc]), np.concatenate([[1.0], g])


def integral_length(r: np.ndarray, g: np.ndarray, L: float, to_first_zero: bool = False) -> float:
    """Trapezoid integral of g from 0 to L/2 (or to its first zero crossing)."""
    r = np.asarray(r, np.float64)
    g = np.asarray(g, np.float64)
    ok = np.isfinite(g) & (r <= 0.5 * L)
    r, g = r[ok], g[ok]
    if to_first_zero:
        neg = np.nonzero(g <= 0)[0]
        if len(neg):
            k = neg[0]
            r0 = r[k - 1] + (r[k] - r[k - 1]) * g[k - 1] / (g[k - 1] - g[k])
            r = np.concatenate([r[:k], [r0]])
            g = np.concatenate([g[:k], [0.0]])
    return float(np.trapezoid(g, r)) if hasattr(np, "trapezoid") else float(np.trapz(g, r))
