"""Pins of the spectral and correlation statistics (Sec. 5.3-5.4, Eqs. 5.5-5.13)
against closed forms and brute force.  CPU only."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import analysis


def _grid(M, L):
    dx = L / M
    c = (np.arange(M) + 0.5) * dx
    Y, X = np.meshgrid(c, c, indexing="ij")
    return X, Y


def test_parseval():
    rng = np.random.default_rng(1)
    u = rng.normal(0, 1, (32, 32, 2))
    uh = analysis.fourier_coefficients(u)
    lhs = 0.5 * (np.abs(uh) ** 2).sum()
    rhs = 0.5 * (u * u).sum(axis=2).mean()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_single_mode_energy():
    # u = U sin(2 pi m y / L) e_x  ->  E(m) = U^2 / 4, zero elsewhere
    M, L, U, m = 64, 100.0, 1.7, 5
    X, Y = _grid(M, L)
    u = np.zeros((M, M, 2))
    u[..., 0] = U * np.sin(2 * math.pi * m * Y / L)
    E = analysis.energy_spectrum(u)
    assert E[m - 1] == pytest.approx(U * U / 4, rel=1e-12)
    E[m - 1] = 0
    assert np.abs(E).max() < 1e-20


def test_fft_matches_direct_dft():
    M = 8
    rng = np.random.default_rng(2)
    u = rng.normal(0, 1, (M, M, 2))
    uh = analysis.fourier_coefficients(u)
    j = np.arange(M)
    for (ky, kx) in [(0, 0), (1, 3), (7, 2), (4, 4)]:
        ph = np.exp(-2j * math.pi * (ky * j[:, None] + kx * j[None, :]) / M)
        direct = (u * ph[..., None]).sum((0, 1)) / M ** 2
        assert np.abs(uh[ky, kx] - direct).max() < 1e-12


def test_slope_fit_recovers_power_law():
    k = np.arange(1, 33, dtype=np.float64)
    E = 3.5 * k ** 0.8
    alpha, C = analysis.slope_fit(E)
    assert alpha == pytest.approx(0.8, abs=1e-12)
    assert C == pytest.approx(1.0, rel=1e-12)
    E = 2.0 * k ** -0.5
    assert analysis.slope_fit(E)[0] == pytest.approx(-0.5, abs=1e-12)


def test_grid_autocorrelation_fft_equals_bruteforce():
    rng = np.random.default_rng(3)
    u = rng.normal(0, 1, (12, 12, 2))
    a = analysis.grid_autocorrelation(u)
    b = analysis.grid_autocorrelation_bruteforce(u)
    assert np.abs(a - b).max() < 1e-12


def test_vcf_single_mode_is_bessel_j0():
    # an isotropic mixture is not needed: the angular average of cos(k . r)
    # over directions is J0(|k| r); a plane wave along x with its rotated copy
    # along y reproduces it up to the anisotropy of a two-direction average,
    # so use many directions on a fine grid.
    M, L = 256, 100.0
    X, Y = _grid(M, L)
    u = np.zeros((M, M, 2))
    m = 3
    k = 2 * math.pi * m / L
    u[..., 0] = np.cos(k * X)
    u[..., 1] = np.cos(k * Y)
    r, g = analysis.vcf_grid(u, L, dr=L / M)
    # two directions: g(r) = <cos(k r cos th) + cos(k r sin th)>_th / 2 = J0(k r)
    sel = (r > 0) & (r < 0.25 * L)
    assert np.nanmax(np.abs(g[sel] - special.j0(k * r[sel]))) < 0.05


def test_vcf_iid_velocities_uncorrelated_and_bruteforce_agrees():
    rng = np.random.default_rng(4)
    L = 30.0
    n = 900
    pos = rng.uniform(0, L, (n, 2))
    V = rng.normal(0, 1, (n, 2))
    r, g, cnt = analysis.vcf_bruteforce(pos, V, L, dr=1.0)
    assert g[0] == 1.0
    assert np.abs(g[1:][cnt[1:] > 200]).max() < 0.2
    # a velocity that is a smooth function of position is correlated at short range
    V2 = np.stack([np.sin(2 * math.pi * pos[:, 0] / L), np.cos(2 * math.pi * pos[:, 1] / L)], 1)
    r, g, cnt = analysis.vcf_bruteforce(pos, V2, L, dr=1.0)
    assert g[1] > 0.9


def test_integral_length_closed_form():
    # g(r) = exp(-r / a) integrates to a (for L/2 >> a)
    a = 2.0
    r = np.linspace(0, 50, 5001)
    g = np.exp(-r / a)
    assert analysis.integral_length(r, g, L=100.0) == pytest.approx(a, rel=1e-4)
    g = np.cos(math.pi * r / 10.0)   # first zero at r = 5: integral 10/pi
    assert analysis.integral_length(r, g, L=100.0, to_first_zero=True) == pytest.approx(10 / math.pi, rel=1e-3)


def test_agent_com_minimum_image():
    L = 10.0
    x = np.array([[9.9, 5.0], [0.3, 5.0]])
    v = np.array([[1.0, 0.0], [3.0, 0.0]])
    com, V = analysis.agent_com(x, v, L)
    assert com[0] == pytest.approx([0.1, 5.0])
    assert V[0] == pytest.approx([2.0, 0.0])


def test_stats_protocol_helpers_match_oracle_routines():
    # the statistics protocol's vectorised correlation function and batched
    # band energies are the oracle's pair loop and per-field spectrum
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    from stats_protocol import PROTOCOL, band_energies, band_energies_batch, vcf_pairs
    rng = np.random.default_rng(21)
    L = 40.0
    pos = rng.uniform(0.0, L, (300, 2))
    V = rng.normal(size=(300, 2)) + 0.2
    a = analysis.vcf_bruteforce(pos, V, L, 0.25)
    b = vcf_pairs(pos, V, L, 0.25)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
    assert np.allclose(a[1], b[1], rtol=1e-12, atol=1e-14, equal_nan=True)
    u = rng.normal(size=(3, PROTOCOL["M"], PROTOCOL["M"], 2))
    got = band_energies_batch(u)
    for f in range(3):
        assert np.allclose(got[f], band_energies(analysis.energy_spectrum(u[f])), rtol=1e-13)


def test_transient_window_accumulator():
    # the 4M protocol's windows: snapshots of window w scaled by (w + 1) give
    # (w + 1)^2 times one snapshot's band energies in that window and the same
    # correlation length (the normalised correlation is scale-free); the
    # ensemble's standard error is the spread over seeds / sqrt(seeds)
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    from stats_protocol import PROTOCOL_4M, WindowAccumulator, band_energies_of, window_ensemble
    rng = np.random.default_rng(22)
    M, L = 32, 250.0
    u = rng.normal(size=(M, M, 2)) + 0.1
    acc = WindowAccumulator(L)
    k = PROTOCOL_4M["window"] // PROTOCOL_4M["every"]
    nw = PROTOCOL_4M["steps"] // PROTOCOL_4M["window"]
    for n in range(k * nw):
        acc.add((n // k + 1) * u)
    res = acc.result()
    E1 = band_energies_of(analysis.energy_spectrum(u), PROTOCOL_4M["bands"])
    r, g = analysis.vcf_grid(u, L, L / PROTOCOL_4M["M"])
    L1 = analysis.integral_length(r, g, L)
    for w in range(nw):
        assert np.allclose(res["E_bands"][w], (w + 1) ** 2 * E1, rtol=1e-12)
        assert res["L_gv"][w] == pytest.approx(L1, rel=1e-12)
    e = window_ensemble([res, dict(res, E_bands=(2 * np.array(res["E_bands"])).tolist())])
    assert np.allclose(e["E_bands"], 1.5 * np.array(res["E_bands"]))
    assert np.allclose(e["E_bands_sem"], np.abs(np.array(res["E_bands"])) * np.sqrt(0.5) / np.sqrt(2))
