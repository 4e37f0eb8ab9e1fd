"""Pins of the oracle's time stepping (velocity-Verlet, Sec. 5) against closed
forms and invariants.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

from paper_1310_0998_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C1 = inputs.physics(inputs.WORKLOADS["dimers_1600"])


def _init(oracle_mod, cfg, x, v, step=0):
    F = oracle_mod.forces(cfg, x, v, step)
    return np.asarray(x, np.float64), np.asarray(v, np.float64), F


def test_momentum_conserved_without_propulsion_and_friction(oracle_mod):
    cfg = dict(C1, f_sp=0.0, gamma_s=0.0)
    x, v = inputs.initial_state(cfg, thermal=True)
    x, v, F = _init(oracle_mod, cfg, x, v)
    P0 = oracle_mod.momentum_ke(cfg, v)
    _, vn, _, _, pk = oracle_mod.step(cfg, x, v, F, 0, 1000, every=50)
    scale = np.abs(v).sum()
    assert np.abs(pk[:, :2] - P0[:2]).max() <= 1e-12 * scale


def test_momentum_decay_with_stokes_friction(oracle_mod):
    # f_sp = 0: pair and bond forces cancel in the sum, so
    # P_n = P_0 (1 - c)^2 (1 - 2c)^(n-1) with c = gamma_s dt / (2m).
    cfg = dict(C1, f_sp=0.0, gamma_s=0.8)
    x, v = inputs.initial_state(cfg, thermal=True)
    v = v + np.float32(0.75)          # a net drift to decay
    x, v, F = _init(oracle_mod, cfg, x, v)
    P0 = oracle_mod.momentum_ke(cfg, v)[:2]
    c = cfg["gamma_s"] * cfg["dt"] / (2 * cfg["mass"])
    _, _, _, _, pk = oracle_mod.step(cfg, x, v, F, 0, 400, every=1)
    n = np.arange(1, 401)
    expect = P0[None, :] * ((1 - c) ** 2 * (1 - 2 * c) ** (n - 1))[:, None]
    scale = np.abs(v).sum()
    assert np.abs(pk[:, :2] - expect).max() <= 1e-12 * scale


def test_stokes_decay_single_dimer(oracle_mod):
    # a translating dimer with F_p = 0: every velocity follows v_n = v_0 (1-c)^2 (1-2c)^(n-1)
    cfg = dict(C1, n_agents=1, L=10.0, f_sp=0.0, gamma_s=0.6)
    x = np.array([[4.0, 5.0], [4.5, 5.0]])
    v0 = np.array([[0.3, -0.2], [0.3, -0.2]])
    x, v, F = _init(oracle_mod, cfg, x, v0)
    c = cfg["gamma_s"] * cfg["dt"] / (2 * cfg["mass"])
    for n in (1, 2, 10, 100):
        _, vn, _, _, _ = oracle_mod.step(cfg, x, v, F, 0, n)
        expect = v0 * (1 - c) ** 2 * (1 - 2 * c) ** (n - 1)
        assert np.abs(vn - expect).max() <= 1e-12


@pytest.mark.parametrize("split", [0, 1])
def test_isolated_dimer_terminal_velocity(oracle_mod, split):
    # |v_COM| -> F_p / (2 zeta) along the director (head = particle 2k)
    cfg = dict(C1, n_agents=1, L=20.0, gamma_s=5.0, f_sp=1.0, sp_split=split)
    th = 0.7
    x = np.array([[10.0 + 0.25 * math.cos(th), 10.0 + 0.25 * math.sin(th)],
                  [10.0 - 0.25 * math.cos(th), 10.0 - 0.25 * math.sin(th)]])
    x, v, F = _init(oracle_mod, cfg, x, np.zeros((2, 2)))
    xn, vn, _, _, _ = oracle_mod.step(cfg, x, v, F, 0, 3000)
    vt = cfg["f_sp"] / (2 * cfg["gamma_s"])
    n = np.array([math.cos(th), math.sin(th)])
    com_v = 0.5 * (vn[0] + vn[1])
    assert com_v == pytest.approx(vt * n, abs=1e-12)
    # steady bond length: l (split) or l + F_p/(2 kappa) (head only)
    d = xn[0] - xn[1]
    d -= cfg["L"] * np.round(d / cfg["L"])
    r = math.hypot(*d)
    expect = cfg["bond_l"] + (cfg["f_sp"] / (2 * cfg["kappa"]) if split else 0.0)
    assert r == pytest.approx(expect, abs=1e-11)


def test_bond_oscillation_verlet_frequency(oracle_mod):
    # along-axis bond oscillation of a free dimer obeys the Stormer-Verlet
    # recurrence d_{n+1} + d_{n-1} = (2 - (omega dt)^2) d_n, omega^2 = 2 kappa / m
    cfg = dict(C1, n_agents=1, L=10.0, f_sp=0.0, gamma_s=0.0)
    x = np.array([[5.0, 5.0], [5.53, 5.0]])
    x, v, F = _init(oracle_mod, cfg, x, np.zeros((2, 2)))
    seps = []
    for _ in range(200):
        x, v, F, _, _ = oracle_mod.step(cfg, x, v, F, 0, 1)
        seps.append(x[1, 0] - x[0, 0] - cfg["bond_l"])
    d = np.array(seps)
    w2dt2 = 2 * cfg["kappa"] / cfg["mass"] * cfg["dt"] ** 2
    resid = d[2:] + d[:-2] - (2 - w2dt2) * d[1:-1]
    assert np.abs(resid).max() <= 1e-9 * 0.03
    # and it oscillates (the sign flips) with the discrete period 2 pi / theta
    theta = math.acos(1 - w2dt2 / 2)
    flips = np.count_nonzero(np.diff(np.sign(d)))
    assert abs(flips - 200 * theta / math.pi) <= 2


def _head_to_head(cfg, s0):
    l = cfg["bond_l"]
    y = 0.5 * cfg["L"]
    xa = 0.4 * cfg["L"]
    return np.array([[xa, y], [xa - l, y], [xa + s0, y], [xa + s0 + l, y]])


def test_head_to_head_balance_closed_form(oracle_mod):
    # Two agents pushing head to head with no noise (kT = 0) and Stokes friction
    # come to rest where propulsion balances the conservative repulsion of the
    # heads: f_sp = A w(s), i.e. s = r_c (1 - f_sp / A)  (Eq. 5.1 balance).
    cfg = dict(C1, n_agents=2, L=20.0, kT=0.0, gamma_s=2.0, gamma=4.5)
    x = _head_to_head(cfg, 0.9)
    x, v, F = _init(oracle_mod, cfg, x, np.zeros((4, 2)))
    xn, vn, _, _, _ = oracle_mod.step(cfg, x, v, F, 0, 20000)
    s = xn[2, 0] - xn[0, 0]
    assert s == pytest.approx(cfg["r_c"] * (1 - cfg["f_sp"] / cfg["A"]), abs=1e-9)
    assert np.abs(vn).max() < 1e-10


def test_paper_force_balance_estimate(oracle_mod):
    # Sec. 5.1, Eq. 5.1: with f_SP = 1, l = 1, a = 4 (r_h = l/(2a)) and r_c = 0.5
    # the paper estimates Phi ~ 1.3 from f_SP ~ Phi w(r_h).  Recover Phi from the
    # oracle's conservative force at r = r_h with unit amplitude.
    g = json.load(open(os.path.join(GOLDEN, "eq5_1_force_balance.json")))
    r_h = g["l"] / (2 * g["a"])
    cfg = dict(C1, A=1.0, gamma=0.0, kT=0.0, r_c=g["r_c"])
    f, _, _ = oracle_mod.pair_force(cfg, [r_h, 0.0], [0.0, 0.0], 0.0)
    phi = g["f_SP"] / f[0]
    assert round(phi, 1) == g["Phi_printed"]
    # the paper's chosen Phi = 1.5 then holds heads apart at r_c (1 - f_SP/Phi)
    cfg = dict(inputs.PAPER_SET, n_agents=2, L=10.0, gamma=8.0, gamma_s=0.5, kT=0.0,
               A=g["Phi_chosen"], seed=1)
    x = _head_to_head(cfg, 0.3)
    x, v, F = _init(oracle_mod, cfg, x, np.zeros((4, 2)))
    xn, _, _, _, _ = oracle_mod.step(cfg, x, v, F, 0, 40000)
    s = xn[2, 0] - xn[0, 0]
    assert s == pytest.approx(g["r_c"] * (1 - g["f_SP"] / g["Phi_chosen"]), abs=1e-8)


def _hamiltonian(oracle_mod, cfg, x, v):
    x = np.asarray(x)
    L, rc = cfg["L"], cfg["r_c"]
    ke = 0.5 * cfg["mass"] * (v * v).sum()
    pr = oracle_mod.pairs(cfg, x, "cells")
    d = x[pr[:, 0]] - x[pr[:, 1]]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(1))
    # potential of the conservative force A w(r): U = A r_c (1 - r/r_c)^2 / 2
    upair = (0.5 * cfg["A"] * rc * (1 - r / rc) ** 2).sum()
    db = x[0::2] - x[1::2]
    db -= L * np.round(db / L)
    rb = np.sqrt((db * db).sum(1))
    ubond = (0.5 * cfg["kappa"] * (rb - cfg["bond_l"]) ** 2).sum()
    return ke + upair + ubond


def test_energy_error_scales_with_dt_squared(oracle_mod):
    # conservative system (gamma = kT = gamma_s = f_sp = 0): velocity-Verlet's
    # energy error shrinks 4x when dt halves
    base = dict(C1, n_agents=200, L=20.0, gamma=0.0, kT=0.0, gamma_s=0.0, f_sp=0.0)
    x0, v0 = inputs.initial_state(base, thermal=True)
    errs = []
    for dt in (0.004, 0.002):
        cfg = dict(base, dt=dt)
        x, v, F = _init(oracle_mod, cfg, x0, v0)
        H0 = _hamiltonian(oracle_mod, cfg, x, v)
        n = int(round(0.4 / dt))
        dev = 0.0
        for _ in range(10):
            x, v, F, _, _ = oracle_mod.step(cfg, x, v, F, 0, n // 10)
            dev = max(dev, abs(_hamiltonian(oracle_mod, cfg, x, v) - H0))
        errs.append(dev)
    assert errs[0] / errs[1] == pytest.approx(4.0, abs=0.5)


def test_fluctuation_dissipation_temperature(oracle_mod):
    # F_p = gamma_s = 0: the DPD thermostat holds T_kin = sum m|v|^2 / (2N - 2) at kT.
    # The random start stores ~2 kT per particle of overlap energy that relaxes
    # over some 30 time units.  In the 40 x 40 box the kinetic temperature then
    # keeps wandering by a few percent over tens of time units (slow structural
    # rearrangements of a system that small); in an 80 x 80 box at the same
    # density a 50-unit average is steady to ~0.1%, so the pin uses that box.
    Ts = []
    for seed in (102, 103):
        cfg = dict(C1, f_sp=0.0, gamma_s=0.0, seed=seed, L=80.0, n_agents=3200)
        x, v = inputs.initial_state(cfg, thermal=True)
        x, v, F = _init(oracle_mod, cfg, x, v)
        x, v, F, s, _ = oracle_mod.step(cfg, x, v, F, 0, 10000)
        _, _, _, _, pk = oracle_mod.step(cfg, x, v, F, s, 10000, every=10)
        n = 2 * cfg["n_agents"]
        Ts.append(2 * pk[:, 2].mean() / (2 * n - 2))
    assert np.mean(Ts) == pytest.approx(C1["kT"], rel=0.005)


def test_trajectory_deterministic_and_resumable(oracle_mod):
    cfg = C1
    x, v = inputs.initial_state(cfg)
    x, v, F = _init(oracle_mod, cfg, x, v)
    a = oracle_mod.step(cfg, x, v, F, 0, 40)
    b = oracle_mod.step(cfg, x, v, F, 0, 40)
    assert all((p == q).all() for p, q in zip(a[:3], b[:3]))
    h = oracle_mod.step(cfg, x, v, F, 0, 20)
    h2 = oracle_mod.step(cfg, h[0], h[1], h[2], h[3], 20)
    assert h2[3] == 40
    assert all((p == q).all() for p, q in zip(a[:3], h2[:3]))


def test_wrap_and_minimum_image(oracle_mod):
    L = 40.0
    assert oracle_mod.wrap(-1e-18, L) == 0.0
    assert oracle_mod.wrap(40.0, L) == 0.0
    assert oracle_mod.wrap(41.5, L) == 1.5
    assert oracle_mod.wrap(-0.5, L) == 39.5
    assert oracle_mod.minimg(39.5, L) == -0.5
    assert oracle_mod.minimg(-39.5, L) == 0.5
    assert oracle_mod.minimg(0.25, L) == 0.25


def test_forces_do_not_depend_on_thread_count():
    # each particle's pair list is summed in j order, so the oracle's forces
    # are the same bits on one thread and on all of them
    import oracle
    cfg = inputs.physics(inputs.WORKLOADS["dimers_1600"])
    x, v = inputs.initial_state(cfg, thermal=True)
    n = oracle.num_threads()
    F_all = oracle.forces(cfg, x, v, 3)
    oracle.set_threads(1)
    try:
        F_one = oracle.forces(cfg, x, v, 3)
    finally:
        oracle.set_threads(n)
    assert (F_all == F_one).all()
    assert oracle.num_threads() == n
