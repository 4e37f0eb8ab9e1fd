"""Long-run statistics of the engine against the oracle's: the energy spectrum
E(k) in log-spaced bands and the integral length of the velocity correlation
function (Sec. 5.3-5.4), as ensemble means over the seeds of the protocol in
tests/golden/stats_protocol.py.  On the GPU the seeds run as the replicas of
one batch, and the statistics of all replicas are taken together (the batched
band energies of the protocol module, and its pair-loop correlation function
evaluated in FP64 on the device).  The oracle's values are stored in
tests/golden/stats_dimers_1600.json (written by make_stats_golden.py, which
calls only the oracle).

Trajectories diverge chaotically, so the comparison is statistical: each
quantity must agree within max(2 %, 3 sigma), sigma being the combined
standard error of the two ensemble means.  Where sigma exceeds 0.5 % of the
value the comparison is underpowered for a 2 % claim, and the test says so in
its output.
"""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

from paper_1310_0998_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def vcf_batch(x, v, R: int, L: float, dr: float, chunk: int = 64):
    """vcf_pairs of stats_protocol for every replica of a batch at once, in
    FP64 on the device: x, v [R N][2] (N particles per replica, agents as
    consecutive pairs).  Returns g [R][nb] (without the g(0) entry)."""
    import torch

    X = x.double().view(R, -1, 2)
    W = v.double().view(R, -1, 2)
    h, t = X[:, 0::2], X[:, 1::2]
    d = h - t
    d -= L * torch.round(d / L)
    com = torch.remainder(t + 0.5 * d, L)
    V = 0.5 * (W[:, 0::2] + W[:, 1::2])
    n = com.shape[1]
    mean = V.mean(1)
    mean2 = (mean * mean).sum(1)
    var = (V * V).sum(2).mean(1) - mean2
    nb = int(np.floor(0.5 * L / dr))
    I, J = torch.triu_indices(n, n, 1, device=x.device)
    # each bin is spread over S partial sums (by pair index), so that the
    # device's atomic adds do not all meet on a few addresses
    S = 256
    sub = torch.arange(I.numel(), device=x.device) % S
    num = torch.zeros(R * nb * S, dtype=torch.float64, device=x.device)
    cnt = torch.zeros(R * nb * S, dtype=torch.float64, device=x.device)
    for c0 in range(0, R, chunk):
        c1 = min(R, c0 + chunk)
        dd = com[c0:c1, J] - com[c0:c1, I]
        dd -= L * torch.round(dd / L)
        r = torch.sqrt((dd * dd).sum(-1))
        b = torch.floor(r / dr).long()
        ok = b < nb
        dots = (V[c0:c1, J] * V[c0:c1, I]).sum(-1)
        key = ((torch.arange(c0, c1, device=x.device)[:, None] * nb + b) * S + sub[None, :])[ok]
        num.index_add_(0, key, dots[ok])
        cnt.index_add_(0, key, torch.ones_like(dots[ok]))
    num, cnt = num.view(R, nb, S).sum(-1), cnt.view(R, nb, S).sum(-1)
    return ((num / cnt - mean2[:, None]) / var[:, None]).cpu().numpy()


def test_energy_spectrum_and_correlation_length_match_oracle():
    import torch

    from oracle import analysis
    from paper_1310_0998_amd import dpd
    from stats_protocol import PROTOCOL, band_energies_batch, ensemble

    with open(os.path.join(HERE, "golden", "stats_dimers_1600.json")) as f:
        ref = json.load(f)
    assert ref["protocol"] == json.loads(json.dumps(PROTOCOL))
    # every seed is one replica of one batch
    seeds = PROTOCOL["seeds"]
    R = len(seeds)
    cfgs = [dict(inputs.physics(inputs.WORKLOADS[PROTOCOL["workload"]]), seed=s) for s in seeds]
    states = [inputs.initial_state(c) for c in cfgs]
    x = np.concatenate([st[0] for st in states])
    v = np.concatenate([st[1] for st in states])
    L, dr = cfgs[0]["L"], PROTOCOL["dr"]
    sim = dpd.Sim(cfgs, device="cuda:0")
    sim.set_state(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(), 0)
    sim.set_graph_chunk(PROTOCOL["every"])
    sim.step(PROTOCOL["warmup"])
    nsnap = PROTOCOL["steps"] // PROTOCOL["every"]
    E = np.zeros((R, len(PROTOCOL["bands"])))
    g = None
    for _ in range(nsnap):
        sim.step(PROTOCOL["every"])
        u, _ = sim.bin_velocity(PROTOCOL["M"], 0.0, 0)
        xs, vs, _, _ = sim.get_state()
        E += band_energies_batch(u.cpu().numpy())
        gs = vcf_batch(xs, vs, R, L, dr)
        g = gs if g is None else g + gs
    sim.close()
    nb = g.shape[1]
    r = np.concatenate([[0.0], (np.arange(nb) + 0.5) * dr])
    per_seed = [dict(E_bands=(E[q] / nsnap).tolist(),
                     L_gv=analysis.integral_length(r, np.concatenate([[1.0], g[q] / nsnap]), L),
                     snapshots=nsnap) for q in range(R)]
    gpu = ensemble(per_seed)
    rows = [(f"E band {a}-{b}", gpu["E_bands"][i], gpu["E_bands_sem"][i], ref["E_bands"][i],
             ref["E_bands_sem"][i]) for i, (a, b) in enumerate(PROTOCOL["bands"])]
    rows.append(("L_gv", gpu["L_gv"], gpu["L_gv_sem"], ref["L_gv"], ref["L_gv_sem"]))
    bad = []
    for name, gv, gs, o, os_ in rows:
        sig = np.hypot(gs, os_) / abs(o)
        tol = max(0.02, 3.0 * sig)
        dev = abs(gv - o) / abs(o)
        note = "  (underpowered: sigma > 0.5 %)" if sig > 0.005 else ""
        print(f"{name:12s} gpu {gv:.5g}  oracle {o:.5g}  diff {100 * dev:.2f} %  "
              f"sigma {100 * sig:.2f} %  tolerance {100 * tol:.2f} %{note}")
        if dev > tol:
            bad.append(name)
    assert not bad, bad


def test_transient_4m_statistics_match_oracle():
    """The 4M-particle workload over t <= 10 from its random start (PROTOCOL_4M:
    seeds 301-304, u_M on 256 x 256 every 20 steps): band energies and the
    integral length of the gridded field's correlation per 400-step window,
    against the oracle's stored values (stats_dimers_4M_transient.json,
    written by make_stats_golden_4m.py from the oracle alone), within
    max(2 %, 3 sigma) of the combined standard error over the four seeds.
    Both sides start from the same states and draw the same noise, so the
    per-seed differences are printed as well."""
    import torch

    from paper_1310_0998_amd import dpd
    from stats_protocol import PROTOCOL_4M, WindowAccumulator, window_ensemble

    path = os.path.join(HERE, "golden", "stats_dimers_4M_transient.json")
    if not os.path.exists(path):
        pytest.skip("stats_dimers_4M_transient.json not written")
    with open(path) as f:
        ref = json.load(f)
    P = PROTOCOL_4M
    assert ref["protocol"] == json.loads(json.dumps(P))
    per_seed = []
    for seed in P["seeds"]:
        cfg = dict(inputs.physics(inputs.WORKLOADS[P["workload"]]), seed=seed, bin_M_max=P["M"])
        x, v = inputs.initial_state(cfg)
        sim = dpd.Sim(cfg, device="cuda:0")
        sim.set_state(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(), 0)
        acc = WindowAccumulator(cfg["L"])
        for _ in range(P["steps"] // P["every"]):
            sim.step(P["every"])
            u, _ = sim.bin_velocity(P["M"], 0.0, 0)
            acc.add(u.cpu().numpy())
        sim.close()
        per_seed.append(acc.result())
    gpu = window_ensemble(per_seed)
    bad = []
    nw = P["steps"] // P["window"]
    for w in range(nw):
        rows = [(f"w{w} E {a}-{b}", gpu["E_bands"][w][i], gpu["E_bands_sem"][w][i], ref["E_bands"][w][i],
                 ref["E_bands_sem"][w][i],
                 max(abs(s["E_bands"][w][i] / o["E_bands"][w][i] - 1) for s, o in zip(per_seed, ref["per_seed"])))
                for i, (a, b) in enumerate(P["bands"])]
        rows.append((f"w{w} L_gv", gpu["L_gv"][w], gpu["L_gv_sem"][w], ref["L_gv"][w], ref["L_gv_sem"][w],
                     max(abs(s["L_gv"][w] / o["L_gv"][w] - 1) for s, o in zip(per_seed, ref["per_seed"]))))
        for name, gv, gs, o, os_, seedmax in rows:
            sig = np.hypot(gs, os_) / abs(o)
            tol = max(0.02, 3.0 * sig)
            dev = abs(gv - o) / abs(o)
            print(f"{name:12s} gpu {gv:.5g}  oracle {o:.5g}  diff {100 * dev:.3f} %  sigma {100 * sig:.2f} %  "
                  f"tolerance {100 * tol:.2f} %  largest per-seed diff {100 * seedmax:.3f} %")
            if dev > tol:
                bad.append(name)
    assert not bad, bad


@pytest.mark.parametrize("n_agents,L,kind", [(800, 40.0, "random"), (420, 29.25, "edge"),
                                             (3000, 60.0, "random")])
def test_agent_vcf_matches_oracle_pair_loop(n_agents, L, kind):
    # the GPU pair sums of dpd_agent_vcf against the oracle's pair loop over
    # the same state: every bin's pair count exactly, g within what the
    # fixed-point pair sums allow (half a step of 2^-20 per pair, over the
    # velocity variance)
    import torch
    from oracle import analysis
    from paper_1310_0998_amd import dpd, fieldstats, inputs
    cfg = dict(inputs.physics(inputs.WORKLOADS["dimers_1600"]), n_agents=n_agents, L=L, seed=n_agents)
    x, v = inputs.initial_state(cfg, kind=kind, thermal=True)
    dr = 0.25
    r, g, c = fieldstats.agent_vcf(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(), L, dr)
    com, V = analysis.agent_com(x, v, L)
    ro, go, co = analysis.vcf_bruteforce(com, V, L, dr)
    assert np.array_equal(r, ro)
    assert np.array_equal(c, co)
    var = float((V * V).sum(axis=1).mean() - V.mean(axis=0) @ V.mean(axis=0))
    ok = co > 0
    assert np.abs(g[ok] - go[ok]).max() <= 2.0 ** -21 / var + 1e-12
    assert fieldstats.integral_length(r, g, L, to_first_zero=False) == pytest.approx(
        analysis.integral_length(ro, go, L), rel=1e-6)
