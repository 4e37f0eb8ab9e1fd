"""Batches of replicas, captured step chunks and tile schedules, through the C
ABI.  A replica in a batch must follow bitwise the trajectory of a handle made
for it alone (which the parity tests pin to the oracle); replayed graph chunks
and every tile schedule must give bitwise the results of the launches one by
one.  Needs an MI355X."""
import numpy as np
import pytest

import oracle
from paper_1310_0998_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

C1 = inputs.physics(inputs.WORKLOADS["dimers_1600"])
DEV = "cuda:0"


@pytest.fixture(scope="module")
def dpd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_0998_amd import dpd as d
    d.lib()
    return d


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def replicas():
    """Five systems of uneven size, box, friction, seed and layout; the last
    one, at areal density 3 (softer repulsion, so that the random start does not
    tear bonds) with 8 x 8 tiles, sends every tile to the overflow kernel."""
    cfgs = [
        dict(C1, n_agents=300, L=23.0, gamma_s=0.0, seed=11),
        dict(C1, n_agents=800, L=40.0, seed=12),
        dict(C1, n_agents=137, L=16.5, gamma=1.0, gamma_s=5.0, seed=13),
        dict(C1, n_agents=1500, L=47.0, gamma=20.0, gamma_s=0.5, seed=14, sp_split=1),
        dict(C1, n_agents=800, L=23.0, A=5.0, seed=15, tile=8),
    ]
    kinds = ["random", "edge", "random", "random", "random"]
    states = [inputs.initial_state(c, kind=k, thermal=True) for c, k in zip(cfgs, kinds)]
    return cfgs, states


def concat(states):
    return (np.concatenate([s[0] for s in states]), np.concatenate([s[1] for s in states]))


def split(a, sizes):
    out, o = [], 0
    for n in sizes:
        out.append(a[o:o + n])
        o += n
    return out


def test_batch_matches_single_handles(dpd):
    cfgs, states = replicas()
    x, v = concat(states)
    b = dpd.Sim(cfgs, device=DEV)
    b.set_state(dev(x), dev(v), 3)
    singles = []
    for c, (xs, vs) in zip(cfgs, states):
        s = dpd.Sim(c, device=DEV)
        s.set_state(dev(xs), dev(vs), 3)
        singles.append(s)
    # forces of the loaded state
    Fb = split(host(b.forces()), b.sizes)
    for s, F in zip(singles, Fb):
        assert (host(s.forces()) == F).all()
    # two calls (the second starts from the prepared step), with records
    pkb = [host(b.step(13, reduce_every=13)), host(b.step(17, reduce_every=17))]
    pks = [[host(s.step(13, reduce_every=13)), host(s.step(17, reduce_every=17))] for s in singles]
    xb, vb, Fb, sb = b.get_state()
    assert sb == 33
    parts = [split(host(t), b.sizes) for t in (xb, vb, Fb)]
    for q, s in enumerate(singles):
        xs, vs, Fs, ss = s.get_state()
        assert ss == 33
        for k, t in enumerate((xs, vs, Fs)):
            assert (host(t) == parts[k][q]).all(), (q, "xvF"[k])
        for rec in range(2):
            # the FP64 sums run over other tile partitions: equal to rounding
            assert pkb[rec][0, q] == pytest.approx(pks[q][rec][0], rel=1e-12, abs=1e-9)
    # velocity fields, plain bins and windows with centre-of-mass velocities
    for eps, mode in ((0.0, 0), (2.5, 1)):
        ub, nb = b.bin_velocity(16, eps, mode)
        for q, s in enumerate(singles):
            us, ns = s.bin_velocity(16, eps, mode)
            assert (host(ns) == host(nb[q])).all()
            assert (host(us) == host(ub[q])).all()
    b.close()
    for s in singles:
        s.close()


def test_batch_forces_match_oracle(dpd):
    cfgs, states = replicas()
    x, v = concat(states)
    b = dpd.Sim(cfgs, device=DEV)
    b.set_state(dev(x), dev(v), 7)
    F = split(host(b.forces()).astype(np.float64), b.sizes)
    for c, (xs, vs), Fq in zip(cfgs, states, F):
        Fo = oracle.forces(c, xs, vs, 7)
        _, scale = oracle.force_parts(c, xs, vs, 7)
        per = np.sqrt(((Fq - Fo) ** 2).sum(1)) / scale
        assert per.max() < 1e-5
    b.close()


def test_batch_cells_concatenated(dpd):
    cfgs, states = replicas()
    x, v = concat(states)
    b = dpd.Sim(cfgs, device=DEV)
    b.set_state(dev(x), dev(v), 0)
    cs, ids = (host(t) for t in b.cells())
    o_c, o_p = 0, 0
    for c, (xs, _) in zip(cfgs, states):
        nc = int(np.floor(c["L"] / c["r_c"]))
        seg = cs[o_c:o_c + nc * nc + 1] - o_p
        cs_o, ids_o = oracle.bin_cells(c, xs)
        assert (seg == cs_o).all()
        assert (ids[o_p:o_p + len(xs)] == ids_o).all()
        o_c += nc * nc
        o_p += len(xs)
    assert cs[-1] == len(x)
    b.close()


@pytest.mark.parametrize("batch", [False, True])
def test_graph_chunks_bitwise(dpd, batch):
    if batch:
        cfgs, states = replicas()
        cfg = cfgs
        x, v = concat(states)
    else:
        cfg = C1
        x, v = inputs.initial_state(C1, thermal=True)
    ref = dpd.Sim(cfg, device=DEV)
    ref.set_state(dev(x), dev(v), 0)
    g = dpd.Sim(cfg, device=DEV)
    g.set_state(dev(x), dev(v), 0)
    g.set_graph_chunk(8)
    # replays with eager work and synchronisation between them; call lengths
    # that start from the B buffers and leave remainders
    for n, red in ((24, 8), (13, 0), (16, 0), (40, 16), (7, 0), (32, 8)):
        pr = ref.step(n, reduce_every=red) if red else ref.step(n)
        pg = g.step(n, reduce_every=red) if red else g.step(n)
        a, b2 = ref.get_state(), g.get_state()
        assert a[3] == b2[3]
        for k in range(3):
            assert (host(a[k]) == host(b2[k])).all(), (n, "xvF"[k])
        if red:
            assert (host(pr) == host(pg)).all()
    ref.close()
    g.close()


@pytest.mark.parametrize("batch", [False, True])
def test_schedules_bitwise(dpd, batch):
    if batch:
        cfgs, states = replicas()
        cfg = cfgs
        x, v = concat(states)
    else:
        cfg = dict(C1, n_agents=1500, L=47.0)
        x, v = inputs.initial_state(cfg, thermal=True)
    ref = dpd.Sim(cfg, device=DEV)
    ref.set_state(dev(x), dev(v), 0)
    ref.step(20)
    want = [host(t) for t in ref.get_state()[:3]]
    for tx, ty, order in ((8, 8, 1), (4, 4, 0), (6, 5, 1), (5, 7, 0)):
        s = dpd.Sim(cfg, device=DEV)
        s.set_schedule(tx, ty, order)
        assert s.schedule() == (tx, ty, order)
        s.set_state(dev(x), dev(v), 0)
        s.step(20)
        got = [host(t) for t in s.get_state()[:3]]
        for k in range(3):
            assert (got[k] == want[k]).all(), (tx, ty, order, "xvF"[k])
        s.close()
    ref.close()


@pytest.mark.parametrize("batch", [False, True])
def test_autotune_keeps_state(dpd, batch):
    if batch:
        cfgs, states = replicas()
        cfg = cfgs
        x, v = concat(states)
    else:
        cfg = C1
        x, v = inputs.initial_state(C1, thermal=True)
    ref = dpd.Sim(cfg, device=DEV)
    ref.set_state(dev(x), dev(v), 0)
    ref.step(5)
    t = dpd.Sim(cfg, device=DEV)
    t.set_state(dev(x), dev(v), 0)
    t.step(5)  # leaves a prepared step behind
    tx, ty, order, ms = t.autotune(4)
    assert 1 <= tx <= 8 and 1 <= ty <= 8 and order in (0, 1) and ms > 0
    assert t.schedule() == (tx, ty, order)
    print(f"autotune: tile {tx} x {ty}, order {order}, {ms:.4f} ms/step")
    a, b2 = ref.get_state(), t.get_state()
    assert a[3] == b2[3] == 5
    for k in range(3):
        assert (host(a[k]) == host(b2[k])).all()
    # the cell list read with the stored state (and the row binning of the
    # velocities that uses it) belongs to that state again, not to a trial
    for u, w in zip(ref.cells(), t.cells()):
        assert (host(u) == host(w)).all()
    for u, w in zip(ref.bin_velocity(32, 0.0, 0), t.bin_velocity(32, 0.0, 0)):
        assert (host(u) == host(w)).all()
    ref.step(11)
    t.step(11)
    a, b2 = ref.get_state(), t.get_state()
    for k in range(3):
        assert (host(a[k]) == host(b2[k])).all()
    ref.close()
    t.close()


def test_autotune_clustered_replica_keeps_state(dpd):
    # a batch whose first replica is one dense cluster (most of its tiles go to
    # the overflow kernel, so the tuner's per-replica refinement has replicas
    # to move) next to a uniform one: whatever tiles the tuner gives each
    # replica, the state comes back exactly and later steps match an untuned
    # run bit for bit
    cfgs = [dict(C1, n_agents=1200, L=40.0, seed=41), dict(C1, n_agents=800, L=40.0, seed=42)]
    states = [inputs.initial_state(cfgs[0], kind="clustered", thermal=True),
              inputs.initial_state(cfgs[1], thermal=True)]
    x, v = concat(states)
    ref = dpd.Sim(cfgs, device=DEV)
    ref.set_state(dev(x), dev(v), 0)
    ref.step(6)
    t = dpd.Sim(cfgs, device=DEV)
    t.set_state(dev(x), dev(v), 0)
    t.step(6)
    tx, ty, order, ms = t.autotune(6)
    print(f"autotune (clustered replica 0): tile {tx} x {ty}, order {order}, {ms:.4f} ms/step")
    assert 1 <= tx <= 8 and 1 <= ty <= 8 and ms > 0
    a, b2 = ref.get_state(), t.get_state()
    assert a[3] == b2[3] == 6
    for k in range(3):
        assert (host(a[k]) == host(b2[k])).all()
    for u, w in zip(ref.cells(), t.cells()):
        assert (host(u) == host(w)).all()
    ref.step(14)
    t.step(14)
    a, b2 = ref.get_state(), t.get_state()
    for k in range(3):
        assert (host(a[k]) == host(b2[k])).all()
    ref.close()
    t.close()


def test_sweep_workload_runs(dpd):
    # the 64-replica sweep, briefly: every replica stays finite and keeps the
    # momentum balance of its own friction (Stokes decay only: no propulsion)
    cfgs = [dict(c, f_sp=0.0) for c in inputs.sweep_replicas()]
    states = [inputs.initial_state(c, thermal=True) for c in cfgs]
    x, v = concat(states)
    b = dpd.Sim([inputs.physics(c) for c in cfgs], device=DEV)
    b.set_state(dev(x), dev(v), 0)
    b.set_graph_chunk(10)
    pk = host(b.step(20, reduce_every=10))
    assert pk.shape == (2, 64, 3)
    assert np.isfinite(pk).all()
    xs, vs, _, s = b.get_state()
    assert s == 20 and np.isfinite(host(xs)).all() and np.isfinite(host(vs)).all()
    b.close()


def test_batch_error_paths(dpd):
    cfgs, _ = replicas()
    with pytest.raises(dpd.DPDError):
        dpd.Sim([dict(cfgs[0], skin=0.3), cfgs[1]], device=DEV)
    b = dpd.Sim(cfgs, device=DEV)
    with pytest.raises(dpd.DPDError):
        b.set_graph_chunk(7)
    with pytest.raises(dpd.DPDError):
        b.set_schedule(9, 4, 0)
    with pytest.raises(dpd.DPDError):
        b.set_schedule(1, 1, 0)  # more tiles than the workspace holds
    with pytest.raises(dpd.DPDError):
        b.autotune(4)  # no state yet
    b.close()


def test_paper_geometry_batch_steps(dpd):
    # the paper's own parameters (bond l = 1 longer than r_c = 0.5) in small
    # boxes, as a batch with windowed 128-point fields: the partner stays in
    # the stencil (no DPD_EBOND) and the state stays finite
    from paper_1310_0998_amd import paper_runs
    cfgs = []
    for i, (phi, g, gs) in enumerate(paper_runs.REPLICAS):
        c = paper_runs.replica_cfg(phi, g, gs, seed=900 + i)
        c = dict(c, L=25.0, n_agents=int(round(4.0e4 * phi / 16)))
        cfgs.append(c)
    states = [inputs.initial_state(c) for c in cfgs]
    x, v = concat(states)
    b = dpd.Sim(cfgs, device=DEV)
    b.set_state(dev(x), dev(v), 0)
    b.set_graph_chunk(50)
    b.step(600)
    u, n = b.bin_velocity(64, 2.0, 0)
    xs, vs, _, s = b.get_state()
    assert s == 600 and np.isfinite(host(xs)).all() and np.isfinite(host(vs)).all()
    assert np.isfinite(host(u)).all() and (host(n).sum(axis=(1, 2)) > 0).all()
    b.close()
