"""GPU engine against the FP64 oracle, element by element on the same seeded
inputs, through the C ABI.  Needs an MI355X."""
import math

import numpy as np
import pytest

import oracle
from paper_1310_0998_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

C1 = inputs.physics(inputs.WORKLOADS["dimers_1600"])
C2 = inputs.physics(inputs.WORKLOADS["dimers_200k"])
C3 = inputs.physics(inputs.WORKLOADS["dimers_4M"])
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


def make_sim(dpd, cfg, x, v, step=0, F=None):
    sim = dpd.Sim(cfg, device=DEV)
    sim.set_state(dev(x), dev(v), step, None if F is None else dev(F))
    return sim


def force_errors(cfg, x, v, step, F_gpu):
    """Per-particle error relative to the scale S_i, and the global relative L2 error."""
    Fo = oracle.forces(cfg, x, v, step)
    _, scale = oracle.force_parts(cfg, x, v, step)
    F = F_gpu.astype(np.float64)
    per = np.sqrt(((F - Fo) ** 2).sum(1)) / scale
    glob = np.sqrt(((F - Fo) ** 2).sum()) / np.sqrt((Fo ** 2).sum())
    return per, glob


# ---------------------------------------------------------------- noise words

@pytest.mark.parametrize("rng_kind,noise_kind", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_rng_words_bit_identical(dpd, rng_kind, noise_kind):
    cfg = dict(C1, rng_kind=rng_kind, noise_kind=noise_kind, seed=0xDEADBEEF12345)
    rng = np.random.default_rng(1)
    n = 3000
    i = rng.integers(0, 2 ** 30, n).astype(np.int32)
    j = rng.integers(0, 2 ** 30, n).astype(np.int32)
    i[:10] = np.arange(10)
    j[:10] = np.arange(10)[::-1]
    for step in (0, 1, 12345, 2 ** 32 + 7):
        w, a = dpd.rng_words(cfg, dev(i), dev(j), step)
        w = host(w).view(np.uint32)
        a = host(a)
        for k in range(0, n, 97):
            wo = oracle.pair_words(cfg, int(i[k]), int(j[k]), step)
            assert (w[k] == wo).all(), (k, w[k], wo)
            ao = oracle.pair_alpha(cfg, int(i[k]), int(j[k]), step)
            assert abs(a[k] - ao) <= 2e-6 * max(1.0, abs(ao)), (k, a[k], ao)


# ------------------------------------------------------------------- binning

BIN_CASES = [
    ("C1", dict(C1), "random"),
    ("C1-edge", dict(C1), "edge"),
    ("ragged-47", dict(C1, L=47.0, n_agents=1100, seed=5), "random"),
    ("w>rc", dict(C1, L=29.25, r_c=1.1, n_agents=420, seed=6), "edge"),
    ("nc3", dict(C1, L=3.0, n_agents=4, seed=7), "random"),
    ("nc4", dict(C1, L=4.5, r_c=1.125, n_agents=8, seed=8), "edge"),
    ("nc5", dict(C1, L=5.0, n_agents=12, seed=9), "random"),
    ("clustered", dict(C1, L=40.0, n_agents=1200, seed=10), "clustered"),
    ("one-agent", dict(C1, L=10.0, n_agents=1, seed=11), "random"),
    # the cell scan works in chunks of 4096 cells up to 2^20 cells, of 16384
    # above: a whole number of chunks; a last chunk of 257 cells (not a whole
    # group of 4); 270 large chunks, more than one look-back window of 256
    ("chunk-exact", dict(C1, L=128.0, n_agents=8000, seed=12), "random"),
    ("chunk-ragged", dict(C1, L=129.0, n_agents=8000, seed=13), "random"),
    ("chunks-270", dict(C1, L=2100.0, n_agents=100000, seed=14), "random"),
    # 2^20 cells: 256 small chunks, one full look-back window; one cell row
    # more: large chunks
    ("small-chunks-256", dict(C1, L=1024.0, n_agents=30000, seed=15), "random"),
    ("large-chunks-65", dict(C1, L=1025.0, n_agents=30000, seed=16), "random"),
]


@pytest.mark.parametrize("name,cfg,kind", BIN_CASES, ids=[c[0] for c in BIN_CASES])
def test_binning_bit_exact(dpd, name, cfg, kind):
    x, v = inputs.initial_state(cfg, kind=kind, thermal=True)
    sim = make_sim(dpd, cfg, x, v)
    cs, ids = sim.cells()
    cso, idso = oracle.bin_cells(cfg, x)
    assert (host(cs) == cso).all()
    assert (host(ids) == idso).all()
    # and again after the particles moved (state positions are FP32)
    sim.step(7)
    xs = host(sim.get_state()[0])
    cs, ids = sim.cells()
    cso, idso = oracle.bin_cells(cfg, xs)
    assert (host(cs) == cso).all()
    assert (host(ids) == idso).all()
    sim.close()


def test_binning_with_multi_cell_jumps(dpd):
    # three agents move ~2 cells per step (|v| dt = 2 cell widths): they take the
    # engine's jumper path; cells must still match the oracle bit for bit and
    # the trajectory must match too
    cfg = dict(C1, L=30.0, n_agents=300, seed=21, gamma=0.0, kT=0.0)
    x, v = inputs.initial_state(cfg)
    v[0:2] = (400.0, 0.0)
    v[2:4] = (-300.0, 410.0)
    v[4:6] = (0.0, -401.0)
    sim = make_sim(dpd, cfg, x, v)
    Fo = oracle.forces(cfg, x, v, 0)
    xo, vo, Fo, so = x.astype(np.float64), v.astype(np.float64), Fo, 0
    for k in range(4):
        sim.step(1)
        xo, vo, Fo, so, _ = oracle.step(cfg, xo, vo, Fo, so, 1)
        xs = host(sim.get_state()[0])
        cs, ids = sim.cells()
        cso, idso = oracle.bin_cells(cfg, xs)
        assert (host(cs) == cso).all() and (host(ids) == idso).all()
    d = xs.astype(np.float64) - xo
    d -= cfg["L"] * np.round(d / cfg["L"])
    assert np.abs(d).max() < 1e-3
    sim.close()


# -------------------------------------------------------------------- forces

FORCE_CASES = [
    ("C1", dict(C1), "random", True),
    ("C1-edge", dict(C1), "edge", True),
    ("ragged-47", dict(C1, L=47.0, n_agents=1100, seed=5), "random", True),
    ("w>rc", dict(C1, L=29.25, r_c=1.1, n_agents=420, seed=6), "edge", True),
    ("nc3", dict(C1, L=3.0, n_agents=4, seed=7), "random", True),
    ("nc4", dict(C1, L=4.5, r_c=1.125, n_agents=8, seed=8), "edge", True),
    ("nc5", dict(C1, L=5.0, n_agents=12, seed=9), "random", True),
    ("clustered", dict(C1, L=40.0, n_agents=1200, seed=10), "clustered", True),
    ("uniform-noise", dict(C1, noise_kind=1, seed=12), "random", True),
    ("philox2x32", dict(C1, rng_kind=1, seed=13), "random", True),
    ("head-only", dict(C1, sp_split=1, seed=14), "random", True),
    ("tile8", dict(C1, tile=8, seed=15), "random", True),
    ("tile1", dict(C1, L=12.0, n_agents=70, tile=1, seed=16), "random", True),
    ("gamma0", dict(C1, gamma=0.0, seed=17), "random", True),
    ("at-rest", dict(C1, seed=18), "random", False),
    # the change of weight exponent of Sec. 6: f_D with w^s, f_R with w^(s/2)
    ("w_exp-0.5", dict(C1, w_exp=0.5, seed=19), "random", True),
    ("w_exp-1", dict(C1, w_exp=1.0, seed=20), "edge", True),
    ("w_exp-3", dict(C1, w_exp=3.0, seed=21), "random", True),
    # the paper's own geometry: bond l = 1 longer than r_c = 0.5 (partner read by id)
    ("l>rc", dict(C1, r_c=0.5, bond_l=1.0, A=1.5, kT=0.05, seed=22), "random", True),
]


@pytest.mark.parametrize("name,cfg,kind,thermal", FORCE_CASES, ids=[c[0] for c in FORCE_CASES])
def test_forces_match_oracle(dpd, name, cfg, kind, thermal):
    x, v = inputs.initial_state(cfg, kind=kind, thermal=thermal)
    step = 31
    sim = make_sim(dpd, cfg, x, v, step=step)
    F = host(sim.forces())
    per, glob = force_errors(cfg, x, v, step, F)
    k = int(per.argmax())
    print(f"{name}: max per-particle error {per.max():.2e} (particle {k}), global {glob:.2e}, "
          f"median {np.median(per):.2e}")
    assert per.max() <= 1e-5, (name, per.max(), k)
    assert glob <= 1e-5, (name, glob)
    # the stored force of set_state is the same evaluation
    _, _, Fs, s = sim.get_state()
    assert s == step
    assert (host(Fs) == F).all()
    sim.close()


def _sampled_errors(cfg, x, v, step, F, idx):
    """Per-particle error of the sampled particles relative to their scale S_i
    (the oracle evaluates the sampled forces one by one; S_i comes from its
    whole-system force parts)."""
    Fo = oracle.forces_subset(cfg, x, v, step, idx)
    _, scale = oracle.force_parts(cfg, x, v, step)
    err = np.sqrt(((F[idx].astype(np.float64) - Fo) ** 2).sum(1))
    return err / scale[idx], Fo


def test_forces_full_size_sampled(dpd):
    # 4M particles in the benchmark's launch configuration: every force is
    # computed on the GPU, a sample is checked against the oracle one by one
    cfg = C3
    x, v = inputs.initial_state(cfg, thermal=True)
    sim = make_sim(dpd, cfg, x, v, step=3)
    F = host(sim.forces())
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(len(x), 3000, replace=False), [0, 1, len(x) - 2, len(x) - 1]])
    per, _ = _sampled_errors(cfg, x, v, 3, F, idx)
    print(f"4M sampled: max per-particle error / S_i {per.max():.2e}")
    assert per.max() <= 1e-5
    # cell list of the full system is bit-exact
    cs, ids = sim.cells()
    cso, idso = oracle.bin_cells(cfg, x)
    assert (host(cs) == cso).all() and (host(ids) == idso).all()
    # after stepping in the benchmark's configuration the state stays sane and
    # its cell list (a scan over hundreds of chunks, many launches later) is
    # still bit-exact
    sim.step(20)
    sim.sync()
    xs = host(sim.get_state()[0])
    assert np.isfinite(xs).all() and (xs >= 0).all() and (xs < cfg["L"]).all()
    cs, ids = sim.cells()
    cso, idso = oracle.bin_cells(cfg, xs)
    assert (host(cs) == cso).all() and (host(ids) == idso).all()
    sim.close()


@pytest.mark.parametrize("k,gz", list(enumerate(inputs.GAMMA_ZETA_GRID_200K)),
                         ids=[f"gamma{g:g}-zeta{z:g}" for g, z in inputs.GAMMA_ZETA_GRID_200K])
def test_forces_200k_grid_sampled(dpd, k, gz):
    # every point of the 200k-particle gamma x zeta grid, from its own seed
    g, z = gz
    cfg = dict(C2, gamma=g, gamma_s=z, seed=201 + k)
    x, v = inputs.initial_state(cfg, thermal=True)
    sim = make_sim(dpd, cfg, x, v, step=11)
    F = host(sim.forces())
    idx = np.random.default_rng(1 + k).choice(len(x), 3000, replace=False)
    per, _ = _sampled_errors(cfg, x, v, 11, F, idx)
    print(f"200k gamma={g} zeta={z}: max per-particle error / S_i {per.max():.2e}")
    assert per.max() <= 1e-5
    sim.close()


# --------------------------------------------------------------- trajectories

def _traj_errors(cfg, xa, va, xb, vb):
    d = xa.astype(np.float64) - xb
    d -= cfg["L"] * np.round(d / cfg["L"])
    dx = np.sqrt((d * d).sum(1)).max() / cfg["r_c"]
    vrms = math.sqrt((vb * vb).sum(1).mean())
    dv = np.sqrt(((va - vb) ** 2).sum(1)).max() / vrms
    return dx, dv


def _r32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _oracle_fp32_storage(cfg, x, v, n, flip_seed=None):
    """The oracle advanced one step at a time with its state (x, v, F) stored
    in FP32 between steps, the precision of the engine's state; the oracle's
    arithmetic is untouched.  With flip_seed, every stored coordinate of x
    and v is also moved by one FP32 ulp up or down (at random) after every
    step: the divergence this causes is what FP32 state precision alone
    allows a chaotic trajectory over the same steps."""
    rng = None if flip_seed is None else np.random.default_rng(flip_seed)
    x, v = _r32(x), _r32(v)
    F = _r32(oracle.forces(cfg, x, v, 0))
    s = 0
    for _ in range(n):
        x, v, F, s, _ = oracle.step(cfg, x, v, F, s, 1)
        x, v = np.asarray(x, np.float32), np.asarray(v, np.float32)
        if rng is not None:
            for a in (x, v):
                sgn = rng.choice([-1.0, 1.0], size=a.shape).astype(np.float32)
                a[...] = np.nextafter(a, sgn * np.float32(np.inf))
        x[(x >= np.float32(cfg["L"])) | (x < 0)] = 0.0
        x, v, F = x.astype(np.float64), v.astype(np.float64), _r32(F)
    return x, v


def _gpu_trajectory(dpd, cfg, x, v, n):
    """GPU states (x, v, F) after each of n steps from (x, v) at step 0."""
    sim = make_sim(dpd, cfg, x, v)
    out = []
    for _ in range(n):
        sim.step(1)
        xs, vs, Fs, _ = sim.get_state()
        out.append((host(xs), host(vs), host(Fs)))
    sim.close()
    return out


def _half_ulp(a):
    a = np.abs(np.asarray(a, np.float32))
    return 0.5 * (np.nextafter(a, np.float32(np.inf)) - a).astype(np.float64)


@pytest.mark.parametrize("gamma", [4.5, 0.0])
def test_trajectory_100_steps(dpd, gamma):
    """100 steps of the 1600-particle workload, two ways.
    Each step: the oracle's step from the GPU's previous state (x_k, v_k, F_k),
    whose FP64 drift the GPU must round correctly (position within half an
    FP32 ulp), whose force at the GPU's new state (x_k+1, u) must match the
    GPU's within 1e-5 S_i, and whose second half kick then bounds the GPU's
    velocity by dt/(2m) 1e-5 S_i plus half an ulp.  No chaos enters: every
    bound follows from FP32 state storage and the force tolerance.
    End point: the GPU against the oracle run with the same FP32 state
    storage, within the divergence that FP32 precision alone allows (the
    same oracle with one ulp of noise on every stored coordinate at every
    step; the smallest of three seeds)."""
    cfg = dict(C1, gamma=gamma)
    L, dt = cfg["L"], cfg["dt"]
    h32 = float(np.float32(dt / (2.0 * cfg["mass"])))
    x, v = inputs.initial_state(cfg)
    traj = _gpu_trajectory(dpd, cfg, x, v, 100)
    worst = [0.0, 0.0, 0.0]
    for k in range(99):
        xk, vk, Fk = (a.astype(np.float64) for a in traj[k])
        xn, vn, Fn = traj[k + 1]
        u = _r32(vk + h32 * Fk)  # the engine's FP32 half-step velocity
        y = xk + dt * u
        y -= L * np.floor(y / L)
        d = xn.astype(np.float64) - y
        d -= L * np.round(d / L)
        worst[0] = max(worst[0], float((np.abs(d) / (_half_ulp(y) * (1 + 1e-9) + 1e-30)).max()))
        Fo = oracle.forces(cfg, xn, u, k + 2)
        _, S = oracle.force_parts(cfg, xn, u, k + 2)
        worst[1] = max(worst[1], float((np.sqrt(((Fn - Fo) ** 2).sum(1)) / S).max()))
        vo = u + h32 * Fo
        tol_v = h32 * 1e-5 * S[:, None] + _half_ulp(vo)
        worst[2] = max(worst[2], float((np.abs(vn - vo) / tol_v).max()))
    print(f"gamma={gamma}: per step, worst position / (ulp/2) {worst[0]:.3f}, force / S_i "
          f"{worst[1]:.2e}, velocity / bound {worst[2]:.3f}")
    assert worst[0] <= 1.0 and worst[1] <= 1e-5 and worst[2] <= 1.0

    xr, vr = _oracle_fp32_storage(cfg, x, v, 100)
    ex, ev = _traj_errors(cfg, traj[-1][0], traj[-1][1], xr, vr)
    yard = [_traj_errors(cfg, *_oracle_fp32_storage(cfg, x, v, 100, flip_seed=sd), xr, vr)
            for sd in (1, 2, 3)]
    yx, yv = min(a[0] for a in yard), min(a[1] for a in yard)
    print(f"gamma={gamma}: step 100, GPU - FP32-storage oracle dx={ex:.2e} dv={ev:.2e}; "
          f"one-ulp-per-step yardstick dx={yx:.2e} dv={yv:.2e}")
    assert ex <= yx and ev <= yv


def test_run_to_run_bitwise_and_resume(dpd):
    cfg = C1
    x, v = inputs.initial_state(cfg, thermal=True)
    a = make_sim(dpd, cfg, x, v)
    a.step(60)
    xa, va, Fa, sa = [t if isinstance(t, int) else host(t) for t in a.get_state()]
    b = make_sim(dpd, cfg, x, v)
    b.step(60)
    xb, vb, Fb, sb = [t if isinstance(t, int) else host(t) for t in b.get_state()]
    assert (xa == xb).all() and (va == vb).all() and (Fa == Fb).all() and sa == sb == 60
    # 30 + 30 from a checkpoint equals 60 in one go
    c = make_sim(dpd, cfg, x, v)
    c.step(30)
    xc, vc, Fc, sc = c.get_state()
    d = make_sim(dpd, cfg, host(xc), host(vc), step=sc, F=host(Fc))
    d.step(30)
    xd, vd, Fd, sd = [t if isinstance(t, int) else host(t) for t in d.get_state()]
    assert sd == 60
    assert (xd == xa).all() and (vd == va).all() and (Fd == Fa).all()
    # and 1 + 59 split inside one handle
    e = make_sim(dpd, cfg, x, v)
    e.step(1)
    e.step(59)
    xe = host(e.get_state()[0])
    assert (xe == xa).all()
    for s in (a, b, c, d, e):
        s.close()


@pytest.mark.parametrize("between", ["nothing", "forces", "bin_velocity_windows",
                                     "bin_velocity_plain", "get_state"])
def test_split_steps_bitwise(dpd, between):
    # a dpd_step call leaves the next step's half kick and drift prepared; the
    # next call starts from it, and every other entry point either leaves it
    # alone or drops it: either way 5 + 5 steps equal 10 steps bit for bit
    cfg = C1
    x, v = inputs.initial_state(cfg, thermal=True)
    ref = make_sim(dpd, cfg, x, v)
    ref.step(10)
    xr, vr, Fr, sr = (host(t) if not isinstance(t, int) else t for t in ref.get_state())
    sim = make_sim(dpd, cfg, x, v)
    sim.step(5)
    if between == "forces":
        sim.forces()
    elif between == "bin_velocity_windows":
        sim.bin_velocity(16, 7.5, 0)
    elif between == "bin_velocity_plain":
        sim.bin_velocity(40, 0.0, 0)
    elif between == "get_state":
        sim.get_state()
    sim.step(5)
    xs, vs, Fs, ss = sim.get_state()
    assert ss == sr == 10
    assert (host(xs) == xr).all() and (host(vs) == vr).all() and (host(Fs) == Fr).all()
    ref.close()
    sim.close()


@pytest.mark.parametrize("skin,kind,steps,L,n_agents", [
    (0.3, "random", 300, 40.0, 800), (0.6, "random", 300, 40.0, 800), (0.3, "edge", 200, 40.0, 800),
    (0.35, "random", 200, 47.0, 1104),
    # density 3 (softer repulsion, so that the random start does not tear
    # bonds): every tile overflows the LDS capacities, on rebuild steps and
    # between them (global-memory path with the slots of the last rebuild)
    (0.3, "dense", 60, 23.0, 800)])
def test_skin_trajectory_bitwise(dpd, skin, kind, steps, L, n_agents):
    # With a Verlet skin the cells are r_c + skin wide and the steps between
    # rebuilds test only the pairs listed at the last rebuild.  The pair set
    # within r_c is the same and the pair sums are exact, so the trajectory is
    # bitwise the one of the path that rebuilds every step with r_c-wide cells.
    cfg = dict(C1, L=L, n_agents=n_agents)
    if kind == "dense":
        cfg["A"] = 5.0
        kind = "random"
    x, v = inputs.initial_state(cfg, kind=kind, thermal=True)
    ref = make_sim(dpd, cfg, x, v)
    sk = make_sim(dpd, dict(cfg, skin=skin), x, v)
    half = steps // 2
    pr = [host(ref.step(half, reduce_every=half)), host(ref.step(steps - half, reduce_every=steps - half))]
    ps = [host(sk.step(half, reduce_every=half)), host(sk.step(steps - half, reduce_every=steps - half))]
    a, b = ref.get_state(), sk.get_state()
    assert a[3] == b[3] == steps
    for k in range(3):
        assert (host(a[k]) == host(b[k])).all(), ("x", "v", "F")[k]
    for p, q in zip(pr, ps):  # the FP64 sums run in another order
        assert q == pytest.approx(p, rel=1e-12, abs=1e-9)
    nreb = sk.rebuilds()
    print(f"skin {skin} {kind}: {nreb} rebuilds in {steps} steps")
    assert ref.rebuilds() == 0
    assert 2 <= nreb < steps // 2  # the lists were used
    ref.close()
    sk.close()


def test_skin_forces_and_bins(dpd):
    # the force call and the binned field with a skin, against the oracle
    cfg = dict(C1, skin=0.4)
    x, v = inputs.initial_state(cfg, thermal=True)
    sim = make_sim(dpd, cfg, x, v)
    sim.step(50)
    xs, vs, _, step = sim.get_state()
    xs, vs = host(xs), host(vs)
    F = host(sim.forces())
    per, glob = force_errors(cfg, xs, vs, step, F)
    assert per.max() <= 1e-5 and glob <= 1e-5
    sim.step(7)
    xs, vs, _, _ = sim.get_state()
    u, n = sim.bin_velocity(40, 0.0, 0)
    uo, no = oracle.bin_velocity(cfg, host(xs), host(vs), 40, 0.0, 0)
    assert (host(n) == no).all()
    sim.close()


def test_momentum_conserved_on_gpu(dpd):
    cfg = dict(C1, f_sp=0.0, gamma_s=0.0)
    x, v = inputs.initial_state(cfg, thermal=True)
    sim = make_sim(dpd, cfg, x, v)
    pk = host(sim.step(1000, reduce_every=10))
    P0 = oracle.momentum_ke(cfg, v.astype(np.float64))
    scale = np.abs(v).sum()
    assert np.abs(pk[:, :2] - P0[:2]).max() <= 1e-5 * scale
    sim.close()


def test_dense_cluster_steps(dpd):
    # a dense cluster overflows the LDS capacities of its tiles, which then take
    # the global-memory kernel in the step, final and force modes; the pair sums
    # are exact in both kernels, so momentum is conserved and the forces of the
    # stepped state match the oracle
    cfg = dict(C1, f_sp=0.0, gamma_s=0.0)
    x, v = inputs.initial_state(cfg, kind="clustered", thermal=True)
    sim = make_sim(dpd, cfg, x, v)
    pk = host(sim.step(6, reduce_every=3))
    P0 = oracle.momentum_ke(cfg, v.astype(np.float64))
    assert np.abs(pk[:, :2] - P0[:2]).max() <= 1e-5 * np.abs(v).sum()
    xs, vs, _, step = sim.get_state()
    xs, vs = host(xs), host(vs)
    v64 = vs.astype(np.float64)
    ref = [math.fsum(v64[:, 0]), math.fsum(v64[:, 1]), 0.5 * math.fsum((v64 * v64).sum(1))]
    assert pk[-1] == pytest.approx(ref, rel=1e-12, abs=1e-12)
    F = host(sim.forces())
    per, glob = force_errors(cfg, xs, vs, step, F)
    assert per.max() <= 1e-5 and glob <= 1e-5, (per.max(), glob)
    sim.close()


def test_large_capacity_retry_path(dpd):
    # at 1.6 particles per cell, 8 x 8 tiles hold about 102 tile particles and
    # 160 staged ones: over the fast kernel's LDS capacities (96 / 128) but
    # within the large ones its overflow kernel tries first, so nearly every
    # tile runs there.  Forces match the oracle, and the trajectory is bitwise
    # the one of 4 x 4 tiles, which stay in the fast kernel.
    n_agents = 2560
    cfg = dict(C1, n_agents=n_agents, L=40.0, seed=23, tile=8)
    x, v = inputs.initial_state(cfg, thermal=True)
    a = make_sim(dpd, cfg, x, v, step=5)
    F = host(a.forces())
    per, glob = force_errors(cfg, x, v, 5, F)
    assert per.max() <= 1e-5 and glob <= 1e-5, (per.max(), glob)
    b = make_sim(dpd, dict(cfg, tile=4), x, v, step=5)
    assert (host(b.forces()) == F).all()
    pa = host(a.step(60, reduce_every=20))
    pb = host(b.step(60, reduce_every=20))
    sa = [host(t) for t in a.get_state()[:3]]
    sb = [host(t) for t in b.get_state()[:3]]
    for u, w in zip(sa, sb):
        assert (u == w).all()
    # the FP64 reductions run over other tiles, so only to rounding
    assert pa == pytest.approx(pb, rel=1e-12, abs=1e-12)
    a.close()
    b.close()


def test_far_bond_partner_by_id(dpd):
    # the paper's geometry: the bond (l = 1) reaches beyond the 3 x 3 stencil
    # of r_c-wide cells (r_c = 0.5), so the partner is read by id.  Forces match
    # the oracle for a random state (fast kernel) and for a dense cluster (the
    # overflow kernel's paths), and a batch of them steps bitwise like single
    # handles.  The replicas' sizes (1606, 22 and 2400 particles) put replica
    # boundaries inside wavefronts, two of them inside one, for the map from
    # input index to replica that the partner lookup is built with
    base = dict(C1, r_c=0.5, bond_l=1.0, A=1.5, kT=0.05, dt=0.003, L=40.0)
    cases = [(dict(base, n_agents=803, seed=31), "random"), (dict(base, n_agents=11, seed=33), "random"),
             (dict(base, n_agents=1200, seed=32), "clustered")]
    singles = []
    for cfg, kind in cases:
        x, v = inputs.initial_state(cfg, kind=kind, thermal=True)
        sim = make_sim(dpd, cfg, x, v, step=4)
        F = host(sim.forces())
        per, glob = force_errors(cfg, x, v, 4, F)
        print(f"far bond, {kind}: max per-particle error {per.max():.2e}, global {glob:.2e}")
        assert per.max() <= 1e-5 and glob <= 1e-5, (kind, per.max(), glob)
        sim.step(40)
        singles.append([host(t) for t in sim.get_state()[:3]])
        sim.close()
    states = [inputs.initial_state(c, kind=k, thermal=True) for c, k in cases]
    b = dpd.Sim([c for c, _ in cases], device=DEV)
    b.set_state(dev(np.concatenate([s_[0] for s_ in states])), dev(np.concatenate([s_[1] for s_ in states])), 4)
    b.step(40)
    got = [host(t) for t in b.get_state()[:3]]
    o = 0
    for q, (c, _) in enumerate(cases):
        n = 2 * c["n_agents"]
        for u, w in zip(got, singles[q]):
            assert (u[o:o + n] == w).all(), q
        o += n
    b.close()


def test_dense_cluster_reductions_run_to_run(dpd):
    # tiles of a dense cluster take the global-memory kernel, whose lanes take
    # the members of each tile in canonical order: the FP64 momentum and
    # kinetic-energy sums, like the states, are bitwise the same in every run
    # (the slot order the members arrive in comes from atomic ranks and varies)
    cfg = dict(C1, f_sp=0.0, gamma_s=0.0)
    x, v = inputs.initial_state(cfg, kind="clustered", thermal=True)
    runs = []
    for _ in range(3):
        sim = make_sim(dpd, cfg, x, v)
        pk = host(sim.step(30, reduce_every=1))
        xs, vs, _, _ = sim.get_state()
        runs.append((pk, host(xs), host(vs)))
        sim.close()
    for pk, xs, vs in runs[1:]:
        assert (pk == runs[0][0]).all()
        assert (xs == runs[0][1]).all() and (vs == runs[0][2]).all()


def test_stokes_momentum_decay_on_gpu(dpd):
    cfg = dict(C1, f_sp=0.0, gamma_s=0.8)
    x, v = inputs.initial_state(cfg, thermal=True)
    v = (v + np.float32(0.75)).astype(np.float32)
    sim = make_sim(dpd, cfg, x, v)
    pk = host(sim.step(400, reduce_every=1))
    P0 = oracle.momentum_ke(cfg, v.astype(np.float64))[:2]
    c = cfg["gamma_s"] * cfg["dt"] / 2
    n = np.arange(1, 401)
    expect = P0[None, :] * ((1 - c) ** 2 * (1 - 2 * c) ** (n - 1))[:, None]
    assert np.abs(pk[:, :2] - expect).max() <= 1e-5 * np.abs(v).sum()
    sim.close()


@pytest.mark.parametrize("split", [0, 1])
def test_isolated_dimer_terminal_velocity_on_gpu(dpd, split):
    cfg = dict(C1, n_agents=1, L=20.0, gamma_s=5.0, sp_split=split)
    th = 0.7
    x = np.array([[10 + 0.25 * math.cos(th), 10 + 0.25 * math.sin(th)],
                  [10 - 0.25 * math.cos(th), 10 - 0.25 * math.sin(th)]], np.float32)
    sim = make_sim(dpd, cfg, x, np.zeros_like(x))
    sim.step(3000)
    _, vs, _, _ = sim.get_state()
    vs = host(vs).astype(np.float64)
    vt = cfg["f_sp"] / (2 * cfg["gamma_s"])
    com = 0.5 * (vs[0] + vs[1])
    assert com == pytest.approx(vt * np.array([math.cos(th), math.sin(th)]), abs=1e-6)
    sim.close()


def test_reductions_are_exact_sums(dpd):
    cfg = C1
    x, v = inputs.initial_state(cfg, thermal=True)
    sim = make_sim(dpd, cfg, x, v)
    pk = host(sim.step(25, reduce_every=25))
    _, vs, _, _ = sim.get_state()
    vs = host(vs).astype(np.float64)
    ref = [math.fsum(vs[:, 0]), math.fsum(vs[:, 1]), 0.5 * math.fsum((vs * vs).sum(1))]
    assert pk[0] == pytest.approx(ref, rel=1e-12, abs=1e-12)
    sim.close()


def test_fluctuation_dissipation_on_gpu(dpd):
    # the oracle's pin in the same 80 x 80 box at density 1 (a smaller box keeps
    # wandering by a few percent), with three seeds and 100 time units each after
    # 50 units of relaxation from the random start
    Ts = []
    for seed in (102, 103, 104):
        cfg = dict(C1, f_sp=0.0, gamma_s=0.0, seed=seed, L=80.0, n_agents=3200)
        x, v = inputs.initial_state(cfg, thermal=True)
        sim = make_sim(dpd, cfg, x, v)
        sim.step(10000)
        pk = host(sim.step(20000, reduce_every=10))
        n = 2 * cfg["n_agents"]
        Ts.append(2 * pk[:, 2].mean() / (2 * n - 2))
        sim.close()
    print("kinetic temperatures", Ts)
    assert np.mean(Ts) == pytest.approx(C1["kT"], rel=0.005)


@pytest.mark.parametrize("w_exp", [0.5, 1.0])
def test_fluctuation_dissipation_weight_exponent(dpd, w_exp):
    # with the dissipative weight w^s and the random weight w^(s/2) the pair
    # thermostat still satisfies fluctuation-dissipation: T_kin -> kT
    Ts = []
    for seed in (105, 106):
        cfg = dict(C1, f_sp=0.0, gamma_s=0.0, seed=seed, L=80.0, n_agents=3200, w_exp=w_exp)
        x, v = inputs.initial_state(cfg, thermal=True)
        sim = make_sim(dpd, cfg, x, v)
        sim.step(6000)
        pk = host(sim.step(12000, reduce_every=10))
        n = 2 * cfg["n_agents"]
        Ts.append(2 * pk[:, 2].mean() / (2 * n - 2))
        sim.close()
    print(f"w_exp {w_exp}: kinetic temperatures", Ts)
    assert np.mean(Ts) == pytest.approx(C1["kT"], rel=0.01)


# ----------------------------------------------------------- velocity field

@pytest.mark.parametrize("M,eps,mode", [(40, 0.0, 0), (64, 0.0, 1), (16, 7.5, 0), (10, 12.0, 1),
                                        (1, 0.0, 0)])
def test_bin_velocity_matches_oracle(dpd, M, eps, mode):
    cfg = C1
    x, v = inputs.initial_state(cfg, thermal=True)
    sim = make_sim(dpd, cfg, x, v)
    sim.step(5)
    xs, vs, _, _ = sim.get_state()
    xs, vs = host(xs), host(vs)
    u, n = sim.bin_velocity(M, eps, mode)
    uo, no = oracle.bin_velocity(cfg, xs, vs, M, eps, mode)
    assert (host(n) == no).all()
    q = 2.0 ** -min(32, 46 - math.ceil(math.log2(len(x) // (1 + mode) + 1)))
    err = np.abs(host(u).astype(np.float64) - uo)
    assert (err <= q + 2.0 ** -23 * np.abs(uo)).all()
    sim.close()


@pytest.mark.parametrize("how", ["set_state_with_F", "after_forces", "edge_layout"])
def test_bin_velocity_row_path_every_entry(dpd, how):
    # plain particle bins are read straight from the stored (cell, id) order;
    # check them after every way of reaching a stored state
    cfg = C1
    kind = "edge" if how == "edge_layout" else "random"
    x, v = inputs.initial_state(cfg, kind=kind, thermal=True)
    sim = make_sim(dpd, cfg, x, v)
    sim.step(3)
    xs, vs, Fs, step = sim.get_state()
    if how == "set_state_with_F":
        sim.set_state(xs, vs, step, Fs)
    elif how == "after_forces":
        sim.forces()
    for M in (40, 64, 7):
        u, n = sim.bin_velocity(M, 0.0, 0)
        uo, no = oracle.bin_velocity(cfg, host(xs), host(vs), M, 0.0, 0)
        assert (host(n) == no).all()
        q = 2.0 ** -min(32, 46 - math.ceil(math.log2(len(x) + 1)))
        assert (np.abs(host(u).astype(np.float64) - uo) <= q + 2.0 ** -23 * np.abs(uo)).all()
    sim.close()


def test_bin_velocity_full_size(dpd):
    cfg = C3
    x, v = inputs.initial_state(cfg, thermal=True)
    sim = make_sim(dpd, cfg, x, v)
    u, n = sim.bin_velocity(256, 0.0, 0)
    uo, no = oracle.bin_velocity(cfg, x, v, 256, 0.0, 0)
    assert (host(n) == no).all()
    assert np.abs(host(u) - uo).max() <= 1e-6
    sim.close()


# ------------------------------------------------------------- error paths

def test_error_paths(dpd):
    cfg = C1
    x, v = inputs.initial_state(cfg)
    sim = dpd.Sim(cfg, device=DEV)
    with pytest.raises(dpd.DPDError) as e:
        sim.step(1)
    assert e.value.code == -5
    with pytest.raises(dpd.DPDError) as e:
        sim.forces()
    assert e.value.code == -5
    bad = x.copy()
    bad[17, 0] = np.nan
    sim.set_state(dev(bad), dev(v))
    with pytest.raises(dpd.DPDError) as e:
        sim.sync()
    assert e.value.code == -4
    # a bond stretched across more than one cell width is reported
    far = x.copy()
    far[1] = far[0] + np.float32(2.5)
    far[1] = np.mod(far[1], np.float32(cfg["L"]))
    sim.set_state(dev(far), dev(v))
    with pytest.raises(dpd.DPDError) as e:
        sim.sync()
    assert e.value.code == -6
    # recovery: a good state works again
    sim.set_state(dev(x), dev(v))
    sim.step(3)
    sim.sync()
    # a blow-up (huge time step) is reported as non-finite
    cfg2 = dict(C1, dt=5.0)
    s2 = make_sim(dpd, cfg2, x, v)
    s2.step(30)
    with pytest.raises(dpd.DPDError) as e:
        s2.sync()
    assert e.value.code in (-4, -6)
    sim.close()
    s2.close()
