"""dpd_forces_noalloc (the library's static device scratch in place of a
workspace) against dpd_forces on a handle with its own workspace, through the
C ABI: bitwise equal forces, and within the force tolerance of the oracle, on
two calls in a row, the second with a smaller system."""
import numpy as np
import pytest

import oracle
from paper_1310_0998_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dpd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_0998_amd import dpd as d
    d.lib()
    return d


def _case(n_agents, L, seed):
    cfg = dict(inputs.physics(inputs.WORKLOADS["dimers_1600"]), n_agents=n_agents, L=L, seed=seed)
    x, v = inputs.initial_state(cfg, thermal=True)
    return cfg, x, v


def test_noalloc_forces_equal_workspace_forces_twice(dpd):
    dev = torch.device("cuda:0")
    # the second call is smaller: it must not see the first call's leftovers
    for n_agents, L, seed, step in ((20000, 200.0, 71, 9), (800, 40.0, 72, 3)):
        cfg, x, v = _case(n_agents, L, seed)
        xd, vd = torch.from_numpy(x).to(dev), torch.from_numpy(v).to(dev)
        F_na = dpd.forces_noalloc(cfg, xd, vd, step)
        sim = dpd.Sim(cfg, device=dev)
        sim.set_state(xd, vd, step)
        F_ws = sim.forces()
        sim.close()
        a, b = F_na.cpu().numpy(), F_ws.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), \
            f"{2 * n_agents} particles: noalloc and workspace forces differ"
        Fo = oracle.forces(cfg, x, v, step)
        _, scale = oracle.force_parts(cfg, x, v, step)
        err = np.sqrt(((a.astype(np.float64) - Fo) ** 2).sum(1)) / scale
        print(f"{2 * n_agents} particles: max per-particle error / S_i = {err.max():.2e}")
        assert err.max() <= 1e-5


def test_noalloc_refuses_oversize(dpd):
    cfg = inputs.physics(inputs.WORKLOADS["dimers_4M"])
    dev = torch.device("cuda:0")
    x = torch.zeros((4, 2), dtype=torch.float32, device=dev)
    with pytest.raises(ValueError):
        dpd.forces_noalloc(cfg, x, x)  # shape check in the binding
    lib = dpd.lib()
    import ctypes
    rc = lib.dpd_forces_noalloc(ctypes.byref(dpd.make_params(cfg)), ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(x.data_ptr()), 0, ctypes.c_void_p(x.data_ptr()), None)
    assert rc == -2 and b"static scratch" in lib.dpd_last_error(None)
