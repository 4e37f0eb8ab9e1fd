"""The C-ABI library loads, exports every entry point include/dpd.h declares,
and its host-only paths (parameter validation, workspace sizing) behave.
CPU only: no call here launches a kernel."""
import ctypes
import os
import re

import pytest

from paper_1310_0998_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpd.h")


@pytest.fixture(scope="module")
def dpd():
    from paper_1310_0998_amd import build as b
    if not os.path.exists(b.LIB):
        b.build(force=True)
    from paper_1310_0998_amd import dpd as d
    d.lib()
    return d


def declared_functions(path=None):
    names = []
    paths = [path] if path else sorted(
        os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    for hp in paths:
        text = open(hp).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+\**\s*(dpd_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions(HEADER)
    for required in ("dpd_create", "dpd_set_state", "dpd_forces", "dpd_step", "dpd_bin_velocity",
                     "dpd_get_state", "dpd_destroy", "dpd_last_error", "dpd_workspace_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol(dpd):
    lib = ctypes.CDLL(dpd.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_params_struct_layout_matches_header(dpd):
    # 1 int64 + 11 doubles + 1 uint64 + 5 int32 + 2 floats + 1 reserved int32 = 128 bytes
    assert ctypes.sizeof(dpd.Params) == 8 + 11 * 8 + 8 + 8 * 4


def test_workspace_and_cells(dpd):
    cfg = inputs.physics(inputs.WORKLOADS["dimers_1600"])
    assert dpd.cells_per_side(cfg) == 40
    n = dpd.workspace_bytes(cfg)
    assert n > 1600 * 100
    big = inputs.physics(inputs.WORKLOADS["dimers_4M"])
    assert dpd.cells_per_side(big) == 2000
    assert dpd.workspace_bytes(big) < 2 * 1024 ** 3
    assert dpd.cells_per_side(dict(cfg, L=7.25, r_c=1.1)) == 6
    # a bond longer than the cutoff keeps cells of width r_c (its partner is
    # read by id), but refuses a Verlet skin too narrow to hold it
    assert dpd.cells_per_side(dict(cfg, L=100.0, r_c=0.5, bond_l=1.0)) == 200
    with pytest.raises(dpd.DPDError):
        dpd.workspace_bytes(dict(cfg, L=100.0, r_c=0.5, bond_l=1.0, skin=0.2))


@pytest.mark.parametrize("bad", [
    dict(n_agents=0), dict(L=2.5), dict(L=40.1), dict(r_c=0.0), dict(dt=0.0), dict(mass=-1.0),
    dict(gamma=-1.0), dict(kT=float("nan")), dict(noise_kind=2), dict(rng_kind=5), dict(sp_split=3),
    dict(tile=99), dict(bin_M_max=-1), dict(w_exp=-1.0), dict(w_exp=9.0), dict(w_exp=float("nan")),
])
def test_invalid_parameters_rejected(dpd, bad):
    cfg = dict(inputs.physics(inputs.WORKLOADS["dimers_1600"]), **bad)
    with pytest.raises(dpd.DPDError) as ei:
        dpd.workspace_bytes(cfg)
    assert ei.value.code == -1
    assert len(dpd.lib().dpd_last_error(None)) > 0


def test_create_rejects_bad_workspace(dpd):
    cfg = inputs.physics(inputs.WORKLOADS["dimers_1600"])
    p = dpd.make_params(cfg)
    h = ctypes.c_void_p()
    lib = dpd.lib()
    assert lib.dpd_create(ctypes.byref(p), None, 0, None, ctypes.byref(h)) == -2
    assert lib.dpd_create(ctypes.byref(p), ctypes.c_void_p(256 * 1000 + 8), 10 ** 9, None,
                          ctypes.byref(h)) == -2          # misaligned
    need = dpd.workspace_bytes(cfg)
    assert lib.dpd_create(ctypes.byref(p), ctypes.c_void_p(256 * 1000), need - 1, None,
                          ctypes.byref(h)) == -2          # too small
    assert b"needs" in lib.dpd_last_error(None)
    assert h.value is None


def test_null_handle_calls_fail_cleanly(dpd):
    lib = dpd.lib()
    assert lib.dpd_step(None, 1, 0, None) == -1
    assert lib.dpd_forces(None, None) == -1
    assert lib.dpd_set_state(None, None, None, 0, None) == -1
    assert lib.dpd_sync(None) == -1
    lib.dpd_destroy(None)


def test_batch_workspace_and_validation(dpd):
    c1 = inputs.physics(inputs.WORKLOADS["dimers_1600"])
    one = dpd.workspace_bytes(c1)
    assert dpd.workspace_bytes([c1]) == one
    two = dpd.workspace_bytes([c1, dict(c1, n_agents=300, L=23.0)])
    assert two > one
    sweep = [inputs.physics(c) for c in inputs.sweep_replicas()]
    assert len(sweep) == 64
    assert dpd.workspace_bytes(sweep) < 2 * 1024 ** 3
    with pytest.raises(dpd.DPDError) as ei:
        dpd.workspace_bytes([c1, dict(c1, skin=0.3)])  # no skin in a batch
    assert ei.value.code == -1
    with pytest.raises(dpd.DPDError) as ei:
        dpd.workspace_bytes([c1, dict(c1, L=2.5)])     # a bad replica names itself
    assert b"replica 1" in dpd.lib().dpd_last_error(None)
    lib = dpd.lib()
    n = ctypes.c_size_t(0)
    assert lib.dpd_batch_workspace_bytes(ctypes.byref(dpd.make_params(c1)), 0, ctypes.byref(n)) == -1


def test_null_handle_batch_calls_fail_cleanly(dpd):
    lib = dpd.lib()
    i = ctypes.c_int32(0)
    assert lib.dpd_set_graph_chunk(None, 8) == -1
    assert lib.dpd_set_schedule(None, 8, 7, 0) == -1
    assert lib.dpd_get_schedule(None, ctypes.byref(i), ctypes.byref(i), ctypes.byref(i)) == -1
    assert lib.dpd_autotune(None, 4, None, None, None, None) == -1


def test_sweep_replicas_recipe():
    # seeded, log-uniform sizes in range, the 16-point grid four times over,
    # boxes exactly representable in FP32 at areal density 2 phi
    import numpy as np
    a = inputs.sweep_replicas()
    assert a == inputs.sweep_replicas()
    na = np.array([c["n_agents"] for c in a])
    assert na.min() >= 2000 and na.max() <= 64000
    grid = {(c["phi"], c["ratio"]) for c in a}
    assert len(grid) == 16
    for c in a:
        assert float(np.float32(c["L"])) == c["L"]
        rho = 2 * c["n_agents"] / c["L"] ** 2
        assert abs(rho / (2 * c["phi"]) - 1) < 1e-3
        assert c["gamma"] == 4.5 and abs(c["gamma"] / c["gamma_s"] - c["ratio"]) < 1e-12


def test_closure_header_and_validation(dpd):
    names = declared_functions(os.path.join(ROOT, "include", "closure.h"))
    for required in ("dpd_nn_create", "dpd_nn_forward", "dpd_nn_gradient", "dpd_nn_adam",
                     "dpd_nn_train_step", "dpd_nn_rollout", "dpd_nn_destroy"):
        assert required in names
    from paper_1310_0998_amd import closure as cl
    from oracle import closure as oc
    assert cl.param_count(64, 4, 32, 4) == oc.param_count(4, 32, 4) == 20258
    lib = cl.lib()
    n = ctypes.c_size_t(0)
    for bad in (dict(M=6), dict(M=0), dict(c_in=3), dict(c_in=36), dict(width=24), dict(layers=0),
                dict(layers=9), dict(max_batch=0)):
        kw = dict(M=64, c_in=4, width=32, layers=4, max_batch=8)
        kw.update(bad)
        assert lib.dpd_nn_workspace_bytes(ctypes.byref(cl.make_params(**kw)), ctypes.byref(n)) == -1
        assert len(lib.dpd_nn_last_error(None)) > 0
    assert lib.dpd_nn_workspace_bytes(ctypes.byref(cl.make_params(64, 4, 32, 4, 8)), ctypes.byref(n)) == 0
    assert lib.dpd_nn_forward(None, None, None, 1, None) == -1
    assert lib.dpd_nn_rollout(None, None, None, 1, 1, None, None, 0, 1, None) == -1
