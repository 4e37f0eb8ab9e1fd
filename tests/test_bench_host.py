"""Host-side logic of bench.py (no GPU): the algorithmic bytes of the pair
pass and of the fused kernel, the gating of the committed counter summaries by
the kernel-source hash, and the JSON sanitising of the output lines."""
import json
import math

import pytest

import bench


def test_pair_pass_bytes():
    # 32 B per particle at one particle per cell: x 8 + u 8 + id 4 read,
    # F 8 written, cell_start 4 per cell (n_cells + 1 entries)
    assert bench.pair_pass_bytes(4_000_000, 4_000_000) == 128_000_004
    assert bench.pair_pass_bytes(0, 0) == 4


def test_fused_kernel_bytes():
    # 60 B per particle of the fused step kernel, the cell_start entries and
    # the clear of the consumed counter array
    assert bench.fused_kernel_bytes(4_000_000, 4_000_000) == 272_000_004
    assert bench.fused_kernel_bytes(0, 0) == 4


def test_committed_counters_are_sane_when_current():
    # a committed summary taken with the current kernel sources must give
    # plausible figures; one taken with other sources is not used at all
    t = bench.measured_traffic()
    v = bench.measured_valu(100.0)
    if t is None and v is None:
        pytest.skip("no counter summary taken with the current kernel sources")
    if t is not None:
        assert 0.5 * 128e6 < t < 4.0 * 128e6
    if v is not None:
        assert 0.0 < v["frac"] and v["peak"] == 256 * 64 * 2.4e9


def test_profile_fields_reject_other_sources(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "x.txt").write_text("kernel_source_hash: 0000\nhbm_bytes_per_launch: 5\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abcd")
    assert bench._profile_fields("x.txt") is None
    (tmp_path / "profiles" / "y.txt").write_text("kernel_source_hash: abcd\nhbm_bytes_per_launch: 5\n")
    assert bench._profile_fields("y.txt")["hbm_bytes_per_launch"] == "5"
    assert bench._profile_fields("missing.txt") is None


def test_finite_sanitising():
    line = {"a": float("inf"), "b": [1.0, float("nan"), {"c": -float("inf")}], "d": 2}
    out = json.loads(json.dumps(bench._finite(line)))
    assert out == {"a": None, "b": [1.0, None, {"c": None}], "d": 2}
    assert not any(isinstance(x, float) and not math.isfinite(x) for x in out["b"][:2] if x is not None)
