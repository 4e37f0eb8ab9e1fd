"""Host-side logic of bench.py (no GPU): the algorithmic bytes of the pair
kernel, the gating of the committed counter summaries by the kernel-source
hash, and the JSON sanitising of the closure line."""
import json
import math

import bench


def test_pair_kernel_bytes():
    # 60 B per particle of traffic plus the 4-byte cell_start entries
    assert bench.pair_kernel_bytes(4_000_000, 4_000_000) == 256_000_004
    assert bench.pair_kernel_bytes(0, 0) == 4


def test_committed_counters_match_sources():
    # the committed summaries were taken with the current kernel sources, so
    # the benchmark reports their traffic and VALU figures
    t = bench.measured_traffic()
    assert t is not None and 0.9 * 256e6 < t < 1.5 * 256e6
    v = bench.measured_valu(170.0)
    assert v is not None and 0.0 < v["frac"] < 1.0 and v["peak"] == 256 * 64 * 2.4e9


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
