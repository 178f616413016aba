"""Host-side logic of bench.py (no GPU): the traffic figures recorded in
profiles/ are used only for the kernel family, source hash, workload and
launch shape they were measured on, and the roofline record's arithmetic."""
import os

import pytest

import bench

FILES = {"k_gemm.hip": "gemm v1", "hz_mfma.h": "mfma", "hz_common.h": "common",
         "k_cellsolve.hip": "cells v1", "k_plr.hip": "plr v1"}


@pytest.fixture
def root(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1510_01831_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name, text in FILES.items():
        (csrc / name).write_text(text)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def _summary(root, name, lines):
    (root / "profiles" / name).write_text("# summary\n\n" + "\n".join(lines) + "\n")


def test_source_hash_follows_the_family_sources(root):
    g, c, p = (bench.kernel_src_hash(f) for f in ("gemm_mfma64_c128", "cell_solve_volume_c64",
                                                  "plr_gemv_c128"))
    assert len({g, c, p}) == 3
    assert bench.kernel_src_hash("gemv_c128") == g          # same sources as the GEMMs
    (root / "paper_1510_01831_amd" / "csrc" / "k_plr.hip").write_text("plr v2")
    assert bench.kernel_src_hash("plr_gemv_c128") != p
    assert bench.kernel_src_hash("gemm_mfma64_c128") == g


def test_recorded_traffic_matches_family_hash_workload_and_shape(root):
    src = bench.kernel_src_hash("gemm_mfma64_c128")
    _summary(root, "a.md", [f"traffic: kernel=gemm_mfma64_c128 src={src} workload=C4 "
                            f"alg_bytes=1.000000e+10 bytes_per_launch=1.100000e+10"])
    assert bench.recorded_traffic("gemm_mfma64_c128", "C4", 1.0e10) == 1.1e10
    assert bench.recorded_traffic("gemm_mfma64_c128", "C4", 1.003e10) == 1.1e10   # within 0.5%
    assert bench.recorded_traffic("gemm_mfma64_c128", "C4", 3.0e9) is None        # other shape
    assert bench.recorded_traffic("gemm_mfma64_c128", "C3", 1.0e10) is None       # other workload
    assert bench.recorded_traffic("gemm_mfma32_c128", "C4", 1.0e10) is None       # other family
    # a changed kernel source invalidates the figure
    (root / "paper_1510_01831_amd" / "csrc" / "k_gemm.hip").write_text("gemm v2")
    assert bench.recorded_traffic("gemm_mfma64_c128", "C4", 1.0e10) is None


def test_recorded_traffic_without_shape_applies_to_any_launch(root):
    src = bench.kernel_src_hash("cell_solve_volume_c128")
    _summary(root, "b.md", [f"traffic: kernel=cell_solve_volume_c128 src={src} workload=C4 "
                            f"bytes_per_launch=9.000000e+10"])
    assert bench.recorded_traffic("cell_solve_volume_c128", "C4", 1.2e11) == 9.0e10
    assert bench.recorded_traffic("cell_solve_volume_c128", "C4") == 9.0e10


def test_roofline_record(root):
    k = {"name": "gemm_mfma64_c128", "launches": 4, "ms": 20.0, "bytes": 8e9, "flops": 2e14}
    r = bench.roofline(k, 64, "C4")
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["avg_launch_ms"] == pytest.approx(5.0)
    assert r["achieved"] == pytest.approx(2e14 / 20e-3 / 1e12)
    assert r["frac"] == pytest.approx(2e14 / 20e-3 / 78.6e12)
    assert r["executed_frac"] == pytest.approx(0.75 * r["frac"])
    assert r["traffic"] is None
    g = {"name": "gemv_c64", "launches": 2, "ms": 1.0, "bytes": 4e9, "flops": 2e9}
    r = bench.roofline(g, 1, "C4")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4e9 / 1e-3 / 1e9)
    assert r["frac"] == pytest.approx(4e9 / 1e-3 / 8e12)
