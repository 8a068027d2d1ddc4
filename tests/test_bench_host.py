"""Host logic of the benchmark (no GPU): the one-GPU rule, the roofline
arithmetic, the hash-gated traffic figure, and the kernel-family table
against the C header's family enum."""
import json
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_family_table_matches_header():
    text = open(os.path.join(ROOT, "include", "isdf.h")).read()
    enum = dict((k, int(v)) for k, v in re.findall(r"ISDF_K_([A-Z_]+) = (\d+)", text))
    nfam = enum.pop("NFAMILY")
    assert sorted(enum.values()) == list(range(nfam)) == sorted(bench.FAMILIES)
    assert bench.ALL_FAMILIES == (1 << nfam) - 1
    for name, fam in enum.items():
        assert bench.FAMILIES[fam][0] == name.lower(), (name, bench.FAMILIES[fam])
        assert bench.FAMILIES[fam][1] in ("hbm", "mfma")


def test_roofline_arithmetic(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda fam, config: None)
    # HBM family: 4 launches, 2 ms in all, 4 GB algorithmic -> 1 GB in 0.5 ms = 2000 GB/s
    st = {"ms": 2.0, "launches": 4, "bytes": 4e9, "flops": 0.0}
    r = bench.roofline(6, st, mixed=set())
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["family"] == "fft"
    assert r["achieved"] == pytest.approx(2000.0) and r["peak"] == bench.PEAK_HBM_GBS
    assert r["frac"] == pytest.approx(2000.0 / bench.PEAK_HBM_GBS, abs=1e-4)
    assert r["avg_launch_us"] == pytest.approx(500.0) and r["alg_bytes_per_launch"] == pytest.approx(1e9)
    assert r["mfma_issue_frac"] is None
    # GEMM family in FP64: 2 launches, 1 ms, 4e10 flop -> 40 TFLOP/s against the FP64 peak
    st = {"ms": 1.0, "launches": 2, "bytes": 0.0, "flops": 4e10}
    r = bench.roofline(4, st, mixed=set())
    assert r["unit"] == "TFLOP/s" and r["peak"] == bench.PEAK_FP64_TFS
    assert r["achieved"] == pytest.approx(40.0)
    # the exchange family in BF16 splits is priced against the BF16 peak, six products per flop
    r = bench.roofline(5, st, mixed={5})
    assert r["peak"] == bench.PEAK_BF16_TFS and "gemm_mixed_kernel" in r["kernel"]
    assert r["mfma_issue_frac"] == pytest.approx(6 * 40.0 / bench.PEAK_BF16_TFS, abs=1e-4)


def test_traffic_figure_needs_the_measured_source(tmp_path, monkeypatch):
    """A committed traffic summary is used only while the hash of the
    kernel source it was measured on matches the source in the tree."""
    import hashlib

    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2404_09373_amd" / "csrc").mkdir(parents=True)
    src = open(os.path.join(ROOT, "paper_2404_09373_amd", "csrc", "kernels_fft.hip")).read()
    srcp = tmp_path / "paper_2404_09373_amd" / "csrc" / "kernels_fft.hip"
    srcp.write_text(src)
    sha = hashlib.sha256(srcp.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "traffic_fft_cfg2.md").write_text(
        f"traffic_bytes_per_launch: 2459581000\nkernel_source_sha256: {sha}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(6, 2) == pytest.approx(2459581000.0)
    # it holds for the workload it was measured on only
    assert bench.measured_traffic(6, 5) is None
    # a changed source voids it; families without a summary have none
    srcp.write_text(src + "\n// changed\n")
    assert bench.measured_traffic(6, 2) is None
    assert bench.measured_traffic(0, 2) is None


def test_cpu_baseline_both_exchange_forms():
    """The bounded oracle sample runs for the full K and for K C, and an
    all-point domain (F = I) adds no selection or fit time."""
    import bench
    from workloads import tiny_system

    s = tiny_system("d_atom", grids=((6, 6, 6), (24, 24, 24)), n_occ=3)
    s.n_mu_ratio = 30.0  # the universal domain takes its 216 points
    for ri in (False, True):
        r = bench.cpu_baseline(s, sample_pts=512, ex_scale=1, occ_ri=ri)
        assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] >= 1
        assert ("occ-RI" in r["sample"]) == ri
        assert r["stages_s"]["select"] > 0  # the window still selects
