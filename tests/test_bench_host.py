"""CPU: the benchmark's host logic (no GPU): the one-GPU guard, the kernel
instance a workload's traffic record must name, the source-hash check that
voids a traffic record once the kernels change, and the roofline constants.
"""
import hashlib
import json
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("grid,edge,name", [
    (64, 0, "rv::k_vote_bin<4, false>"),     # one solve: 16^3 bricks up to G = 128
    (128, 0, "rv::k_vote_bin<4, false>"),
    (129, 0, "rv::k_vote_bin<5, false>"),
    (256, 0, "rv::k_vote_bin<5, false>"),
    (257, 0, "rv::k_vote_bin<5, true>"),     # wide run layout above 256
    (360, 0, "rv::k_vote_bin<5, true>"),
    (64, 32, "rv::k_vote_bin<5, false>"),    # a batch names its tuned edge
    (64, 16, "rv::k_vote_bin<4, false>"),
])
def test_vote_kernel_name(grid, edge, name):
    assert bench.vote_kernel_name(grid, edge) == name
    # the key strategy has one kernel instance (the source's configuration)
    assert bench.vote_kernel_name(grid, edge, "keys") == bench.KEY_VOTE_KERNEL
    src = (ROOT / "paper_2506_11547_amd" / "csrc" / "rv_bin.hip").read_text()
    assert "using Keys = KeyPack<16, 32, 1>;" in src


def make_record(tmp_path, workload, kernel, digests):
    rec = {"kernel": kernel, "workload": workload, "fetch_kib_per_dispatch": 1.0,
           "write_kib_per_dispatch": 2.0, "fetch_scale": 2.0, "write_scale": 1.0,
           "sources_sha256": digests, "traffic_bytes_per_launch": 4096.0}
    p = tmp_path / f"{workload}.json"
    p.write_text(json.dumps(rec))
    return p


def test_traffic_record_follows_the_sources(tmp_path, monkeypatch):
    src = "paper_2506_11547_amd/csrc/rv_bin.hip"
    good = {src: hashlib.sha256((ROOT / src).read_bytes()).hexdigest()}
    kernel = "rv::k_vote_bin<5, false>"
    monkeypatch.setitem(bench.TRAFFIC_RECORDS, "large",
                        [make_record(tmp_path, "large", kernel, good)])
    assert bench.measured_traffic("large", kernel) == 4096.0
    # another kernel instance or workload than the record's: no figure
    assert bench.measured_traffic("large", "rv::k_vote_bin<5, true>") is None
    assert bench.measured_traffic("medium", kernel) is None
    # the record of the kernel the solve ran, among the workload's records
    keys = tmp_path / "keys"
    keys.mkdir()
    monkeypatch.setitem(bench.TRAFFIC_RECORDS, "large",
                        [tmp_path / "missing.json", make_record(keys, "large", bench.KEY_VOTE_KERNEL, good),
                         make_record(tmp_path, "large", kernel, good)])
    assert bench.measured_traffic("large", kernel) == 4096.0
    assert bench.measured_traffic("large", bench.KEY_VOTE_KERNEL) == 4096.0
    # a source changed since the profile: no figure
    monkeypatch.setitem(bench.TRAFFIC_RECORDS, "large",
                        [make_record(tmp_path, "large", kernel, {src: "0" * 64})])
    assert bench.measured_traffic("large", kernel) is None
    # an unreadable record: no figure
    monkeypatch.setitem(bench.TRAFFIC_RECORDS, "large", [tmp_path / "missing.json"])
    assert bench.measured_traffic("large", kernel) is None
    # the committed records are the workloads' bin and key profiles
    assert bench.TRAFFIC_RECORDS["paper_default"][1].name == "vote_keys__paper_default_traffic.json"


def test_roofline_constants():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit operation per lane per clock
    assert bench.ALU_PEAK_GOPS == pytest.approx(39321.6)
    assert bench.HBM_PEAK_GBS == 8000.0
    # the rule's operations per sample: 4 mul + 4 fma, 1 sign test, 1 add + 1
    # reciprocal + 1 mul, 3 fma + 3 floor + 6 clamp compares + 2 index
    # multiply-adds, 1 vote add
    assert bench.OPS_PER_SAMPLE == 4 + 4 + 1 + 1 + 1 + 1 + 3 + 3 + 6 + 2 + 1
