"""Host-side measurement tools: the rocprofv3 summaries behind bench.py's roofline figure and the
algorithmic byte model it divides by (no GPU needed)."""
import csv
import glob
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1703_06999_amd import profiling  # noqa: E402


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Value": value})


def _evaluation(scale):
    """Dispatches of one potential evaluation in launch order, counter values scaled."""
    names = ["void vdwxc::k_theta_zfwd<float, 8, true>(...)", "void vdwxc::k_ypass<float, 8, -1>(...)",
             "void vdwxc::k_xcontract<float, 20, 32, 4>(...)", "void vdwxc::k_ypass<float, 8, 1>(...)",
             "void vdwxc::k_zinv_assemble<float, 4, 4, 1>(...)", "void vdwxc::k_div_z<float, 8>(...)",
             "void vdwxc::k_div_y<float, 8>(...)", "void vdwxc::k_div_x<float, 8>(...)"]
    return [(nm, scale * (k + 1)) for k, nm in enumerate(names)]


def test_traffic_summary_scales_by_the_calibration_kernel(tmp_path):
    # a plain streaming kernel that moves 1 MiB each way reads as 512 KiB fetched, 1024 KiB written
    calib = 1 << 20
    fetch = _evaluation(10.0) + _evaluation(30.0) + [("void at::native::neg_kernel(...)", 512.0)]
    write = _evaluation(1.0) + _evaluation(1.0) + [("void at::native::neg_kernel(...)", 1024.0)]
    _write_counters(tmp_path / "f.csv", fetch)
    _write_counters(tmp_path / "w.csv", write)
    text = profiling.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "t", "cmd1 ;; cmd2", calib)
    assert f"source_sha256: {profiling.source_hash()}" in text
    rows = {}
    for line in text.splitlines():
        if line.startswith("| `"):
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            rows[cells[0]] = float(cells[-1])
    # stage k (1-based) fetched the mean of 10k and 30k KiB = 20k KiB, scaled by 2; wrote k KiB
    for k, stage in enumerate(["theta_zfwd", "y_fwd", "x_contract", "y_inv", "z_assemble", "div_z", "div_y",
                               "div_x"], start=1):
        assert rows[stage] == pytest.approx((2 * 20.0 * k + 1.0 * k) * 1024, rel=1e-9), stage


def test_kernel_stats_lists_library_kernels_only(tmp_path):
    p = tmp_path / "stats.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "MaxNs"])
        w.writeheader()
        w.writerow({"Name": "void vdwxc::k_xcontract<float, 20, 32, 4>(...)", "Calls": 3, "AverageNs": 190000,
                    "MinNs": 180000, "MaxNs": 200000})
        w.writerow({"Name": "void at::native::elementwise_kernel(...)", "Calls": 9, "AverageNs": 1000,
                    "MinNs": 1000, "MaxNs": 1000})
    text = profiling.kernel_stats(str(p), "title", "the command")
    assert "`k_xcontract<float, 20, 32, 4>` | 3 | 190.0 | 180.0 | 200.0 |" in text
    assert "elementwise" not in text and "the command" in text


def test_committed_traffic_profiles_are_consistent():
    """Every committed counter summary is read by bench.py only when it was taken with the kernel
    sources as they are now.  Then the y passes move exactly the field bytes of the byte model
    (within 1 %), and the contraction pass at least them and at most 1.25 times: on top of the
    fields it fetches the kernel table again after L2 evictions (about 3-7 GB per launch at
    512^3).  A summary taken with other sources is reported as None (stale), never as a number."""
    grids = {"slater_128": (128,) * 3, "slater_192": (192,) * 3, "nanoparticle_512": (512,) * 3}
    paths = glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md"))
    assert paths
    current = profiling.source_hash()
    for path in paths:
        name = os.path.basename(path)[len("traffic_"):-len(".md")]
        workload, precision = name.rsplit("_", 1)
        recorded = [line.split(":", 1)[1].strip() for line in open(path) if line.startswith("source_sha256:")]
        t = bench.profiled_traffic(workload, precision, "x_contract")
        if recorded and recorded[0] == current:
            alg = bench.stage_bytes("x_contract", grids[workload], precision)
            assert t is not None and alg <= t <= 1.25 * alg, (name, t, alg)
            ty = bench.profiled_traffic(workload, precision, "y_fwd")
            alg_y = bench.stage_bytes("y_fwd", grids[workload], precision)
            assert ty is not None and abs(ty - alg_y) <= 0.01 * alg_y, (name, ty, alg_y)
        else:
            assert t is None, name


def test_stage_bytes_model():
    g = (8, 6, 10)
    N, Nk = 8 * 6 * 10, 8 * 6 * 6
    assert bench.stage_bytes("y_fwd", g, "fp32") == 2 * 20 * Nk * 8
    assert bench.stage_bytes("y_fwd", g, "fp64") == 2 * 20 * Nk * 16
    assert bench.stage_bytes("div_y", g, "fp32") == 5 * 4 * N
    assert bench.stage_bytes("no_such_stage", g, "fp32") == 0.0


def test_serving_pool_plan_is_greedy_by_size_class():
    """The server's buffer pool: repeatedly the largest work-memory class that still fits the
    budget, at most one buffer per slot."""
    from paper_1703_06999_amd.serving import plan_pool
    w = {g: g ** 3 for g in (48, 64, 96, 128, 160)}
    assert plan_pool(w.values(), 1.25 * w[160], 4) == [w[160], w[96], w[48]]
    assert plan_pool(w.values(), 64 * w[160], 4) == [w[160]] * 4
    assert plan_pool(w.values(), 0.5 * w[48], 4) == []
    assert plan_pool([w[64], w[64]], 10 * w[64], 3) == [w[64]] * 3
