"""Host logic of bench.py (no GPU): the one-GPU contract, the committed counter
figures it reports, the roofline arithmetic, and the element Jacobian's operation
count following from the committed instruction counts."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one" in line["error"].lower()


def test_counter_traffic_follows_the_committed_runs():
    tr = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    # counted bytes are reported only while the fused pass is the one the counters saw
    current = tr["source_hash"] == bench.kernel_source_hash(tr["kernel_function"])
    for name, w in tr["workloads"].items():
        expect = (tr["fetch_factor"] * w["fetch_kib_mean"] + tr["write_factor"] * w["write_kib_mean"]) * 1024
        assert abs(w["traffic_bytes_per_launch"] - expect) <= 1e-6 * expect, name
        got = bench.counter_traffic(name, tr["family"], w["precision"])
        assert got == (w["traffic_bytes_per_launch"] if current else None), name
        assert bench.counter_traffic(name, "krylov_spmv_fine", w["precision"]) is None
        other = "fp64" if w["precision"] == "mixed" else "mixed"
        assert bench.counter_traffic(name, tr["family"], other) is None
    assert bench.counter_traffic("no-such-workload", tr["family"], "fp64") is None


def test_roofline_of_picks_the_dominant_family():
    fams = {f: (0, 0.0, 0.0) for f in bench.FAMILIES}
    fams["vanka_pass_fine"] = (1000, 50.0, 1000 * 200e6)      # 50 ms over 1000 launches of 200 MB
    fams["krylov_spmv_fine"] = (100, 5.0, 100 * 150e6)
    r = bench.roofline_of(fams, None, "fp64")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["launches"] == 1000 and abs(r["mean_launch_us"] - 50.0) < 1e-9
    assert abs(r["achieved"] - 4000.0) < 1e-6 and abs(r["frac"] - 0.5) < 1e-12
    assert r["traffic"] is None


@pytest.mark.parametrize("dim", ["2d", "3d"])
def test_element_jacobian_operation_count(dim):
    f = json.load(open(os.path.join(ROOT, "profiles", "flops.json")))["k_elem_jacobian"][dim]
    c = f["wave_instructions_per_launch"]
    ops = 64 * (2 * c["SQ_INSTS_VALU_FMA_F64"] + c["SQ_INSTS_VALU_MUL_F64"] + c["SQ_INSTS_VALU_ADD_F64"]
                + c["SQ_INSTS_VALU_TRANS_F64"])
    assert abs(f["flop_per_cell"] - ops / f["cells_per_launch"]) <= 1e-9 * f["flop_per_cell"]
