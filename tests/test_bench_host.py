"""Host logic of the benchmark (no GPU): the single-GPU contract, the
algorithmic byte count against a hand count, the profile-hash guard and the
rocprofv3 summaries on synthetic counter files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

torch = pytest.importorskip("torch")


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_algorithmic_bytes_hand_count():
    # degrees: node 0: 1, node 1: 3, node 2: 40
    deg = torch.tensor([1, 3, 40], dtype=torch.int64)
    # one walk 0 -> 1 -> 2 -> 1 and a padded walk 2 -> 0
    Y = torch.tensor([[0, 1, 2, 1], [2, 0, -1, -1]], dtype=torch.int32)
    lens = torch.tensor([4, 2], dtype=torch.int32)
    steps, fo = bench.algorithmic_bytes(torch, Y, lens, deg, "fo_weighted")
    assert steps == 4
    # first order: 24 + 4 ceil(log2(d_v + 1)) per step from v
    c = lambda d: 24 + 4 * (d).bit_length()  # ceil(log2(d + 1)) == bit_length(d)
    assert fo == c(1) + c(3) + c(40) + c(40)
    _, gen = bench.algorithmic_bytes(torch, Y, lens, deg, "generic")
    # node2vec: the first step of a walk as first order, later steps
    # 32 + min(probe, stream, merge) + 4 ceil(log2(d_v + 1)) with t the previous node
    L = lambda d: d.bit_length()
    later = lambda dt, dv: 32 + min(4 * dt + 4 * dt * L(dv), 4 * dv + 4 * dv * L(dt), 4 * dv + 4 * dt) + 4 * L(dv)
    assert gen == c(1) + later(1, 3) + later(3, 40) + c(40)
    # two long rows (d_t = 40, d_v = 50): merging both rows (360 B) beats probing (1120 B)
    # and streaming (1400 B)
    Y2 = torch.tensor([[2, 3, 2]], dtype=torch.int32)
    deg2 = torch.tensor([1, 3, 40, 50], dtype=torch.int64)
    _, g2 = bench.algorithmic_bytes(torch, Y2, torch.tensor([3], dtype=torch.int32), deg2, "generic")
    assert g2 == c(40) + 32 + (4 * 50 + 4 * 40) + 4 * L(50)
    # with stored edge lists a later step may read its 16 B list record instead of building the list
    _, g3 = bench.algorithmic_bytes(torch, Y2, torch.tensor([3], dtype=torch.int32), deg2, "generic", lists=True)
    assert g3 == c(40) + 32 + 16 + 4 * L(50)
    _, g4 = bench.algorithmic_bytes(torch, Y, lens, deg, "generic", lists=True)
    tiny = lambda dt, dv: 32 + min(4 * dt + 4 * dt * L(dv), 4 * dv + 4 * dv * L(dt), 4 * dv + 4 * dt, 16) + 4 * L(dv)
    assert g4 == c(1) + tiny(1, 3) + tiny(3, 40) + c(40)


def test_traffic_needs_matching_source_hash(tmp_path):
    f = tmp_path / "t.txt"
    f.write_text("source_hash: 0000000000000000\nk_walk_n2v hbm_bytes_per_launch: 1.5e9\n")
    assert bench.traffic_from_profiles("k_walk_n2v", str(f)) is None
    f.write_text(f"source_hash: {bench.kernel_source_hash()}\nk_walk_n2v hbm_bytes_per_launch: 1.5e9\n")
    assert bench.traffic_from_profiles("k_walk_n2v", str(f)) == 1.5e9
    assert bench.traffic_from_profiles("k_walk_lane", str(f)) is None


def test_l2_hit_needs_matching_source_hash(tmp_path):
    f = tmp_path / "c.txt"
    # the counter summary's layout: derived figures, then the hit rate on a line of its own
    line = "k_walk_n2v valu_insts_per_wave: 1.0 vmem_rd_insts_per_wave: 1.0 lds_insts_per_wave: 0.0 " \
           "wait_any_share_of_wave_cycles: 0.5\nk_walk_n2v l2_hit_rate: 0.375\n"
    f.write_text("source_hash: 0000000000000000\n" + line)
    assert bench.l2_hit_from_profiles("k_walk_n2v", str(f)) is None
    f.write_text(f"source_hash: {bench.kernel_source_hash()}\n" + line)
    assert bench.l2_hit_from_profiles("k_walk_n2v", str(f)) == 0.375
    assert bench.l2_hit_from_profiles("k_walk_lane", str(f)) is None


def _pmc_csv(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_profile_summaries_scale_by_the_copy(tmp_path, monkeypatch):
    t = tmp_path / "trace"
    os.makedirs(t)
    with open(t / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"])
        w.writeheader()
        w.writerow({"Name": "void k_walk_n2v<64>(WalkArgs)", "Calls": 2, "TotalDurationNs": 4000,
                    "AverageNs": 2000, "MinNs": 1900, "MaxNs": 2100})
    # two dispatches of the walk kernel, per-XCD partial counts summed per dispatch
    _pmc_csv(tmp_path / "fetch", [
        {"Dispatch_Id": 1, "Kernel_Name": "k_walk_n2v<64>", "Counter_Name": "FETCH_SIZE", "Counter_Value": 100},
        {"Dispatch_Id": 1, "Kernel_Name": "k_walk_n2v<64>", "Counter_Name": "FETCH_SIZE", "Counter_Value": 100},
        {"Dispatch_Id": 2, "Kernel_Name": "k_walk_n2v<64>", "Counter_Name": "FETCH_SIZE", "Counter_Value": 400}])
    _pmc_csv(tmp_path / "write", [
        {"Dispatch_Id": 1, "Kernel_Name": "k_walk_n2v<64>", "Counter_Name": "WRITE_SIZE", "Counter_Value": 10}])
    # the 1 GiB copy reads half of what it moves and writes all of it
    _pmc_csv(tmp_path / "cf", [{"Dispatch_Id": 9, "Kernel_Name": "copyBuffer", "Counter_Name": "FETCH_SIZE",
                                "Counter_Value": (1 << 30) / 1024 / 2}])
    _pmc_csv(tmp_path / "cw", [{"Dispatch_Id": 9, "Kernel_Name": "copyBuffer", "Counter_Name": "WRITE_SIZE",
                                "Counter_Value": (1 << 30) / 1024}])
    trace_file, traffic_file = tmp_path / "tr.txt", tmp_path / "pmc.txt"
    cmds = {k: k for k in ("trace", "fetch", "write", "cal_fetch", "cal_write")}
    bench.summarize_profiles(str(t), str(tmp_path / "fetch"), str(tmp_path / "write"), str(tmp_path / "cf"),
                             str(tmp_path / "cw"), cmds, trace_file=str(trace_file), traffic_file=str(traffic_file))
    txt = traffic_file.read_text()
    assert "fetch_scale: 2.000000" in txt and "write_scale: 1.000000" in txt
    # mean fetch per dispatch (200 + 400) / 2 KiB, doubled; write 10 KiB
    exp = 300 * 1024 * 2 + 10 * 1024
    assert bench.traffic_from_profiles("k_walk_n2v", str(traffic_file)) == pytest.approx(exp, rel=1e-6)
    assert "2000" in trace_file.read_text()
