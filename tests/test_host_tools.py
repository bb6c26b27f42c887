"""Host-side tools: the benchmark's one-GPU guard, the rocprofv3 summary script and the tuning file (CPU only)."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def _write_counter_csv(path, rows):
    cols = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
            "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (name, counter, value) in enumerate(rows):
            w.writerow({c: 0 for c in cols} | {"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter,
                                                "Counter_Value": value, "Grid_Size": 64})


def test_traffic_summary_scales_by_the_copy(tmp_path):
    """FETCH_SIZE / WRITE_SIZE are scaled by (known copy bytes) / (what the counter read for the copy)."""
    from paper_1711_03836_amd import profile_summary as ps
    kib = 1024 * 1024  # a 1 GiB copy in KiB
    fdir, wdir = tmp_path / "f", tmp_path / "w"
    fdir.mkdir()
    wdir.mkdir()
    _write_counter_csv(fdir / "x_counter_collection.csv",
                       [("__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 2)] +
                       [("k_hop<...>", "FETCH_SIZE", 1000.0)] * 4)
    _write_counter_csv(wdir / "x_counter_collection.csv",
                       [("__amd_rocclr_copyBuffer", "WRITE_SIZE", kib)] +
                       [("k_hop<...>", "WRITE_SIZE", 300.0)] * 4)
    out = tmp_path / "t.json"
    ps.main(["traffic", str(fdir), str(wdir), str(out), "--kernel", "k_hop", "--launches", "3", "--copy-mib", "1024",
             "--tune", "12,3,128,0", "--algorithmic-bytes", "1000000"])
    d = json.load(open(out))
    assert abs(d["fetch"]["factor"] - 2.0) < 1e-12 and abs(d["write"]["factor"] - 1.0) < 1e-12
    assert abs(d["traffic_bytes"] - (2000.0 + 300.0) * 1024) < 1e-6
    assert d["tune"] == [12, 3, 128, 0] and d["source_digest"] == ps.source_digest()


def test_tuning_file_round_trip(tmp_path):
    """Context.save_tuning / load_tuning write and apply the (prec, nrhs) -> (recon, R, bs, march, lds, order)
    table through tune_get / tune_set only; checked here on stand-in contexts (no device)."""
    sys.path.insert(0, ROOT)
    from paper_1711_03836_amd import bqhip as bq

    class Src:
        table = {(1, 12): (12, 1, 64, 0, 1, 1), (0, 1): (18, 1, 64, 16, 0, 0)}

        def tune_get(self, prec, nrhs):
            return self.table[(prec, nrhs)]

    class Dst:
        def __init__(self):
            self.set = []

        def tune_set(self, prec, nrhs, recon, R, bs, march=0, lds=0, order=0):
            self.set.append((prec, nrhs, recon, R, bs, march, lds, order))

    path = tmp_path / "tune.json"
    bq.Context.save_tuning(Src(), path, [(1, 12), (0, 1)], lattice=(32, 32, 32, 64))
    doc = json.loads(path.read_text())
    assert doc["lattice"] == [32, 32, 32, 64]
    dst = Dst()
    assert bq.Context.load_tuning(dst, path) == [(1, 12), (0, 1)]
    assert dst.set == [(1, 12, 12, 1, 64, 0, 1, 1), (0, 1, 18, 1, 64, 16, 0, 0)]
