"""Host-side logic of bench.py (CPU): the refusal of several GPUs, and the counter files that
`--write-traffic` builds from rocprofv3 --pmc runs (kernel names as the bench reports them,
FETCH_SIZE and WRITE_SIZE averaged per dispatch and scaled by a plain copy of known size, the
SHA-256 of the listed sources), checked on synthetic counter tables with known answers."""
import csv
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_kernel_labels():
    assert bench._kernel_label("void elmfb::k_mv_blocks<3, 2>(elmfb::Geo, int)") == \
        "k_mv_blocks<FP16,2>"
    assert bench._kernel_label("void elmfb::k_rmv_chunks<0, 1>(elmfb::Geo)") == \
        "k_rmv_chunks<FP64>"
    assert bench._kernel_label("void elmfb::k_bt_mvb<1, 16>(elmfb::DevBlock const*)") == \
        "k_bt_mvb<FP32,16>"
    assert bench._kernel_label("elmfb::k_gather_rows(elmfb::Geo, int const*)") == "k_gather_rows"
    assert bench._kernel_label("void elmfb::k_bt_fold<1, false, 8, 2>(x)") == \
        "k_bt_fold<1,false,8,2>"
    assert bench._kernel_label("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def _pmc_run(path, counter, rows):
    os.makedirs(path)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_write_traffic_scales_and_hashes(tmp_path):
    gib = 1 << 30
    copy = "__amd_rocclr_copyBuffer"
    # the copy reads FETCH_SIZE = half its bytes (scale 2) and WRITE_SIZE = all of them (scale 1);
    # a small copy of another size is left out of the reference
    _pmc_run(tmp_path / "cf", "FETCH_SIZE", [(copy, gib / 2 / 1024)] * 3 + [(copy, 4.0)])
    _pmc_run(tmp_path / "cw", "WRITE_SIZE", [(copy, gib / 1024)] * 3)
    mv = "void elmfb::k_mv_blocks<3, 2>(elmfb::Geo, int)"
    gr = "elmfb::k_gather_rows(elmfb::Geo)"
    _pmc_run(tmp_path / "f", "FETCH_SIZE", [(mv, 100.0), (mv, 300.0), (gr, 10.0)])
    _pmc_run(tmp_path / "w", "WRITE_SIZE", [(mv, 5.0), (mv, 7.0), (gr, 1.0)])
    out = tmp_path / "traffic.json"
    srcs = "paper_2409_01949_amd/csrc/k_matvec.hip,paper_2409_01949_amd/csrc/common.h"
    subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--write-traffic", "t",
                    "--pmc-fetch", str(tmp_path / "f"), "--pmc-write", str(tmp_path / "w"),
                    "--copy-fetch", str(tmp_path / "cf"), "--copy-write", str(tmp_path / "cw"),
                    "--traffic-kernels", "k_mv_blocks<FP16,2>;k_gather_rows",
                    "--traffic-sources", srcs, "--traffic-out", str(out)],
                   check=True, capture_output=True, cwd=ROOT)
    d = json.loads(out.read_text())
    assert d["scale"]["fetch"] == 2.0 and d["scale"]["write"] == 1.0
    k = d["kernels"]["k_mv_blocks<FP16,2>"]
    assert k["read_bytes"] == 200.0 * 1024 * 2 and k["write_bytes"] == 6.0 * 1024
    assert k["hbm_bytes_per_launch"] == k["read_bytes"] + k["write_bytes"]
    assert k["dispatches_fetch"] == 2 and k["dispatches_write"] == 2
    assert d["kernels"]["k_gather_rows"]["read_bytes"] == 10.0 * 1024 * 2
    h = hashlib.sha256()
    for s in srcs.split(","):
        with open(os.path.join(ROOT, s), "rb") as fh:
            h.update(fh.read())
    assert d["source_sha256"] == h.hexdigest()


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2 and "single-GPU" in r.stdout
