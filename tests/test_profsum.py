"""Host-side checks of the profile summarizer that feeds bench.py's roofline.traffic."""
import csv
import json

from paper_2605_05330_amd import profsum


def _write_pmc(d, counter, rows):
    d.mkdir()
    with open(d / "pmc_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, grid, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Grid_Size": grid, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": val})


def test_traffic_scales_by_the_copy_and_averages_the_last_dispatches(tmp_path):
    step = "wrgn_step_kernel(StepArgs)"
    copy = "__amd_rocclr_copyBuffer"
    # early dispatches (a different phase) must not enter the average of the last 2
    _write_pmc(tmp_path / "f", "FETCH_SIZE", [(step, "100", 999.0), (copy, "64", 32768.0), (step, "100", 10.0),
                                             (step, "100", 30.0), (copy, "64", 5.0)])
    _write_pmc(tmp_path / "w", "WRITE_SIZE", [(copy, "64", 65536.0), (step, "100", 4.0), (step, "100", 4.0)])
    out = profsum.traffic(str(tmp_path / "f"), str(tmp_path / "w"), None, 2)
    doc = json.loads([l for l in out.splitlines() if l.startswith("TRAFFIC_JSON ")][0][13:])
    assert doc["fetch_bytes"] == 20.0 * 2.0 * 1024      # mean 20 KiB, scale 65536/32768
    assert doc["write_bytes"] == 4.0 * 1024
    assert doc["traffic_bytes"] == doc["fetch_bytes"] + doc["write_bytes"]
    assert doc["source_hash"] == profsum.kernel_source_hash()


def test_read_traffic_rejects_a_stale_kernel(tmp_path):
    good = {"traffic_bytes": 1.0, "source_hash": profsum.kernel_source_hash()}
    stale = dict(good, source_hash="0" * 16)
    p = tmp_path / "s.txt"
    p.write_text("header\nTRAFFIC_JSON " + json.dumps(good) + "\n")
    assert profsum.read_traffic(str(p))["traffic_bytes"] == 1.0
    p.write_text("TRAFFIC_JSON " + json.dumps(stale) + "\n")
    assert profsum.read_traffic(str(p)) is None
    assert profsum.read_traffic(str(tmp_path / "missing.txt")) is None
