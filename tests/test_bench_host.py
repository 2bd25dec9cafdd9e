"""Host logic of bench.py's offline summaries (no GPU): the SQ counter
summary's VALU issue fraction and the batched form's per-stage figure read
back from it, which is withheld when the kernel sources have changed."""
import csv
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _write_csv(path, rows):
    keys = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value",
            "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=keys)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(keys, r)))


def test_counter_summary_and_batched_valu_issue(tmp_path, monkeypatch, capsys):
    out = tmp_path / "counters_valu.json"
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(out))
    # two dispatches of one batched R2C shape (100 us each), one batched
    # accumulation (200 us) after it, one C2R (50 us)
    us = 1000  # ns per us
    rows = []
    for d, (name, grid, wg, valu, dur) in enumerate([
            ("void arkcos::r2c_batch_kernel<float, 256, 0>(...)", 256 * 1000, 256, 6.0e6, 100),
            ("void arkcos::r2c_batch_kernel<float, 256, 0>(...)", 256 * 1000, 256, 6.0e6, 100),
            ("void arkcos::accumulate_batch_u_kernel<float, 8, 2, 8>(...)", 512 * 1024, 512, 3.0e6, 200),
            ("void arkcos::c2r_batch_kernel<float, 256, 0>(...)", 256 * 500, 256, 9.0e6, 50)]):
        for cn, v in (("SQ_INSTS_VALU", valu), ("SQ_INSTS_SALU", 1.0e6)):
            rows.append((d + 1, name, grid, wg, cn, v, 0, dur * us))
    path = tmp_path / "run_counter_collection.csv"
    _write_csv(path, rows)
    bench.summarize_counters(str(path), "cmd", "title")
    md = capsys.readouterr().out
    assert "`r2c_batch_kernel` | 1000 | 256 | 2 | 100.0 |" in md
    data = json.loads(out.read_text())
    ent = {e["kernel"]: e for e in data["kernels"]}
    # VALU issue = VALU x 4 cycles / (1024 SIMDs x 2.4 GHz x duration)
    assert abs(ent["r2c_batch_kernel"]["valu_issue"] - 6.0e6 * 4 / (1024 * 2.4e9 * 100e-6)) < 1e-3
    assert ent["accumulate_batch_u_kernel"]["source_sha"] == bench.kernel_source_hash("accumulate", batched=True)
    got = bench.batched_valu_issue()
    assert got is not None
    st = got["stages"]
    assert abs(st["ring_r2c"] - 6.0e6 * 4 / (1024 * 2.4e9 * 100e-6)) < 1e-3
    assert abs(st["accumulate"] - 3.0e6 * 4 / (1024 * 2.4e9 * 200e-6)) < 1e-3
    assert abs(st["fold_c2r"] - 9.0e6 * 4 / (1024 * 2.4e9 * 50e-6)) < 1e-3
    # a summary taken on other sources is not used
    data["kernels"][0]["source_sha"] = "0" * 16
    out.write_text(json.dumps(data))
    assert bench.batched_valu_issue() is None


def test_committed_counter_summary_is_readable():
    """The committed summary parses; its figures are used only while the
    kernel sources match (None otherwise, never an error)."""
    got = bench.batched_valu_issue()
    assert got is None or set(got["stages"]) <= set(bench.BATCH_KERNELS)
