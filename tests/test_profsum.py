"""Host checks of the rocprofv3 summary tools: FETCH/WRITE readings summed
over one operation's dispatches, scaled by the copy calibration, kept per
run length, dropped when the kernel sources change; bench.py looks records
up by the run length it ran."""
import csv
import json

from paper_2008_00672_amd import profsum

HDR = ["Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        w.writerows(rows)
    return str(path)


def _files(tmp_path, fetch_kib, write_kib):
    rx = "void fcx::fc_rx_kernel<2, 4096>(fcx::LaunchArgs, int)"
    tx = "void fcx::fc_tx_pruned_kernel<1, 2048, 1, false, 0>(fcx::LaunchArgs, int)"
    f = _csv(tmp_path / "f.csv", [[rx, "FETCH_SIZE", fetch_kib]] * 3 + [[tx, "FETCH_SIZE", 999.0]])
    w = _csv(tmp_path / "w.csv", [[rx, "WRITE_SIZE", write_kib]] * 3 + [[tx, "WRITE_SIZE", 999.0]])
    # three 256 MiB copies (the median is taken) plus a small unrelated copy;
    # the fetch counter reads half the bytes, the write counter all of them
    kib = (256 << 20) / 1024.0
    cf = _csv(tmp_path / "cf.csv", [["copy_kernel", "FETCH_SIZE", v] for v in (kib / 2, kib / 2, kib / 2, 7.0)])
    cw = _csv(tmp_path / "cw.csv", [["copy_kernel", "WRITE_SIZE", v] for v in (kib, kib, kib, 7.0)])
    return f, w, cf, cw


def test_traffic_records_per_run_length(tmp_path):
    out = str(tmp_path / "traffic_fc_rx.json")
    d = profsum.traffic("fc_rx", *_files(tmp_path, 1000.0, 400.0), 3, out, "cmd a", 2)
    r = d["by_run_len"]["2"]
    assert abs(r["copy_factor_fetch"] - 2.0) < 1e-12 and abs(r["copy_factor_write"] - 1.0) < 1e-12
    assert r["dispatches"] == [3, 3]
    # per call: (3 x 1000 KiB x 2 + 3 x 400 KiB x 1) / 3 calls
    assert abs(r["bytes_per_launch"] - (2000.0 + 400.0) * 1024.0) < 1e-6
    d = profsum.traffic("fc_rx", *_files(tmp_path, 1500.0, 400.0), 3, out, "cmd b", 4)
    assert sorted(d["by_run_len"]) == ["2", "4"]
    assert abs(d["by_run_len"]["4"]["bytes_per_launch"] - (3000.0 + 400.0) * 1024.0) < 1e-6
    assert d["by_run_len"]["2"]["command"] == "cmd a"
    # records taken from other kernel sources are dropped on the next write
    j = json.load(open(out))
    j["kernel_hash"] = "0" * 16
    json.dump(j, open(out, "w"))
    d = profsum.traffic("fc_rx", *_files(tmp_path, 1000.0, 400.0), 3, out, "cmd c", 1)
    assert sorted(d["by_run_len"]) == ["1"] and d["kernel_hash"] == profsum.kernel_hash()
    md = str(tmp_path / "t.md")
    profsum.traffic_md([out], md, ["cmd c"])
    text = open(md).read()
    assert "| fc_rx | 1 | 1 |" in text and profsum.kernel_hash() in text


def test_bench_looks_up_its_run_length():
    import bench
    path = bench.os.path.join(bench.ROOT, "profiles", "traffic_fc_rx.json")
    j = json.load(open(path))
    if j["kernel_hash"] != profsum.kernel_hash():
        assert bench.traffic("fc_rx", 2) is None       # sources changed since the counters
        return
    for k, rec in j["by_run_len"].items():
        assert bench.traffic("fc_rx", int(k)) == round(rec["bytes_per_launch"])
    assert bench.traffic("fc_rx", 3) is None             # never measured at 3 blocks per task
