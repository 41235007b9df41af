"""Summaries of rocprofv3 output for this library's kernels.

  python -m paper_2008_00672_amd.profsum stats <kernel_stats.csv> <out.md> "<command>"
  python -m paper_2008_00672_amd.profsum traffic <op> <fetch.csv> <write.csv> \
         <calib_fetch.csv> <calib_write.csv> <calls> <out.json> "<command>" <run_len>

`stats` turns a --kernel-trace --stats summary into a short markdown table.
`traffic` sums FETCH_SIZE / WRITE_SIZE (KiB per dispatch) over the dispatches
of one operation (all fc_tx_* kernels, or fc_rx_kernel), divides by the number
of calls, and scales each counter by known-bytes / reading of a plain 256 MiB
device copy profiled with the same counter. The traffic depends on the work
split (blocks per task: a run re-reads the input its first block overlaps),
so each record is kept under the run length it was taken at, several per
file. The file records a hash of the kernel sources so bench.py can tell
whether it is still current; records of another hash are dropped.
"""
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 << 20


def kernel_hash():
    """Hash of the kernel sources without their line comments and blank
    lines, so that edits to comments alone keep the counters current."""
    import re
    h = hashlib.sha256()
    for f in ("fc_device.h", "fc_internal.h", "fc_kern_io.hip"):
        for line in open(os.path.join(HERE, "csrc", f)).read().split("\n"):
            code = re.sub(r"//.*$", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _short(name):
    n = name.replace("void fcx::", "").replace("fcx::", "")
    return n.split("(")[0]


def stats_md(path, out, command):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel trace", "", "Command (repo root, MI355X):", "", "    " + command, "",
             "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    tx_avg = 0.0
    for r in rows:
        k = _short(r["Name"])
        avg = float(r["AverageNs"]) / 1e3
        if OPS["fc_tx"](k):
            tx_avg += avg
        lines.append("| %s | %s | %.1f | %.2f | %.1f |" % (k, r["Calls"], avg, float(r["TotalDurationNs"]) / 1e6,
                                                          float(r["Percentage"])))
    lines += ["", "Sum of the TX class averages (template argument false: input is the low-rate signal): %.1f us. "
              "The TX classes of one call run concurrently on side streams, so this exceeds the call's wall "
              "time, which bench.py measures; the kernels with template argument true are the grid-input "
              "TX (fc_tx_modulate), fc_rxd_kernel the demodulating RX, both timed outside the step." % tx_avg, ""]
    open(out, "w").write("\n".join(lines))


def _dispatch_values(path, counter, select):
    tot, n = 0.0, 0
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter or not select(_short(r["Kernel_Name"])):
            continue
        tot += float(r["Counter_Value"])
        n += 1
    return tot, n


def _copy_reading(path, counter):
    """Counter value of the 256 MiB copies: the median of the three largest
    copy dispatches (the run makes exactly three such copies)."""
    vals = sorted(float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                  if r["Counter_Name"] == counter and "copy" in r["Kernel_Name"].lower())
    top = vals[-3:]
    return top[len(top) // 2]


def _tx_front(k):
    """The FRONT template argument of a TX kernel name (fc_tx_pruned_kernel<IO,
    L, log2 I, FRONT, plan> or fc_tx_full_kernel<IO, N, FRONT>), else None."""
    if not k.startswith("fc_tx_") or "<" not in k:
        return None
    args = [a.strip() for a in k[k.index("<") + 1:k.rindex(">")].split(",")]
    return next((a for a in args if a in ("true", "false")), None)


# kernels of one call of each operation
OPS = {
    "fc_tx": lambda k: _tx_front(k) == "false",       # TX from the low-rate signal
    "fc_tx_grid": lambda k: _tx_front(k) == "true",   # TX from the QAM grid
    "fc_rx": lambda k: k.startswith("fc_rx_kernel"),
    "fc_rxd": lambda k: k.startswith("fc_rxd_kernel"),
}


def traffic(op, fetch, write, cfetch, cwrite, calls, out, command, run_len):
    """Add (or replace) the record of op at blocks-per-task run_len in out."""
    sel = OPS[op]
    f_kib, nf = _dispatch_values(fetch, "FETCH_SIZE", sel)
    w_kib, nw = _dispatch_values(write, "WRITE_SIZE", sel)
    ff = COPY_BYTES / (_copy_reading(cfetch, "FETCH_SIZE") * 1024.0)
    fw = COPY_BYTES / (_copy_reading(cwrite, "WRITE_SIZE") * 1024.0)
    per_call = (f_kib * 1024.0 * ff + w_kib * 1024.0 * fw) / calls
    h = kernel_hash()
    d = json.load(open(out)) if os.path.exists(out) else {}
    if d.get("kernel_hash") != h or "by_run_len" not in d:
        d = {"op": op, "kernel_hash": h, "by_run_len": {}}
    d["by_run_len"][str(int(run_len))] = {
        "bytes_per_launch": per_call, "fetch_kib_per_call": f_kib / calls, "write_kib_per_call": w_kib / calls,
        "copy_factor_fetch": ff, "copy_factor_write": fw, "dispatches": [nf, nw], "calls": calls,
        "command": command}
    d["by_run_len"] = dict(sorted(d["by_run_len"].items(), key=lambda kv: int(kv[0])))
    json.dump(d, open(out, "w"), indent=1)
    return d


def traffic_md(jsons, out, commands):
    """Markdown table of the traffic summaries (one row per op and run length)."""
    ds = [json.load(open(j)) for j in jsons]
    recs = [(d["op"], int(k), r) for d in ds for k, r in d["by_run_len"].items()]
    lines = ["# HBM traffic per call (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
             "Counter runs (repo root, MI355X), one counter per run; `--tuning` fixes the blocks per task "
             "(tx_run_len,tx_conc,rx_run_len,rx_conc; the grid-input TX and the demodulating RX take the TX "
             "and RX values):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Calibration: a plain 256 MiB device copy under the same counters gives the scale factors "
                  "FETCH x%.4f, WRITE x%.4f (known bytes / counter reading)." % (recs[0][2]["copy_factor_fetch"],
                                                                                  recs[0][2]["copy_factor_write"]),
              "", "| op | blocks per task | dispatches per call | FETCH KiB/call | WRITE KiB/call | "
                  "calibrated HBM bytes/call |",
              "|---|---|---|---|---|---|"]
    for op, k, r in recs:
        lines.append("| %s | %d | %d | %.0f | %.0f | %.4g |" % (op, k, r["dispatches"][0] // r["calls"],
                                                               r["fetch_kib_per_call"], r["write_kib_per_call"],
                                                               r["bytes_per_launch"]))
    lines += ["", "Kernel source hash: %s (code lines, comments excluded)" % ds[0]["kernel_hash"], ""]
    open(out, "w").write("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats_md(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic_md":
        traffic_md(sys.argv[2].split(","), sys.argv[3], sys.argv[4:])
    elif sys.argv[1] == "traffic":
        print(traffic(sys.argv[2], *sys.argv[3:7], int(sys.argv[7]), sys.argv[8], sys.argv[9], int(sys.argv[10])))
