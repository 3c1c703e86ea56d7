"""Helpers of the committed rocprofv3 measurements (measurement tooling, not
part of the compute path).

    python -m paper_1704_00131_amd.profiling copy
        a plain 64 MiB device-to-device copy, three times: the kernel whose
        FETCH_SIZE / WRITE_SIZE counters calibrate the HBM byte counts
    python -m paper_1704_00131_amd.profiling stats OUT TITLE COMMAND KERNEL_STATS_CSV
        a short text table of the kernels with the largest total time from a
        rocprofv3 --kernel-trace --stats CSV, headed by the command that made it
    python -m paper_1704_00131_amd.profiling summarize OUT KERNEL SRC FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB
        per-dispatch averages of FETCH_SIZE and WRITE_SIZE (KiB) of KERNEL from
        two rocprofv3 --pmc result databases, scaled by the copy kernel's
        counters against its known byte count, written to OUT (JSON) with the
        sha256 of the kernel source SRC
"""
import hashlib
import json
import sqlite3
import statistics
import sys

COPY_BYTES = 64 << 20


def copy():
    import torch
    n = COPY_BYTES // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x %d bytes" % COPY_BYTES)


def _values(db, counter, kernel_prefix=None):
    con = sqlite3.connect(db)
    rows = con.execute("select name, counter_value from pmc_events where counter_name = ?", (counter,)).fetchall()
    con.close()
    if kernel_prefix is None:
        return [v for _, v in rows]
    return [v for n, v in rows if kernel_prefix in n]


def summarize(out, kernel, src, fetch_db, write_db, copy_fetch_db, copy_write_db):
    f = _values(fetch_db, "FETCH_SIZE", kernel)
    w = _values(write_db, "WRITE_SIZE", kernel)
    # the copy kernel is the largest dispatch of the calibration run
    cf = max(_values(copy_fetch_db, "FETCH_SIZE"))
    cw = max(_values(copy_write_db, "WRITE_SIZE"))
    ff = COPY_BYTES / 1024.0 / cf
    wf = COPY_BYTES / 1024.0 / cw
    with open(src, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()[:16]
    fr, wr = statistics.mean(f), statistics.mean(w)
    d = {"kernel": kernel, "dispatches": len(f), "kernel_source_sha256_16": sha,
         "fetch_kib_per_launch_raw": fr, "write_kib_per_launch_raw": wr,
         "calibration": {"copy_bytes": COPY_BYTES, "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
                         "fetch_factor": ff, "write_factor": wf},
         "hbm_bytes_per_launch": 1024.0 * (fr * ff + wr * wf)}
    with open(out, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d))


def stats(out, title, command, csv_path, top=14):
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# %s" % title, "#", "# command: %s" % command,
             "# total kernel time %.1f ms over %d kernels; times in microseconds" % (total / 1e6, len(rows)), "",
             "| kernel | calls | total ms | avg us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append("| `%s` | %d | %.2f | %.2f | %.2f | %.2f | %.1f%% |" % (
            r["Name"].replace("|", "/"), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "copy":
        copy()
    elif sys.argv[1] == "stats":
        stats(*sys.argv[2:6])
    elif sys.argv[1] == "summarize":
        summarize(*sys.argv[2:9])
    else:
        raise SystemExit(__doc__)
