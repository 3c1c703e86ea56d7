"""Helpers of the committed rocprofv3 measurements (measurement tooling, not
part of the compute path).

    python -m paper_1704_00131_amd.profiling copy
        a plain 64 MiB device-to-device copy, three times: the kernel whose
        FETCH_SIZE / WRITE_SIZE counters calibrate the HBM byte counts
    python -m paper_1704_00131_amd.profiling sweep L1 BETA SWEEPS
        SWEEPS sweeps with the equal-time estimators of the honeycomb L1 x L1
        Hubbard chain (U = 5, dtau = 0.1, n_wrap = 10, two-valued field, seed
        0) after its set-up: the workload of the counter runs (a short beta
        keeps a counter-collecting run to seconds; the per-launch figures of
        the block update and the products depend on N, not on L)
    python -m paper_1704_00131_amd.profiling mfma OUT DB N WORKLOAD COMMAND
        per-kernel averages of the FP64 MFMA counters of one rocprofv3 --pmc
        run (SQ_INSTS_VALU_MFMA_MOPS_F64, in units of 512 flops, and the
        derived MfmaUtil, the percentage of SIMD cycles with the MFMA unit
        busy) with the dispatch durations of that run, the product kernels'
        counted flops against their algorithmic 2 N^3, written to OUT (JSON)
    python -m paper_1704_00131_amd.profiling dbstats OUT TITLE COMMAND RESULTS_DB
        the same table from the database of a rocprofv3 --kernel-trace run
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


def sweep(L1, beta, sweeps):
    import torch

    import paper_1704_00131_amd as pa
    from inputs import honeycomb_lattice
    lat = honeycomb_lattice(L1, L1)
    dtau, U = 0.1, 5.0
    m = pa.make_model(lat.n, beta, dtau, 10, pa.hubbard_coupling(U, dtau), U=U, trotter="sym", seed=0)
    ch = pa.Chain(m, lat.K)
    ch.random_field().init()
    print("set up honeycomb %dx%d N=%d L=%d" % (L1, L1, lat.n, m.n_slices), flush=True)
    for s in range(sweeps):
        st = ch.sweep(1, measure=True)
        torch.cuda.synchronize()
        print("sweep %d done: %d proposals, %d accepted" % (s, st.proposals, st.accepted), flush=True)
    ch.close()


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


def mfma(out, db, n, workload, command):
    n = int(n)
    con = sqlite3.connect(db)
    rows = con.execute("select name, dispatch_id, duration, counter_name, counter_value from pmc_events").fetchall()
    con.close()
    # a raw SQ counter comes as one row per shader engine: summed per
    # dispatch; the derived MfmaUtil is one row per dispatch
    per = {}
    for name, disp, dur, cname, val in rows:
        key = name.split("(")[0]
        if key.startswith("void "):   # template instances are listed with their return type
            key = key[5:]
        d = per.setdefault(key, {}).setdefault(disp, {"duration_ns": dur})
        d[cname] = d.get(cname, 0.0) + val
    kernels = []
    for key, disps in per.items():
        vals = list(disps.values())
        mops = [v.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) for v in vals]
        util = [v["MfmaUtil"] for v in vals if "MfmaUtil" in v]
        dur = [v["duration_ns"] for v in vals]
        flops = 512.0 * statistics.mean(mops)
        if flops <= 0.0:
            continue
        k = {"kernel": key, "dispatches": len(vals), "mfma_flops_per_dispatch": flops,
             "avg_duration_us": statistics.mean(dur) / 1e3,
             "counted_tflops": flops / (statistics.mean(dur) * 1e-9) / 1e12,
             "mfma_util_pct": statistics.mean(util) if util else None}
        if key.startswith("k_gemm") and "group" not in key:
            k["algorithmic_flops_per_dispatch"] = 2.0 * n ** 3
            k["counted_over_algorithmic"] = flops / (2.0 * n ** 3)
        kernels.append(k)
    kernels.sort(key=lambda k: -k["dispatches"] * k["avg_duration_us"])
    d = {"workload": workload, "N": n, "command": command,
         "note": "durations are those of the counter run (dispatches serialised); MfmaUtil = busy MFMA cycles "
                 "over active cycles of all SIMDs, in percent; the peak is 78.6 TFLOP/s (FP64 MFMA, dense)",
         "kernels": kernels}
    with open(out, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d))


def dbstats(out, title, command, db, top=16):
    con = sqlite3.connect(db)
    q = ("select s.display_name, count(*), sum(d.end - d.start), avg(d.end - d.start), min(d.end - d.start), "
         "max(d.end - d.start) from rocpd_kernel_dispatch d join rocpd_info_kernel_symbol s "
         "on d.kernel_id = s.id group by s.display_name order by 3 desc")
    rows = con.execute(q).fetchall()
    con.close()
    total = sum(r[2] for r in rows)
    lines = ["# %s" % title, "#", "# command: %s" % command,
             "# total kernel time %.1f ms over %d kernels; times in microseconds" % (total / 1e6, len(rows)), "",
             "| kernel | calls | total ms | avg us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for name, calls, tot, avg, mn, mx in rows[:top]:
        lines.append("| `%s` | %d | %.2f | %.2f | %.2f | %.2f | %.1f%% |" % (
            name.replace("|", "/"), calls, tot / 1e6, avg / 1e3, mn / 1e3, mx / 1e3, 100.0 * tot / total))
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


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
    elif sys.argv[1] == "dbstats":
        dbstats(*sys.argv[2:6])
    elif sys.argv[1] == "summarize":
        summarize(*sys.argv[2:9])
    elif sys.argv[1] == "sweep":
        sweep(int(sys.argv[2]), float(sys.argv[3]), int(sys.argv[4]))
    elif sys.argv[1] == "mfma":
        mfma(*sys.argv[2:7])
    else:
        raise SystemExit(__doc__)
