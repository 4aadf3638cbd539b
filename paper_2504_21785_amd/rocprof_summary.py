"""Summaries of rocprofv3 result databases (rocpd SQLite), as plain text.

    python -m paper_2504_21785_amd.rocprof_summary kernels RUN_results.db
        per kernel: calls, total and mean duration, share of GPU time
    python -m paper_2504_21785_amd.rocprof_summary counter RUN_results.db COUNTER [--calib-mib M]
        per kernel: mean counter value per dispatch; with --calib-mib, the
        value of the plain elementwise copy kernel (reads and writes M MiB)
        gives the factor that turns the counter's KiB into bytes
    python -m paper_2504_21785_amd.rocprof_summary traffic FETCH.db WRITE.db --calib-mib M
            --workload W --command CMD --out FILE.json
        HBM bytes per launch of each FGGC stage (FETCH_SIZE + WRITE_SIZE,
        calibrated), stamped with the digest of the kernel sources
    python -m paper_2504_21785_amd.rocprof_summary valu SQ.db --workload W --command CMD --out FILE.json
        mean SQ_* counter values per dispatch of the direct-sum kernel (and
        the other kernels), stamped with the digest of the kernel sources

Only reads the database; nothing here touches a GPU.
"""
import argparse
import hashlib
import json
import os
import re
import sqlite3
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# stage name -> kernel-name fragments (the kernels that make up the stage)
STAGE_KERNELS = {
    "fggc_coef": ["fggc_coef_kernel"],
    "fggc_accum": ["fggc_agg1_kernel", "fggc_stencil1_kernel", "fggc_stencil_fft1_kernel", "fggc_accum_wave_kernel",
                   "fggc_accum_kernel", "fggc_accum_generic_kernel"],
    # bucket_pos_kernel and the two-level sort's kernels also serve the
    # direct sum's sort; their dispatches count here
    "fggc_sort": ["fggc_key_kernel", "fggc_rank_kernel", "count_rowscan_kernel", "count_binscan_kernel",
                  "bucket_pos_kernel", "bucket_rank_kernel", "coarse_perm_kernel", "fine_sort_kernel"],
    "fggc_band_mac": ["band_mac"],
    "fggc_fused": ["fggc_fused_kernel"],
    "fggc_contract": ["fft_contract_kernel", "fft_contract2_kernel", "band_table_kernel"],
    "fggc_ifft": ["fft_axis_kernel", "fft_axis_mr_kernel"],
    "ds_kernel": ["ds_kernel"],
    "ds_sep2": ["ds_sep2_kernel"],
}


def source_digest() -> str:
    """SHA-256 over the kernel sources (csrc/*.hip, *.h, *.cpp), in name order."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("fggc::", "")
    n = re.sub(r"^void ", "", n)
    n = re.sub(r"\(.*$", "", n)
    return n[:90]


def kernels(db):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                     "group by name order by sum(duration) desc").fetchall()
    tot = sum(r[2] for r in rows) or 1
    out = [f"{'kernel':90s} {'calls':>6s} {'total_us':>12s} {'avg_us':>10s} {'pct':>6s}"]
    for name, n, s, a in rows:
        out.append(f"{short(name):90s} {n:6d} {s / 1e3:12.1f} {a / 1e3:10.2f} {100 * s / tot:6.2f}")
    return "\n".join(out)


def counter(db, name, calib_mib=None):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                     "where counter_name = ? group by kernel_name, dispatch_id", (name,)).fetchall()
    per = {}
    for k, _, v in rows:
        per.setdefault(k, []).append(v)
    factor = None
    lines = []
    if calib_mib:
        cal = [sum(v) / len(v) for k, v in per.items() if "elementwise" in k]
        if cal:
            expect_kib = calib_mib * 1024.0
            factor = expect_kib / max(cal)
            lines.append(f"calibration: elementwise copy of {calib_mib} MiB reads {max(cal):.0f} KiB of "
                         f"{name} per dispatch (expected {expect_kib:.0f}); factor {factor:.4f}")
    lines.append(f"{'kernel':90s} {'dispatches':>10s} {'value/dispatch':>16s} {'x1024xfactor':>14s}")
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        m = sum(v) / len(v)
        b = m * 1024.0 * (factor if factor else 1.0)
        lines.append(f"{short(k):90s} {len(v):10d} {m:16.1f} {b:14.4g}")
    return "\n".join(lines)


def per_dispatch(db, name):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                     "where counter_name = ? group by kernel_name, dispatch_id", (name,)).fetchall()
    per = {}
    for k, _, v in rows:
        per.setdefault(k, []).append(v)
    return {k: sum(v) / len(v) for k, v in per.items()}


def traffic(fetch_db, write_db, calib_mib, workload, command):
    out = {"workload": workload, "command": command, "source_sha256": source_digest(),
           "calibration_mib": calib_mib, "stages": {}}
    for cname, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        per = per_dispatch(db, cname)
        cal = [v for k, v in per.items() if "elementwise" in k]
        factor = calib_mib * 1024.0 / max(cal) if cal else 1.0
        out[cname.lower() + "_factor"] = factor
        for stage, frags in STAGE_KERNELS.items():
            ks = [k for k in per if any(f in k for f in frags)]
            if not ks:
                continue
            b = sum(per[k] for k in ks) * 1024.0 * factor
            out["stages"].setdefault(stage, {})[cname.lower() + "_bytes"] = b
            out["stages"][stage]["kernels"] = sorted(short(k) for k in ks)
    return out


def valu(db, workload, command):
    """Mean value per dispatch of every SQ_* counter in the run, per kernel
    family (the template arguments dropped), e.g. kernels["ds_kernel"]."""
    c = sqlite3.connect(db)
    names = [r[0] for r in c.execute("select distinct counter_name from counters_collection")]
    out = {"workload": workload, "command": command, "source_sha256": source_digest(), "kernels": {}}
    for name in names:
        for k, v in per_dispatch(db, name).items():
            fam = re.sub(r"<.*$", "", short(k))
            out["kernels"].setdefault(fam, {})[name] = v
            out["kernels"][fam].setdefault("instances", [])
            if short(k) not in out["kernels"][fam]["instances"]:
                out["kernels"][fam]["instances"].append(short(k))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["kernels", "counter", "traffic", "valu"])
    ap.add_argument("db")
    ap.add_argument("name", nargs="?")
    ap.add_argument("--calib-mib", type=float, default=None)
    ap.add_argument("--workload", default="cfg1")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.what == "kernels":
        print(kernels(a.db))
    elif a.what == "valu":
        t = valu(a.db, a.workload, a.command)
        text = json.dumps(t, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text + "\n")
        print(text)
    elif a.what == "traffic":
        t = traffic(a.db, a.name, a.calib_mib or 256.0, a.workload, a.command)
        text = json.dumps(t, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text + "\n")
        print(text)
    else:
        if not a.name:
            sys.exit("counter name required")
        print(counter(a.db, a.name, a.calib_mib))


if __name__ == "__main__":
    main()
