"""Summaries of rocprofv3 result databases (the default rocpd SQLite output).

    python -m paper_1904_08616_amd.profile_summary trace RUN.db --command "..."
        per-kernel call count and duration statistics (the --stats table)
    python -m paper_1904_08616_amd.profile_summary pmc RUN.db [RUN2.db ...] --kernel NAME --command "..."
        average value per dispatch of every counter collected, for kernels matching NAME
    python -m paper_1904_08616_amd.profile_summary counters --fetch F.db --write W.db \
        --kernel k_dslash_stream --fetch-command "..." --write-command "..." [--json OUT]
        FETCH_SIZE / WRITE_SIZE per dispatch of one kernel, scaled by what the
        same counters read for the largest plain copy in the run, as HBM bytes

The copy is the runtime's buffer copy (torch's device-to-device copy of a
known size, --copy-gib): its read and write volumes are known, so (known
KiB) / (counted KiB) is the factor that turns a counter into bytes on this
chip.  It must be the largest buffer copy in the run.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


# The sources the headline kernel (the float64 streaming Dslash) is compiled
# from: its counters are stale once any of them changes.
HEADLINE_SOURCES = ("common.h", "dslash_impl.h", "dslash_stream.h", "dslash_f64.hip")


def kernel_sources_sha256(names=HEADLINE_SOURCES) -> str:
    """Hash of the kernel's source files: counters taken on other sources are stale."""
    h = hashlib.sha256()
    for name in sorted(names):
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_stats(db):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
                     "grid_x, workgroup_x, lds_size, vgpr_count, scratch_size from kernels "
                     "group by name, grid_x order by sum(duration) desc").fetchall()
    return rows


def counters(db, counter):
    c = sqlite3.connect(db)
    return c.execute("select p.name, count(*), avg(p.counter_value), min(p.counter_value), max(p.counter_value), "
                     "k.grid_x from pmc_events p join kernels k on p.dispatch_id = k.dispatch_id "
                     "where p.counter_name = ? group by p.name, k.grid_x", (counter,)).fetchall()


def trace_report(db, command):
    out = [f"command: {command}", "", "rocprofv3 --kernel-trace --stats, per kernel (durations in ns)", ""]
    out.append("%-8s %12s %10s %10s %10s %9s %5s %7s %5s %4s  %s" % (
        "calls", "total", "average", "min", "max", "grid", "wg", "lds", "vgpr", "scr", "kernel"))
    for r in kernel_stats(db):
        out.append("%-8d %12d %10.0f %10d %10d %9d %5d %7d %5d %4d  %s" % (tuple(r[1:]) + (r[0],)))
    return "\n".join(out)


def counter_report(fetch_db, write_db, kernel, fetch_cmd, write_cmd, copy_gib=1.0):
    res = {}
    lines = [f"FETCH_SIZE command: {fetch_cmd}", f"WRITE_SIZE command: {write_cmd}", ""]
    for db, name in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        rows = counters(db, name)
        copies = [r for r in rows if "copyBuffer" in r[0]]
        if not copies:
            raise SystemExit(f"{db}: no buffer copy to calibrate {name} against")
        cmax = max(r[4] for r in copies)  # KiB counted for the largest copy
        known = copy_gib * (1 << 20)  # KiB the calibration copy moves each way
        scale = known / cmax
        ks = [r for r in rows if kernel in r[0]]
        if not ks:
            raise SystemExit(f"{db}: no dispatch of {kernel}")
        k = max(ks, key=lambda r: r[1])
        res[name] = {"kernel": k[0], "dispatches": k[1], "kib_avg": k[2], "kib_min": k[3], "kib_max": k[4],
                     "copy_kib_per_gib": cmax, "scale": scale, "bytes": k[2] * scale * 1024}
        lines.append(f"{name}: {k[0]}")
        lines.append(f"  dispatches {k[1]}, KiB per dispatch avg {k[2]:.1f} (min {k[3]:.1f}, max {k[4]:.1f})")
        lines.append(f"  a {copy_gib:g} GiB copy counts {cmax:.1f} KiB -> scale {scale:.5f}; "
                     f"bytes per dispatch {k[2] * scale * 1024:.4e}")
    total = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    lines.append(f"HBM bytes per dispatch (scaled FETCH + WRITE): {total:.4e}")
    res["traffic_bytes"] = total
    return "\n".join(lines), res


def pmc_report(dbs, command, kernels):
    """Average value per dispatch of every counter in the runs, per kernel."""
    out = [f"command: {command}", "", "average per dispatch (dispatches)", ""]
    for db in dbs:
        c = sqlite3.connect(db)
        rows = c.execute("select name, counter_name, count(*), avg(counter_value), max(counter_value) "
                         "from pmc_events group by name, counter_name order by name, counter_name").fetchall()
        for r in rows:
            if any(k in r[0] for k in kernels):
                out.append("%-26s %16.1f  (n %3d, max %14.1f)  %s" % (r[1], r[3], r[2], r[4], r[0]))
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--fetch-command", required=True)
    c.add_argument("--write-command", required=True)
    c.add_argument("--json")
    c.add_argument("--launch", help="launch configuration (JSON) the counters were taken with")
    c.add_argument("--copy-gib", type=float, default=1.0,
                   help="size of the calibration copy (the largest buffer copy in the runs; it must be larger "
                        "than any other device copy there, such as clones of the inputs)")
    q = sub.add_parser("pmc")
    q.add_argument("dbs", nargs="+")
    q.add_argument("--command", required=True)
    q.add_argument("--kernel", action="append", required=True)
    a = ap.parse_args(argv)
    if a.mode == "trace":
        print(trace_report(a.db, a.command))
        return 0
    if a.mode == "pmc":
        print(pmc_report(a.dbs, a.command, a.kernel))
        return 0
    text, res = counter_report(a.fetch, a.write, a.kernel, a.fetch_command, a.write_command, a.copy_gib)
    print(text)
    if a.json:
        res["kernel_sources_sha256"] = kernel_sources_sha256()
        res["launch"] = json.loads(a.launch) if a.launch else None
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)
            f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
