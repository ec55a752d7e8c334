"""Text summaries of rocprofv3 result databases (SQLite), for the kernel timing and byte-counter files kept
beside the code.

  python -m paper_1404_1066_amd.prof_summary kernels <results.db> "<command that produced it>" <runs> <title>
  python -m paper_1404_1066_amd.prof_summary traffic <fetch.db> <write.db> "<command>" <title> <kernel> <source>
  python -m paper_1404_1066_amd.prof_summary counters <results.db> "<command>" <title> [<kernel name part>]

`traffic` reads one FETCH_SIZE run and one WRITE_SIZE run (KiB per dispatch). Each counter is scaled by what
it reads for the 256 MiB device copy of `bench.py --copy-probe` (known bytes read and written), and the
scaled bytes per dispatch of every kernel are listed. The last line is a JSON record for `kernel`, with the
SHA-256 of its source file, so a reader can tell whether the kernel changed after the counters were taken.
"""

import collections
import hashlib
import json
import os
import sqlite3
import sys


def kernels(db, cmd, runs, title):
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    tot = sum(r[2] for r in rows)
    out = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", f"    {cmd}", "",
           f"rocprofv3 kernel-trace statistics over {runs} runs in the process. Total kernel time "
           f"{tot / 1e3:.1f} ms ({tot / 1e3 / runs:.1f} ms per run).", "",
           "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, total, avg, pct in rows[:30]:  # the summary table holds microseconds
        out.append(f"| `{name.split('(')[0].replace('void ', '')}` | {calls} | {total / 1e3:.2f} | {avg:.2f} "
                   f"| {pct:.1f} |")
    return "\n".join(out)


def _per_kernel(db):
    d = collections.defaultdict(list)
    for name, v in sqlite3.connect(db).execute("select kernel_name, value from counters_collection"):
        d[name.split("(")[0].replace("void ", "")].append(v)
    return d


def traffic(fdb, wdb, cmd, title, kernel, source):
    f, w = _per_kernel(fdb), _per_kernel(wdb)
    probe = 256 * 1024  # KiB read and written by the copy probe
    cf = [v for k, vs in f.items() if "copyBuffer" in k for v in vs if v > probe / 4]
    cw = [v for k, vs in w.items() if "copyBuffer" in k for v in vs if v > probe / 2]
    sf, sw = probe / (sum(cf) / len(cf)), probe / (sum(cw) / len(cw))
    out = [f"# {title}", "", "Commands (from the repository root, one MI355X; one counter per run):", "",
           f"    {cmd.replace('<COUNTER>', 'FETCH_SIZE')}", f"    {cmd.replace('<COUNTER>', 'WRITE_SIZE')}", "",
           f"Copy probe (256 MiB read + 256 MiB written): FETCH_SIZE reads {sum(cf) / len(cf):.0f} KiB, WRITE_SIZE "
           f"{sum(cw) / len(cw):.0f} KiB, so FETCH_SIZE is scaled by {sf:.3f} and WRITE_SIZE by {sw:.3f}.", "",
           "| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | HBM bytes/dispatch (scaled) |",
           "|---|---|---|---|---|"]
    rows = []
    for k in f:
        if k in w and "copyBuffer" not in k:
            a, b = sum(f[k]) / len(f[k]), sum(w[k]) / len(w[k])
            rows.append((len(f[k]) * (a * sf + b * sw), k, len(f[k]), a, b))
    rec = None
    for _, k, c, a, b in sorted(rows, reverse=True)[:20]:
        out.append(f"| `{k}` | {c} | {a:.1f} | {b:.1f} | {(a * sf + b * sw) * 1024:.4g} |")
        if rec is None and (k.endswith(kernel) or k.split("<")[0].endswith(kernel)):  # the largest variant
            with open(source, "rb") as fh:
                sha = hashlib.sha256(fh.read()).hexdigest()
            rec = {"kernel": k, "bytes_per_dispatch": (a * sf + b * sw) * 1024, "fetch_kib": a, "write_kib": b,
                   "fetch_scale": sf, "write_scale": sw, "source": os.path.relpath(source), "source_sha256": sha}
    out += ["", "Record read by bench.py:", "", json.dumps(rec)]
    return "\n".join(out)


def counters(db, cmd, title, match=""):
    """Average of every collected counter per dispatch, for the kernels whose name contains `match` (all when
    empty), the twelve with the most GPU cycles over all their dispatches first (dispatch count when no cycle
    counter was collected); derived ratios for the MFMA counters when present."""
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, counter, v in sqlite3.connect(db).execute("select kernel_name, counter_name, value from counters_collection"):
        k = name.split("(")[0].replace("void ", "")
        if match in k:
            d[k][counter].append(v)
    out = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", f"    {cmd}", "",
           "Per-dispatch averages (counters summed over the device's units by rocprofv3).", ""]
    def weight(cs):
        v = cs.get("GRBM_GUI_ACTIVE")
        return sum(v) if v else max(len(x) for x in cs.values())

    for k, cs in sorted(d.items(), key=lambda kv: -weight(kv[1]))[:12]:
        n = max(len(v) for v in cs.values())
        avg = {c: sum(v) / len(v) for c, v in cs.items()}
        out.append(f"## `{k}` ({n} dispatches)")
        out.append("")
        for c in sorted(avg):
            out.append(f"* {c}: {avg[c]:.6g}")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in avg and "GRBM_GUI_ACTIVE" in avg and avg["GRBM_GUI_ACTIVE"] > 0:
            # GRBM_GUI_ACTIVE arrives summed over the 8 XCDs (each counts the kernel's cycles); MFMA busy cycles
            # are summed over the 1024 SIMDs (256 CUs x 4)
            cyc = avg["GRBM_GUI_ACTIVE"] / 8
            out.append(f"* GPU cycles per XCD: {cyc:.6g}")
            out.append(f"* MFMA busy fraction: {avg['SQ_VALU_MFMA_BUSY_CYCLES'] / (cyc * 1024):.4f}")
        out.append("")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "kernels":
        print(kernels(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5]))
    elif sys.argv[1] == "counters":
        print(counters(*sys.argv[2:6]))
    else:
        print(traffic(*sys.argv[2:8]))
