"""Summaries of rocprofv3 output for the hopping-matrix kernels.

    python -m paper_1311_4521_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR OUT_JSON
    python -m paper_1311_4521_amd.rocprof_summary stats STATS_CSV OUT_MD

``traffic`` reads two ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
runs of ``bench.py`` (``--output-format csv``).  Both counters are in KiB per
dispatch.  Each is scaled by the factor that makes the streaming copy kernel
(``tmh_stream_copy``, same run, known size) read exactly the bytes it moves;
the scaled per-dispatch average of the dominant kernel is written as JSON
together with a hash of the kernel sources, so that ``bench.py`` can tell
counters taken on older code from current ones.

``stats`` turns a ``rocprofv3 --kernel-trace --stats`` kernel_stats.csv into
a short markdown table.
"""

from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
HOP_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("hop.hip", "hop_body.h", "common.h", "kernels.h")]
DOMINANT = "tmh::hop_kernel<double, 0, 0>"
COPY = "stream_copy_kernel"


def hop_source_hash() -> str:
    h = hashlib.sha256()
    for f in HOP_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = []
    for f in files:
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def _per_kernel(rows, counter):
    acc = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
    return acc


def _pick(acc, key):
    vals = [v for k, lst in acc.items() if key in k for v in lst]
    if not vals:
        raise SystemExit(f"kernel {key!r} not in the counter output")
    return sum(vals) / len(vals), len(vals)


def traffic(fetch_dir, write_dir, out_json, copy_bytes=None, sites=None):
    fetch = _per_kernel(_rows(fetch_dir), "FETCH_SIZE")
    write = _per_kernel(_rows(write_dir), "WRITE_SIZE")
    cf, _ = _pick(fetch, COPY)
    cw, _ = _pick(write, COPY)
    if copy_bytes is None:
        copy_bytes = cw  # the write counter is taken as exact for the copy
    kf, kw = copy_bytes / cf, copy_bytes / cw
    hf, nf = _pick(fetch, DOMINANT)
    hw, nw = _pick(write, DOMINANT)
    res = {
        "kernel": DOMINANT,
        "sites": sites,
        "source_hash": hop_source_hash(),
        "copy_bytes": copy_bytes,
        "fetch_scale": round(kf, 4),
        "write_scale": round(kw, 4),
        "fetch_bytes_per_launch": hf * kf,
        "write_bytes_per_launch": hw * kw,
        "bytes_per_launch": hf * kf + hw * kw,
        "dispatches": [nf, nw],
        "other_kernels": {k[:80]: {"fetch": sum(v) / len(v) * kf} for k, v in fetch.items()
                          if "tmh::" in k},
    }
    with open(out_json, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


def stats(stats_csv, out_md):
    """Per-kernel table from rocprofv3's kernel statistics.  When the kernel
    trace of the same run sits beside it (``*_kernel_trace.csv``), the table
    also gives the average over the dispatches that did work: a CG enqueues
    its iterations 8 at a time, and dispatches of iterations past convergence
    return at once (a few microseconds); a dispatch shorter than a tenth of
    its kernel's median is counted as such an early exit."""
    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    work = {}
    trace = glob.glob(os.path.join(os.path.dirname(stats_csv), "*kernel_trace.csv"))
    if trace:
        durs = {}
        with open(trace[0]) as fh:
            for r in csv.DictReader(fh):
                durs.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        for name, d in durs.items():
            d = sorted(d)
            med = d[len(d) // 2]
            kept = [x for x in d if x >= 0.1 * med]
            work[name] = (len(d) - len(kept), sum(kept) / len(kept) / 1e3)
    lines = ["| kernel | calls | total ms | avg us | % | early exits | avg us of the rest |",
             "|---|---|---|---|---|---|---|"]
    for r in rows[:24]:
        name = r["Name"]
        short = name if len(name) <= 70 else name[:67] + "..."
        ex, avg = work.get(name, (None, None))
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} | "
                     f"{'' if ex is None else ex} | {'' if avg is None else f'{avg:.2f}'} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "traffic":
        extra = {}
        if len(sys.argv) > 5:
            extra["sites"] = int(sys.argv[5])
        if len(sys.argv) > 6:
            extra["copy_bytes"] = float(sys.argv[6])
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4], **extra), indent=1))
    elif cmd == "stats":
        stats(sys.argv[2], sys.argv[3])
    else:
        raise SystemExit(__doc__)
