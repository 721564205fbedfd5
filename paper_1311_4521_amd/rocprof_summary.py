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

    python -m paper_1311_4521_amd.rocprof_summary requests READ_DIR WRITE_DIR OUT_MD SITES COPY_BYTES

``requests`` reads two counter runs that bin the L2-to-memory requests by
size: ``TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum
TCC_EA0_RDREQ_sum`` and ``TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum
TCC_EA0_RDREQ_DRAM_sum``.  Read bytes are 32, 64 and 128 times the binned
counts, write bytes 64 times the 64-byte and 32 times the other write
requests: no scale factor, and the streaming copy of known size in the same
run checks them.  It writes a per-kernel table (bytes per launch and per
site).

    python -m paper_1311_4521_amd.rocprof_summary units OUT_MD DIR [DIR ...]

``units`` reads counter runs that each include ``GRBM_GUI_ACTIVE`` and, per
kernel, averages every other counter divided by the ``GRBM_GUI_ACTIVE`` of
the same dispatch (busy and stall cycles of the texture-address, texture-data
and L1 units, wave and instruction levels of the sequencers), leaving out
dispatches shorter than a quarter of the kernel's longest (the early exits of
iterations past convergence).  The streaming copy of the same run gives the
reference row.

    python -m paper_1311_4521_amd.rocprof_summary gaps TRACE_CSV PATTERN [LAST_N]

``gaps`` measures, from a kernel trace, how much of the wall time of the
last LAST_N dispatches whose names contain PATTERN (default: all of them)
lies between kernels rather than inside one: the launch-boundary share of a
stretch of back-to-back launches.
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


def short_name(name: str, width: int = 70) -> str:
    """Kernel name without the namespace, the return type and the parameter
    list (the template arguments stay), cut to `width` characters."""
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("tmh::(anonymous namespace)::", "").replace("tmh::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            n = n[:i]
            break
    return n if len(n) <= width else n[: width - 3] + "..."


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
        short = short_name(name)
        ex, avg = work.get(name, (None, None))
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} | "
                     f"{'' if ex is None else ex} | {'' if avg is None else f'{avg:.2f}'} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


RD_BINS = (("TCC_EA0_RDREQ_32B_sum", 32), ("TCC_EA0_RDREQ_64B_sum", 64), ("TCC_EA0_RDREQ_128B_sum", 128))


def _mean_per_kernel(rows, counter):
    acc = {}
    for r in rows:
        if r["Counter_Name"] == counter:
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def requests(read_dir, write_dir, out_md, sites, copy_bytes, command=""):
    """Bytes per launch from the size-binned request counters (see module
    docstring).  Returns {kernel: (read bytes, write bytes, launches)}."""
    rrows, wrows = _rows(read_dir), _rows(write_dir)
    rd = {}
    counts = {}
    for counter, size in RD_BINS:
        m, n = _mean_per_kernel(rrows, counter)
        for k, v in m.items():
            rd[k] = rd.get(k, 0.0) + size * v
            counts[k] = n[k]
    wall, _ = _mean_per_kernel(wrows, "TCC_EA0_WRREQ_sum")
    w64, _ = _mean_per_kernel(wrows, "TCC_EA0_WRREQ_64B_sum")
    dram, _ = _mean_per_kernel(wrows, "TCC_EA0_RDREQ_DRAM_sum")
    wr = {k: 64.0 * w64.get(k, 0.0) + 32.0 * (v - w64.get(k, 0.0)) for k, v in wall.items()}
    copy = [k for k in rd if COPY in k]
    if not copy:
        raise SystemExit("no streaming copy in the counter output")
    cr, cw = rd[copy[0]], wr.get(copy[0], 0.0)
    res = {k: (rd[k], wr.get(k, 0.0), counts[k], dram.get(k)) for k in rd if "tmh::" in k}
    lines = [f"Counters binned by request size: read bytes = 32 n32 + 64 n64 + 128 n128, write bytes = "
             f"64 n64 + 32 (n - n64), no scale factor.  Check: the streaming copy of {copy_bytes:,.0f} bytes "
             f"reads {cr:,.0f} and writes {cw:,.0f} bytes per launch ({cr / copy_bytes:.4f} / "
             f"{cw / copy_bytes:.4f}).", "",
             "| kernel | launches | read MB | write MB | read B/site | write B/site | DRAM read requests |",
             "|---|---|---|---|---|---|---|"]
    for k, (r, w, n, d) in sorted(res.items(), key=lambda kv: -kv[1][0]):
        short = short_name(k, 90)
        lines.append(f"| `{short}` | {n} | {r / 1e6:.1f} | {w / 1e6:.1f} | {r / sites:.1f} | {w / sites:.1f} | "
                     f"{'' if d is None else f'{d:,.0f}'} |")
    with open(out_md, "w") as fh:
        if command:
            fh.write(command.rstrip() + "\n\n")
        fh.write("\n".join(lines) + "\n")
    return res


def units(out_md, dirs, command=""):
    """Per kernel, the mean over its dispatches of counter / GRBM_GUI_ACTIVE
    (see module docstring).  Returns {kernel: {counter: (mean, dispatches)}}."""
    ratios = {}
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {d}")
        for f in files:
            disp = {}
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    e = disp.setdefault(r["Dispatch_Id"], {"": r["Kernel_Name"]})
                    e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            longest = {}
            for e in disp.values():
                longest[e[""]] = max(longest.get(e[""], 0.0), e.get("GRBM_GUI_ACTIVE", 0.0))
            for e in disp.values():
                g = e.get("GRBM_GUI_ACTIVE", 0.0)
                if g <= 0.0 or g < 0.25 * longest[e[""]]:
                    continue
                for c, v in e.items():
                    if c not in ("", "GRBM_GUI_ACTIVE"):
                        ratios.setdefault(e[""], {}).setdefault(c, []).append(v / g)
    res = {k: {c: (sum(v) / len(v), len(v)) for c, v in cs.items()} for k, cs in ratios.items()
           if "tmh::" in k or COPY in k}
    counters = sorted({c for cs in res.values() for c in cs})
    lines = ["Each entry: counter / GRBM_GUI_ACTIVE of the same dispatch, averaged over the kernel's "
             "dispatches (early exits left out).", "",
             "| kernel | " + " | ".join(f"`{c}`" for c in counters) + " |",
             "|---|" + "---|" * len(counters)]
    for k in sorted(res, key=lambda k: (COPY not in k, short_name(k, 90))):
        cells = [f"{res[k][c][0]:.4g}" if c in res[k] else "" for c in counters]
        lines.append(f"| `{short_name(k, 90)}` | " + " | ".join(cells) + " |")
    with open(out_md, "w") as fh:
        if command:
            fh.write(command.rstrip() + "\n\n")
        fh.write("\n".join(lines) + "\n")
    return res


def gaps(trace_csv, pattern, last_n=None):
    """(kernel busy ns, wall ns, dispatches) over the last `last_n` dispatches
    whose names contain `pattern`, taken as one back-to-back stretch."""
    with open(trace_csv) as fh:
        rows = [r for r in csv.DictReader(fh) if pattern in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    if last_n:
        rows = rows[-int(last_n):]
    if not rows:
        raise SystemExit(f"no dispatch matches {pattern!r}")
    busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows)
    wall = int(rows[-1]["End_Timestamp"]) - int(rows[0]["Start_Timestamp"])
    return busy, wall, len(rows)


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
    elif cmd == "requests":
        requests(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]), float(sys.argv[6]),
                 command=os.environ.get("TMH_PROFILE_COMMAND", ""))
    elif cmd == "units":
        units(sys.argv[2], sys.argv[3:], command=os.environ.get("TMH_PROFILE_COMMAND", ""))
    elif cmd == "gaps":
        b, wl, n = gaps(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else None)
        print(f"{n} dispatches: kernels busy {b / 1e6:.3f} ms of {wl / 1e6:.3f} ms wall, "
              f"between kernels {100.0 * (wl - b) / wl:.1f} %")
    else:
        raise SystemExit(__doc__)
