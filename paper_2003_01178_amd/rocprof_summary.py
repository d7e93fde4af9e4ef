"""Summaries of rocprofv3 CSV output for the measurement records in profiles/.

    python -m paper_2003_01178_amd.rocprof_summary stats  <kernel_stats.csv> <out.md> <title> <command>
    python -m paper_2003_01178_amd.rocprof_summary traffic <out.json> <kernel substring> \
        <fetch_dir> <write_dir> <copy_fetch_dir> <copy_write_dir> <copy_bytes> [sources=a.hip,b.hpp] <command...>

`traffic` scales the per-dispatch FETCH_SIZE and WRITE_SIZE of a kernel by
what the same counters read for a plain device copy of known size (bytes
read = bytes written = copy_bytes), and records the hash of the kernel
sources they were taken with, so a later change of the kernel voids them
(the star kernel's sources unless `sources=` names others, relative to the
package directory).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
STAR_SOURCES = ("csrc/star.hip", "csrc/block.hpp")
# the part of internal.hpp that the star kernel compiles against
STAR_DECLS = ("csrc/internal.hpp", b"// Device form of a star query", b"// ----------------------------------------------------------- shared scan")


def source_hash(files=STAR_SOURCES, decls=STAR_DECLS):
    """Hash of the sources the star kernel is built from."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    path, begin, end = decls
    with open(os.path.join(HERE, path), "rb") as fh:
        text = fh.read()
    i, j = text.find(begin), text.find(end)
    if i < 0 or j < i:
        raise ValueError(f"star declarations not found in {path}")
    h.update(text[i:j])
    return h.hexdigest()[:16]


def _counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def per_dispatch(d, kernel_substring, counter):
    vals = [float(r["Counter_Value"]) for r in _counter_rows(d)
            if kernel_substring in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise ValueError(f"no {counter} rows for {kernel_substring} in {d}")
    return sum(vals) / len(vals), len(vals)


def stats(csv_path, out_md, title, command):
    with open(csv_path) as f:
        rows = list(csv.DictReader(f))
    lines = [f"# {title}", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def file_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(out_json, kernel, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, command,
            sources=None):
    copy_bytes = int(copy_bytes)
    cf, _ = per_dispatch(copy_fetch_dir, "copyBuffer", "FETCH_SIZE")
    cw, _ = per_dispatch(copy_write_dir, "copyBuffer", "WRITE_SIZE")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    kf, nf = per_dispatch(fetch_dir, kernel, "FETCH_SIZE")
    kw, nw = per_dispatch(write_dir, kernel, "WRITE_SIZE")
    rec = {"kernel": kernel, "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw,
           "dispatches": [nf, nw], "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "traffic_bytes": kf * 1024.0 * f_scale + kw * 1024.0 * w_scale,
           "source_hash": source_hash() if not sources else file_hash(sources),
           "sources": list(sources) if sources else [*STAR_SOURCES, STAR_DECLS[0]], "command": command}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[5:]))
    elif sys.argv[1] == "traffic":
        rest = sys.argv[9:]
        srcs = None
        if rest and rest[0].startswith("sources="):
            srcs = rest[0][len("sources="):].split(",")
            rest = rest[1:]
        traffic(*sys.argv[2:9], " ".join(rest), sources=srcs)
    else:
        raise SystemExit(__doc__)
