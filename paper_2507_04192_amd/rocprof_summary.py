"""Summaries of rocprofv3 CSV output for the kernels of this library.

    python -m paper_2507_04192_amd.rocprof_summary trace DIR
        per-kernel calls and average duration (from *_kernel_stats.csv)
    python -m paper_2507_04192_amd.rocprof_summary pmc DIR
        per-kernel average of each collected counter (*_counter_collection.csv)
    python -m paper_2507_04192_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR COPY_BYTES OUT.json
        HBM bytes per dispatch of every kernel from a FETCH_SIZE run and a
        WRITE_SIZE run (KiB per dispatch), each scaled by what the same
        counter reads for a plain device copy of COPY_BYTES bytes recorded
        in the same runs; the result is keyed by the hash of the kernel
        sources so that a later change of the kernels invalidates it.

Kernel names are shortened to the template name and its arguments
("k_p2g<float, 3, 1>"); the copy is the largest dispatch whose name
contains "copy".
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_sources_hash() -> str:
    """SHA-256 over the HIP sources and the public header, in name order."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*"))) + [os.path.join(HERE, "..", "include", "mpm.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    m = re.search(r"(?:mpm::)?(\w+<[^()]*>)\(", name)
    if m:
        return m.group(1)
    m = re.search(r"(\w+)\(", name)
    return m.group(1) if m else name[:80]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def trace(d: str):
    """[(short name, calls, avg_us, total_ms, percent)] by total time."""
    rows = []
    with open(_find(d, "_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    rows.sort(key=lambda r: -r[3])
    return rows


def pmc(d: str):
    """{short name: {counter: mean value per dispatch}} and {name: dispatches}."""
    acc = defaultdict(lambda: defaultdict(list))
    with open(_find(d, "_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            acc[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    means = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}
    counts = {k: max(len(v) for v in cs.values()) for k, cs in acc.items()}
    return means, counts


def _copy_value(d: str, counter: str) -> float:
    best = 0.0
    with open(_find(d, "_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if "copy" in r["Kernel_Name"].lower() and r["Counter_Name"] == counter:
                best = max(best, float(r["Counter_Value"]))
    if best <= 0:
        raise RuntimeError(f"no copy dispatch with {counter} in {d}")
    return best


def traffic(fetch_dir: str, write_dir: str, copy_bytes: int):
    fm, _ = pmc(fetch_dir)
    wm, _ = pmc(write_dir)
    cf = _copy_value(fetch_dir, "FETCH_SIZE")
    cw = _copy_value(write_dir, "WRITE_SIZE")
    sf, sw = copy_bytes / cf, copy_bytes / cw      # bytes per counter unit
    out = {"csrc_sha256": kernel_sources_hash(), "copy_bytes": copy_bytes,
           "copy_fetch_counter": cf, "copy_write_counter": cw,
           "bytes_per_fetch_unit": sf, "bytes_per_write_unit": sw, "kernels": {}}
    for k in sorted(set(fm) | set(wm)):
        fb = fm.get(k, {}).get("FETCH_SIZE")
        wb = wm.get(k, {}).get("WRITE_SIZE")
        out["kernels"][k] = {"fetch_bytes": None if fb is None else fb * sf,
                             "write_bytes": None if wb is None else wb * sw}
    return out


def main(argv=None):
    a = list(sys.argv[1:] if argv is None else argv)
    if not a:
        print(__doc__)
        return 2
    if a[0] == "trace":
        print("| kernel | calls | avg us | total ms | % |")
        print("|---|---:|---:|---:|---:|")
        for n, c, us, ms, p in trace(a[1]):
            print(f"| `{n}` | {c} | {us:.2f} | {ms:.2f} | {p:.1f} |")
    elif a[0] == "pmc":
        means, counts = pmc(a[1])
        ctrs = sorted({c for v in means.values() for c in v})
        print("| kernel | dispatches | " + " | ".join(ctrs) + " |")
        print("|---|---:|" + "---:|" * len(ctrs))
        for k in sorted(means):
            print(f"| `{k}` | {counts[k]} | " + " | ".join(f"{means[k].get(c, float('nan')):.4g}" for c in ctrs)
                  + " |")
    elif a[0] == "traffic":
        out = traffic(a[1], a[2], int(a[3]))
        with open(a[4], "w") as f:
            json.dump(out, f, indent=1)
        for k, v in out["kernels"].items():
            fb, wb = v["fetch_bytes"], v["write_bytes"]
            print(f"{k:40s} fetch {fb and fb / 2**20:10.2f} MiB  write {wb and wb / 2**20:10.2f} MiB")
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main())
