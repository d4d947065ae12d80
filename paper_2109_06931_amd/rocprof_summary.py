"""Summaries of rocprofv3 CSV output (``--output-format csv``).

    python -m paper_2109_06931_amd.rocprof_summary stats DIR [--top N]
        kernel table from *kernel_stats.csv: calls, average and total duration
    python -m paper_2109_06931_amd.rocprof_summary pmc DIR
        per-kernel average of every counter in *counter_collection.csv
    python -m paper_2109_06931_amd.rocprof_summary bytes --fetch D1 --write D2 \\
            --copy-fetch D3 --copy-write D4 --copy-bytes B
        table of read and written bytes per dispatch for every kernel, scaled
        as below
    python -m paper_2109_06931_amd.rocprof_summary traffic --fetch D1 --write D2 \\
            --copy-fetch D3 --copy-write D4 --copy-bytes B --kernel NAME --source FILE [--source FILE ...] --out JSON
        HBM bytes per launch of kernel NAME: FETCH_SIZE and WRITE_SIZE (KiB per
        dispatch) scaled by what the same counters read for a plain copy of B
        bytes; records the sha256 of the kernel's sources (concatenated in the
        order given) so that readers can tell when the figures no longer
        describe the code.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict


def _files(d, suffix):
    out = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not out:
        sys.exit(f"no *{suffix} under {d}")
    return out


def _short(name, width=70):
    name = name.replace("hpa::(anonymous namespace)::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(d, top=15):
    rows = []
    for f in _files(d, "kernel_stats.csv"):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    return "\n".join(lines)


def pmc_table(d):
    acc = defaultdict(lambda: defaultdict(list))
    for f in _files(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                acc[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} | {"dispatches": max(len(v) for v in cs.values())}
            for k, cs in acc.items()}


def _pick(table, kernel):
    hits = {k: v for k, v in table.items() if kernel in k}
    if not hits:
        sys.exit(f"kernel {kernel!r} not in the counter output")
    # the busiest matching kernel (template instances share a name prefix)
    return max(hits.values(), key=lambda v: v.get("dispatches", 0))


def _scales(a):
    cf = max(pmc_table(a.copy_fetch).values(), key=lambda v: v.get("FETCH_SIZE", 0))["FETCH_SIZE"]
    cw = max(pmc_table(a.copy_write).values(), key=lambda v: v.get("WRITE_SIZE", 0))["WRITE_SIZE"]
    return cf, cw, a.copy_bytes / (cf * 1024.0), a.copy_bytes / (cw * 1024.0)


def bytes_table(a):
    fetch, write = pmc_table(a.fetch), pmc_table(a.write)
    _, _, sf, sw = _scales(a)
    rows = []
    for k in set(fetch) | set(write):
        f = fetch.get(k, {}).get("FETCH_SIZE", 0.0)
        w = write.get(k, {}).get("WRITE_SIZE", 0.0)
        rows.append((f * 1024.0 * sf + w * 1024.0 * sw, k, f, w))
    rows.sort(reverse=True)
    lines = ["| kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | read GB (scaled) | written GB (scaled) |",
             "|---|---:|---:|---:|---:|"]
    for _, k, f, w in rows:
        if k.startswith("__amd_rocclr") or k.startswith("void at::"):
            continue
        lines.append(f"| `{_short(k)}` | {f:,.0f} | {w:,.0f} | {f * 1024 * sf / 1e9:.3f} | {w * 1024 * sw / 1e9:.3f} |")
    return "\n".join(lines)


def sources_sha256(files):
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic(a):
    f = _pick(pmc_table(a.fetch), a.kernel)["FETCH_SIZE"]
    w = _pick(pmc_table(a.write), a.kernel)["WRITE_SIZE"]
    cf, cw, sf, sw = _scales(a)
    out = {"kernel": a.kernel, "sources": [os.path.relpath(f) for f in a.source], "source_sha256": sources_sha256(a.source),
           "fetch_kib_per_launch": f, "write_kib_per_launch": w,
           "copy_bytes": a.copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": sf, "write_scale": sw,
           "fetch_bytes_per_launch": f * 1024.0 * sf, "write_bytes_per_launch": w * 1024.0 * sw}
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=15)
    p = sub.add_parser("pmc")
    p.add_argument("dir")
    t = sub.add_parser("traffic")
    for k in ["fetch", "write", "copy-fetch", "copy-write", "kernel", "out"]:
        t.add_argument(f"--{k}", required=True)
    t.add_argument("--source", action="append", required=True)
    b = sub.add_parser("bytes")
    for k in ["fetch", "write", "copy-fetch", "copy-write"]:
        b.add_argument(f"--{k}", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats(a.dir, a.top))
    elif a.cmd == "pmc":
        for k, v in sorted(pmc_table(a.dir).items(), key=lambda kv: kv[0]):
            print(_short(k), json.dumps({c: round(x, 1) for c, x in v.items()}))
    elif a.cmd == "bytes":
        print(bytes_table(a))
    else:
        print(json.dumps(traffic(a), indent=1))


if __name__ == "__main__":
    main()
