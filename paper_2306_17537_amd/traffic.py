"""Profile summaries: HBM traffic per kernel launch from two rocprofv3 counter runs (FETCH_SIZE,
then WRITE_SIZE), and the top of a rocprofv3 kernel-trace statistics table.

Both counters are reported in KiB per dispatch but do not read one-to-one on this GPU, so each is
scaled by what it reads for a kernel of known traffic run in the same process: a 1 GiB fill
(writes 1 GiB, reads nothing) for WRITE_SIZE and a 1 GiB device-to-device copy (reads 1 GiB) for
FETCH_SIZE.  ``calibrate()`` issues both; bench.py runs it first under ``--pmc-calibration``.

Summaries are written as markdown with one machine-readable line per kernel variant:
    traffic-json: {"kernel": ..., "fetch_bytes": ..., "write_bytes": ..., "sources": ...}
``sources`` is a hash of the kernel source files at measurement time; ``lookup()`` returns
nothing once the sources have changed, so a stale figure is never reported.  Kernel-trace
summaries carry the same kind of line per kernel (``trace-json:``, average duration), read by
``trace_lookup()``.

Usage (from the repository root, after the profiler runs):
    python -m paper_2306_17537_amd.traffic summarize --fetch DIR1 --write DIR2 \\
        --kernel 'k_xconv<float, 128' --out profiles/NAME.md --command '...'
    python -m paper_2306_17537_amd.traffic stats --dir DIR --out profiles/NAME.md \\
        --command '...' [--top 20] [--extra TEXT]
    python -m paper_2306_17537_amd.traffic counters --dir DIR --kernel REGEX \\
        --out profiles/NAME.md --command '...' (any --pmc counters, median per launch)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
CAL_BYTES = 1 << 30
KERNEL_SOURCES = ("csrc/passes.hpp", "csrc/fft.hpp", "csrc/operator.hip")


def _code_only(text):
    """Source text without comments and blank lines (a comment edit changes no kernel)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def sources_hash():
    """Hash of the kernel sources the operator passes are built from, comments excluded."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(_HERE, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def calibrate():
    """1 GiB fill and 1 GiB copy on the current device (for the counter scale factors)."""
    import torch
    a = torch.empty(CAL_BYTES // 4, dtype=torch.float32, device="cuda:0")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def _rows(directory):
    paths = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not paths:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    out = []
    with open(paths[0]) as f:
        for r in csv.DictReader(f):
            out.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return out


def _factor(rows, counter, pattern):
    vals = [v for k, c, v in rows if c == counter and re.search(pattern, k)]
    if not vals:
        raise ValueError(f"calibration kernel /{pattern}/ not found for {counter}")
    kib = max(vals)  # the 1 GiB dispatch is the largest of its kind
    return CAL_BYTES / (kib * 1024.0)


def summarize(fetch_dir, write_dir, kernel):
    """Per kernel whose name matches the regular expression `kernel`: median scaled
    bytes per launch."""
    fr, wr = _rows(fetch_dir), _rows(write_dir)
    ff = _factor(fr, "FETCH_SIZE", r"copyBuffer")
    wf = _factor(wr, "WRITE_SIZE", r"FillFunctor")
    res = {}
    for rows, counter, fac, key in ((fr, "FETCH_SIZE", ff, "fetch_bytes"),
                                    (wr, "WRITE_SIZE", wf, "write_bytes")):
        per = {}
        for k, c, v in rows:
            if c != counter or not re.search(kernel, k):
                continue
            m = re.search(r"(k_\w+<[^>]*>)", k)
            per.setdefault(m.group(1) if m else k, []).append(v * 1024.0 * fac)
        for name, vals in per.items():
            res.setdefault(name, {})[key] = statistics.median(vals)
            res[name]["launches_" + key.split("_")[0]] = len(vals)
    return dict(fetch_factor=ff, write_factor=wf, kernels=res)


def write_markdown(summary, path, command, title):
    src = sources_hash()
    lines = [f"# {title}", "", "Commands (from /tmp with TMPDIR=/tmp, repository at $R):", "",
             "```", command, "```", "",
             f"Counter scale factors from the in-process 1 GiB calibration kernels: "
             f"FETCH_SIZE x {summary['fetch_factor']:.4f}, WRITE_SIZE x "
             f"{summary['write_factor']:.4f}.", "",
             "| kernel | launches | fetched MB/launch | written MB/launch |", "|---|---|---|---|"]
    for name, d in sorted(summary["kernels"].items()):
        lines.append(f"| `{name}` | {d.get('launches_fetch', 0)} | "
                     f"{d.get('fetch_bytes', 0) / 1e6:.2f} | {d.get('write_bytes', 0) / 1e6:.2f} |")
    lines.append("")
    for name, d in sorted(summary["kernels"].items()):
        lines.append("traffic-json: " + json.dumps(dict(kernel=name, sources=src, **{
            k: v for k, v in d.items() if k.endswith("_bytes")})))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def lookup(kernel, profiles_dir=None):
    """fetch + write bytes per launch of `kernel` (exact template name) from the committed
    summaries, or None if absent or measured on different kernel sources."""
    profiles_dir = profiles_dir or os.path.join(ROOT, "profiles")
    src = sources_hash()
    for path in sorted(glob.glob(os.path.join(profiles_dir, "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-json: "):
                    continue
                d = json.loads(line[len("traffic-json: "):])
                if d["kernel"] == kernel and d.get("sources") == src:
                    return d.get("fetch_bytes", 0.0) + d.get("write_bytes", 0.0), d, path
    return None


def trace_lookup(kernel, profiles_dir=None, summary=None):
    """(average microseconds, calls, summary path) of `kernel` (exact template name) in the
    committed kernel-trace summaries measured on the current kernel sources (only the file
    named `summary` if given: one kernel can serve several grids in a run), or None."""
    profiles_dir = profiles_dir or os.path.join(ROOT, "profiles")
    src = sources_hash()
    pattern = summary if summary else "*.md"
    for path in sorted(glob.glob(os.path.join(profiles_dir, pattern))):
        with open(path) as f:
            for line in f:
                if not line.startswith("trace-json: "):
                    continue
                d = json.loads(line[len("trace-json: "):])
                if d["kernel"] == kernel and d.get("sources") == src:
                    return d["avg_us"], d["calls"], path
    return None


def kernel_stats(directory, top=20):
    """Rows (name, calls, avg us, min us, max us, percent) of a --kernel-trace --stats run."""
    paths = glob.glob(os.path.join(directory, "**", "*kernel_stats.csv"), recursive=True)
    if not paths:
        raise FileNotFoundError(f"no kernel_stats.csv under {directory}")
    rows = []
    with open(paths[0]) as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    rows.sort(key=lambda x: -x[5])
    return rows[:top]


def write_stats_markdown(rows, path, command, title, extra=""):
    lines = [f"# {title}", "", "Command (from /tmp with TMPDIR=/tmp, repository at $R):", "", "```",
             command, "```", "", "| kernel | calls | avg us | min us | max us | % time |",
             "|---|---|---|---|---|---|"]
    src = sources_hash()
    js = []
    for n, c, a, lo, hi, pc in rows:
        m = re.search(r"(k_\w+(?:<[^>]*>)?|__amd\w+)", n)
        name = m.group(1) if m else re.sub(r"^void ", "", n)
        lines.append(f"| `{name[:80]}` | {c} | {a:.2f} | {lo:.2f} | {hi:.2f} | {pc:.2f} |")
        js.append("trace-json: " + json.dumps(dict(kernel=name, sources=src, calls=c, avg_us=a)))
    if extra:
        lines += ["", extra]
    lines += [""] + js
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(directory, kernel):
    """Median value per launch of every counter of a --pmc run, per kernel whose name matches
    the regular expression `kernel`: {kernel: {counter: (median, launches)}}."""
    per = {}
    for k, c, v in _rows(directory):
        if not re.search(kernel, k):
            continue
        m = re.search(r"(k_\w+<[^>]*>)", k)
        per.setdefault(m.group(1) if m else k, {}).setdefault(c, []).append(v)
    return {k: {c: (statistics.median(vs), len(vs)) for c, vs in d.items()}
            for k, d in per.items()}


def write_counters_markdown(res, path, command, title, extra=""):
    names = sorted({c for d in res.values() for c in d})
    lines = [f"# {title}", "", "Command (from /tmp with TMPDIR=/tmp, repository at $R):", "",
             "```", command, "```", "",
             "Median per launch over the launches of each kernel (counters as rocprofv3 reports "
             "them, summed over the GPU's instances).", "",
             "| kernel | launches | " + " | ".join(names) + " |",
             "|---|---|" + "---|" * len(names)]
    for k in sorted(res):
        d = res[k]
        n = max(v[1] for v in d.values())
        lines.append(f"| `{k}` | {n} | " + " | ".join(
            f"{d[c][0]:.4g}" if c in d else "" for c in names) + " |")
    if extra:
        lines += ["", extra]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("summarize")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--kernel", required=True, help="regular expression on the kernel name")
    s.add_argument("--out", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="HBM traffic per launch")
    k = sub.add_parser("stats")
    k.add_argument("--dir", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--title", default="Kernel trace statistics")
    k.add_argument("--top", type=int, default=20)
    k.add_argument("--extra", default="")
    c = sub.add_parser("counters")
    c.add_argument("--dir", required=True)
    c.add_argument("--kernel", required=True, help="regular expression on the kernel name")
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="Counters per launch")
    c.add_argument("--extra", default="")
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        write_counters_markdown(counters(a.dir, a.kernel), a.out, a.command, a.title, a.extra)
        return 0
    if a.cmd == "stats":
        write_stats_markdown(kernel_stats(a.dir, a.top), a.out, a.command, a.title, a.extra)
        return 0
    summ = summarize(a.fetch, a.write, a.kernel)
    write_markdown(summ, a.out, a.command, a.title)
    print(json.dumps(summ, indent=1))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
