"""Markdown summaries of rocprofv3 output for the kernels of librbsog.so.

    python3 -m paper_2205_13824_amd.profsummary trace <dir> <prefix>
        kernel durations from <prefix>_kernel_stats.csv (every dispatch) and
        <prefix>_kernel_trace.csv (the steady-state dispatches: those of the
        grid size most dispatches of the kernel used, without the ones that
        returned at once, steps with a near-list build apart)
    python3 -m paper_2205_13824_amd.profsummary counters <dir> <prefix> [...]
        per-dispatch counter means from <prefix>_counter_collection.csv files
        (steady-state dispatches as above)
    python3 -m paper_2205_13824_amd.profsummary traffic <dir> <fetch_prefix> <write_prefix> <copy_mib>
        HBM bytes per dispatch: FETCH_SIZE and WRITE_SIZE (KiB) scaled by what
        they read for the plain device-to-device copies of <copy_mib> MiB that
        bench.py --copy-probe-mib runs last; each row carries the hash of
        its kernel's source file and the shared headers, which bench.py
        compares before it reports the bytes

Only files that rocprofv3 wrote are read; nothing here runs on the GPU.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import re
import statistics
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def sources_sha256() -> str:
    """Hash of the kernel sources (csrc/*.hip and *.h, sorted by name)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# the source file that defines each kernel of the library
KERNEL_FILES = {
    "k_rho": "kernels_far.hip", "k_rho_reduce": "kernels_far.hip", "k_far": "kernels_far.hip",
    "k_far_side": "kernels_far.hip", "k_far_finish": "kernels_far.hip",
    "k_near_list": "kernels_near.hip", "k_near_cells": "kernels_near.hip", "k_list_build": "kernels_near.hip",
    "k_neighbors": "kernels_near.hip",
    "k_kdq": "kernels_md.hip", "k_bin": "kernels_md.hip", "k_scan_blocks": "kernels_md.hip",
    "k_scan_apply": "kernels_md.hip", "k_cell_scatter": "kernels_md.hip", "k_sort_gather": "kernels_md.hip",
    "k_kinetic": "kernels_md.hip", "k_msd": "kernels_md.hip", "k_fill_i32": "kernels_md.hip",
    "k_refill": "kernels_sample.hip", "k_sf_partial": "structure_factor.hip", "k_sf_reduce": "structure_factor.hip",
    "k_probe": "probe_rates.hip",
}


def kernel_sha16(kernel: str):
    """First 16 hex digits of the hash of the file that defines `kernel`
    (short name, template arguments allowed) and the shared headers; None
    for kernels outside the library."""
    base = kernel.split("<")[0]
    src = KERNEL_FILES.get(base)
    if src is None:
        return None
    h = hashlib.sha256()
    for name in (src, "rbsog_internal.h", "rbsog_math.h"):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """`rbsog::(anonymous namespace)::k_rho<false>(rbsog::EvalArgs, ...)` -> `k_rho<false>`."""
    name = name.strip()
    name = re.sub(r"^.*::(?=k_\w+)", "", name)
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _grid(r):
    for k in ("Grid_Size", "Grid_Size_X"):
        if k in r:
            g = int(float(r[k]))
            for extra in ("Grid_Size_Y", "Grid_Size_Z"):
                if extra in r:
                    g *= int(float(r[extra]))
            return g
    return 0


def steady(dispatches):
    """dispatches: list of (grid, duration_ns, payload).  The grid size most
    dispatches used, minus those shorter than a tenth of that group's median
    (kernels that return at once when no work is due)."""
    by_grid = defaultdict(list)
    for d in dispatches:
        by_grid[d[0]].append(d)
    grid = max(by_grid, key=lambda g: (len(by_grid[g]), g))
    group = by_grid[grid]
    med = statistics.median(d[1] for d in group)
    return grid, [d for d in group if d[1] >= 0.1 * med]


def trace(directory, prefix):
    out = []
    stats = os.path.join(directory, f"{prefix}_kernel_stats.csv")
    if os.path.exists(stats):
        rows = _rows(stats)
        out.append("Every dispatch (`--stats`):\n")
        out.append("| kernel | calls | avg us | min us | max us | % of GPU time |")
        out.append("|---|---:|---:|---:|---:|---:|")
        for r in rows:
            out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                       f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                       f"{float(r['Percentage']):.2f} |")
        out.append("")
    tr = os.path.join(directory, f"{prefix}_kernel_trace.csv")
    if os.path.exists(tr):
        rows = []
        for r in _rows(tr):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]), _grid(r)))
        rows.sort()
        windows = build_windows(rows)
        per, per_b = defaultdict(list), defaultdict(list)
        for s0, e0, k, g in rows:
            (per_b if in_windows(windows, s0) else per)[k].append((g, e0 - s0, None))
        out.append(f"Steady-state dispatches of steps without a near-list build ({len(windows)} steps with one left "
                   "out; the grid size most dispatches used; dispatches shorter than a tenth of that group's "
                   "median, which returned at once, left out):\n")
        out += _steady_table(per)
        if per_b:
            out.append("Steps with a near-list build (same filters):\n")
            out += _steady_table(per_b)
    return "\n".join(out)


def _steady_table(per):
    out = ["| kernel | grid | dispatches | mean us | median us | min us | max us |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    rows = []
    for k, ds in per.items():
        grid, st = steady(ds)
        t = [d[1] / 1e3 for d in st]
        rows.append((sum(t), f"| `{k}` | {grid} | {len(t)} / {len(ds)} | {statistics.mean(t):.1f} | "
                             f"{statistics.median(t):.1f} | {min(t):.1f} | {max(t):.1f} |"))
    out += [r for _, r in sorted(rows, key=lambda x: -x[0])]
    out.append("")
    return out


def build_windows(rows):
    """[start, end] of the steps that built a near list: from the last k_kdq
    dispatch before a working k_list_build (one longer than a quarter of the
    longest) to the end of the first far-force dispatch after it.  rows:
    sorted (start, end, kernel, grid)."""
    builds = [(s, e) for s, e, k, _ in rows if k.startswith("k_list_build")]
    if not builds:
        return []
    longest = max(e - s for s, e in builds)
    out = []
    for s, e in builds:
        if e - s < 0.25 * longest:
            continue
        w0 = max((r[0] for r in rows if r[2] == "k_kdq" and r[0] <= s), default=s)
        w1 = min((r[1] for r in rows if r[2].startswith(("k_far<", "k_far_finish")) and r[0] >= e), default=e)
        out.append((w0, w1))
    return out


def in_windows(windows, t):
    return any(w0 <= t <= w1 for w0, w1 in windows)


def _counter_table(paths):
    per = defaultdict(lambda: defaultdict(list))  # kernel -> dispatch -> [(counter, value, grid, dur)]
    for p in paths:
        for r in _rows(p):
            k = short_name(r["Kernel_Name"])
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            per[k][(p, r["Dispatch_Id"])].append((r["Counter_Name"], float(r["Counter_Value"]), _grid(r), dur))
    result = {}
    for k, disp in per.items():
        ds = [(v[0][2], v[0][3], v) for v in disp.values()]
        grid, st = steady(ds)
        sums = defaultdict(list)
        for _, _, v in st:
            for name, val, _, _ in v:
                sums[name].append(val)
        result[k] = (grid, len(st), len(ds), {n: statistics.mean(v) for n, v in sums.items()})
    return result


def counters(directory, prefixes):
    paths = [os.path.join(directory, f"{p}_counter_collection.csv") for p in prefixes]
    tab = _counter_table([p for p in paths if os.path.exists(p)])
    names = sorted({n for v in tab.values() for n in v[3]})
    out = ["Mean per steady-state dispatch (the grid size most dispatches used, without dispatches that "
           "returned at once):\n",
           "| kernel | dispatches | " + " | ".join(names) + " |",
           "|---|---:|" + "---:|" * len(names)]
    for k in sorted(tab, key=lambda k: -tab[k][3].get(names[0], 0.0) if names else 0.0):
        grid, n, nall, vals = tab[k]
        out.append(f"| `{k}` | {n} / {nall} | " + " | ".join(f"{vals[c]:.4g}" if c in vals else "-" for c in names)
                   + " |")
    return "\n".join(out) + "\n"


def traffic(directory, fetch_prefix, write_prefix, copy_mib):
    f = _counter_table([os.path.join(directory, f"{fetch_prefix}_counter_collection.csv")])
    w = _counter_table([os.path.join(directory, f"{write_prefix}_counter_collection.csv")])
    kib = copy_mib * 1024

    def probe(path, counter):
        # the copies: the non-library dispatches with the largest count (the
        # copy probe moves far more than any other copy of the run), mean of
        # those within 10 % of it
        vals = [(short_name(r["Kernel_Name"]), float(r["Counter_Value"])) for r in _rows(path)
                if r["Counter_Name"] == counter and not short_name(r["Kernel_Name"]).startswith("k_")]
        if not vals:
            return None
        top = max(v for _, v in vals)
        sel = [(k, v) for k, v in vals if v >= 0.9 * top]
        return sel[0][0], statistics.mean(v for _, v in sel)

    pf = probe(os.path.join(directory, f"{fetch_prefix}_counter_collection.csv"), "FETCH_SIZE")
    pw = probe(os.path.join(directory, f"{write_prefix}_counter_collection.csv"), "WRITE_SIZE")
    if pf is None or pw is None:
        raise SystemExit("no copy-probe dispatch in the counter files")
    sf, sw = kib / pf[1], kib / pw[1]
    out = [f"Scale factors from the plain copy (`{pf[0]}`, {copy_mib} MiB read and written per dispatch):\n",
           f"* FETCH_SIZE reads {pf[1]:.0f} KiB per copy: scale {sf:.4f}",
           f"* WRITE_SIZE reads {pw[1]:.0f} KiB per copy: scale {sw:.4f}", "",
           "| kernel | dispatches | FETCH_SIZE KiB | read bytes / launch | WRITE_SIZE KiB | written bytes / launch | source sha256 |",
           "|---|---:|---:|---:|---:|---:|---|"]
    for k in sorted(f, key=lambda k: -f[k][3].get("FETCH_SIZE", 0.0)):
        if not k.startswith("k_"):
            continue
        fv = f[k][3].get("FETCH_SIZE")
        wv = w.get(k, (0, 0, 0, {}))[3].get("WRITE_SIZE")
        if fv is None or wv is None:
            continue
        out.append(f"| `{k}` | {f[k][1]} / {f[k][2]} | {fv:.0f} | {fv * sf * 1024:.4g} | {wv:.0f} | "
                   f"{wv * sw * 1024:.4g} | {kernel_sha16(k)} |")
    out.append("")
    return "\n".join(out) + "\n"


def read_traffic(path):
    """{kernel: (read bytes, written bytes)} of a traffic summary, for the
    kernels whose source still hashes to the value recorded there."""
    tab = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"\| `(k_[^`]+)` \| [^|]+\| [^|]+\| ([0-9.e+]+) \| [^|]+\| ([0-9.e+]+) \| ([0-9a-f]+) \|",
                         line)
            if m and m.group(4) == kernel_sha16(m.group(1)):
                tab[m.group(1)] = (float(m.group(2)), float(m.group(3)))
    return tab


def main(argv):
    if len(argv) < 3:
        raise SystemExit(__doc__)
    if argv[0] == "trace":
        print(trace(argv[1], argv[2]))
    elif argv[0] == "counters":
        print(counters(argv[1], argv[2:]))
    elif argv[0] == "traffic":
        print(traffic(argv[1], argv[2], argv[3], int(argv[4])))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
