"""Counter audit: parse rocprofv3 CSV output and summarise it.

Section 3 ("Hardware counters") and Section 4.2 ("Counter audit") fix the
rules: counters are collected in a separate run from the timing, are used
only to check how many bytes moved (never for timing), the short warm-up
launch is excluded by rule, failed profiles are excluded, and each figure
is reported as the median with its range over the remaining launches.

Counter scaling: FETCH_SIZE / WRITE_SIZE are read in KiB per dispatch and
scaled by what the same counter reads for a plain device copy of known size
(a copy of B bytes reads B and writes B bytes), so a counter that samples
only part of the memory channels is corrected.

    python -m paper_2608_15764_amd.rocprof summary --trace DIR --fetch DIR \\
        --write DIR --kernel plain_kload --calib-bytes 1073741824 ...
"""
import argparse
import csv
import glob
import math
import os
import statistics
import sys


def _num(v):
    try:
        x = float(v)
    except (TypeError, ValueError):
        return None
    return x if math.isfinite(x) else None


def _csv(path_or_dir, suffix):
    if os.path.isdir(path_or_dir):
        hits = sorted(glob.glob(os.path.join(path_or_dir, "**", f"*{suffix}"),
                                recursive=True))
        if not hits:
            raise FileNotFoundError(f"no *{suffix} under {path_or_dir}")
        path_or_dir = hits[0]
    with open(path_or_dir, newline="") as f:
        return list(csv.DictReader(f))


def counter_rows(path_or_dir):
    """Rows of a rocprofv3 counter_collection CSV, in dispatch order.

    A row whose value is missing or not finite is marked failed.
    """
    out = []
    for r in _csv(path_or_dir, "counter_collection.csv"):
        out.append({"dispatch": int(r.get("Dispatch_Id") or 0),
                    "kernel": r.get("Kernel_Name", ""),
                    "grid": int(_num(r.get("Grid_Size")) or 0),
                    "counter": r.get("Counter_Name", ""),
                    "value": _num(r.get("Counter_Value")),
                    "failed": _num(r.get("Counter_Value")) is None})
    out.sort(key=lambda r: r["dispatch"])
    return out


def trace_rows(path_or_dir):
    """Rows of a rocprofv3 kernel_trace CSV, in start order."""
    out = []
    for r in _csv(path_or_dir, "kernel_trace.csv"):
        s, e = _num(r.get("Start_Timestamp")), _num(r.get("End_Timestamp"))
        out.append({"dispatch": int(r.get("Dispatch_Id") or 0),
                    "kernel": r.get("Kernel_Name", ""),
                    "start": s, "end": e,
                    "ns": (e - s) if (s is not None and e is not None) else None})
    out.sort(key=lambda r: (r["start"] or 0))
    return out


def exclude_warmup(rows, key="kernel"):
    """Drop the first dispatch of every kernel name (the warm-up launch)."""
    seen = set()
    out = []
    for r in rows:
        k = r[key]
        if k in seen:
            out.append(r)
        else:
            seen.add(k)
    return out


def med_range(values):
    v = [x for x in values if x is not None]
    if not v:
        return None
    return {"median": statistics.median(v), "min": min(v), "max": max(v), "n": len(v)}


def counter_values(rows, counter, kernel_substr):
    """Per-dispatch values of one counter for kernels matching a substring,
    warm-up excluded per kernel name, failed dispatches dropped (counted)."""
    sel = [r for r in rows if r["counter"] == counter and kernel_substr in r["kernel"]]
    failed = sum(r["failed"] for r in sel)
    sel = exclude_warmup([r for r in sel if not r["failed"]])
    return [r["value"] for r in sel], failed


def calib_scale(rows, counter, calib_bytes, calib_substr="copyBuffer"):
    """Scale turning the counter's KiB reading into true bytes, from the
    largest device copies (one read and one write of calib_bytes each)."""
    vals = [r["value"] for r in rows
            if r["counter"] == counter and calib_substr in r["kernel"] and not r["failed"]]
    if not vals:
        return None
    top = max(vals)
    big = [v for v in vals if v >= 0.5 * top]
    return calib_bytes / (statistics.median(big) * 1024.0)


def kernel_durations(rows, kernel_substr, exclude_first=True):
    sel = [r for r in rows if kernel_substr in r["kernel"] and r["ns"] is not None]
    if exclude_first:
        sel = exclude_warmup(sel)
    return [r["ns"] for r in sel]


def summary(trace, fetch, write, kernel, calib_bytes, algorithmic_bytes=None):
    out = {"kernel": kernel}
    if trace:
        ns = kernel_durations(trace_rows(trace), kernel)
        out["dispatches"] = len(ns)
        out["mean_ns"] = statistics.fmean(ns) if ns else None
        out["duration_ns"] = med_range(ns)
    total = 0.0
    ok = True
    for name, path, counter in (("fetch", fetch, "FETCH_SIZE"),
                                ("write", write, "WRITE_SIZE")):
        if not path:
            ok = False
            continue
        rows = counter_rows(path)
        vals, failed = counter_values(rows, counter, kernel)
        scale = calib_scale(rows, counter, calib_bytes)
        out[f"{name}_kib"] = med_range(vals)
        out[f"{name}_failed_dispatches"] = failed
        out[f"{name}_scale"] = scale
        if vals and scale:
            b = statistics.fmean(vals) * 1024.0 * scale
            out[f"{name}_bytes_per_launch"] = b
            total += b
        else:
            ok = False
    if ok:
        out["hbm_bytes_per_launch"] = total
    if algorithmic_bytes:
        out["algorithmic_bytes_per_launch"] = algorithmic_bytes
        if ok:
            out["traffic_over_algorithmic"] = total / algorithmic_bytes
        if out.get("mean_ns"):
            out["achieved_gbps"] = algorithmic_bytes / out["mean_ns"]
    return out


def format_summary(s, commands, source_hash=None, notes=()):
    lines = ["# rocprofv3 summary (generated by paper_2608_15764_amd.rocprof)"]
    for c in commands:
        lines.append(f"# command: {c}")
    for n in notes:
        lines.append(f"# {n}")
    if source_hash:
        lines.append(f"source_hash: {source_hash}")
    for k, v in s.items():
        if isinstance(v, dict):
            v = ", ".join(f"{a}={b:.6g}" if isinstance(b, float) else f"{a}={b}"
                          for a, b in v.items())
        elif isinstance(v, float):
            v = f"{v:.6g}" if abs(v) < 1e6 else f"{v:.0f}"
        lines.append(f"{k}: {v}")
    return "\n".join(lines) + "\n"


def per_kernel_stats(trace):
    """Calls and mean duration per kernel name from a kernel trace."""
    agg = {}
    for r in trace_rows(trace):
        if r["ns"] is None:
            continue
        agg.setdefault(r["kernel"], []).append(r["ns"])
    return {k: {"calls": len(v), "mean_ns": statistics.fmean(v)} for k, v in agg.items()}


def attribute(rows, manifest, kernel_substr="plain_kload"):
    """Pair the matching kernel dispatches of one counter run, in order, with
    a launch manifest (a list of dicts, one per launch).  Returns
    {counter: [(manifest entry, value or None)]}."""
    out = {}
    counters = sorted({r["counter"] for r in rows if kernel_substr in r["kernel"]})
    for c in counters:
        sel = [r for r in rows if r["counter"] == c and kernel_substr in r["kernel"]]
        if len(sel) != len(manifest):
            raise ValueError(f"{c}: {len(sel)} dispatches for {len(manifest)} launches")
        out[c] = [(m, r["value"]) for m, r in zip(manifest, sel)]
    return out


CELL_KEYS = ("path", "policy", "bytes", "waves_per_cu", "layout", "K", "order", "mask")


def cell_key(m):
    """The cell a manifest entry belongs to (fields it has, in a fixed order)."""
    return tuple(m[k] for k in CELL_KEYS if k in m)


def cell_table(runs, manifest, fetch_scale=None, kernel_substr="plain_kload",
               cus=None, xccs=None):
    """Per cell: median of every counter over the non-warm-up launches, plus
    the derived L2 hit rate, scaled bytes, mean L1 latencies and, given the
    device's CU and XCC counts, the fraction of CU cycles the LDS was busy
    (SQ_LDS_IDX_ACTIVE is summed over every CU; GRBM_GUI_ACTIVE over every
    XCC)."""
    cells = {}
    for rows in runs:
        for c, pairs in attribute(rows, manifest, kernel_substr).items():
            for m, v in pairs:
                if m["warmup"] or v is None:
                    continue
                key = cell_key(m)
                cells.setdefault(key, {}).setdefault(c, []).append(v)
    table = {}
    for key, cs in sorted(cells.items()):
        row = {c: statistics.median(v) for c, v in cs.items()}
        hit = row.get("TCC_HIT_sum")
        miss = row.get("TCC_MISS_sum")
        if hit is not None and miss is not None and hit + miss > 0:
            row["l2_hit_rate"] = hit / (hit + miss)
        if fetch_scale and "FETCH_SIZE" in row:
            row["fetch_bytes"] = row["FETCH_SIZE"] * 1024.0 * fetch_scale
        gui = row.get("GRBM_GUI_ACTIVE")
        if cus and xccs and gui and "SQ_LDS_IDX_ACTIVE" in row:
            row["lds_busy_frac"] = row["SQ_LDS_IDX_ACTIVE"] / (gui / xccs * cus)
        # mean cycles per L1-to-L2 read request, and per wave instruction
        # in the L1 (the counters' own definitions: totals over requests
        # or over TA state reads)
        for name, total, count in (
                ("tcp_tcc_read_latency", "TCP_TCC_READ_REQ_LATENCY_sum", "TCP_TCC_READ_REQ_sum"),
                ("tcp_wave_latency", "TCP_TCP_LATENCY_sum", "TCP_TA_TCP_STATE_READ_sum")):
            if row.get(count) and total in row:
                row[name] = row[total] / row[count]
        table[key] = row
    return table


def trace_cells(trace, manifest, kernel_substr):
    """Per cell of a launch manifest: the kernel durations of a trace run,
    paired in start order with the manifest's launches, warm-ups dropped;
    median, range and count in ns, and decimal GB/s at the median where the
    manifest gives each launch's issued bytes (``issued_bytes``)."""
    sel = [r for r in trace_rows(trace) if kernel_substr in r["kernel"]]
    if len(sel) != len(manifest):
        raise ValueError(f"{len(sel)} {kernel_substr} dispatches for {len(manifest)} launches")
    cells = {}
    for m, r in zip(manifest, sel):
        if m["warmup"] or r["ns"] is None:
            continue
        c = cells.setdefault(cell_key(m), {"ns": [], "bytes": m.get("issued_bytes")})
        c["ns"].append(r["ns"])
    out = {}
    for key, c in sorted(cells.items()):
        row = med_range(c["ns"])
        if c["bytes"]:
            row["gbps"] = c["bytes"] / row["median"]
        out[key] = row
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="rocprofv3 CSV summaries")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("summary")
    s.add_argument("--trace")
    s.add_argument("--fetch")
    s.add_argument("--write")
    s.add_argument("--kernel", required=True)
    s.add_argument("--calib-bytes", type=int, default=1 << 30)
    s.add_argument("--algorithmic-bytes", type=int, default=None)
    s.add_argument("--source-hash", default=None)
    s.add_argument("--command", action="append", default=[])
    s.add_argument("--note", action="append", default=[])
    s.add_argument("--out", default=None)
    k = sub.add_parser("kernels")
    k.add_argument("--trace", required=True)
    c3 = sub.add_parser("cells", help="per-cell counter table from a manifest")
    c3.add_argument("--manifest", required=True)
    c3.add_argument("--counters", nargs="+", required=True,
                    help="counter_collection CSVs (or directories), one per pass")
    c3.add_argument("--fetch-scale", type=float, default=None)
    c3.add_argument("--calib-bytes", type=int, default=None,
                    help="size of the device copies in the FETCH_SIZE pass: the "
                         "fetch scale is read from them (instead of --fetch-scale)")
    c3.add_argument("--kernel", default="plain_kload",
                    help="substring naming the manifest's kernels")
    c3.add_argument("--cus", type=int, default=None)
    c3.add_argument("--xccs", type=int, default=None)
    c3.add_argument("--command", action="append", default=[])
    c3.add_argument("--out", default=None)
    tc = sub.add_parser("trace-cells", help="per-cell kernel durations from a manifest")
    tc.add_argument("--manifest", required=True)
    tc.add_argument("--trace", required=True)
    tc.add_argument("--kernel", required=True, help="substring naming the manifest's kernels")
    tc.add_argument("--command", action="append", default=[])
    tc.add_argument("--note", action="append", default=[])
    tc.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "trace-cells":
        import json
        with open(a.manifest) as f:
            man = json.load(f)
        tab = trace_cells(a.trace, man, a.kernel)
        lines = ["# rocprofv3 per-cell kernel durations (generated by paper_2608_15764_amd.rocprof)"]
        lines += [f"# command: {c}" for c in a.command]
        lines += [f"# {n}" for n in a.note]
        keys = [k for k in CELL_KEYS if man and k in man[0]]
        lines.append(f"# {' '.join(keys)}: median / min / max ns over non-warm-up launches, "
                     "GB/s at the median")
        for key, row in tab.items():
            gb = f" gbps={row['gbps']:.1f}" if "gbps" in row else ""
            lines.append(f"{' '.join(map(str, key))}: median_ns={row['median']:.0f} "
                         f"min_ns={row['min']:.0f} max_ns={row['max']:.0f} n={row['n']}{gb}")
        text = "\n".join(lines) + "\n"
        if a.out:
            with open(a.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)
        return 0
    if a.cmd == "cells":
        import json
        with open(a.manifest) as f:
            man = json.load(f)
        runs = [counter_rows(p) for p in a.counters]
        scale = a.fetch_scale
        if scale is None and a.calib_bytes:
            scales = [calib_scale(r, "FETCH_SIZE", a.calib_bytes) for r in runs]
            scales = [x for x in scales if x is not None]
            if not scales:
                raise SystemExit("--calib-bytes: no device copy with FETCH_SIZE in any pass")
            scale = scales[0]
        tab = cell_table(runs, man, scale, a.kernel, a.cus, a.xccs)
        lines = ["# rocprofv3 per-cell counters (generated by paper_2608_15764_amd.rocprof)"]
        lines += [f"# command: {c}" for c in a.command]
        if scale:
            lines.append(f"# FETCH_SIZE scale (device copies of known size): {scale:.6g}")
        keys = [k for k in CELL_KEYS if man and k in man[0]]
        lines.append(f"# {' '.join(keys)}: counter medians over non-warm-up launches")
        for key, row in tab.items():
            vals = " ".join(f"{c}={v:.6g}" for c, v in sorted(row.items()))
            lines.append(f"{' '.join(map(str, key))}: {vals}")
        text = "\n".join(lines) + "\n"
        if a.out:
            with open(a.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)
        return 0
    if a.cmd == "summary":
        sm = summary(a.trace, a.fetch, a.write, a.kernel, a.calib_bytes,
                     a.algorithmic_bytes)
        text = format_summary(sm, a.command, a.source_hash, a.note)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)
    else:
        for name, v in sorted(per_kernel_stats(a.trace).items(),
                              key=lambda kv: -kv[1]["calls"] * kv[1]["mean_ns"]):
            print(f"{v['calls']:6d} {v['mean_ns'] / 1e3:10.2f} us  {name}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
