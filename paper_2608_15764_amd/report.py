"""The benchmark's result line.

A benchmark run produces a large result (every curve, every extra
configuration).  That detail goes to a JSON file; standard output ends with
one compact JSON object that carries the headline figures: the metric and
its value, the step time, the roofline of the dominant kernel, the CPU
baseline and one summary figure per extra configuration.  The compact line
is bounded in size so that a reader keeping only the tail of the output
still has all of it.

Bandwidth throughout is issued logical bytes per calibrated nanosecond, in
decimal GB/s (Section 3, "Timing, residency, statistics").
"""
import json
import os

LINE_LIMIT = 4000          # bytes of the compact line, newline excluded

# Keys the compact line always carries.
REQUIRED = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
            "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
            "roofline", "cpu_baseline")

# Optional sections, dropped last-first if the line would exceed the limit.
OPTIONAL = ("curve_peak_gbps", "curve_peak_frac_of_hbm", "best_waves_per_cu",
            "peak_K_at_best", "decline_2_8_at_best", "paper_like", "strict_cg",
            "gap", "fabric", "xcd_weighting", "eager", "c5a", "c5b", "streaming_gate", "f4", "f4_fixed_iters",
            "detail")


def _r(x, nd=4):
    if isinstance(x, float):
        return round(x, nd)
    return x


def _pick(d, keys, nd=4):
    if not isinstance(d, dict):
        return None
    return {k: _r(d[k], nd) for k in keys if k in d}


def _config(cfg):
    c = dict(cfg or {})
    out = {"workload": c.get("workload")}
    for k in ("buffer_bytes", "vec_width", "L", "cache_policy", "cells_per_step"):
        if k in c:
            out[k] = c[k]
    ks = c.get("Ks")
    if ks:
        out["Ks"] = f"{min(ks)}..{max(ks)}"
    ws = c.get("waves_per_cu")
    if ws:
        out["waves_per_cu"] = f"{min(ws)}..{max(ws)} step {ws[1] - ws[0]}" if len(ws) > 1 else ws[0]
    if c.get("orders"):
        out["orders"] = c["orders"]
    if c.get("infeasible_cells") is not None:
        out["infeasible_cells"] = len(c["infeasible_cells"])
    return out


def _cpu(cb):
    if not isinstance(cb, dict):
        return None
    out = _pick(cb, ("value", "unit", "cores", "kind", "sample", "host_cpu",
                     "matches_gpu", "checksum_s", "error"), 3)
    mp = cb.get("multi_process")
    if isinstance(mp, dict):
        out["multi_process"] = _pick(mp, ("value", "cores", "matches_gpu", "error"), 3)
    return out


def _c5a(row):
    if not isinstance(row, dict):
        return None
    return _pick(row, ("batched_aggregate_gbps", "batched_aggregate_frac",
                       "hbm_aggregate_gbps", "hbm_aggregate_frac",
                       "batched_best_point_gbps", "node_per_point_aggregate_gbps",
                       "plain_aggregate_gbps", "fused_launches", "chosen_plan",
                       "matches_oracle", "points_checked", "sizes"), 4)


def _c5b(row):
    if not isinstance(row, dict):
        return None
    out = {}
    for kind, v in row.items():
        if isinstance(v, dict) and "median_gbps" in v:
            out[kind] = {"gbps": _r(v.get("median_gbps"), 1),
                         "frac": _r(v.get("frac_of_hbm_peak"), 4),
                         "abs_err": v.get("abs_err"), "rel_err": v.get("rel_err"),
                         "within_bound": v.get("within_bound")}
    return out or None


def compact(result, detail_path=None):
    """The compact headline dict of a full benchmark result."""
    r = result
    out = {k: r.get(k) for k in REQUIRED if k not in ("config", "roofline", "cpu_baseline")}
    out["config"] = _config(r.get("config"))
    rl = r.get("roofline") or {}
    out["roofline"] = _pick(rl, ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                 "algorithmic_bytes_per_launch", "mean_launch_us",
                                 "launches", "kernel"), 4)
    out["cpu_baseline"] = _cpu(r.get("cpu_baseline"))
    for k in ("curve_peak_gbps", "curve_peak_frac_of_hbm", "best_waves_per_cu",
              "peak_K_at_best", "decline_2_8_at_best"):
        if k in r:
            out[k] = _r(r[k])
    pl = r.get("paper_like_cell")
    if isinstance(pl, dict):
        bo = pl.get("by_order") or {}
        med = pl.get("median_gbps") or {}
        out["paper_like"] = {
            "waves_per_cu": pl.get("waves_per_cu"), "peak_K": pl.get("peak_K"),
            "decline_2_8": _r(pl.get("decline_2_8")),
            "decline_2_8_asc": _r((bo.get("asc") or {}).get("decline_2_8")),
            "decline_2_8_rev": _r((bo.get("rev") or {}).get("decline_2_8")),
            "gbps_K2": _r(med.get(2), 1), "gbps_K8": _r(med.get(8), 1)}
    cg = r.get("strict_cg")
    if isinstance(cg, dict):
        out["strict_cg"] = _pick(cg, ("policy", "value", "ms_per_step", "curve_peak_gbps",
                                      "curve_peak_frac_of_hbm", "best_waves_per_cu",
                                      "peak_K_at_best", "paper_like_decline_2_8",
                                      "paper_like_decline_2_8_asc",
                                      "paper_like_decline_2_8_rev",
                                      "paper_like_paired_decline_median"), 4)
    gap = r.get("gap")
    if isinstance(gap, dict):
        out["gap"] = _pick(gap, ("hbm_latency_ns", "kernel_frac", "ceiling_frac_of_peak",
                                 "tail_loss", "residual_frac", "frac_of_ceiling"), 4)
    fb = r.get("fabric_by_xcd")
    if isinstance(fb, dict) and fb:
        # [min, max] GB/s per class of XCD subset at the lowest occupancy
        w = min(fb, key=lambda k: int(k))
        out["fabric"] = fb[w].get("by_class")
    xw = r.get("xcd_weighting")
    if isinstance(xw, dict) and xw:
        # per occupancy: rate gain of the re-weighted split, even/odd share
        out["xcd_weighting"] = {w: [v.get("gain"), v.get("even_over_odd_share")]
                                for w, v in xw.items()}
    ea = r.get("eager_sweep")
    if isinstance(ea, dict):
        out["eager"] = _pick(ea, ("step_ms", "aggregate_gbps", "dispatch_event_gbps"), 1)
    rows = r.get("rows") or {}
    c5a = _c5a(rows.get("c5a_batched"))
    if c5a:
        out["c5a"] = c5a
    c5b = _c5b(rows.get("c5b_precision"))
    if c5b:
        out["c5b"] = c5b
    f4 = rows.get("f4_regime_map")
    if isinstance(f4, dict) and isinstance(f4.get("backends"), dict):
        # [saturating, rising-censored, peak-decline] curves per backend
        out["f4"] = {name: [b["counts"].get(k, 0) for k in
                            ("saturating", "rising-censored", "peak-decline")]
                     for name, b in f4["backends"].items() if "counts" in b}
        fi = {name: [b["fixed_iters"]["counts"].get(k, 0) for k in
                     ("saturating", "rising-censored", "peak-decline")]
              for name, b in f4["backends"].items() if "fixed_iters" in b}
        if fi:
            out["f4_fixed_iters"] = fi
    sg = r.get("streaming_gate")
    if isinstance(sg, dict):
        out["streaming_gate"] = _pick(sg, ("median_gbps", "median_frac",
                                           "littles_law_ceiling_gbps", "frac_of_ceiling",
                                           "verdict"), 4)
    if detail_path:
        out["detail"] = detail_path
    return out


def headline_line(result, detail_path=None, limit=LINE_LIMIT):
    """The compact line as text, at most ``limit`` bytes: optional sections
    are dropped, last first, until it fits; their names are listed under
    ``"dropped"``."""
    c = compact(result, detail_path)
    dropped = []
    line = json.dumps(c, separators=(",", ":"), default=str)
    for k in reversed(OPTIONAL):
        if len(line.encode()) <= limit:
            break
        if k in c:
            del c[k]
            dropped.append(k)
            c["dropped"] = dropped
            line = json.dumps(c, separators=(",", ":"), default=str)
    if len(line.encode()) > limit:
        raise ValueError(f"headline line of {len(line)} bytes exceeds {limit}")
    return line


def write_detail(result, path):
    """Write the full result as JSON to ``path`` (directories created)."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        json.dump(result, f, default=str)
        f.write("\n")


def emit(result, detail_path, out):
    """Write the detail file, then print the compact line as the last line
    of ``out``."""
    if detail_path:
        write_detail(result, detail_path)
    line = headline_line(result, detail_path)
    out.write(line + "\n")
    out.flush()
    return line


def summarize(result):
    """A short plain-text reading of a full result (the detail file): the
    headline, the roofline, where the gap goes, and one line per extra
    configuration that the run holds."""
    c = compact(result)
    rl = c.get("roofline") or {}
    lines = [f"{c.get('metric')}: {c.get('value')} {c.get('unit')} "
             f"({c.get('steps')} steps, {c.get('ms_per_step')} ms per step)"]
    if rl:
        tr = rl.get("traffic")
        ab = rl.get("algorithmic_bytes_per_launch")
        ratio = f", HBM traffic {tr / ab:.5f}x algorithmic" if tr and ab else ""
        lines.append(f"roofline: {rl.get('achieved')} of {rl.get('peak')} {rl.get('unit')} "
                     f"({100 * rl.get('frac', 0):.1f} %, {rl.get('bound')}-bound){ratio}")
    if "curve_peak_gbps" in c:
        lines.append(f"best cell: {c['curve_peak_gbps']} GB/s at {c.get('best_waves_per_cu')} "
                     f"waves/CU, K = {c.get('peak_K_at_best')}")
    pl = c.get("paper_like")
    if pl:
        lines.append(f"paper-like cell ({pl.get('waves_per_cu')} waves/CU): K = 2->8 change "
                     f"{100 * pl.get('decline_2_8', 0):+.2f} %")
    g = c.get("gap")
    if g:
        lines.append(f"gap: design ceiling {g.get('ceiling_frac_of_peak')} x (1 - tail "
                     f"{g.get('tail_loss')}) x residual {g.get('residual_frac')} = kernel "
                     f"{g.get('kernel_frac')}")
    if c.get("fabric"):
        lines.append("fabric by XCD subset (GB/s, min-max): " + ", ".join(
            f"{k} {v[0]}-{v[1]}" for k, v in c["fabric"].items()))
    if c.get("c5a"):
        a = c["c5a"]
        lines.append(f"batched sweep: {a.get('batched_aggregate_gbps')} GB/s "
                     f"({a.get('chosen_plan')}, oracle match {a.get('matches_oracle')})")
    if c.get("c5b"):
        lines.append("precision sums: " + ", ".join(
            f"{k} {v.get('gbps')} GB/s (within bound {v.get('within_bound')})"
            for k, v in c["c5b"].items()))
    cb = c.get("cpu_baseline")
    if cb:
        lines.append(f"CPU oracle: {cb.get('value')} {cb.get('unit')} on {cb.get('cores')} "
                     f"core(s), matches GPU {cb.get('matches_gpu')}")
    errs = [k for k in result if k.endswith("_error")]
    for k in errs:
        lines.append(f"{k}: {result[k]}")
    return "\n".join(lines)


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="Summarize a bench detail file")
    ap.add_argument("detail", nargs="?", default=os.path.join("results", "bench_detail.json"))
    a = ap.parse_args(argv)
    with open(a.detail) as f:
        print(summarize(json.load(f)))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
