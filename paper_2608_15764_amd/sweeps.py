"""Sweep drivers: the experiment designs of the method on top of the C ABI.

Each driver builds cells, runs them through the native sweep driver
(``sweep_run``: back-to-back launches, per-cell dispatch-stamped events and
clock windows, one synchronisation) or a captured graph
(``sweep_graph_create`` once, ``sweep_graph_launch`` per pass: per-cell
clock windows), and summarises the launches with :mod:`stats`.

plain_k_sweep      Section 3 / Section 4.2: fixed-work K sweep at several
                   occupancies, ascending and reversed order.
allocation_sweep   Section 3 "Allocation-size sweep" / Section 4.2: the
                   same fixed work over allocations of different size.
path_comparison    Section 4.3: LDS-direct loads against the matched
                   register path at equal in-flight depth.
two_stream         Section 4.4: two co-resident streams in one workgroup,
                   displacement against each stream running solo.
batched_autotuned  64 uneven sweep points with per-size-class tuned
                   (vector width, K, waves, cache policy), captured in one
                   hipGraph, against the same points launched one by one
                   at the untuned default.
precision_sum      streaming FP32 / BF16 / FP8 sum with compensated FP32
                   accumulation and an FP64 final combine.

Buffers are dropped with ``del`` and stay in torch's caching allocator;
nothing here returns device memory to the driver.  A hipFree of VRAM makes
later HBM reads about 6 % slower for a while (under 0.1 s after 1 GiB,
0.1-0.25 s after 8 GiB, 0.5-1 s after 20 GiB on MI355X), which would leak
into whatever is timed next.
"""
import json
import os

import torch

from . import ilpsweep as isw
from . import stats

SEED_BASE = 0x1D5EED00
GIB = 1 << 30
MIB = 1 << 20


def device_buffer(nbytes, seed):
    """A seeded device buffer (SplitMix64 words) of ``nbytes`` bytes."""
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    isw.sweep_fill_u32(buf, int(nbytes), seed)
    torch.cuda.synchronize()
    return buf


def _feasible(cell):
    """True if the cell's kernel can reach the cell's residency."""
    try:
        isw.sweep_run([cell])
        return True
    except isw.SweepError as e:
        if e.code == isw.EOCCUPANCY:
            return False
        raise


def _median(v):
    return stats.median(v) if v else None


# ------------------------------------------------------------- K sweep (C2)
def plain_k_cells(buf, nbytes, L, policy, waves_list, Ks, orders=("asc", "rev"),
                  vec_width=16):
    """Cells of a K sweep, grouped by occupancy, each order in turn."""
    cells, meta = [], []
    for w in waves_list:
        for order in orders:
            ks = list(Ks) if order == "asc" else list(reversed(list(Ks)))
            for K in ks:
                c = isw.make_cell(buf, nbytes, K, vec_width, w, L,
                                  cache_policy=policy)
                cells.append(c)
                meta.append({"waves_per_cu": w, "order": order, "K": K,
                             "bytes": nbytes})
    return cells, meta


def drop_infeasible(cells, meta):
    seen = {}
    keep_c, keep_m, dropped = [], [], []
    for c, m in zip(cells, meta):
        key = (c.kind, c.K, c.vec_width, c.waves_per_cu, c.cache_policy)
        if key not in seen:
            seen[key] = _feasible(c)
        if seen[key]:
            keep_c.append(c)
            keep_m.append(m)
        else:
            dropped.append(dict(m))
    return keep_c, keep_m, dropped


def summarize_k_sweep(meta, runs, vec_width=16):
    """Summary of repeated K-sweep passes (``runs``: list of result lists).
    Every ``meta`` entry names its cell's allocation (``bytes``), which the
    residency screen needs: a cache-resident buffer may be read faster than
    HBM allows however many bytes a launch issues over it."""
    missing = [m for m in meta if "bytes" not in m]
    if missing:
        raise ValueError("cell metadata must carry the allocation size 'bytes'")
    by = {}
    checks = {}
    for results in runs:
        for m, r in zip(meta, results):
            key = (m["waves_per_cu"], m["order"])
            by.setdefault(key, {}).setdefault(m["K"], []).append(r["gbps"])
            checks.setdefault(r["issued_loads"], set()).add((r["sum32"], r["xor32"]))
    out = {"curves": {}, "checksums_consistent": all(len(v) == 1 for v in checks.values())}
    waves = sorted({k[0] for k in by})
    for w in waves:
        samples = {}
        per_order = {}
        for order in ("asc", "rev"):
            s = by.get((w, order))
            if not s:
                continue
            per_order[order] = stats.summarize_curve(s)
            for K, v in s.items():
                samples.setdefault(K, []).extend(v)
        summ = stats.summarize_curve(samples)
        summ["by_order"] = {o: {"decline_2_8": v.get("decline_2_8"),
                                "peak_K": v["peak_K"]}
                            for o, v in per_order.items()}
        n_waves = None
        for m, r in zip(meta, runs[0]):
            if m["waves_per_cu"] == w:
                n_waves = r["waves"]
                break
        summ["in_flight_bytes"] = {
            K: stats.in_flight_bytes(n_waves, K, vec_width) for K in summ["median_gbps"]}
        summ["implied_latency_ns"] = {
            K: stats.implied_latency_ns(summ["in_flight_bytes"][K], g)
            for K, g in summ["median_gbps"].items() if g > 0}
        out["curves"][w] = summ
    issued = [r["issued_loads"] for r in runs[0]]
    out["kset_mismatch"] = stats.kset_mismatch(issued) if issued else None
    anom = [(w, k, x, r) for w, c in out["curves"].items() for k, x, r in c["anomalous"]]
    out["anomalous_launches"] = {
        "rule": "launch < 0.9 x its cell's median",
        "count": len(anom),
        "launches": sum(c["launches"] for c in out["curves"].values()),
        "worst": (None if not anom else
                  dict(zip(("waves_per_cu", "K", "gbps", "ratio"),
                           min(anom, key=lambda a: a[3]))))}
    out["residency_flags"] = sum(
        stats.residency_flag(r["gbps"], m["bytes"]) for res in runs
        for m, r in zip(meta, res))
    best_w = max(out["curves"], key=lambda w: max(out["curves"][w]["median_gbps"].values()))
    out["best_waves_per_cu"] = best_w
    out["peak_gbps"] = max(out["curves"][best_w]["median_gbps"].values())
    return out


def plain_k_sweep(buf, nbytes, L, policy, waves_list, Ks, passes=3, warmup=1):
    cells, meta = plain_k_cells(buf, nbytes, L, policy, waves_list, Ks)
    cells, meta, dropped = drop_infeasible(cells, meta)
    for _ in range(warmup):
        isw.sweep_run(cells)
    runs = [isw.sweep_run(cells) for _ in range(passes)]
    out = summarize_k_sweep(meta, runs)
    out["infeasible"] = dropped
    return out


def completion_spread(buf, nbytes, L, policy, waves_list, K=4, reps=3):
    """When each wave of a K-sweep cell finishes, as a fraction of the cell's
    window (from the per-wave clock records), per occupancy: the 10th, 50th
    and 90th percentile of the wave end times, the earliest and latest last
    end over the XCDs, and the latest wave start.  Every wave has the same
    share of the work, so a spread of end times is unequal service; the
    mean wave duration per XCD against the chip mean shows whether that
    service differs by XCD."""
    import numpy as np
    dt = np.dtype([("sum32", "<u4"), ("xor32", "<u4"), ("hw_id", "<u4"),
                   ("xcc_id", "<u4"), ("t0", "<u8"), ("t1", "<u8")])
    out = {}
    for w in waves_list:
        n = isw.sweep_device_info()["num_cus"] * w
        rec = torch.zeros(n * dt.itemsize, dtype=torch.uint8, device="cuda")
        rows, per_xcd = [], []
        for _ in range(reps + 1):                  # the first launch is the warm-up
            r = isw.sweep_plain(buf, nbytes, K, 16, w, L,
                                isw.make_opts(cache_policy=policy, wave_out=rec))
            a = rec.cpu().numpy().view(dt)[: r["waves"]]
            t0 = a["t0"].astype(np.int64)
            t1 = a["t1"].astype(np.int64)
            base, win = t0.min(), max(int(t1.max() - t0.min()), 1)
            ends = (t1 - base) / win
            xcc = a["xcc_id"] & 0xF
            xs = np.unique(xcc)
            last = [ends[xcc == x].max() for x in xs]
            dur = (t1 - t0).astype(np.float64)
            per_xcd.append([dur[xcc == x].mean() / dur.mean() for x in xs])
            rows.append((np.percentile(ends, 10), np.median(ends), np.percentile(ends, 90),
                         min(last), max(last), ((t0 - base) / win).max(), r["gbps"]))
        m = np.median(np.array(rows[1:]), axis=0)
        px = np.median(np.array(per_xcd[1:]), axis=0)
        out[w] = {"K": K, "end_p10": round(m[0], 3), "end_p50": round(m[1], 3),
                  "end_p90": round(m[2], 3), "xcd_last_end_min": round(m[3], 3),
                  "xcd_last_end_max": round(m[4], 3), "last_start": round(m[5], 3),
                  "xcd_mean_duration_ratio": [round(v, 3) for v in px],
                  "gbps": round(m[6], 1)}
    return out


# -------------------------------------------------- allocation sweep (C3)
def allocation_sweep(sizes, Ks=(1, 2, 4, 8), waves_list=(16,), L=1 << 30,
                     policy=isw.CACHE_BYPASS_L1, n=3, seed=SEED_BASE + 2):
    """Fixed-work K sweep over prefixes of one buffer of the largest size.
    The whole allocation x occupancy x K sweep is captured into one hipGraph;
    one untimed replay, then ``n`` replays whose per-cell clock windows are
    summarised."""
    top = max(sizes)
    buf = device_buffer(top, seed)
    cells, meta = [], []
    for size in sizes:
        c, m = plain_k_cells(buf, size, L, policy, waves_list, Ks)
        c, m, _ = drop_infeasible(c, m)
        cells += c
        meta += [dict(x, bytes=size) for x in m]
    g = isw.sweep_graph_create(cells)
    try:
        isw.sweep_graph_launch(g)                  # warm-up replay, excluded
        runs = [isw.sweep_graph_launch(g)[0] for _ in range(n)]
    finally:
        isw.sweep_graph_destroy(g)
    out = {}
    for size in sizes:
        idx = [i for i, m in enumerate(meta) if m["bytes"] == size]
        s_meta = [meta[i] for i in idx]
        s_runs = [[run[i] for i in idx] for run in runs]
        summ = summarize_k_sweep(s_meta, s_runs)
        issued = {m["K"]: r["issued_loads"] for m, r in zip(s_meta, s_runs[0])}
        out[size] = {
            "issued_bytes": s_runs[0][0]["issued_bytes"],
            "volume_to_allocation": s_runs[0][0]["issued_bytes"] / size,
            # exact unique-line coverage of every K's cell, from the address map
            "coverage": {K: _coverage_row(size, 16, n) for K, n in sorted(issued.items())},
            "curves": {w: {"median_gbps": c["median_gbps"],
                           "decline_2_8": c.get("decline_2_8"),
                           "by_order": c["by_order"]}
                       for w, c in summ["curves"].items()},
            "checksums_consistent": summ["checksums_consistent"],
            "anomalous_launches": summ["anomalous_launches"]["count"],
        }
    del buf
    return out


def _coverage_row(alloc_bytes, vec_bytes, issued_loads):
    c = stats.line_coverage(alloc_bytes, vec_bytes, issued_loads)
    return {"coverage": round(c["coverage"], 6), "re_reads": c["re_reads"],
            "max_reads": c["max_reads"],
            "re_read_frac": round(c["re_reads"] / c["line_reads"], 6)
            if c["line_reads"] else 0.0}


# ------------------------------------------------- path comparison (C4)
def path_comparison(buf, nbytes, L, depths=range(1, 17), waves_list=(1, 2, 4, 8),
                    policy=isw.CACHE_DEFAULT, n=3):
    """LDS-direct against matched register path (Section 4.3) at every
    (waves per CU, depth).  One warm-up pass, then n passes; a pass runs
    every depth ascending and then reversed, so each cell has 2n timed
    launches, whose median is the cell's figure."""
    cells, meta = [], []
    for W in waves_list:
        for order in ("asc", "rev"):
            ds = list(depths) if order == "asc" else list(reversed(list(depths)))
            for D in ds:
                for kind in (isw.KIND_LDS_ASYNC, isw.KIND_LDS_MATCHED):
                    cells.append(isw.make_cell(buf, nbytes, D, 16, W, L, kind=kind,
                                               cache_policy=policy))
                    meta.append((W, D, kind))
    warm = isw.sweep_run(cells)
    samples = {}
    sums = {}
    for _ in range(n):
        for m, r in zip(meta, isw.sweep_run(cells)):
            samples.setdefault(m, []).append(r["gbps"])
            sums.setdefault(m[:2], set()).add((r["sum32"], r["xor32"]))
    # both kinds read the same map at each (waves, depth): equal sinks
    out = {"checksums_equal_across_paths": all(len(v) == 1 for v in sums.values()),
           "policy": {v: k for k, v in isw.POLICY_NAMES.items()}[policy],
           # the fixed-work control carried over to the LDS paths: every
           # depth issues 64 D floor(L / 64 D) requests of the same L
           "depth_set_mismatch": stats.kset_mismatch([r["issued_loads"] for r in warm]),
           "launches_per_cell": 2 * n}
    for W in waves_list:
        row = {}
        for D in depths:
            a = _median(samples[(W, D, isw.KIND_LDS_ASYNC)])
            b = _median(samples[(W, D, isw.KIND_LDS_MATCHED)])
            row[D] = {"async_gbps": a, "matched_gbps": b, "ratio": a / b}
        out[W] = row
    return out


def two_stream(buf, nbytes, L, depths=(4, 8), pairs=((4, 4),), n=3,
               policy=isw.CACHE_DEFAULT, kind_b=isw.KIND_LDS_ASYNC, split=False):
    """Displacement of each stream by the other (Section 4.4): for every
    depth and (stream-A waves, stream-B waves) pair per workgroup, the
    co-resident bandwidth of each stream against the same stream solo.
    Stream A runs plain loads; stream B the LDS-direct ring (``kind_b =
    KIND_LDS_ASYNC``, cross-mechanism) or plain loads too (``KIND_PLAIN``,
    the section's same-mechanism measurement).  With ``split`` the streams
    run on different CUs (sweep_two_stream_split), and the solo runs keep
    that placement."""
    opts = isw.make_opts(cache_policy=policy)
    call = isw.sweep_two_stream_split if split else isw.sweep_two_stream_kind
    out = {}

    def run(D, wa, wb):
        return call(buf, nbytes, D, wa, wb, kind_b, L, opts)

    for D in depths:
        for wa, wb in pairs:
            res = {"co": [], "solo_a": [], "solo_b": []}
            run(D, wa, wb)
            for _ in range(n):
                a, b = run(D, wa, wb)
                res["co"].append((a["gbps"], b["gbps"]))
                a, _ = run(D, wa, 0)
                res["solo_a"].append(a["gbps"])
                _, b = run(D, 0, wb)
                res["solo_b"].append(b["gbps"])
            co_a = _median([x[0] for x in res["co"]])
            co_b = _median([x[1] for x in res["co"]])
            sa, sb = _median(res["solo_a"]), _median(res["solo_b"])
            out[f"D{D}_A{wa}_B{wb}"] = {
                "depth": D, "waves": [wa, wb], "co_a_gbps": co_a, "co_b_gbps": co_b,
                "solo_a_gbps": sa, "solo_b_gbps": sb,
                "displacement_a": 1 - co_a / sa, "displacement_b": 1 - co_b / sb}
    return out


# ------------------------------------------ autotuned batched sweep (C5a)
def point_sizes(n=64, lo_log2=20, hi_log2=31, align=64 * 1024):
    """n log-spaced sizes from 2**lo_log2 to 2**hi_log2 bytes, aligned."""
    out = []
    for i in range(n):
        s = 2.0 ** (lo_log2 + (hi_log2 - lo_log2) * i / (n - 1))
        out.append(max(align, int(round(s / align)) * align))
    return out


SIZE_CLASS_EDGES = [4 * MIB, 16 * MIB, 64 * MIB, 256 * MIB, GIB]


def size_class(nbytes):
    for i, e in enumerate(SIZE_CLASS_EDGES):
        if nbytes < e:
            return i
    return len(SIZE_CLASS_EDGES)


# The tuner's candidates: every vector width, K = 1..16, 1..8 waves per SIMD
# and every cache policy.  A point whose size 64 K V does not divide is read
# up to its last whole wave-group (the fixed-work rule), at most 64 K V - V
# bytes short of the whole point; the issued bytes are what is timed and
# what the sinks cover.
DEFAULT_SPACE = {"vec_widths": [4, 8, 16], "Ks": list(range(1, 17)),
                 "waves_per_cu": [4 * w for w in range(1, 9)],
                 "policies": [isw.CACHE_DEFAULT, isw.CACHE_NT,
                              isw.CACHE_BYPASS_L1, isw.CACHE_BYPASS_L1_NT]}


def autotune(buf_for_size, sizes, space=None, reps=3, cache_path=None,
             device_key=None):
    """Best (V, K, waves, policy) per size class; cached as JSON if asked."""
    space = space or DEFAULT_SPACE
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f).get(device_key or "default", {})
    classes = {}
    for s in sizes:
        classes.setdefault(size_class(s), []).append(s)
    table = {}
    for cls, members in sorted(classes.items()):
        if str(cls) in cache:
            table[cls] = cache[str(cls)]
            continue
        rep = members[len(members) // 2]
        buf = buf_for_size(rep)
        best, best_g = None, -1.0
        for pol in space["policies"]:
            cfg, g = isw.sweep_autotune(buf, rep, space["vec_widths"], space["Ks"],
                                        space["waves_per_cu"], pol, reps)
            if g > best_g:
                best, best_g = cfg, g
        best["tuned_gbps"] = best_g
        best["tuned_at_bytes"] = rep
        table[cls] = best
    if cache_path:
        allc = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                allc = json.load(f)
        allc[device_key or "default"] = {str(k): v for k, v in table.items()}
        with open(cache_path, "w") as f:
            json.dump(allc, f, indent=1)
    return table


# (K, vec_width, waves_per_cu, policy) of the K sweep's best cells at HBM
# sizes: 1 wave/SIMD at K = 7-8, 2 waves/SIMD at K = 3, 3 waves/SIMD at K = 2
STREAMING_SEEDS = ((8, 16, 4, isw.CACHE_NT), (7, 16, 4, isw.CACHE_NT),
                   (3, 16, 8, isw.CACHE_NT), (2, 16, 12, isw.CACHE_NT))


def batched_autotuned(n_points=64, n=10, default=(16, 2, 16, isw.CACHE_BYPASS_L1),
                      seed=SEED_BASE + 4, cache_path=None, space=None, verify=None,
                      hi_log2=31, fixed=None):
    """64 sweep points of uneven size (1 MiB .. 2 GiB), laid out back to
    back in one seeded buffer, each read once per pass at its size class's
    tuned (V, K, waves, policy): captured once as a hipGraph, in which the
    consecutive points of one tuned configuration run as one fused
    persistent launch, and replayed ``n`` times; against the same graph
    with one kernel node per point, and the same points launched one by one
    at the untuned default.  ``verify``, if given, is called with one (seed, first word,
    words, sum32, xor32) tuple per launch of the first tuned replay and of
    the first untuned pass, and returns one bool per tuple: whether those
    sinks are the ones the words' oracle gives.  ``fixed`` = (K, V, waves
    per CU, policy) skips the tuning and runs every point with it (for
    counter runs that must repeat the same launches)."""
    sizes = point_sizes(n_points, hi_log2=hi_log2)
    offs, off = [], 0
    for s in sizes:
        offs.append(off)
        off += s
    big = device_buffer(off, seed)
    base = big.data_ptr()

    def buf_for(size):
        # tune on the largest point's region of a class-sized prefix
        return base

    if fixed is None:
        table = autotune(buf_for, sizes, space=space, cache_path=cache_path)
    else:
        K, V, w, pol = fixed
        table = {c: {"K": K, "vec_width": V, "waves_per_cu": w, "cache_policy": pol}
                 for c in {size_class(s) for s in sizes}}

    def cells_of(cfgs):
        return [isw.make_cell(base + o, s, t["K"], t["vec_width"], t["waves_per_cu"],
                              s // t["vec_width"], cache_policy=t["cache_policy"])
                for s, o, t in zip(sizes, offs, cfgs)]

    def key(t):
        return (t["K"], t["vec_width"], t["waves_per_cu"], t["cache_policy"])

    # batch-level choice: the per-class configurations (one fused launch per
    # run of equal ones), or one class's configuration for every point (a
    # single fused launch); each plan's fused graph timed over 3 replays
    plans = {"per_class": [table[size_class(s)] for s in sizes]}
    uniform = {key(t): t for t in table.values()}
    if not fixed:
        # the streaming shapes the K sweep finds best at HBM sizes (few waves
        # each holding 6-8 KiB in flight), so that the search starts from
        # them whatever the per-class picks were
        sp = space or DEFAULT_SPACE
        for K, V, w, pol in STREAMING_SEEDS:
            if K in sp["Ks"] and V in sp["vec_widths"] and w in sp["waves_per_cu"] \
                    and pol in sp["policies"]:
                uniform.setdefault((K, V, w, pol), {"K": K, "vec_width": V,
                                                    "waves_per_cu": w, "cache_policy": pol})
    for t in sorted(uniform.values(), key=key):
        plans["uniform_K{}_V{}_w{}_p{}".format(*key(t))] = [t] * len(sizes)
    plan_gbps = {}

    def score(name, cfgs, replays=3):
        try:
            with isw.sweep_graph_create(cells_of(cfgs), isw.make_opts(fuse=True)) as pg:
                isw.sweep_graph_launch(pg)
                runs = [isw.sweep_graph_launch(pg) for _ in range(replays)]
        except isw.SweepError as e:
            if e.code in (isw.EOCCUPANCY, isw.EINVAL):
                return None                    # a configuration some point cannot run
            raise
        plans[name] = cfgs
        plan_gbps[name] = sum(r["issued_bytes"] for r in runs[0][0]) / (
            _median([ms for _, ms in runs]) * 1e6)
        return plan_gbps[name]

    for name, cfgs in list(plans.items()):
        score(name, cfgs)
    # then a local search around the best single configuration: neighbouring
    # K, occupancy, width and policy, three rounds at most
    for _ in range(0 if fixed else 3):
        best = max((n for n in plan_gbps if n != "per_class"), key=plan_gbps.get)
        t0 = plans[best][0]
        K, V, w, pol = key(t0)
        cand = [(K + d, V, w, pol) for d in (-2, -1, 1, 2)] + \
               [(K, V, w + d, pol) for d in (-4, 4)] + \
               [(K, v, w, pol) for v in (4, 8, 16) if v != V] + \
               [(K, V, w, q) for q in (isw.CACHE_NT, isw.CACHE_BYPASS_L1_NT) if q != pol]
        improved = False
        for k2, v2, w2, p2 in cand:
            if not (1 <= k2 <= 16 and 4 <= w2 <= 32):
                continue
            name = f"uniform_K{k2}_V{v2}_w{w2}_p{p2}"
            if name in plan_gbps:
                continue
            t = {"K": k2, "vec_width": v2, "waves_per_cu": w2, "cache_policy": p2}
            g = score(name, [t] * len(sizes))
            if g is not None and g > plan_gbps[best]:
                improved = True
        if not improved:
            break
    # the three best plans timed again over more replays, so that one noisy
    # score does not decide
    if not fixed:
        for name in sorted(plan_gbps, key=plan_gbps.get, reverse=True)[:3]:
            score(name, plans[name], replays=9)
    chosen = max(plan_gbps, key=plan_gbps.get)
    cfgs = plans[chosen]
    tuned = cells_of(cfgs)
    V0, K0, w0, p0 = default
    plain = [isw.make_cell(base + o, s, K0, V0, w0, s // V0, cache_policy=p0)
             for s, o in zip(sizes, offs)]
    # the chosen plan captured once and replayed: fused, and beside it the
    # same configurations with one kernel node per point
    graph = isw.sweep_graph_create(tuned, isw.make_opts(fuse=True))
    nodes = isw.sweep_graph_create(tuned)
    g_runs, g_ms, p_runs, u_runs, u_ms = [], [], [], [], []
    try:
        isw.sweep_graph_launch(graph)
        isw.sweep_graph_launch(nodes)
        isw.sweep_run(plain)
        for _ in range(n):
            r, ms = isw.sweep_graph_launch(graph)
            g_runs.append(r)
            g_ms.append(ms)
            r, ms = isw.sweep_graph_launch(nodes)
            u_runs.append(r)
            u_ms.append(ms)
            p_runs.append(isw.sweep_run(plain))
    finally:
        isw.sweep_graph_destroy(graph)
        isw.sweep_graph_destroy(nodes)
    pts = []
    for i, s in enumerate(sizes):
        t = cfgs[i]
        pts.append({"bytes": s, "issued_bytes": g_runs[0][i]["issued_bytes"],
                    "K": t["K"], "vec_width": t["vec_width"],
                    "waves_per_cu": t["waves_per_cu"], "cache_policy": t["cache_policy"],
                    # alone in its own graph node, and inside the fused launch
                    # (where neighbouring points overlap its window)
                    "batched_gbps": _median([r[i]["gbps"] for r in u_runs]),
                    "fused_window_gbps": _median([r[i]["gbps"] for r in g_runs]),
                    "plain_gbps": _median([r[i]["gbps"] for r in p_runs]),
                    "hbm_targeted": s > stats.INFINITY_CACHE_BYTES})
    issued = sum(p["issued_bytes"] for p in pts)
    hbm = [i for i, p in enumerate(pts) if p["hbm_targeted"]]
    # every HBM-targeted point's bytes over its own median window, each
    # point alone in its graph node
    hbm_bytes = sum(pts[i]["issued_bytes"] for i in hbm)
    hbm_ns = sum(_median([r[i]["window_ns"] for r in u_runs]) for i in hbm)
    plain_ms = _median([sum(r["event_ms"] for r in run) for run in p_runs])
    out = {
        "sizes": len(sizes),
        "total_bytes": off,
        "issued_bytes": issued,
        "tuned": {str(k): v for k, v in table.items()},
        "plans_gbps": {k: round(v, 1) for k, v in plan_gbps.items()},
        "chosen_plan": chosen,
        "space": {k: (v if k != "policies" else [int(p) for p in v])
                  for k, v in (space or DEFAULT_SPACE).items()},
        "points": pts,
        "graph_ms": _median(g_ms),
        "plain_kernel_ms_sum": plain_ms,
        # the headline: the whole batch's issued bytes over the graph's time
        "batched_aggregate_gbps": issued / (_median(g_ms) * 1e6),
        # runs of consecutive points with one configuration: one launch each
        "fused_launches": 1 + sum(
            1 for a, b in zip(pts, pts[1:])
            if (a["K"], a["vec_width"], a["waves_per_cu"], a["cache_policy"])
            != (b["K"], b["vec_width"], b["waves_per_cu"], b["cache_policy"])),
        "node_per_point_graph_ms": _median(u_ms),
        "node_per_point_aggregate_gbps": issued / (_median(u_ms) * 1e6),
        "hbm_points": len(hbm),
        "hbm_aggregate_gbps": hbm_bytes / hbm_ns if hbm_ns else None,
        "batched_best_point_gbps": max(p["batched_gbps"] for i, p in enumerate(pts)
                                       if i in hbm) if hbm else None,
        "plain_aggregate_gbps": sum(r["issued_bytes"] for r in p_runs[0]) / (plain_ms * 1e6),
        "plain_best_point_gbps": max(p["plain_gbps"] for i, p in enumerate(pts)
                                     if i in hbm) if hbm else None,
    }
    out["batched_aggregate_frac"] = out["batched_aggregate_gbps"] / stats.HBM_PEAK_GBPS
    if out["hbm_aggregate_gbps"]:
        out["hbm_aggregate_frac"] = out["hbm_aggregate_gbps"] / stats.HBM_PEAK_GBPS
    if verify is not None:
        checks = []
        for runs in (g_runs[0], p_runs[0]):
            for o, r in zip(offs, runs):
                checks.append((seed, o // 4, r["issued_bytes"] // 4, r["sum32"], r["xor32"]))
        ok = verify(checks)
        out["matches_oracle"] = bool(all(ok))
        out["points_checked"] = len(ok)
        out["mismatched_points"] = [i for i, v in enumerate(ok) if not v]
    del big
    return out


# ----------------------------------------------- precision reduction (C5b)
def precision_sum(payload_bytes=4 * GIB, n=10, waves_choices=(4, 8, 12, 16, 24, 32),
                  seed=SEED_BASE + 5, waves_fixed=None, on_payload=None):
    """Streaming FP32 / BF16 / FP8 sums of N(0,1) payloads.  The occupancy
    is tuned per payload type (median of 3 launches per choice), then n
    launches are timed at the chosen occupancy.  ``waves_fixed`` ({kind:
    waves_per_cu}) skips the tuning for the kinds it names.  ``on_payload``,
    if given, is called as on_payload(kind, payload, n_elements, row) after a
    kind's launches, while its payload is still on the device; what it
    returns (a dict) is merged into the kind's row."""
    import synth
    out = {}
    for kind, dt in (("f32", isw.F32), ("bf16", isw.BF16), ("fp8_e4m3", isw.FP8_E4M3)):
        eb = synth.ELEM_BYTES[kind]
        n_el = payload_bytes // eb
        p = synth.normal_payload(kind, n_el, seed, device="cuda")
        torch.cuda.synchronize()
        tune = {}
        if waves_fixed and kind in waves_fixed:
            best_w = waves_fixed[kind]
        else:
            isw.sweep_reduce_fp(p, n_el, dt, waves_choices[0])
            for w in waves_choices:
                tune[w] = _median([isw.sweep_reduce_fp(p, n_el, dt, w)[1]["gbps"]
                                   for _ in range(3)])
            best_w = max(tune, key=tune.get)
        isw.sweep_reduce_fp(p, n_el, dt, best_w)    # warm-up at the chosen occupancy
        gs, sums = [], []
        for _ in range(n):
            s, r = isw.sweep_reduce_fp(p, n_el, dt, best_w)
            gs.append(r["gbps"])
            sums.append(s)
        out[kind] = {"elements": n_el, "sum": sums[0],
                     "deterministic": len(set(sums)) == 1,
                     "waves_per_cu": best_w,
                     "tuning_gbps": {w: round(g, 1) for w, g in tune.items()},
                     "median_gbps": _median(gs),
                     "frac_of_hbm_peak": _median(gs) / stats.HBM_PEAK_GBPS,
                     "waves": r["waves"], "grid_wgs": r["grid_wgs"]}
        if on_payload is not None:
            out[kind].update(on_payload(kind, p, n_el, out[kind]))
        del p
    return out


# ------------------------------------------------------ counter pass (C3)
def allocation_counter_pass(sizes, Ks=(2, 8), waves_per_cu=16, L=1 << 30,
                            policy=isw.CACHE_BYPASS_L1, reps=3,
                            seed=SEED_BASE + 2, manifest=None):
    """Cells of the allocation sweep, one launch per call, for a separate
    rocprofv3 counter run.  The first launch of every cell is its warm-up.
    Returns (and optionally writes) the manifest of plain-load launches in
    launch order, so the counter rows can be attributed to cells."""
    buf = device_buffer(max(sizes), seed)
    order = []
    for size in sizes:
        for direction in ("asc", "rev"):
            ks = list(Ks) if direction == "asc" else list(reversed(list(Ks)))
            for K in ks:
                c = isw.make_cell(buf, size, K, 16, waves_per_cu, L, cache_policy=policy)
                for rep in range(reps):
                    r = isw.sweep_run([c])[0]
                    order.append({"bytes": size, "K": K, "order": direction,
                                  "rep": rep, "warmup": rep == 0,
                                  "issued_bytes": r["issued_bytes"],
                                  "gbps": r["gbps"]})
    del buf
    if manifest:
        with open(manifest, "w") as f:
            json.dump(order, f)
    return order


# --------------------------- order and footprint experiment (next rows f2, f3)
def order_footprint(sizes, Ks=(1, 2, 4, 8), waves_per_cu=16, L=1 << 26,
                    policy=isw.CACHE_BYPASS_L1_NT, n=3, seed=SEED_BASE + 6):
    """The fixed-work K sweep under three address orderings, at allocations
    below, around and above the caches (4 MiB L2 per XCD, 256 MiB last-level
    cache).  Coalescing, occupancy and logical bytes are the same in every
    cell; only the address ordering and the footprint change: round robin
    (a group's K loads are adjacent segments, neighbouring waves read
    neighbouring groups), blocked (every wave streams its own range) and
    strided (round robin, but a group's K loads go to K regions Q segments
    apart, so the K-dependent part of the aggregate order changes)."""
    buf = device_buffer(max(sizes), seed)
    out = {}
    for size in sizes:
        row = {}
        for order, oname in ((isw.ORDER_ROUND_ROBIN, "round_robin"),
                             (isw.ORDER_BLOCKED, "blocked"),
                             (isw.ORDER_STRIDED, "strided")):
            cells, meta = [], []
            for direction in ("asc", "rev"):
                ks = list(Ks) if direction == "asc" else list(reversed(list(Ks)))
                for K in ks:
                    cells.append(isw.make_cell(buf, size, K, 16, waves_per_cu, L,
                                               cache_policy=policy, order=order))
                    meta.append({"waves_per_cu": waves_per_cu, "order": direction, "K": K,
                                 "bytes": size})
            arr = isw.cell_array(cells)
            isw.sweep_run(arr, raw=True)
            runs = [isw.sweep_run(arr) for _ in range(n)]
            summ = summarize_k_sweep(meta, runs)
            c = summ["curves"][waves_per_cu]
            n_waves = runs[0][0]["waves"]
            issued = {m["K"]: r["issued_loads"] for m, r in zip(meta, runs[0])}
            row[oname] = {"median_gbps": {k: round(v, 1) for k, v in c["median_gbps"].items()},
                          "coverage": {K: _coverage_row(size, 16, n)
                                       for K, n in sorted(issued.items())},
                          "front_duplicates": {
                              K: round(stats.front_duplicates(
                                  order, K, n_waves, L // (64 * K), size // 16), 4)
                              for K in Ks},
                          "decline_2_8": c.get("decline_2_8"),
                          "by_order": c["by_order"],
                          "residency_flags": summ["residency_flags"],
                          "checksums_consistent": summ["checksums_consistent"]}
        out[size] = row
    del buf
    return out


# ----------------------------------------------- regime map (next row f4)
REGIME_BACKENDS = (("hbm", GIB), ("infinity_cache", 128 * MIB), ("l2", 4 * MIB))


REGIME_ARMS = ("fixed_work", "fixed_iters")


def _regime_curve(buf, nbytes, V, w, g, Ks, policy, n, mode, L, iters):
    """One response curve of the regime map: the feasible K, each timed in
    2n launches (n passes ascending then descending after a warm-up pass),
    or None when fewer than three K are feasible."""
    def cell(K):
        return isw.make_cell(buf, nbytes, K, V, w, L, cache_policy=policy, mode=mode,
                             fixed_iters=iters, grid_wgs=(g * w // 4) if g else 0)
    keep = [K for K in Ks if _feasible(cell(K))]
    if len(keep) < 3:
        return None
    seq = keep + keep[::-1]
    arr = isw.cell_array([cell(K) for K in seq])
    isw.sweep_run(arr, raw=True)                 # warm-up pass
    samples = {K: [] for K in keep}
    by_order = {"asc": {K: [] for K in keep}, "rev": {K: [] for K in keep}}
    for _ in range(n):
        for i, (K, r) in enumerate(zip(seq, isw.sweep_run(arr))):
            samples[K].append(r["gbps"])
            by_order["asc" if i < len(keep) else "rev"][K].append(r["gbps"])
    med = stats.per_k_medians(samples)
    return {"regime": stats.classify(med), "peak_K": stats.peak_k(med),
            "peak_gbps": round(max(med.values()), 1),
            "decline_2_8": (stats.decline(med[2], med[8])
                            if 2 in med and 8 in med else None),
            "regime_by_order": {o: stats.classify(stats.per_k_medians(v))
                                for o, v in by_order.items()}}


def regime_map(waves_list=(4, 8, 12, 16, 20, 24, 28, 32), widths=(4, 8, 16),
               Ks=range(1, 17), half_grid=True, backends=REGIME_BACKENDS,
               work_bytes=GIB, policy=isw.CACHE_BYPASS_L1_NT, n=3, seed=SEED_BASE + 7,
               arms=REGIME_ARMS, iters_K=8):
    """Response curves over occupancy x vector width (x full / half-CU
    grids), each classified saturating / rising-censored / peak-decline by
    the 95 % plateau rule with a three-cell tail, on every backend: a buffer
    far above the caches (HBM), one inside the 256 MiB last-level cache and
    one inside the 4 MiB L2 of an XCD (Section 4.2, "Prevalence", compares
    the prevalence of the decline on the L2-targeted and the HBM backends).

    Two arms.  Fixed work: every curve reads the same logical volume,
    ``work_bytes`` (half of it on the half grid), at every K.  Fixed
    iterations, the sweep the paper's qualification grid ran: every K runs
    the same iteration count, chosen so that K = ``iters_K`` reads that same
    volume, so the volume grows with K.  Both wrap over the smaller buffers.
    A pass runs every K ascending, then descending; after one warm-up pass
    ``n`` passes are timed, so every cell has 2n launches, whose median is
    its figure."""
    info = isw.sweep_device_info()
    grids = [0] + ([info["num_cus"] // 2] if half_grid else [])
    out = {}
    for name, nbytes in backends:
        buf = device_buffer(nbytes, seed)
        entry = {"bytes": nbytes, "launches_per_cell": 2 * n}
        for arm in arms:
            curves, iters_used = {}, {}
            counts = {"saturating": 0, "rising-censored": 0, "peak-decline": 0,
                      "infeasible": 0}
            for g in grids:
                for V in widths:
                    for w in waves_list:
                        curve_bytes = work_bytes if g == 0 else work_bytes // 2
                        key = f"{'half' if g else 'full'}_V{V}_w{w}"
                        if arm == "fixed_work":
                            mode, L, iters = isw.FIXED_WORK, curve_bytes // V, 0
                        else:
                            n_waves = (g or info["num_cus"]) * w
                            iters = max(1, curve_bytes // (V * iters_K * 64 * n_waves))
                            mode, L = isw.FIXED_ITERS, 0
                            iters_used[key] = iters
                        c = _regime_curve(buf, nbytes, V, w, g, Ks, policy, n, mode, L,
                                          iters)
                        if c is None:
                            counts["infeasible"] += 1
                            continue
                        counts[c["regime"]] += 1
                        curves[key] = c
            if arm == "fixed_work":
                entry.update(counts=counts, curves=curves)
            else:
                entry[arm] = {"counts": counts, "curves": curves, "iters": iters_used,
                              "iters_K": iters_K}
        out[name] = entry
        del buf
    return {"backends": out,
            "counts": {name: v["counts"] for name, v in out.items() if "counts" in v},
            "counts_fixed_iters": {name: v["fixed_iters"]["counts"]
                                   for name, v in out.items() if "fixed_iters" in v},
            "work_bytes": work_bytes}


# ------------------------------------------- latency ladder (next row f1)
def latency_ladder(footprints=None, stride=128, hops=8192, n_samples=4096,
                   policies=(isw.CACHE_DEFAULT, isw.CACHE_BYPASS_L1), seed=SEED_BASE + 8,
                   evict_bytes=2 * GIB):
    """Unloaded dependent-load latency against footprint (Section 4.1):
    mean ns per hop over an unsampled run, and p5/p50/p95/p99 of the
    per-hop shader-clock samples of a second run.

    Footprints that fit the last-level cache are warmed by walking the chain
    first.  Larger ones are measured cold: before every run a 2 GiB stream
    evicts the caches, and every run continues the chain where the previous
    one stopped, so no timed hop revisits a node an earlier run touched."""
    import synth
    if footprints is None:
        footprints = [8 << 10 << i for i in range(19)]          # 8 KiB .. 2 GiB
    names = {0: "default", 1: "nt", 2: "bypass_l1", 3: "bypass_l1_nt"}
    evict_buf = device_buffer(evict_bytes, seed + 1)

    def evict():
        isw.sweep_plain(evict_buf, evict_bytes, 4, 16, 32, evict_bytes // 16)

    out = {}
    for fp in footprints:
        chain, start = synth.chase_chain(fp, stride, seed + fp.bit_length(), device="cuda")
        nodes = fp // stride
        cold = fp > stats.INFINITY_CACHE_BYTES
        idx = start
        row = {}
        samples = torch.zeros(n_samples, dtype=torch.int32, device="cuda")
        for pol in policies:
            res = []
            for ns_ in (0, n_samples):
                if cold:
                    evict()
                    warm = 0
                else:
                    warm = min(nodes, 1 << 15)
                r = isw.sweep_chase(chain, fp, idx, warm, hops, pol,
                                    samples if ns_ else None, ns_)
                res.append(r)
                if cold:
                    idx = r["final_index"]
            mean, dist = res
            cyc = samples.cpu().numpy().astype("float64")
            v = sorted(cyc / dist["shader_clock_hz"] * 1e9)
            q = lambda p: float(v[min(len(v) - 1, int(p * len(v)))])
            row[names[pol]] = {
                "mean_ns": round(mean["ns_per_hop"], 2),
                "p5_ns": round(q(0.05), 1), "p50_ns": round(q(0.50), 1),
                "p95_ns": round(q(0.95), 1), "p99_ns": round(q(0.99), 1),
                "cold": cold, "shader_clock_hz": dist["shader_clock_hz"]}
        out[fp] = row
        del chain, samples
    del evict_buf
    return out


FABRIC_MASKS = (("one", tuple(1 << x for x in range(8))),
                ("group_of_four", (0x0F, 0xF0)),
                ("two_per_group", (0x55, 0xAA, 0x3C, 0xC3)),
                ("three_per_group", (0x77, 0xEE, 0xDD, 0xBB)),
                ("all", (0xFF,)))


def fabric_by_xcd(buf, nbytes, waves_list=(4, 8), policy=isw.CACHE_BYPASS_L1_NT, n=5,
                  masks=FABRIC_MASKS, manifest=None):
    """Where the plateau's ceiling sits: the plain K = 8 read run only by the
    workgroups of chosen XCDs (one XCD, a group of four that share a path,
    two or three from each group, all eight), each mask timed in ``n``
    launches after a warm-up.  Every active wave's XCC_ID is checked against
    the XCD its workgroup index names (``misplaced_waves``).  With
    ``manifest`` (a path), every launch is listed in order for a separate
    kernel-trace run."""
    import numpy as np
    dt = wave_rec_dtype()
    n_cus = isw.sweep_device_info()["num_cus"]
    rec = torch.zeros(n_cus * max(waves_list) * dt.itemsize, dtype=torch.uint8, device="cuda")
    out, launches = {}, []
    for w in waves_list:
        rows, by_class = {}, {}
        for cls, ms in masks:
            for m in ms:
                opts = isw.make_opts(cache_policy=policy, wave_out=rec)
                r0 = isw.sweep_xcd_subset(buf, nbytes, w, m, opts)      # warm-up
                runs = [isw.sweep_xcd_subset(buf, nbytes, w, m, opts) for _ in range(n)]
                r = runs[-1]
                for i, x in enumerate([r0] + runs):
                    launches.append({"path": "xcd_subset", "waves_per_cu": w,
                                     "mask": f"{m:#04x}", "issued_bytes": x["issued_bytes"],
                                     "rep": i, "warmup": i == 0})
                a = rec[: r["waves"] * dt.itemsize].cpu().numpy().view(dt)
                bits = [x for x in range(8) if m >> x & 1]
                want = np.array([bits[(aw // 4) % len(bits)] for aw in range(r["waves"])])
                got = a["xcc_id"].astype(np.int64) & 0xF
                g = _median([x["gbps"] for x in runs])
                ev = _median([x["issued_bytes"] / (x["event_ms"] * 1e6) for x in runs
                              if x["event_ms"] > 0])
                rows[f"{m:#04x}"] = {"class": cls, "xcds": len(bits), "waves": r["waves"],
                                     "bytes": r["issued_bytes"], "gbps": round(g, 1),
                                     "event_gbps": round(ev, 1) if ev else None,
                                     "misplaced_waves": int((got != want).sum())}
                by_class.setdefault(cls, []).append(g)
        out[w] = {"masks": rows,
                  "by_class": {c: [round(min(v), 1), round(max(v), 1)] for c, v in by_class.items()}}
    del rec
    if manifest:
        with open(manifest, "w") as f:
            json.dump(launches, f)
    return out


def xcd_weighting(buf, nbytes, waves_list=(4, 8, 16), rounds=4, n=3,
                  policy=isw.CACHE_BYPASS_L1_NT):
    """What the method's equal split costs when the XCDs are served unequally:
    the K = 8 read with a contiguous share of the groups per XCD, starting
    from equal shares and re-weighted ``rounds`` times by each XCD's measured
    speed (its share over its finish time, from the per-wave clock records).
    Per occupancy and round: the shares, each XCD's finish time relative to
    the mean, and the rate (median of ``n`` launches after a warm-up)."""
    import numpy as np
    dt = wave_rec_dtype()
    n_cus = isw.sweep_device_info()["num_cus"]
    rec = torch.zeros(n_cus * max(waves_list) * dt.itemsize, dtype=torch.uint8, device="cuda")
    out = {}
    for w in waves_list:
        weights = [1.0] * 8
        per_xcd = n_cus * w // 8           # waves per XCD
        rows = []
        for rnd in range(rounds + 1):
            opts = isw.make_opts(cache_policy=policy, wave_out=rec)
            isw.sweep_xcd_split(buf, nbytes, w, weights, opts)          # warm-up
            gb, fin = [], []
            for _ in range(n):
                r = isw.sweep_xcd_split(buf, nbytes, w, weights, opts)
                a = rec[: r["waves"] * dt.itemsize].cpu().numpy().view(dt)
                t0 = int(a["t0"].min())
                ends = a["t1"].astype(np.int64).reshape(8, per_xcd).max(axis=1) - t0
                x = (a["xcc_id"].astype(np.int64) & 0xF).reshape(8, per_xcd)
                if not (x == np.arange(8)[:, None]).all():
                    raise RuntimeError("a wave ran on another XCD than its share's")
                gb.append(r["gbps"])
                fin.append(ends)
            ends = np.median(np.array(fin), axis=0)
            total = sum(weights)
            shares = [v / total for v in weights]
            rows.append({"round": rnd, "gbps": round(_median(gb), 1),
                         "shares": [round(v, 4) for v in shares],
                         "finish_rel": [round(float(e / ends.mean()), 3) for e in ends]})
            weights = [shares[i] / float(ends[i]) for i in range(8)]
        even = np.mean([rows[-1]["shares"][i] for i in (0, 2, 4, 6)])
        odd = np.mean([rows[-1]["shares"][i] for i in (1, 3, 5, 7)])
        out[w] = {"rounds": rows, "gain": round(rows[-1]["gbps"] / rows[0]["gbps"] - 1, 4),
                  "even_over_odd_share": round(float(even / odd), 4)}
    del rec
    return out


XCD_FOOTPRINTS = (("l2", 1 * MIB), ("infinity_cache", 64 * MIB), ("hbm", 2 * GIB))


def latency_by_xcd(footprints=XCD_FOOTPRINTS, walkers=(8, 64), hops=4096, stride=128,
                   policy=isw.CACHE_BYPASS_L1, seed=SEED_BASE + 9, evict_bytes=2 * GIB):
    """Unloaded dependent-load latency resolved by XCD (the latency ladder of
    Section 4.1 run from every XCD at once): ``n`` walkers spread evenly
    along one chain, one per workgroup, so the dispatcher puts n / 8 on each
    XCD.  Cache-resident footprints are warmed by every walker walking the
    whole cycle first (each XCD's L2 then holds what fits); the HBM one is
    measured cold after a 2 GiB eviction stream.  Per footprint and walker
    count: mean ns per hop on each XCD, the spread across XCDs, and the odd
    minus even XCD means."""
    import synth
    evict_buf = device_buffer(evict_bytes, seed + 1)
    out = {}
    for name, fp in footprints:
        nodes = fp // stride
        cold = fp > stats.INFINITY_CACHE_BYTES
        row = {}
        for n in walkers:
            chain, starts = synth.chase_chain_starts(fp, stride, seed + fp.bit_length(), n,
                                                     device="cuda")
            if cold:
                isw.sweep_plain(evict_buf, evict_bytes, 4, 16, 32, evict_bytes // 16)
            warm = 0 if cold else nodes
            res = isw.sweep_chase_walkers(chain, fp, starts, warm, hops, policy)
            by = {}
            for r in res:
                by.setdefault(r["xcc_id"], []).append(r["ns_per_hop"])
            per = {x: sum(v) / len(v) for x, v in sorted(by.items())}
            odd = [v for x, v in per.items() if x % 2]
            even = [v for x, v in per.items() if not x % 2]
            row[n] = {"per_xcd_ns": {x: round(v, 2) for x, v in per.items()},
                      "walkers_per_xcd": {x: len(v) for x, v in sorted(by.items())},
                      "spread": round(max(per.values()) / min(per.values()) - 1, 4),
                      "odd_minus_even_ns": (round(sum(odd) / len(odd) - sum(even) / len(even), 2)
                                            if odd and even else None),
                      "cold": cold, "warm_hops": warm}
            del chain
        out[name] = {"bytes": fp, "walkers": row}
    del evict_buf
    return out


# ------------------------------- baseline arm and streaming gate (Table 1)
def fixed_iteration_arm(buf, nbytes, Ks=(1, 2, 4, 8), waves_per_cu=16, iters=None,
                        policy=isw.CACHE_BYPASS_L1_NT, n=3):
    """The paper's baseline arm (Section 4.2, Table 1, first row): every wave
    runs the same iteration count at every K, so issued work grows with K.
    ``iters`` defaults to one pass of the buffer at K = 1."""
    info = isw.sweep_device_info()
    n_waves = info["num_cus"] * waves_per_cu
    if iters is None:
        iters = max(1, nbytes // 16 // (64 * n_waves))
    cells, meta = [], []
    for direction in ("asc", "rev"):
        ks = list(Ks) if direction == "asc" else list(reversed(list(Ks)))
        for K in ks:
            cells.append(isw.make_cell(buf, nbytes, K, 16, waves_per_cu, 0,
                                       cache_policy=policy, mode=isw.FIXED_ITERS,
                                       fixed_iters=iters))
            meta.append({"waves_per_cu": waves_per_cu, "order": direction, "K": K,
                         "bytes": nbytes})
    arr = isw.cell_array(cells)
    isw.sweep_run(arr, raw=True)
    runs = [isw.sweep_run(arr) for _ in range(n)]
    summ = summarize_k_sweep(meta, runs)
    c = summ["curves"][waves_per_cu]
    issued = {m["K"]: r["issued_bytes"] for m, r in zip(meta, runs[0])}
    return {"iters_per_wave": iters, "issued_bytes": issued,
            "median_gbps": {k: round(v, 1) for k, v in c["median_gbps"].items()},
            "decline_2_8": c.get("decline_2_8"), "by_order": c["by_order"]}


def streaming_gate(buf, nbytes, vec_width=4, K=1, waves_per_cu=32, launches=31,
                   policy=isw.CACHE_BYPASS_L1_NT, latency_ns=None, pass_frac=0.85):
    """The streaming-read ceiling row of Section 4.1 ("read, 4 B width, ILP
    1"): median and best of ``launches`` one-pass launches, as a fraction
    of the HBM datasheet figure.

    With ``latency_ns`` (the unloaded HBM round trip) the row also carries
    its Little's-law ceiling, min(datasheet, bytes in flight / latency),
    and a verdict: "pass" if the median reaches ``pass_frac`` of the
    datasheet; "latency-bound" if the form offers too few bytes in flight
    for the datasheet (ceiling below ``pass_frac`` of it), so that it cannot
    pass on this part whatever the memory system does; "fail" otherwise."""
    c = isw.make_cell(buf, nbytes, K, vec_width, waves_per_cu, nbytes // vec_width,
                      cache_policy=policy)
    arr = isw.cell_array([c] * (launches + 1))
    res = isw.sweep_run(arr)[1:]
    g = sorted(r["gbps"] for r in res)
    med = stats.median(g)
    out = {"vec_width": vec_width, "K": K, "waves_per_cu": waves_per_cu,
           "launches": launches, "median_gbps": round(med, 1),
           "best_gbps": round(g[-1], 1),
           "median_frac": med / stats.HBM_PEAK_GBPS,
           "best_frac": g[-1] / stats.HBM_PEAK_GBPS}
    if latency_ns:
        fl = stats.in_flight_bytes(res[0]["waves"], K, vec_width)
        ceil = stats.littles_ceiling_gbps(fl, latency_ns)
        if med >= pass_frac * stats.HBM_PEAK_GBPS:
            verdict = "pass"
        elif ceil < pass_frac * stats.HBM_PEAK_GBPS:
            verdict = "latency-bound"
        else:
            verdict = "fail"
        out.update({"in_flight_bytes": fl, "latency_ns": round(latency_ns, 1),
                    "littles_law_ceiling_gbps": round(ceil, 1),
                    "frac_of_ceiling": med / ceil,
                    "implied_latency_ns": round(stats.implied_latency_ns(fl, med), 1),
                    "pass_frac": pass_frac, "verdict": verdict})
    return out


def hbm_latency_ns(footprint=GIB, policy=isw.CACHE_BYPASS_L1, seed=SEED_BASE + 8):
    """Unloaded HBM round trip: the cold pointer-chase mean over one
    footprint far above the last-level cache (the latency ladder's own
    method, one rung)."""
    row = latency_ladder(footprints=[footprint], policies=(policy,), seed=seed)
    name = {v: k for k, v in isw.POLICY_NAMES.items()}[policy]
    return row[footprint][name]["mean_ns"]


def wave_rec_dtype():
    """NumPy dtype of the 32-byte per-wave record (sweep_wave_rec_t)."""
    import numpy as np
    return np.dtype([("sum32", "<u4"), ("xor32", "<u4"), ("hw_id", "<u4"),
                     ("xcc_id", "<u4"), ("t0", "<u8"), ("t1", "<u8")])


def gap_breakdown(buf, nbytes, L, policy, summ, latency_ns, waves_list, Ks,
                  vec_width=16):
    """Split the K sweep's distance from the datasheet figure into the part
    the design offers (cells whose bytes in flight over the HBM latency fall
    below the datasheet), the tail loss of the static equal split (the
    ceiling lost while only some waves still run, from one untimed launch
    per cell with its per-wave clock records) and a residual.  ``summ`` is
    the timed sweep's summary; its per-cell medians are the measured
    rates."""
    dt = wave_rec_dtype()
    n_cus = isw.sweep_device_info()["num_cus"]
    rec = torch.zeros(n_cus * max(waves_list) * dt.itemsize, dtype=torch.uint8,
                      device="cuda")
    cells, per_w = [], {}
    for w in waves_list:
        curve = summ["curves"].get(w)
        if curve is None:
            continue
        rows = {}
        for K in Ks:
            g = curve["median_gbps"].get(K)
            if g is None:
                continue
            opts = isw.make_opts(cache_policy=policy, wave_out=rec)
            isw.sweep_plain(buf, nbytes, K, vec_width, w, L, opts)     # warm-up
            r = isw.sweep_plain(buf, nbytes, K, vec_width, w, L, opts)
            a = rec[: r["waves"] * dt.itemsize].cpu().numpy().view(dt)
            t0 = a["t0"].astype("int64").tolist()
            t1 = a["t1"].astype("int64").tolist()
            per_wave = 64 * K * vec_width
            fl = stats.in_flight_bytes(r["waves"], K, vec_width)
            ceil = stats.littles_ceiling_gbps(fl, latency_ns)
            act = stats.active_ceiling_gbps(t0, t1, per_wave, latency_ns)
            c = {"bytes": r["issued_bytes"], "gbps": g, "ceiling_gbps": ceil,
                 "active_ceiling_gbps": act}
            cells.append(c)
            rows[K] = {"gbps": round(g, 1), "ceiling_gbps": round(ceil, 1),
                       "active_ceiling_gbps": round(act, 1),
                       "idle_slots": round(stats.idle_slots(t0, t1), 4)}
        if rows:
            split = stats.gap_split([c for c in cells[-len(rows):]])
            per_w[w] = {"cells": rows,
                        "split": {k: (round(v, 4) if isinstance(v, float) else v)
                                  for k, v in split.items()}}
    out = stats.gap_split(cells)
    out = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}
    out["hbm_latency_ns"] = round(latency_ns, 1)
    out["by_waves_per_cu"] = per_w
    out["method"] = ("design ceiling = min(8 TB/s, bytes in flight of all waves / "
                     "unloaded HBM latency); active ceiling = its time average with "
                     "only the waves running at each moment, from one untimed launch "
                     "per cell with per-wave clock records; times summed over cells")
    return out


def write_records(path, meta, runs, extra=None):
    """Append one JSON line per launch (cell, pass index, raw result): the
    raw log kept beside the reported medians."""
    with open(path, "a") as f:
        for i, run in enumerate(runs):
            for m, r in zip(meta, run):
                rec = dict(m)
                rec["pass"] = i
                rec.update({k: r[k] for k in ("issued_bytes", "sum32", "xor32", "gbps",
                                              "window_ns", "event_ms", "waves")})
                if extra:
                    rec.update(extra)
                f.write(json.dumps(rec) + "\n")


def k_counter_pass(nbytes=GIB, waves_list=(4, 16), Ks=(1, 2, 4, 8, 16), L=1 << 26,
                   policy=isw.CACHE_BYPASS_L1_NT, reps=3, seed=SEED_BASE + 1,
                   manifest=None):
    """The K sweep cell by cell, one launch per call, for a separate
    rocprofv3 run with stall-reason and occupancy counters.  The first
    launch of every cell is its warm-up.  Returns (and optionally writes)
    the launch manifest."""
    buf = device_buffer(nbytes, seed)
    order = []
    for w in waves_list:
        for K in Ks:
            c = isw.make_cell(buf, nbytes, K, 16, w, L, cache_policy=policy)
            for rep in range(reps):
                r = isw.sweep_run([c])[0]
                order.append({"bytes": nbytes, "waves_per_cu": w, "K": K, "order": "asc",
                              "rep": rep, "warmup": rep == 0,
                              "issued_bytes": r["issued_bytes"], "gbps": r["gbps"]})
    del buf
    if manifest:
        with open(manifest, "w") as f:
            json.dump(order, f)
    return order


def order_counter_pass(sizes=(16 * MIB, 128 * MIB, GIB), waves_per_cu=16, Ks=(1, 2, 4, 8),
                       L=1 << 26, policy=isw.CACHE_BYPASS_L1_NT, reps=3,
                       seed=SEED_BASE + 6, manifest=None):
    """The order/footprint cells (three address layouts) one launch per
    call, for a separate rocprofv3 counter run: does the L2 catch the
    repeats the lock-step sharing model counts?  The first launch of every
    cell is its warm-up.  Returns (and optionally writes) the launch
    manifest; each entry carries the model's share for its cell."""
    layouts = ((isw.ORDER_ROUND_ROBIN, "round_robin"), (isw.ORDER_BLOCKED, "blocked"),
               (isw.ORDER_STRIDED, "strided"))
    n_waves = isw.sweep_device_info()["num_cus"] * waves_per_cu
    order = []
    for size in sizes:
        buf = device_buffer(size, seed)
        for code, name in layouts:
            for K in Ks:
                c = isw.make_cell(buf, size, K, 16, waves_per_cu, L, cache_policy=policy,
                                  order=code)
                share = stats.front_duplicates(code, K, n_waves, L // (64 * K), size // 16)
                for rep in range(reps):
                    r = isw.sweep_run([c])[0]
                    order.append({"bytes": size, "waves_per_cu": waves_per_cu, "K": K,
                                  "layout": name, "rep": rep, "warmup": rep == 0,
                                  "front_duplicates": share,
                                  "issued_bytes": r["issued_bytes"], "gbps": r["gbps"]})
        del buf
    if manifest:
        with open(manifest, "w") as f:
            json.dump(order, f)
    return order


def lds_counter_pass(nbytes=2 * GIB, waves_list=(1, 4), depths=(1, 4, 8, 16),
                     L=1 << 27, policy=isw.CACHE_DEFAULT, reps=3,
                     seed=SEED_BASE + 3, manifest=None, policies=None):
    """The LDS-direct and matched register paths cell by cell, one launch
    per call, for a separate rocprofv3 counter run (is the LDS itself ever
    the limit?  where do register loads wait?).  With ``policies`` every
    cell runs under each of those cache policies and its manifest entries
    name the policy.  The first launch of every cell is its warm-up.
    Returns (and optionally writes) the launch manifest."""
    buf = device_buffer(nbytes, seed)
    names = {v: k for k, v in isw.POLICY_NAMES.items()}
    order = []
    for pol in (policies or (policy,)):
        for w in waves_list:
            for D in depths:
                for kind, path in ((isw.KIND_LDS_ASYNC, "lds_async"),
                                   (isw.KIND_LDS_MATCHED, "lds_matched")):
                    c = isw.make_cell(buf, nbytes, D, 16, w, L, kind=kind, cache_policy=pol)
                    for rep in range(reps):
                        r = isw.sweep_run([c])[0]
                        e = {"path": path, "bytes": nbytes, "waves_per_cu": w,
                             "K": D, "order": "asc", "rep": rep, "warmup": rep == 0,
                             "issued_bytes": r["issued_bytes"], "gbps": r["gbps"],
                             "window_ns": r["window_ns"]}
                        if policies:
                            e["policy"] = names[pol]
                        order.append(e)
    del buf
    if manifest:
        with open(manifest, "w") as f:
            json.dump(order, f)
    return order
