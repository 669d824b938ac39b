#!/usr/bin/env python3
"""Benchmark of the offered-ILP streaming-load path on one MI355X.

One step is one pass of the fixed-work plain-load K sweep: a 1 GiB seeded
u32 buffer, 16-byte loads, K = 1..16, 2**26 logical loads per cell, at
1..8 waves per SIMD (4..32 waves per CU), each occupancy swept in ascending
and then reversed K order (Section 3, "Fixed-work control"; Section 4.2).
The sweep is captured once into a hipGraph; a step is one replay of it.
The buffer is resident in HBM before timing starts.  W untimed warm-up
steps are followed by exactly K timed steps between two device
synchronisations; the value is the issued bytes of the timed steps over
their wall time.

Reported beside it:
  roofline      the plain-load kernel's algorithmic bytes per launch over
                its mean duration (hipEvent time of the timed replays over
                the kernels they ran), against 8 TB/s, plus the HBM traffic
                measured by rocprofv3 counters when the committed summary
                matches the current kernel source
  eager_sweep   the same sweep launched cell by cell, with every kernel's
                own dispatch-stamped event time
  cpu_baseline  the CPU oracle computing the per-wave checksums of one
                occupancy's whole K curve (16 full 1 GiB cells; bounded
                sample), checked against the GPU's records of those cells
  rows          the other configurations: allocation sweep, LDS-direct vs
                matched paths, two-stream displacement (both mechanisms),
                autotuned graph-batched sweep, precision sums, latency
                ladder, order/footprint and regime map (--no-extras skips)

The full result goes to a JSON file (--json-out); standard output ends
with one compact JSON line (under 4 KB) holding the headline figures, the
roofline, the CPU baseline and one summary per extra configuration.
--gpus N with N > 1 exits: the benchmark measures one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PLAIN_SOURCES = ["paper_2608_15764_amd/csrc/kernels_plain.hip",
                 "paper_2608_15764_amd/csrc/device.hpp"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "plain_kload_1GiB_ksweep_pmc.txt")
HBM_PEAK_GBPS = 8000.0


def source_hash():
    h = hashlib.sha256()
    for p in PLAIN_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per plain-load launch from the committed counter summary,
    or None if there is none or the kernel source changed since."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    kv = {}
    with open(PMC_SUMMARY) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--policy", default="bypass_l1_nt",
                    choices=["default", "nt", "bypass_l1", "bypass_l1_nt"],
                    help="cache policy of the swept loads: bypass_l1 is the "
                         "L1-bypassing analogue of the paper's .cg operator, "
                         "bypass_l1_nt adds the streaming hint (default)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other configurations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run plain device copies of 1 GiB (counter scale)")
    ap.add_argument("--only", default=None,
                    choices=["c3", "c4", "c5a", "c5b", "c3counters", "c2counters",
                             "c4counters", "c4stalls", "f3counters", "f3ksweep", "next",
                             "fabric"],
                    help="run only one extra configuration (no K sweep); "
                         "the *counters modes and c4stalls run cells one launch "
                         "per call for a separate rocprofv3 counter run")
    ap.add_argument("--manifest", default=None,
                    help="launch manifest path for the counter-run modes")
    ap.add_argument("--c5b-waves", default=None,
                    help="fixed waves per CU for the precision sums instead of "
                         "tuning, e.g. f32=8,bf16=8,fp8_e4m3=4 (for profiling "
                         "the tuned launches alone)")
    ap.add_argument("--c5a-config", default=None,
                    help="fixed K,V,waves_per_cu,policy for every batched point "
                         "instead of tuning, e.g. 3,16,8,1 (for counter runs that "
                         "must repeat the same launches)")
    ap.add_argument("--json-out", default=None,
                    help="file for the full result (default "
                         "results/bench_detail.json); standard output ends "
                         "with a compact headline line")
    ap.add_argument("--record", default=None,
                    help="append one JSON line per timed launch (raw log) to this file")
    return ap.parse_args()


_WORDS = None


def _oracle_cell(task):
    """One cell's global sinks from the oracle (runs in a worker process)."""
    from oracle import checksums, plan as oplan
    K, n_waves, L = task
    p = oplan.wave_group(L, K, n_waves)
    s, x = checksums.per_wave(_WORDS, 16, K, p["Q"], n_waves)
    return K, checksums.combine(s, x)


def cpu_oracle_worker(spec):
    """Child-process side of the multi-process CPU baseline: never imports
    torch and never touches the GPU; forks its pool workers from here."""
    global _WORDS
    import multiprocessing as mp
    from oracle import splitmix
    a = json.loads(spec)
    t0 = time.perf_counter()
    _WORDS = splitmix.buffer_words(a["seed"], a["nbytes"])
    t1 = time.perf_counter()
    tasks = [(K, a["n_waves"], a["L"]) for K in a["Ks"]]
    with mp.get_context("fork").Pool(a["procs"]) as pool:
        res = pool.map(_oracle_cell, tasks, chunksize=1)
    t2 = time.perf_counter()
    print(json.dumps({"sinks": {str(K): list(v) for K, v in res},
                      "generate_s": t1 - t0, "checksum_s": t2 - t1, "procs": a["procs"]}))
    return 0


def cpu_baseline_multi(seed, nbytes, L, Ks, n_waves, gpu_sinks, issued_bytes):
    """The same oracle over the same cells, one cell per worker process, in
    a child process started for it (the measuring process keeps the GPU)."""
    import subprocess
    procs = max(1, min(16, os.cpu_count() or 1, len(Ks)))
    spec = json.dumps({"seed": seed, "nbytes": nbytes, "L": L, "Ks": list(Ks),
                       "n_waves": n_waves, "procs": procs})
    try:
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                            "--cpu-oracle-worker", spec], cwd=ROOT, capture_output=True,
                           text=True, timeout=300)
        out = json.loads(r.stdout.strip().splitlines()[-1])
    except Exception as e:          # reported, never fatal for the bench line
        return {"error": f"{type(e).__name__}: {e}"}
    ok = all(tuple(out["sinks"][str(K)]) == gpu_sinks[K] for K in Ks)
    return {"value": issued_bytes / out["checksum_s"] / 1e9, "unit": "GB/s",
            "cores": out["procs"], "checksum_s": out["checksum_s"],
            "generate_s": out["generate_s"], "matches_gpu": ok,
            "sample": "the same cells, one per worker process (fork pool in a child "
                      "process); buffer generation excluded"}


def cpu_baseline(buf_seed, nbytes, L, Ks, waves_per_cu, gpu_buf, num_cus):
    """Oracle per-wave checksums of one occupancy's whole K curve (one full
    cell per K), timed on the host and checked against the GPU's records."""
    import numpy as np
    import torch
    from oracle import checksums, plan as oplan, splitmix
    from paper_2608_15764_amd import environment, ilpsweep as isw

    dt = np.dtype([("sum32", "<u4"), ("xor32", "<u4"), ("hw_id", "<u4"),
                   ("xcc_id", "<u4"), ("t0", "<u8"), ("t1", "<u8")])
    gpu = {}
    for K in Ks:
        rec = torch.zeros(num_cus * waves_per_cu * 32, dtype=torch.uint8, device="cuda")
        r = isw.sweep_plain(gpu_buf, nbytes, K, 16, waves_per_cu, L,
                            isw.make_opts(wave_out=rec))
        gpu[K] = (r, rec.cpu().numpy().view(dt)[: r["waves"]])
    t0 = time.perf_counter()
    words = splitmix.buffer_words(buf_seed, nbytes)
    t1 = time.perf_counter()
    issued, ok = 0, True
    for K in Ks:
        r, recs = gpu[K]
        p = oplan.wave_group(L, K, r["waves"])
        s, x = checksums.per_wave(words, 16, K, p["Q"], r["waves"])
        issued += p["issued"] * 16
        ok = ok and bool(np.array_equal(s, recs["sum32"]) and np.array_equal(x, recs["xor32"])
                         and p["issued"] == r["issued_loads"])
    t2 = time.perf_counter()
    multi = cpu_baseline_multi(buf_seed, nbytes, L, Ks, gpu[Ks[0]][0]["waves"],
                               {K: (gpu[K][0]["sum32"], gpu[K][0]["xor32"]) for K in Ks},
                               issued)
    return {
        "value": issued / (t2 - t1) / 1e9,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{len(Ks)} full cells of the sweep (K={Ks[0]}..{Ks[-1]} at "
                   f"{waves_per_cu} waves/CU, {gpu[Ks[0]][0]['waves']} waves): per-wave "
                   f"sum/xor checksums of {issued >> 30} GiB issued, NumPy, one "
                   f"process; buffer generation {t1 - t0:.1f} s excluded"),
        "checksum_s": t2 - t1,
        "generate_s": t1 - t0,
        "host_cores_available": os.cpu_count(),
        "host_cpu": environment.cpu_model(),
        "matches_gpu": ok,
        "multi_process": multi,
    }


def timed_graph(isw, cells, steps, warmup):
    """Capture ``cells`` once as a hipGraph, replay it ``warmup`` times
    untimed, then ``steps`` times between two device synchronisations.
    Returns (per-replay result lists, per-replay event ms, wall seconds)."""
    import torch
    arr = isw.cell_array(cells)
    graph = isw.sweep_graph_create(arr)
    try:
        for _ in range(warmup):
            isw.sweep_graph_launch(graph, raw=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = [isw.sweep_graph_launch(graph, raw=True) for _ in range(steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    finally:
        isw.sweep_graph_destroy(graph)
    return [isw.result_dicts(r) for r, _ in outs], [ms for _, ms in outs], t1 - t0


def curve_rows(summ, peak):
    return {w: {"median_gbps": {k: round(v, 1) for k, v in c["median_gbps"].items()},
                "min_gbps": {k: round(v, 1) for k, v in c["min_gbps"].items()},
                "best_gbps": {k: round(v, 1) for k, v in c["best_gbps"].items()},
                "pct_of_best_cell": {k: round(100 * v / peak, 1)
                                     for k, v in c["median_gbps"].items()},
                "in_flight_mib": {k: v / 2**20 for k, v in c["in_flight_bytes"].items()},
                "littles_law_latency_ns": {k: round(v, 1) for k, v in
                                           c["implied_latency_ns"].items()},
                "peak_K": c["peak_K"], "knee_K": c["knee_K"],
                "regime": c["regime"], "decline_2_8": c.get("decline_2_8"),
                "paired_declines_2_8": [round(x, 4) for x in c.get("paired_declines_2_8", [])],
                "by_order": c["by_order"]}
            for w, c in summ["curves"].items()}


def paper_like(summ, w=16):
    c = summ["curves"].get(w)
    if c is None:
        return None
    return {"waves_per_cu": w, "median_gbps": c["median_gbps"],
            "peak_K": c["peak_K"], "decline_2_8": c.get("decline_2_8"),
            "paired_declines_2_8": sorted(round(x, 4) for x in c.get("paired_declines_2_8", [])),
            "regime": c["regime"], "by_order": c["by_order"]}


def strict_cg_sweep(a, isw, sweeps, stats, buf, nbytes, L, waves_list, Ks):
    """The same K sweep under the strict analogue of the paper's .cg
    operator (L1 bypass, no streaming hint), captured as its own graph and
    replayed with the headline's steps and warm-up (Section 4.2, Table 1
    primary cell; "Repeatability")."""
    pol = isw.CACHE_BYPASS_L1
    cells, meta = sweeps.plain_k_cells(buf, nbytes, L, pol, waves_list, Ks)
    cells, meta, _ = sweeps.drop_infeasible(cells, meta)
    runs, ms, wall = timed_graph(isw, cells, a.steps, a.warmup)
    summ = sweeps.summarize_k_sweep(meta, runs)
    step_bytes = sum(r["issued_bytes"] for r in runs[0])
    best_w = summ["best_waves_per_cu"]
    pl = paper_like(summ)
    bo = (pl or {}).get("by_order", {})
    paired = (pl or {}).get("paired_declines_2_8") or []
    return {
        "policy": "bypass_l1",
        "value": round(a.steps * step_bytes / wall / 1e9, 1),
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "curve_peak_gbps": round(summ["peak_gbps"], 1),
        "curve_peak_frac_of_hbm": round(summ["peak_gbps"] / stats.HBM_PEAK_GBPS, 4),
        "best_waves_per_cu": best_w,
        "peak_K_at_best": summ["curves"][best_w]["peak_K"],
        "paper_like_decline_2_8": None if pl is None else pl["decline_2_8"],
        "paper_like_decline_2_8_asc": (bo.get("asc") or {}).get("decline_2_8"),
        "paper_like_decline_2_8_rev": (bo.get("rev") or {}).get("decline_2_8"),
        "paper_like_paired_decline_median": stats.median(paired) if paired else None,
        "paper_like_cell": pl,
        "curves": curve_rows(summ, summ["peak_gbps"]),
        "kset_mismatch": summ["kset_mismatch"],
        "checksums_consistent": summ["checksums_consistent"],
        "residency_flags": summ["residency_flags"],
        "anomalous_launches": summ["anomalous_launches"],
        "graph_replay_event_ms_median": round(sorted(ms)[len(ms) // 2], 3),
    }


def _reduce_lane_terms(kind, n, waves, waves_per_cu):
    """Most terms one lane of the streaming sum adds in its TwoSum chain:
    its share of the full wave-groups (8 loads per lane at 4 waves per CU,
    4 above; FP8 adds one term per four vectors), one remainder vector and
    the trailing elements."""
    per_vec = {"f32": 4, "bf16": 8, "fp8_e4m3": 16}[kind]
    eb = {"f32": 4, "bf16": 2, "fp8_e4m3": 1}[kind]
    loads = 8 if waves_per_cu == 4 else 4
    groups = (n * eb // 16) // (64 * loads)
    g_lane = -(-groups // waves) if waves else 0
    per_group = loads * per_vec if kind != "fp8_e4m3" else loads // 4
    return g_lane * per_group + per_vec + 16


def cpu_precision_hook(store, threads):
    """The oracle's side of the precision rows: the exact sum (and sum |x|)
    of each payload the GPU summed, from a host copy, computed in slices on
    ``threads`` threads and combined exactly; the GPU sum's error against it
    and the rigorous bound.  Timings go to ``store`` (part of the CPU
    baseline)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from oracle import fpsum

    def exact(kind, host, absolute):
        if kind == "f32":
            b = host.view(np.uint32)
            b = b & np.uint32(0x7FFFFFFF) if absolute else b
            fn = lambda a: fpsum.exact_sum_f32_bits(a, rational=True)
        elif kind == "bf16":
            b = host.view(np.uint16)
            b = b & np.uint16(0x7FFF) if absolute else b
            fn = lambda a: fpsum.exact_sum_bf16_bits(a, rational=True)
        else:
            b = host & np.uint8(0x7F) if absolute else host
            fn = lambda a: fpsum.exact_sum_e4m3_hist(a, rational=True)
        step = 1 << 24
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(fn, [b[i:i + step] for i in range(0, b.size, step)]))
        return sum(parts)

    def hook(kind, payload, n_el, row):
        host = payload.cpu().numpy()
        t0 = time.perf_counter()
        s_exact = exact(kind, host, False)
        t1 = time.perf_counter()
        abs_sum = float(exact(kind, host, True))
        del host
        from fractions import Fraction
        err = abs(Fraction(row["sum"]) - s_exact)
        n_lane = _reduce_lane_terms(kind, n_el, row["waves"], row["waves_per_cu"])
        bound = fpsum.sum2_bound(abs_sum, n_lane, 8, row["grid_wgs"])
        store[kind] = {"exact_sum": float(s_exact), "seconds": t1 - t0,
                       "gbps": payload.numel() / (t1 - t0) / 1e9, "threads": threads}
        return {"exact_sum": float(s_exact), "abs_err": float(err),
                "rel_err": float(err) / abs_sum if abs_sum else 0.0,
                "bound": bound, "within_bound": float(err) <= bound}
    return hook


def cpu_batch_verifier(store, threads):
    """The oracle's side of the batched row: every launch's sinks against
    the global sums of the words it read (its issued prefix of its point),
    computed on ``threads`` threads; the time goes to ``store``."""
    from oracle import checksums

    def verify(checks):
        t0 = time.perf_counter()
        want = checksums.range_sinks_many([c[:3] for c in checks], threads=threads)
        store["seconds"] = time.perf_counter() - t0
        store["threads"] = threads
        store["words"] = sum(n for _, _, n in {c[:3] for c in checks})
        store["gbps"] = 4 * store["words"] / store["seconds"] / 1e9
        return [w == (c[3], c[4]) for w, c in zip(want, checks)]
    return verify


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--cpu-oracle-worker":
        return cpu_oracle_worker(sys.argv[2])
    a = parse()
    if a.steps < 1 or a.warmup < 0:
        print("bench.py needs --steps >= 1 and --warmup >= 0", file=sys.stderr)
        return 2
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the path is single-GPU (several GPUs "
              "would each stream their own HBM and combine 16 bytes of sinks and "
              "window end points per cell at the end); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch
    from paper_2608_15764_amd import ilpsweep as isw
    from paper_2608_15764_amd import report, stats, sweeps

    from paper_2608_15764_amd import environment
    torch.cuda.set_device(0)
    env_before = environment.sysfs_metrics()
    info = isw.sweep_device_info()
    hz = isw.sweep_calibrate_clock(0.5)
    policy = isw.POLICY_NAMES[a.policy]
    out_extra = {}
    if a.calib_copy:
        # plain 1 GiB device copies: the known-size reference that scales
        # the FETCH_SIZE / WRITE_SIZE counters of a separate counter run
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if a.only == "c3counters":
        GIB = 1 << 30
        sizes = [512 << 20, GIB, 2 * GIB, 4 * GIB, 8 * GIB, 20 * GIB]
        man = sweeps.allocation_counter_pass(sizes, policy=policy, manifest=a.manifest)
        print(json.dumps({"only": a.only, "launches": len(man)}))
        return 0
    if a.only == "c4counters":
        man = sweeps.lds_counter_pass(policy=policy, manifest=a.manifest)
        print(json.dumps({"only": a.only, "launches": len(man)}))
        return 0
    if a.only == "c4stalls":
        # both LDS paths under the default policy and the swept one, for
        # counter runs on where each path's loads wait
        pols = sorted({isw.CACHE_DEFAULT, policy})
        man = sweeps.lds_counter_pass(waves_list=(1, 4), depths=(8, 16), policies=pols,
                                      manifest=a.manifest)
        print(json.dumps({"only": a.only, "launches": len(man)}))
        return 0
    if a.only == "f3counters":
        man = sweeps.order_counter_pass(policy=policy, manifest=a.manifest)
        print(json.dumps({"only": a.only, "launches": len(man)}))
        return 0
    if a.only == "f3ksweep":
        # every K from 1 to 16 over the 128 MiB allocation, at 2 and 4
        # waves/SIMD: where the wrapped volume realigns with the allocation
        man = []
        for w in (8, 16):
            man += sweeps.order_counter_pass(sizes=(128 << 20,), waves_per_cu=w,
                                             Ks=range(1, 17), policy=policy)
        if a.manifest:
            with open(a.manifest, "w") as f:
                json.dump(man, f)
        print(json.dumps({"only": a.only, "launches": len(man)}))
        return 0
    if a.only == "fabric":
        # the XCD-subset and per-XCD-share reads of the 1 GiB sweep buffer
        # alone, for a kernel trace of their own
        buf = sweeps.device_buffer(1 << 30, sweeps.SEED_BASE + 1)
        rows = {}
        for name, fn, kw in (("fabric_by_xcd", sweeps.fabric_by_xcd, {"manifest": a.manifest}),
                             ("xcd_weighting", sweeps.xcd_weighting, {})):
            try:
                rows[name] = fn(buf, 1 << 30, policy=policy, **kw)
            except isw.SweepError as e:
                rows[name + "_error"] = str(e)
        if a.json_out:
            report.write_detail({"only": a.only, "rows": rows}, a.json_out)
        print(json.dumps({"only": a.only, "detail": a.json_out, "rows": sorted(rows)}))
        return 0
    if a.only == "c2counters":
        man = sweeps.k_counter_pass(policy=policy, manifest=a.manifest)
        print(json.dumps({"only": a.only, "launches": len(man)}))
        return 0
    if a.only:
        out_extra = run_extras(a, isw, sweeps, only=a.only)
        if a.json_out:
            report.write_detail({"only": a.only, "rows": out_extra}, a.json_out)
        print(json.dumps({"only": a.only, "detail": a.json_out,
                          "rows": sorted(out_extra)}, default=str))
        return 0

    nbytes, L = 1 << 30, 1 << 26
    seed = sweeps.SEED_BASE + 1
    buf = sweeps.device_buffer(nbytes, seed)
    waves_list = [4 * w for w in range(1, 9)]
    Ks = list(range(1, 17))
    cells, meta = sweeps.plain_k_cells(buf, nbytes, L, policy, waves_list, Ks)
    cells, meta, dropped = sweeps.drop_infeasible(cells, meta)

    # the step is one replay of the sweep captured once as a hipGraph (one
    # kernel node per cell, then the finishing node); each replay is timed
    # with a hipEvent pair on the stream it is launched on
    runs, graph_ms, wall = timed_graph(isw, cells, a.steps, a.warmup)
    if a.record:
        sweeps.write_records(a.record, meta, runs,
                             {"policy": a.policy, "buffer_bytes": nbytes, "L": L})

    env_after = environment.sysfs_metrics()
    step_bytes = sum(r["issued_bytes"] for r in runs[0])
    value = a.steps * step_bytes / wall / 1e9
    # average launch duration = replay time / kernels per replay: an upper
    # bound on the mean kernel time (it holds the gaps between graph nodes
    # and the small finishing kernel), so `achieved` is a lower bound
    kernel_ms = sum(graph_ms)
    launches = sum(len(run) for run in runs)
    achieved = a.steps * step_bytes / (kernel_ms * 1e6)
    traffic = traffic_from_profile()
    summ = sweeps.summarize_k_sweep(meta, runs)
    best_w = summ["best_waves_per_cu"]
    cb = summ["curves"][best_w]

    result = {
        "metric": "attained HBM GB/s vs offered loads/thread K; % of HBM peak; K=2\u21928 decline %",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (SplitMix64-seeded uint32 buffer, resident in HBM)",
        "config": {
            "workload": ("fixed-work plain-load K sweep: 1 GiB seeded u32 buffer, "
                         "16-byte loads, K=1..16, 2^26 logical loads per cell, "
                         "1..8 waves/SIMD, ascending then reversed K"),
            "buffer_bytes": nbytes, "vec_width": 16, "L": L, "Ks": Ks,
            "waves_per_cu": waves_list, "orders": ["asc", "rev"],
            "cache_policy": a.policy, "cells_per_step": len(cells),
            "infeasible_cells": dropped,
        },
        "curve_peak_gbps": round(summ["peak_gbps"], 1),
        "curve_peak_frac_of_hbm": round(summ["peak_gbps"] / HBM_PEAK_GBPS, 4),
        "best_waves_per_cu": best_w,
        "peak_K_at_best": cb["peak_K"],
        "decline_2_8_at_best": cb.get("decline_2_8"),
        "paper_like_cell": paper_like(summ),
        "curves": curve_rows(summ, summ["peak_gbps"]),
        "kset_mismatch": summ["kset_mismatch"],
        "checksums_consistent": summ["checksums_consistent"],
        "residency_flags": summ["residency_flags"],
        "anomalous_launches": summ["anomalous_launches"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "kernel": "ilp::plain_kload<K,16,policy>",
                     "launches": launches,
                     "mean_launch_us": round(kernel_ms / launches * 1e3, 2),
                     "timing": "hipEvent pair per graph replay / kernels per replay",
                     "algorithmic_bytes_per_launch": step_bytes // len(cells)},
        "device": {"arch": info["arch"], "cus": info["num_cus"],
                   "clock_hz_calibrated": hz},
        "environment": {"static": environment.static_info(),
                        "gpu_before": env_before, "gpu_after": env_after},
    }
    # the strict .cg analogue, timed like the headline
    if a.policy != "bypass_l1" and not a.no_extras:
        result["strict_cg"] = strict_cg_sweep(a, isw, sweeps, stats, buf, nbytes, L,
                                              waves_list, Ks)
    # the same sweep launched eagerly, cell by cell (sweep_run): the cost of
    # one host launch per kernel against the graph replay timed above, and
    # every kernel's own duration from the events its dispatch stamps
    arr = isw.cell_array(cells)
    isw.sweep_run(arr, raw=True)
    torch.cuda.synchronize()
    eager = []
    for _ in range(3):
        e0 = time.perf_counter()
        er = isw.sweep_run(arr, raw=True)
        eager.append(time.perf_counter() - e0)
    eager_ms = sorted(eager)[1] * 1e3
    disp_ms = sum(r.event_ms for r in er)
    result["eager_sweep"] = {
        "cells": len(cells), "step_ms": round(eager_ms, 3),
        "aggregate_gbps": round(step_bytes / (eager_ms * 1e6), 1),
        "dispatch_event_mean_us": round(disp_ms / len(cells) * 1e3, 2),
        "dispatch_event_gbps": round(step_bytes / (disp_ms * 1e6), 1),
        "graph_step_ms": result["ms_per_step"],
        "graph_replay_event_ms": round(sorted(graph_ms)[len(graph_ms) // 2], 3)}
    lat = None
    if not a.no_extras:
        # the unloaded HBM round trip, then where the sweep's distance from
        # the datasheet goes (ceilings by design, tail loss, residual)
        lat = sweeps.hbm_latency_ns()
        result["gap"] = sweeps.gap_breakdown(buf, nbytes, L, policy, summ, lat,
                                             waves_list, Ks)
        # the ceiling the plateau meets: the same read by subsets of the XCDs;
        # and what the equal split costs: shares re-weighted by each XCD's
        # speed.  Both rely on the dispatcher dealing one workgroup to every
        # XCD per round of eight and check it; where that fails, the row
        # records why and the rest of the run goes on.
        for name, fn in (("fabric_by_xcd", sweeps.fabric_by_xcd),
                         ("xcd_weighting", sweeps.xcd_weighting)):
            try:
                result[name] = fn(buf, nbytes, policy=policy)
            except isw.SweepError as e:
                result[name + "_error"] = str(e)
        # one untimed pass of the same sweep under the other cache policies
        pc = {}
        for name, pol in isw.POLICY_NAMES.items():
            pcells, pmeta = sweeps.plain_k_cells(buf, nbytes, L, pol, waves_list, Ks)
            pcells, pmeta, _ = sweeps.drop_infeasible(pcells, pmeta)
            s2 = sweeps.summarize_k_sweep(pmeta, [isw.sweep_run(pcells)])
            c16 = s2["curves"].get(16, {})
            c4 = s2["curves"].get(4, {})
            pc[name] = {"peak_gbps": round(s2["peak_gbps"], 1),
                        "best_waves_per_cu": s2["best_waves_per_cu"],
                        "paper_like_decline_2_8": c16.get("decline_2_8"),
                        "paper_like_median_gbps": {k: round(v, 1) for k, v in
                                                   c16.get("median_gbps", {}).items()},
                        # one wave per SIMD, the lowest occupancy of the sweep
                        "one_wave_per_simd_gbps": {k: round(v, 1) for k, v in
                                                   c4.get("median_gbps", {}).items()}}
        result["policy_curves"] = pc
        result["baseline_fixed_iterations"] = sweeps.fixed_iteration_arm(buf, nbytes)
        result["completion_spread"] = sweeps.completion_spread(
            buf, nbytes, L, isw.POLICY_NAMES[a.policy], waves_list, K=4)
        result["streaming_gate"] = sweeps.streaming_gate(buf, nbytes, latency_ns=lat)
        # the same gate form with 16-byte loads: four times the bytes in flight
        result["streaming_gate_16B"] = sweeps.streaming_gate(buf, nbytes, vec_width=16,
                                                             latency_ns=lat)
        result["library_reads"] = library_reads(buf, nbytes)
    if not a.no_cpu_baseline:
        ks_best = sorted({m["K"] for m in meta if m["waves_per_cu"] == best_w})
        result["cpu_baseline"] = cpu_baseline(seed, nbytes, L, ks_best, best_w, buf,
                                              info["num_cus"])
    del buf
    if not a.no_extras:
        result["rows"] = run_extras(a, isw, sweeps, best_w=best_w)
        # the oracle's exact sums behind the precision rows' errors
        prec = result["rows"].pop("c5b_cpu_oracle", None)
        if prec and "cpu_baseline" in result:
            result["cpu_baseline"]["precision"] = prec
        bat = result["rows"].pop("c5a_cpu_oracle", None)
        if bat and "cpu_baseline" in result:
            result["cpu_baseline"]["batched"] = bat
    detail = a.json_out or os.path.join("results", "bench_detail.json")
    report.emit(result, detail, sys.stdout)
    return 0


def library_reads(buf, nbytes, reps=10):
    """Context for the roofline, not part of the path: the rate of torch's
    own kernels over the same resident 1 GiB buffer, each timed with a
    hipEvent pair on torch's current stream (the one they run on), median
    of ``reps`` after a warm-up.  Reductions read the buffer once; the
    device copy reads it and writes as many bytes."""
    import torch
    x = buf.view(torch.int32)[: nbytes // 4]
    y = torch.empty_like(x)
    xf = x.view(torch.float32)
    ops = {"sum_float32": (lambda: xf.sum(), nbytes),
           "sum_int32_to_int64": (lambda: x.sum(dtype=torch.int64), nbytes),
           "amax_int32": (lambda: torch.amax(x), nbytes),
           "copy_read_plus_write": (lambda: y.copy_(x), 2 * nbytes)}
    out = {}
    for name, (fn, moved) in ops.items():
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = sorted(ms)[len(ms) // 2]
        out[name] = {"bytes_moved": moved, "median_ms": round(med, 4),
                     "gbps": round(moved / (med * 1e6), 1),
                     "frac_of_hbm_peak": round(moved / (med * 1e6) / 8000.0, 4)}
    del y
    return out


def run_extras(a, isw, sweeps, only=None, best_w=None):
    """The other configurations.  ``best_w`` is the K sweep's best
    occupancy (waves per CU); without it (``--only c3``) one short pass of
    the same K sweep finds it."""
    import torch
    rows = {}
    GIB = 1 << 30
    if only in (None, "c3"):
        t = time.perf_counter()
        pol = isw.POLICY_NAMES[a.policy]
        if best_w is None:
            kbuf = sweeps.device_buffer(GIB, sweeps.SEED_BASE + 1)
            best_w = sweeps.plain_k_sweep(kbuf, GIB, 1 << 26, pol, range(4, 33, 4),
                                          range(1, 17), passes=2)["best_waves_per_cu"]
            del kbuf
        # the paper-like occupancy (4 waves/SIMD) and the K sweep's best
        waves = (16,) if best_w == 16 else (16, best_w)
        sizes = [512 << 20, GIB, 2 * GIB, 4 * GIB, 8 * GIB, 20 * GIB]
        rows["c3_allocation_sweep"] = sweeps.allocation_sweep(sizes, waves_list=waves,
                                                              policy=pol)
        rows["c3_allocation_sweep"]["waves_per_cu"] = list(waves)
        rows["c3_allocation_sweep"]["wall_s"] = time.perf_counter() - t
    if only in (None, "c4"):
        t = time.perf_counter()
        nbytes = 2 * GIB
        buf = sweeps.device_buffer(nbytes, sweeps.SEED_BASE + 3)
        L = nbytes // 16
        # both paths and both streams use the swept loads' cache policy;
        # the path comparison is repeated under every other policy beside it
        pol = isw.POLICY_NAMES[a.policy]
        grid = [(wa, wb) for wa in (1, 2, 4, 8) for wb in (1, 2, 4, 8)]
        rows["c4_path_comparison"] = sweeps.path_comparison(buf, nbytes, L, policy=pol, n=5)
        rows["c4_path_comparison_other_policies"] = {
            name: sweeps.path_comparison(buf, nbytes, L, policy=v)
            for name, v in isw.POLICY_NAMES.items() if v != pol}
        rows["c4_two_stream"] = sweeps.two_stream(buf, nbytes, L, policy=pol)
        rows["c4_two_stream_grid"] = sweeps.two_stream(
            buf, nbytes, L, depths=(4,), pairs=grid, n=2, policy=pol)
        # the section's own measurement: plain loads in both streams
        rows["c4_two_stream_same_mechanism_grid"] = sweeps.two_stream(
            buf, nbytes, L, depths=(4,), pairs=grid, n=2, policy=pol,
            kind_b=isw.KIND_PLAIN)
        # the same streams on different CUs: twice the waves per workgroup
        # on half of the CUs, so each stream keeps its total waves
        split_pairs = [(2 * wa, 2 * wb) for wa, wb in grid]
        rows["c4_two_stream_split_same_mechanism_grid"] = sweeps.two_stream(
            buf, nbytes, L, depths=(4,), pairs=split_pairs, n=2, policy=pol,
            kind_b=isw.KIND_PLAIN, split=True)
        rows["c4_two_stream_split_grid"] = sweeps.two_stream(
            buf, nbytes, L, depths=(4,), pairs=split_pairs, n=2, policy=pol, split=True)
        rows["c4_wall_s"] = time.perf_counter() - t
        del buf
    if only in (None, "c5a"):
        t = time.perf_counter()
        verify = None
        if not a.no_cpu_baseline:
            vstore = rows.setdefault("c5a_cpu_oracle", {})
            verify = cpu_batch_verifier(vstore, max(1, min(16, os.cpu_count() or 1)))
        fixed = tuple(int(v) for v in a.c5a_config.split(",")) if a.c5a_config else None
        rows["c5a_batched"] = sweeps.batched_autotuned(verify=verify, fixed=fixed)
        rows["c5a_batched"]["wall_s"] = time.perf_counter() - t
    if only in (None, "c5b"):
        t = time.perf_counter()
        fixed = None
        if a.c5b_waves:
            fixed = {k: int(v) for k, v in (kv.split("=") for kv in a.c5b_waves.split(","))}
        hook = None
        if not a.no_cpu_baseline:
            store = rows.setdefault("c5b_cpu_oracle", {})
            hook = cpu_precision_hook(store, max(1, min(16, os.cpu_count() or 1)))
        rows["c5b_precision"] = sweeps.precision_sum(waves_fixed=fixed, on_payload=hook)
        rows["c5b_precision"]["wall_s"] = time.perf_counter() - t
    if only in (None, "next"):
        t = time.perf_counter()
        MIB = 1 << 20
        # K = 3 and 6 beside the powers of two: around the caches the
        # wrapped volume lands concurrent loads on shared segments only at
        # some K, and the unaligned ones show the loads' own response
        rows["f2_f3_order_footprint"] = sweeps.order_footprint(
            [2 * MIB, 4 * MIB, 8 * MIB, 16 * MIB, 128 * MIB, GIB, 4 * GIB],
            Ks=(1, 2, 3, 4, 6, 8))
        rows["f2_f3_order_footprint"]["wall_s"] = time.perf_counter() - t
        t = time.perf_counter()
        rows["f4_regime_map"] = sweeps.regime_map()
        rows["f4_regime_map"]["wall_s"] = time.perf_counter() - t
        t = time.perf_counter()
        rows["f1_latency_ladder"] = sweeps.latency_ladder()
        rows["f1_latency_ladder"]["wall_s"] = time.perf_counter() - t
        t = time.perf_counter()
        rows["f1_latency_by_xcd"] = sweeps.latency_by_xcd()
        rows["f1_latency_by_xcd"]["wall_s"] = time.perf_counter() - t
    return rows


if __name__ == "__main__":
    sys.exit(main())
