"""Host-side helpers of the sweep drivers (no GPU)."""
import json

from paper_2608_15764_amd import sweeps


def test_point_sizes_span_1MiB_to_2GiB_aligned():
    s = sweeps.point_sizes(64)
    assert len(s) == 64 and s[0] == 1 << 20 and s[-1] == 2 << 30
    assert all(x % (64 * 1024) == 0 for x in s)
    assert all(b >= a for a, b in zip(s, s[1:]))


def test_size_classes():
    M = 1 << 20
    assert [sweeps.size_class(x) for x in (M, 4 * M, 20 * M, 100 * M, 300 * M, 2 << 30)] == \
        [0, 1, 2, 3, 4, 5]


def test_raw_records_roundtrip(tmp_path):
    meta = [{"waves_per_cu": 16, "order": "asc", "K": 1, "bytes": 1 << 30},
            {"waves_per_cu": 16, "order": "asc", "K": 2, "bytes": 1 << 30}]
    r = {"issued_bytes": 1, "sum32": 2, "xor32": 3, "gbps": 4.0, "window_ns": 5.0,
         "event_ms": 6.0, "waves": 7}
    p = tmp_path / "raw.jsonl"
    sweeps.write_records(str(p), meta, [[r, r], [r, r]], {"policy": "nt"})
    lines = [json.loads(l) for l in open(p)]
    assert len(lines) == 4 and lines[3]["pass"] == 1 and lines[1]["K"] == 2
    assert lines[0]["policy"] == "nt" and lines[0]["gbps"] == 4.0


def test_summarize_k_sweep_on_synthetic_results():
    meta, runs = [], [[], []]
    for order in ("asc", "rev"):
        for K in ((1, 2, 4, 8) if order == "asc" else (8, 4, 2, 1)):
            meta.append({"waves_per_cu": 16, "order": order, "K": K, "bytes": 1 << 30})
    base = {1: 5000.0, 2: 7000.0, 4: 7100.0, 8: 7050.0}
    for p in range(2):
        for m in meta:
            runs[p].append({"gbps": base[m["K"]] + p, "issued_loads": 1 << 26,
                            "issued_bytes": 1 << 30, "sum32": 9, "xor32": 9,
                            "waves": 4096})
    s = sweeps.summarize_k_sweep(meta, runs)
    c = s["curves"][16]
    assert c["peak_K"] == 4 and s["checksums_consistent"]
    assert abs(c["decline_2_8"] - (7050.5 - 7000.5) / 7000.5) < 1e-12
    assert s["kset_mismatch"] == 0.0 and s["residency_flags"] == 0
    assert c["in_flight_bytes"][2] == 4096 * 64 * 2 * 16
    assert s["anomalous_launches"]["count"] == 0
    assert s["anomalous_launches"]["launches"] == 16 and s["anomalous_launches"]["worst"] is None


def test_summarize_k_sweep_discloses_a_slow_launch():
    meta = [{"waves_per_cu": 8, "order": "asc", "K": K, "bytes": 1 << 30} for K in (1, 2, 4)]
    runs = []
    for p in range(5):
        runs.append([{"gbps": (3000.0 if (p == 3 and m["K"] == 2) else 6000.0),
                      "issued_loads": 1, "issued_bytes": 1 << 30, "sum32": 0, "xor32": 0,
                      "waves": 2048} for m in meta])
    s = sweeps.summarize_k_sweep(meta, runs)
    a = s["anomalous_launches"]
    assert a["count"] == 1 and a["launches"] == 15
    assert a["worst"] == {"waves_per_cu": 8, "K": 2, "gbps": 3000.0, "ratio": 0.5}


def _flat_sweep(alloc_bytes, gbps):
    meta = [{"waves_per_cu": 16, "order": o, "K": K, "bytes": alloc_bytes}
            for o in ("asc", "rev") for K in (1, 2, 4, 8)]
    runs = [[{"gbps": gbps, "issued_loads": 1 << 26, "issued_bytes": 1 << 30,
              "sum32": 1, "xor32": 2, "waves": 4096} for _ in meta]]
    return meta, runs


def test_residency_screen_uses_the_allocation_not_the_issued_bytes():
    """A 2 MiB buffer read 512 times over (1 GiB issued) sits in the caches:
    more than the HBM datasheet figure is expected there and never flagged.
    The same rate over a 1 GiB buffer is flagged on every launch."""
    s = sweeps.summarize_k_sweep(*_flat_sweep(2 << 20, 25000.0))
    assert s["residency_flags"] == 0
    s = sweeps.summarize_k_sweep(*_flat_sweep(1 << 30, 8500.0))
    assert s["residency_flags"] == 8
    s = sweeps.summarize_k_sweep(*_flat_sweep(1 << 30, 7900.0))
    assert s["residency_flags"] == 0


def test_summarize_k_sweep_needs_the_allocation():
    import pytest
    meta, runs = _flat_sweep(1 << 30, 7000.0)
    del meta[3]["bytes"]
    with pytest.raises(ValueError):
        sweeps.summarize_k_sweep(meta, runs)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU and says so for --gpus N > 1 (no GPU used)."""
    import subprocess
    import sys
    from conftest import ROOT
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr


def test_bench_cpu_oracle_worker():
    """The multi-process CPU baseline's child mode (no GPU): one cell per
    worker, global sinks equal to the oracle's, in one JSON line."""
    import subprocess
    import sys
    from conftest import ROOT
    from oracle import checksums, plan as oplan, splitmix
    spec = {"seed": 5, "nbytes": 4 << 20, "L": (4 << 20) // 16 + 640, "Ks": [1, 3, 5],
            "n_waves": 96, "procs": 3}
    r = subprocess.run([sys.executable, "bench.py", "--cpu-oracle-worker", json.dumps(spec)],
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout.strip().splitlines()[-1])
    words = splitmix.buffer_words(5, 4 << 20)
    for K in spec["Ks"]:
        p = oplan.wave_group(spec["L"], K, spec["n_waves"])
        want = checksums.combine(*checksums.per_wave(words, 16, K, p["Q"], spec["n_waves"]))
        assert tuple(out["sinks"][str(K)]) == want
    assert out["procs"] == 3 and out["checksum_s"] > 0


def test_bench_rejects_zero_steps():
    import subprocess
    import sys
    from conftest import ROOT
    r = subprocess.run([sys.executable, "bench.py", "--steps", "0"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "--steps" in r.stderr and r.stdout == ""
