"""Counter-audit parser on synthetic rocprofv3 CSVs (no GPU)."""
import csv

import pytest

from paper_2608_15764_amd import rocprof

CC_FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id",
             "Thread_Id", "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size",
             "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
             "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp",
             "End_Timestamp"]


def _write_cc(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=CC_FIELDS)
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": k, "Grid_Size": 1024,
                        "Counter_Name": c, "Counter_Value": v})


def test_warmup_failed_and_scale(tmp_path):
    p = tmp_path / "x_counter_collection.csv"
    K = "void ilp::plain_kload<2, 16, 2>(ilp::PlainArgs)"
    rows = [(K, "FETCH_SIZE", 100.0),          # warm-up: excluded by rule
            (K, "FETCH_SIZE", 524288.0),
            (K, "FETCH_SIZE", ""),              # failed dispatch: excluded
            (K, "FETCH_SIZE", 524300.0),
            ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 8.0),
            ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0),
            ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 524290.0)]
    _write_cc(p, rows)
    r = rocprof.counter_rows(str(p))
    vals, failed = rocprof.counter_values(r, "FETCH_SIZE", "plain_kload")
    assert vals == [524288.0, 524300.0] and failed == 1
    sc = rocprof.calib_scale(r, "FETCH_SIZE", 1 << 30)
    assert sc == pytest.approx((1 << 30) / (524289.0 * 1024))
    mr = rocprof.med_range(vals)
    assert mr["median"] == 524294.0 and mr["min"] == 524288.0 and mr["n"] == 2


def test_summary_traffic_over_algorithmic(tmp_path):
    K = "void ilp::plain_kload<4, 16, 3>(ilp::PlainArgs)"
    f = tmp_path / "f_counter_collection.csv"
    w = tmp_path / "w_counter_collection.csv"
    _write_cc(f, [(K, "FETCH_SIZE", 1.0), (K, "FETCH_SIZE", 524288.0),
                  ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0)])
    _write_cc(w, [(K, "WRITE_SIZE", 1.0), (K, "WRITE_SIZE", 160.0),
                  ("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0)])
    s = rocprof.summary(None, str(f), str(w), "plain_kload", 1 << 30, 1 << 30)
    assert s["fetch_scale"] == pytest.approx(2.0)
    assert s["write_scale"] == pytest.approx(1.0)
    assert s["hbm_bytes_per_launch"] == pytest.approx((1 << 30) + 160 * 1024)
    assert s["traffic_over_algorithmic"] == pytest.approx(1 + 160 * 1024 / (1 << 30))
    txt = rocprof.format_summary(s, ["cmd"], "abc")
    assert "source_hash: abc" in txt and "hbm_bytes_per_launch:" in txt


def test_missing_counter_gives_no_traffic(tmp_path):
    K = "plain_kload"
    f = tmp_path / "f_counter_collection.csv"
    _write_cc(f, [(K, "FETCH_SIZE", ""), (K, "FETCH_SIZE", "nan")])
    s = rocprof.summary(None, str(f), None, "plain_kload", 1 << 30)
    assert "hbm_bytes_per_launch" not in s
    assert s["fetch_failed_dispatches"] == 2


def test_cell_table_keys_on_occupancy(tmp_path):
    K4 = "void ilp::plain_kload<4, 16, 3>(ilp::PlainArgs)"
    man = []
    rows = []
    for w in (4, 16):
        for rep in range(3):
            man.append({"bytes": 1 << 30, "waves_per_cu": w, "K": 4, "order": "asc",
                        "rep": rep, "warmup": rep == 0})
            rows.append((K4, "TCC_HIT_sum", 10.0 * w + rep))
            rows.append((K4, "TCC_MISS_sum", 90.0))
    # counters of one dispatch appear as consecutive rows with one dispatch id
    p = tmp_path / "c_counter_collection.csv"
    with open(p, "w", newline="") as f:
        w_ = csv.DictWriter(f, fieldnames=CC_FIELDS)
        w_.writeheader()
        for i in range(len(man)):
            for j in range(2):
                k, c, v = rows[2 * i + j]
                w_.writerow({"Dispatch_Id": i + 1, "Kernel_Name": k, "Grid_Size": 1,
                             "Counter_Name": c, "Counter_Value": v})
    tab = rocprof.cell_table([rocprof.counter_rows(str(p))], man)
    assert set(tab) == {(1 << 30, 4, 4, "asc"), (1 << 30, 16, 4, "asc")}
    row = tab[(1 << 30, 4, 4, "asc")]
    assert row["TCC_HIT_sum"] == 41.5                 # warm-up (40) excluded
    assert row["l2_hit_rate"] == pytest.approx(41.5 / 131.5)


def test_cell_table_keys_on_path_and_kernel(tmp_path):
    """LDS-path manifests carry a path field and name other kernels."""
    KA = "void ilp::lds_kernel_t<1, 4, 0>(ilp::LdsArgs)"
    KM = "void ilp::lds_kernel_t<2, 4, 0>(ilp::LdsArgs)"
    man, rows = [], []
    for path, k in (("lds_async", KA), ("lds_matched", KM)):
        for rep in range(3):
            man.append({"path": path, "bytes": 1 << 31, "waves_per_cu": 1, "K": 4,
                        "order": "asc", "rep": rep, "warmup": rep == 0})
            rows.append((k, "SQ_LDS_BANK_CONFLICT", 5.0 if path == "lds_async" else 7.0))
    rows.insert(1, ("void ilp::plain_kload<4, 16, 3>(ilp::PlainArgs)",
                    "SQ_LDS_BANK_CONFLICT", 99.0))        # not in the manifest
    p = tmp_path / "l_counter_collection.csv"
    _write_cc(p, rows)
    tab = rocprof.cell_table([rocprof.counter_rows(str(p))], man,
                             kernel_substr="lds_kernel_t")
    assert tab[("lds_async", 1 << 31, 1, 4, "asc")]["SQ_LDS_BANK_CONFLICT"] == 5.0
    assert tab[("lds_matched", 1 << 31, 1, 4, "asc")]["SQ_LDS_BANK_CONFLICT"] == 7.0
    with pytest.raises(ValueError):        # plain dispatches do not match it
        rocprof.cell_table([rocprof.counter_rows(str(p))], man)


def test_lds_busy_fraction(tmp_path):
    K = "void ilp::lds_kernel_t<1, 8, 0>(ilp::LdsArgs)"
    man = [{"path": "lds_async", "bytes": 1, "waves_per_cu": 4, "K": 8, "order": "asc",
            "rep": r, "warmup": r == 0} for r in range(2)]
    rows = []
    for r in range(2):
        rows += [(K, "SQ_LDS_IDX_ACTIVE", 8.0e6), (K, "GRBM_GUI_ACTIVE", 8.0e6)]
    p = tmp_path / "b_counter_collection.csv"
    _write_cc(p, rows)
    tab = rocprof.cell_table([rocprof.counter_rows(str(p))], man, kernel_substr="lds_kernel_t",
                             cus=256, xccs=8)
    # 8e6 busy CU-cycles over 1e6 cycles x 256 CUs
    assert tab[("lds_async", 1, 4, 8, "asc")]["lds_busy_frac"] == pytest.approx(8e6 / 256e6)


def test_cell_table_keys_on_policy_and_derives_latencies(tmp_path):
    """Manifests that name a cache policy key their cells on it; the L1
    latency totals are divided by their request and wave counts."""
    K = "void ilp::lds_kernel_t<2, 8, 0>(ilp::LdsArgs)"
    man, rows = [], []
    for pol, lat in (("default", 900.0), ("bypass_l1_nt", 600.0)):
        for rep in range(2):
            man.append({"path": "lds_matched", "policy": pol, "bytes": 1 << 31,
                        "waves_per_cu": 1, "K": 8, "order": "asc", "rep": rep,
                        "warmup": rep == 0})
            rows += [(K, "TCP_TCC_READ_REQ_LATENCY_sum", lat * 1000),
                     (K, "TCP_TCC_READ_REQ_sum", 1000.0),
                     (K, "TCP_TCP_LATENCY_sum", 5000.0),
                     (K, "TCP_TA_TCP_STATE_READ_sum", 0.0)]
    p = tmp_path / "t_counter_collection.csv"
    _write_cc(p, rows)
    tab = rocprof.cell_table([rocprof.counter_rows(str(p))], man, kernel_substr="lds_kernel_t")
    assert set(tab) == {("lds_matched", "default", 1 << 31, 1, 8, "asc"),
                        ("lds_matched", "bypass_l1_nt", 1 << 31, 1, 8, "asc")}
    row = tab[("lds_matched", "default", 1 << 31, 1, 8, "asc")]
    assert row["tcp_tcc_read_latency"] == pytest.approx(900.0)
    assert "tcp_wave_latency" not in row           # zero state reads: no ratio


def test_cell_table_keys_on_layout(tmp_path):
    """Order/footprint manifests name the address layout: cells of equal
    size, occupancy and K but different layouts stay apart."""
    K2 = "void ilp::plain_kload<2, 16, 3>(ilp::PlainArgs)"
    man, rows = [], []
    for layout, hits in (("round_robin", 10.0), ("strided", 50.0)):
        for rep in range(3):
            man.append({"bytes": 128 << 20, "waves_per_cu": 16, "K": 2, "layout": layout,
                        "rep": rep, "warmup": rep == 0})
            rows.append((K2, "TCC_HIT_sum", hits + rep))
    p = tmp_path / "d_counter_collection.csv"
    _write_cc(p, rows)
    tab = rocprof.cell_table([rocprof.counter_rows(str(p))], man)
    assert set(tab) == {(128 << 20, 16, "round_robin", 2), (128 << 20, 16, "strided", 2)}
    assert tab[(128 << 20, 16, "strided", 2)]["TCC_HIT_sum"] == 51.5


def test_cells_cli_reads_the_fetch_scale_from_the_copies(tmp_path, capsys):
    """`cells --calib-bytes` takes the FETCH_SIZE scale from the device
    copies of the FETCH_SIZE pass, and says so in the header."""
    import json
    K4 = "void ilp::plain_kload<4, 16, 3>(ilp::PlainArgs)"
    man = [{"bytes": 1 << 30, "waves_per_cu": 4, "K": 4, "order": "asc", "warmup": r == 0}
           for r in range(3)]
    m = tmp_path / "m.json"
    m.write_text(json.dumps(man))
    f = tmp_path / "f_counter_collection.csv"
    _write_cc(f, [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0),
                  (K4, "FETCH_SIZE", 1.0), (K4, "FETCH_SIZE", 524288.0),
                  (K4, "FETCH_SIZE", 524290.0)])
    h = tmp_path / "h_counter_collection.csv"
    _write_cc(h, [(K4, "TCC_HIT_sum", 5.0)] * 3)
    out = tmp_path / "cells.txt"
    assert rocprof.main(["cells", "--manifest", str(m), "--counters", str(f), str(h),
                         "--calib-bytes", str(1 << 30), "--out", str(out)]) == 0
    text = out.read_text()
    assert "# FETCH_SIZE scale (device copies of known size): 2" in text
    row = [ln for ln in text.splitlines() if ln.startswith(f"{1 << 30} 4 4 asc:")][0]
    assert f"fetch_bytes={524289.0 * 1024 * 2:.6g}" in row
    with pytest.raises(SystemExit):
        rocprof.main(["cells", "--manifest", str(m), "--counters", str(h),
                      "--calib-bytes", str(1 << 30)])
    capsys.readouterr()


def _write_trace(path, rows):
    fields = ["Kernel_Name", "Dispatch_Id", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for i, (k, s, e) in enumerate(rows):
            w.writerow({"Kernel_Name": k, "Dispatch_Id": i + 1, "Start_Timestamp": s,
                        "End_Timestamp": e})


def test_trace_cells_pairs_durations_with_the_manifest(tmp_path, capsys):
    """Kernel durations of a trace, paired in start order with a launch
    manifest: warm-ups dropped, other kernels ignored, GB/s at the median."""
    import json
    X = "void ilp::xcd_subset<3>(ilp::XcdArgs)"
    man, rows, t = [], [], 1000
    for mask, dur in (("0x01", 800), ("0xff", 150)):
        for rep in range(4):
            man.append({"path": "xcd_subset", "waves_per_cu": 4, "mask": mask,
                        "issued_bytes": 1200, "rep": rep, "warmup": rep == 0})
            d = 5000 if rep == 0 else dur + rep
            rows.append((X, t, t + d))
            rows.append(("ilp::finish_cells(...)", t + d + 10, t + d + 20))
            t += d + 100
    p = tmp_path / "x_kernel_trace.csv"
    _write_trace(p, rows[::-1])                       # file order does not matter
    tab = rocprof.trace_cells(str(p), man, "xcd_subset")
    assert set(tab) == {("xcd_subset", 4, "0x01"), ("xcd_subset", 4, "0xff")}
    r = tab[("xcd_subset", 4, "0xff")]
    assert (r["median"], r["min"], r["max"], r["n"]) == (152, 151, 153, 3)
    assert r["gbps"] == pytest.approx(1200 / 152)
    with pytest.raises(ValueError):
        rocprof.trace_cells(str(p), man[:-1], "xcd_subset")
    m = tmp_path / "m.json"
    m.write_text(json.dumps(man))
    out = tmp_path / "t.txt"
    assert rocprof.main(["trace-cells", "--manifest", str(m), "--trace", str(p),
                         "--kernel", "xcd_subset", "--out", str(out)]) == 0
    text = out.read_text()
    assert "xcd_subset 4 0x01: median_ns=802 min_ns=801 max_ns=803 n=3 gbps=1.5" in text
    capsys.readouterr()
