"""The C ABI library: it loads, exports every declared symbol, its structs
match the header's layout, and its host-only planner agrees with the oracle
(no GPU needed)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from conftest import ROOT
from oracle import plan as oplan

HEADER = os.path.join(ROOT, "include", "ilpsweep.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sweep_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def isw():
    from paper_2608_15764_amd import ilpsweep
    return ilpsweep


def test_every_declared_symbol_is_exported(isw):
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(isw.lib, n), n
    assert set(names) == set(isw._SIG)


def test_version_and_errors(isw):
    assert "gfx950" in isw.sweep_version()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert isw.sweep_strerror(code)
    assert isw.sweep_strerror(-99) == "unknown error"


STRUCTS = {
    "sweep_wave_rec_t": ["sum32", "xor32", "hw_id", "xcc_id", "t0", "t1"],
    "sweep_opts_t": ["stream", "cache_policy", "mode", "fixed_iters",
                     "grid_wgs", "pin_occupancy", "wave_out", "lane_out",
                     "order", "wave_out_cap", "lane_out_cap", "fuse"],
    "sweep_result_t": ["target_loads", "issued_loads", "issued_bytes",
                       "mismatch", "sum32", "xor32", "grid_wgs", "wg_threads",
                       "waves", "iters_min", "iters_max", "max_wgs_per_cu",
                       "vgprs", "sgprs", "lds_bytes", "scratch_bytes",
                       "window_ticks", "window_ns", "event_ms", "gbps"],
    "sweep_plan_t": ["grid_wgs", "wg_threads", "waves", "n_vec", "Q",
                     "issued_loads", "issued_bytes", "iters_min", "iters_max",
                     "mismatch", "lds_pad_bytes"],
    "sweep_device_t": ["ordinal", "arch", "num_cus", "lds_per_cu",
                       "lds_per_wg_max", "l2_bytes", "hbm_bytes",
                       "wall_clock_hz", "calibrated_hz", "clock_khz",
                       "mem_clock_khz", "mem_bus_bits"],
    "sweep_chase_t": ["final_index", "hops", "wall_ticks", "ns_per_hop",
                      "shader_clock_hz"],
    "sweep_walker_t": ["final_index", "xcc_id", "hops", "wall_ticks", "ns_per_hop"],
    "sweep_cell_t": ["kind", "K", "vec_width", "waves_per_cu", "cache_policy",
                     "mode", "fixed_iters", "grid_wgs", "buf", "bytes",
                     "total_logical_loads", "order"],
}


def test_struct_layouts_match_the_header(isw):
    # compile a C probe of the header with gcc and compare sizes / offsets
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ilpsweep.h"',
             "int main(void) {"]
    for s, fields in STRUCTS.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fields:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe],
                       check=True)
        out = subprocess.run([exe], check=True, capture_output=True,
                             text=True).stdout
    want = dict(l.rsplit(" ", 1) for l in out.strip().splitlines())
    for s, fields in STRUCTS.items():
        cls = getattr(isw, s)
        assert ctypes.sizeof(cls) == int(want[s]), s
        for f in fields:
            assert getattr(cls, f).offset == int(want[f"{s}.{f}"]), f"{s}.{f}"


@pytest.mark.parametrize("K", [1, 2, 3, 7, 13, 16])
@pytest.mark.parametrize("w", [4, 12, 32])
def test_planner_matches_oracle_fixed_work(isw, K, w):
    L = 2**26
    p = isw.sweep_plan(2**30, K, 16, w, L, num_cus=256)
    n_waves = 256 * w
    o = oplan.wave_group(L, K, n_waves)
    assert p["waves"] == n_waves and p["grid_wgs"] == 256 * w // 4
    assert p["Q"] == o["Q"] and p["issued_loads"] == o["issued"]
    assert (p["iters_min"], p["iters_max"]) == (o["iters_min"], o["iters_max"])
    assert p["issued_bytes"] == 16 * o["issued"]
    assert p["mismatch"] == pytest.approx(oplan.target_mismatch(L, o["issued"]),
                                          abs=1e-15)


def test_planner_other_modes(isw):
    p = isw.sweep_plan(1 << 20, 4, 16, 8, 0, mode=isw.FIXED_ITERS,
                       fixed_iters=3, num_cus=256)
    o = oplan.fixed_iters(3, 4, 256 * 8)
    assert p["issued_loads"] == o["issued"] and p["mismatch"] == 0.0
    T = 256 * 8 * 64
    p = isw.sweep_plan(1 << 20, 3, 16, 8, 10**8, mode=isw.PER_THREAD_FLOOR,
                       num_cus=256)
    o = oplan.per_thread_floor(10**8, T, 3)
    assert p["issued_loads"] == o["issued"]
    assert p["iters_min"] == p["iters_max"] == o["iters"]


@pytest.mark.parametrize("K,w,L", [(1, 4, 2**26), (3, 12, 2**26 + 999), (16, 32, 10**6),
                                   (5, 8, 64 * 5 * 7)])
def test_planner_blocked_order(isw, K, w, L):
    p = isw.sweep_plan(2**30, K, 16, w, L, num_cus=256, order=isw.ORDER_BLOCKED)
    o = oplan.wave_group(L, K, 256 * w, order=oplan.BLOCKED)
    assert p["Q"] == o["Q"] and p["issued_loads"] == o["issued"]
    assert (p["iters_min"], p["iters_max"]) == (o["iters_min"], o["iters_max"])


@pytest.mark.parametrize("K,w,L", [(1, 4, 2**26), (3, 12, 2**26 + 999), (16, 32, 10**6)])
def test_planner_strided_layout(isw, K, w, L):
    """The strided layout deals its groups round robin: the same plan."""
    p = isw.sweep_plan(2**30, K, 16, w, L, num_cus=256, order=isw.ORDER_STRIDED)
    o = oplan.wave_group(L, K, 256 * w, order=oplan.STRIDED)
    assert p["Q"] == o["Q"] and p["issued_loads"] == o["issued"]
    assert (p["iters_min"], p["iters_max"]) == (o["iters_min"], o["iters_max"])
    with pytest.raises(isw.SweepError):
        isw.sweep_plan(2**30, K, 16, w, L, num_cus=256, order=3)


def test_planner_explicit_grid(isw):
    p = isw.sweep_plan(64 << 20, 2, 4, 4, 2**24, num_cus=0, grid_wgs=256)
    assert p["grid_wgs"] == 256 and p["waves"] == 1024
    assert p["Q"] == 2**24 // 128


@pytest.mark.parametrize("args,code", [
    ((1 << 20, 0, 16, 8, 1000), -1),      # K = 0
    ((1 << 20, 17, 16, 8, 1000), -1),     # K = 17
    ((1 << 20, 2, 12, 8, 1000), -1),      # width 12
    ((1 << 20, 2, 16, 6, 1000), -1),      # waves not a multiple of 4
    ((1 << 20, 2, 16, 36, 1000), -1),     # too many waves
    ((0, 2, 16, 8, 1000), -1),            # empty buffer
    ((1000, 2, 16, 8, 1000), -2),         # not a multiple of 1024
    ((1 << 20, 2, 16, 8, 0), -1),         # L = 0
    ((1 << 20, 4, 16, 8, 255), -1),       # less than one wave-group
])
def test_planner_rejects(isw, args, code):
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plan(*args, num_cus=256)
    assert e.value.code == code


def test_planner_rejects_unknown_mode(isw):
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plan(1 << 20, 2, 16, 8, 1000, mode=7, num_cus=256)
    assert e.value.code == -1
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plan(1 << 20, 2, 16, 8, 1000, num_cus=256, order=3)
    assert e.value.code == -1


def test_argument_checks_that_precede_any_device_work(isw):
    """Checks every entry point makes before it touches a device, run on the
    host: sizes whose byte counts overflow, NULL and misaligned pointers."""
    cases = [
        (lambda: isw.sweep_reduce_fp(16, 2**63, isw.F32, 4), isw.EINVAL),
        (lambda: isw.sweep_reduce_fp(16, 10, 9, 4), isw.EINVAL),
        (lambda: isw.sweep_reduce_fp(8, 10, isw.F32, 4), isw.EALIGN),
        (lambda: isw.sweep_reduce_fp(16, 10, isw.F32, 6), isw.EINVAL),
        (lambda: isw.sweep_fill_u32(0, 64, 1), isw.EINVAL),
        (lambda: isw.sweep_fill_u32(16, 6, 1), isw.EALIGN),
        (lambda: isw.sweep_chase(16, 1 << 32, 0, 0, 10), isw.EINVAL),
        (lambda: isw.sweep_chase(16, 4096, 1024, 0, 10), isw.EINVAL),
    ]
    for call, code in cases:
        with pytest.raises(isw.SweepError) as e:
            call()
        assert e.value.code == code
