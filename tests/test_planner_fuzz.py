"""The host-only planner under AddressSanitizer and UndefinedBehaviorSanitizer,
fed random (mostly valid, some invalid) cells and checked against the oracle."""
import os
import random
import shutil
import subprocess

import pytest

from conftest import ROOT
from oracle import plan as oplan

CSRC = os.path.join(ROOT, "paper_2608_15764_amd", "csrc")


@pytest.fixture(scope="module")
def fuzz_exe(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("fuzz") / "plan_fuzz")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
                    "-I", CSRC, os.path.join(ROOT, "tests", "plan_fuzz.cpp"),
                    os.path.join(CSRC, "plan.cpp"), "-o", exe], check=True)
    return exe


def _case(rnd):
    V = rnd.choice([4, 8, 16, 16, 12])
    kind = rnd.choice([0, 0, 0, 1, 2])
    K = rnd.choice([0, 1, 2, 3, 5, 8, 13, 16, 17])
    waves = rnd.choice([4, 8, 16, 32, 6, 36, 1, 2, 16]) if kind == 0 else rnd.choice([1, 4, 8, 16, 17])
    bytes_ = rnd.choice([0, 1000, 64 * V * rnd.randint(1, 1 << 16), 1 << 30, 20 << 30])
    L = rnd.choice([0, 1, 255, 64 * K * rnd.randint(1, 5000) + rnd.randint(0, 100), 1 << 26, 1 << 30])
    mode = rnd.choice([0, 0, 1, 2, 5])
    fixed = rnd.choice([0, 1, 7, 1000])
    cus = rnd.choice([256, 256, 80, 1])
    grid = rnd.choice([0, 0, 0, 3, 1000])
    order = rnd.choice([0, 0, 1, 3])
    return (bytes_, K, V, kind, waves, L, mode, fixed, cus, grid, order)


def test_random_cells_match_the_oracle(fuzz_exe):
    rnd = random.Random(1234)
    cases = [_case(rnd) for _ in range(20000)]
    inp = "\n".join(" ".join(map(str, c)) for c in cases) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([fuzz_exe], input=inp, capture_output=True, text=True, env=env,
                         check=True, timeout=120).stdout.split("\n")
    n_ok = 0
    for c, line in zip(cases, out):
        bytes_, K, V, kind, waves, L, mode, fixed, cus, grid, order = c
        f = line.split()
        if int(f[0]) != 0:
            continue
        n_ok += 1
        Q, issued, imin, imax, g, nw, stride, G, pad = map(int, f[1:])
        wg_waves = 4 if kind == 0 else waves
        assert g == (grid or cus * (waves // 4 if kind == 0 else 1)) and nw == g * wg_waves
        if mode == 0:
            o = oplan.wave_group(L, K, nw, order=order)
        elif mode == 1:
            o = oplan.fixed_iters(fixed, K, nw)
            if order == 1:
                o = {"Q": o["Q"], "issued": o["issued"],
                     **{k: v for k, v in oplan.wave_group(o["issued"], K, nw, order=1).items()
                        if k in ("iters_min", "iters_max")}}
        else:
            t = oplan.per_thread_floor(L, nw * 64, K)
            o = {"Q": nw * t["iters"], "issued": t["issued"], "iters_min": t["iters"],
                 "iters_max": t["iters"]}
            if order == 1:
                o.update({k: v for k, v in oplan.wave_group(o["issued"], K, nw, order=1).items()
                          if k in ("iters_min", "iters_max")})
        assert (Q, issued) == (o["Q"], o["issued"]), c
        assert (imin, imax) == (o["iters_min"], o["iters_max"]), c
        n_vec = bytes_ // V
        assert stride == ((K * 64) % n_vec if order == 1 else (nw * K * 64) % n_vec)
        assert G == -(-Q // nw)
        assert bytes_ % (64 * V) == 0 and 1 <= K <= 16 and Q > 0
    assert n_ok > 300
