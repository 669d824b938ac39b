"""Parity of the HIP path against the CPU oracle, at sizes the oracle
finishes in seconds (several tiles, ragged tails, wrap-around)."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_util import (decode_lanes, decode_recs, dev_bytes, host_words,
                      lanes, recs, reduce_lane_terms)
from oracle import checksums, fpsum, plan as oplan, splitmix
from paper_2608_15764_amd import ilpsweep as isw
import synth

SEED = 0x1D5EED00


def test_device_is_gfx950():
    info = isw.sweep_device_info()
    print("device:", info, flush=True)
    assert info["arch"].startswith("gfx950")
    assert info["num_cus"] > 0 and info["lds_per_cu"] > 0


@pytest.mark.parametrize("nbytes", [4, 12, 16, 1 << 20, (1 << 20) + 12,
                                    3 * (1 << 20) + 4])
def test_fill_matches_oracle(nbytes):
    buf = torch.zeros(((nbytes + 15) // 16) * 16, dtype=torch.uint8, device="cuda")
    isw.sweep_fill_u32(buf, nbytes, SEED + 7)
    torch.cuda.synchronize()
    got = host_words(buf)[:nbytes // 4]
    assert np.array_equal(got, splitmix.words(SEED + 7, 0, nbytes // 4))
    # nothing beyond the requested bytes is touched
    assert not buf[nbytes:].any()


@pytest.mark.parametrize("K", [1, 2, 4, 8])
def test_plumbing_cell_per_thread(K):
    """64 MiB seeded buffer, 256 workgroups x 256 threads, 4-byte loads."""
    nbytes = 64 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED)
    L = nbytes // 4
    n_waves = 1024
    lo = lanes(n_waves * 64)
    ro = recs(n_waves)
    opts = isw.make_opts(grid_wgs=256, lane_out=lo, wave_out=ro)
    r = isw.sweep_plain(buf, nbytes, K, 4, 4, L, opts)
    p = oplan.wave_group(L, K, n_waves)
    assert r["issued_loads"] == p["issued"] == L
    words = splitmix.buffer_words(SEED, nbytes)
    ws, wx = checksums.per_lane(words, 4, K, p["Q"], n_waves)
    gs, gx = decode_lanes(lo, n_waves)
    assert np.array_equal(gs, ws) and np.array_equal(gx, wx)
    rr = decode_recs(ro)
    os_, ox = checksums.per_wave(words, 4, K, p["Q"], n_waves)
    assert np.array_equal(rr["sum32"], os_) and np.array_equal(rr["xor32"], ox)
    assert (r["sum32"], r["xor32"]) == checksums.whole_buffer(words)


PLAIN_CASES = [
    # V, K, waves_per_cu, grid_wgs, n_vec, L (vectors)  -- wrap and ragged
    (4, 1, 4, 3, 64 * 40, 64 * 40 * 3 + 77),
    (4, 5, 8, 2, 64 * 17, 64 * 17 * 5 + 1000),
    (8, 3, 4, 5, 64 * 33, 64 * 33 * 2),
    (8, 16, 32, 1, 64 * 9, 64 * 16 * 11),
    (16, 2, 4, 3, 64 * 64, 64 * 64 * 3 + 129),
    (16, 7, 12, 2, 64 * 50, 64 * 7 * 23),
    (16, 16, 8, 3, 64 * 20, 64 * 16 * 13),
    (16, 1, 32, 4, 64 * 1024, 64 * 1024),
]


def _random_plain_cases(n=48, seed=20261203):
    """Seeded random cells: width, K, occupancy, explicit grid, allocation
    (whole 64-vector segments), a target with a ragged remainder, address
    order and cache policy; the volume wraps the allocation in most."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        V = int(rng.choice([4, 8, 16]))
        K = int(rng.integers(1, 17))
        w = int(rng.choice([4, 8, 12, 16, 20, 24, 28, 32]))
        grid = int(rng.integers(1, 7))
        n_vec = 64 * int(rng.integers(1, 201))
        Q = int(rng.integers(1, 301))
        L = 64 * K * Q + int(rng.integers(0, 64 * K))
        out.append((V, K, w, grid, n_vec, L, int(rng.integers(0, 3)), int(rng.integers(0, 4))))
    return out


@pytest.mark.parametrize("V,K,w,grid,n_vec,L,order,policy", _random_plain_cases())
def test_plain_random_cells_match_oracle(V, K, w, grid, n_vec, L, order, policy):
    """Per lane, per wave and global sinks against the oracle."""
    nbytes = n_vec * V
    buf = synth.random_bytes(nbytes, seed=n_vec + K + 7 * V, device="cuda")
    n_waves = grid * 4
    lo = lanes(n_waves * 64)
    ro = recs(n_waves)
    opts = isw.make_opts(grid_wgs=grid, cache_policy=policy, lane_out=lo,
                         wave_out=ro, order=order)
    r = isw.sweep_plain(buf, nbytes, K, V, w, L, opts)
    p = oplan.wave_group(L, K, n_waves, order=order)
    assert r["issued_loads"] == p["issued"]
    assert (r["iters_min"], r["iters_max"]) == (p["iters_min"], p["iters_max"])
    words = host_words(buf)
    ws, wx = checksums.per_lane(words, V, K, p["Q"], n_waves, order=order)
    gs, gx = decode_lanes(lo, n_waves)
    assert np.array_equal(gs, ws) and np.array_equal(gx, wx)
    rr = decode_recs(ro)
    os_, ox = checksums.per_wave(words, V, K, p["Q"], n_waves, order=order)
    assert np.array_equal(rr["sum32"], os_) and np.array_equal(rr["xor32"], ox)
    assert (r["sum32"], r["xor32"]) == checksums.combine(ws, wx)


@pytest.mark.parametrize("policy", [0, 1, 2, 3])
@pytest.mark.parametrize("V,K,w,grid,n_vec,L", PLAIN_CASES)
def test_plain_matches_oracle(V, K, w, grid, n_vec, L, policy):
    nbytes = n_vec * V
    buf = synth.random_bytes(nbytes, seed=V * 1000 + K, device="cuda")
    n_waves = grid * 4
    lo = lanes(n_waves * 64)
    ro = recs(n_waves)
    opts = isw.make_opts(grid_wgs=grid, cache_policy=policy, lane_out=lo,
                         wave_out=ro)
    r = isw.sweep_plain(buf, nbytes, K, V, w, L, opts)
    p = oplan.wave_group(L, K, n_waves)
    assert r["issued_loads"] == p["issued"]
    assert (r["iters_min"], r["iters_max"]) == (p["iters_min"], p["iters_max"])
    words = host_words(buf)
    ws, wx = checksums.per_lane(words, V, K, p["Q"], n_waves)
    gs, gx = decode_lanes(lo, n_waves)
    assert np.array_equal(gs, ws) and np.array_equal(gx, wx)
    rr = decode_recs(ro)
    assert np.array_equal(rr["sum32"], ws.astype(np.uint64).sum(1).astype(np.uint32))
    assert (r["sum32"], r["xor32"]) == checksums.combine(ws, wx)
    assert (rr["t1"] >= rr["t0"]).all()


@pytest.mark.parametrize("mode", ["fixed_iters", "per_thread_floor"])
def test_plain_other_modes(mode):
    V, K, grid = 16, 3, 2
    n_vec = 64 * 30
    nbytes = n_vec * V
    buf = synth.random_bytes(nbytes, seed=5, device="cuda")
    n_waves = grid * 4
    ro = recs(n_waves)
    if mode == "fixed_iters":
        opts = isw.make_opts(grid_wgs=grid, mode=isw.FIXED_ITERS,
                             fixed_iters=7, wave_out=ro)
        r = isw.sweep_plain(buf, nbytes, K, V, 8, 0, opts)
        o = oplan.fixed_iters(7, K, n_waves)
    else:
        L = 100000
        opts = isw.make_opts(grid_wgs=grid, mode=isw.PER_THREAD_FLOOR, wave_out=ro)
        r = isw.sweep_plain(buf, nbytes, K, V, 8, L, opts)
        o = oplan.per_thread_floor(L, n_waves * 64, K)
    assert r["issued_loads"] == o["issued"]
    Q = o["issued"] // (64 * K)
    s, x = checksums.per_wave(host_words(buf), V, K, Q, n_waves)
    rr = decode_recs(ro)
    assert np.array_equal(rr["sum32"], s) and np.array_equal(rr["xor32"], x)


LDS_CASES = [
    # kind, D, waves per WG, grid, n_vec, L
    (1, 1, 1, 3, 64 * 40, 64 * 40 * 2 + 5),
    (1, 4, 4, 2, 64 * 50, 64 * 4 * 31),
    (1, 16, 8, 3, 64 * 20, 64 * 16 * 9),
    (1, 5, 16, 1, 64 * 64, 64 * 5 * 40),
    (2, 1, 1, 3, 64 * 40, 64 * 40 * 2 + 5),
    (2, 4, 4, 2, 64 * 50, 64 * 4 * 31),
    (2, 16, 8, 3, 64 * 20, 64 * 16 * 9),
    (2, 3, 16, 1, 64 * 64, 64 * 3 * 40),
]


@pytest.mark.parametrize("policy", [0, 1, 2, 3])
@pytest.mark.parametrize("kind,D,W,grid,n_vec,L", LDS_CASES)
def test_lds_paths_match_oracle(kind, D, W, grid, n_vec, L, policy):
    nbytes = n_vec * 16
    buf = synth.random_bytes(nbytes, seed=D * 100 + W, device="cuda")
    n_waves = grid * W
    lo = lanes(n_waves * 64)
    ro = recs(n_waves)
    opts = isw.make_opts(grid_wgs=grid, cache_policy=policy, lane_out=lo,
                         wave_out=ro)
    fn = isw.sweep_lds_async if kind == 1 else isw.sweep_lds_matched_plain
    r = fn(buf, nbytes, D, 16, W, L, opts)
    p = oplan.wave_group(L, D, n_waves)
    assert r["issued_loads"] == p["issued"]
    words = host_words(buf)
    ws, wx = checksums.per_lane(words, 16, D, p["Q"], n_waves)
    gs, gx = decode_lanes(lo, n_waves)
    assert np.array_equal(gs, ws) and np.array_equal(gx, wx)
    assert (r["sum32"], r["xor32"]) == checksums.combine(ws, wx)


def _random_lds_cases(n=32, seed=20261204):
    """Seeded random LDS-path cells: path, depth, waves per workgroup (ring
    within 64 KiB), grid, allocation, ragged target and cache policy."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        W = int(rng.choice([1, 2, 4, 8, 16]))
        D = int(rng.integers(1, 17))
        if W * D > 64:
            continue
        grid = int(rng.integers(1, 7))
        n_vec = 64 * int(rng.integers(1, 151))
        Q = int(rng.integers(1, 201))
        L = 64 * D * Q + int(rng.integers(0, 64 * D))
        out.append((int(rng.integers(1, 3)), D, W, grid, n_vec, L, int(rng.integers(0, 4))))
    return out


@pytest.mark.parametrize("kind,D,W,grid,n_vec,L,policy", _random_lds_cases())
def test_lds_paths_random_cells_match_oracle(kind, D, W, grid, n_vec, L, policy):
    """Per lane, per wave and global sinks of both LDS paths against the
    oracle on seeded random cells (most of them wrap the allocation)."""
    nbytes = n_vec * 16
    buf = synth.random_bytes(nbytes, seed=n_vec + 3 * D + W, device="cuda")
    n_waves = grid * W
    lo = lanes(n_waves * 64)
    ro = recs(n_waves)
    opts = isw.make_opts(grid_wgs=grid, cache_policy=policy, lane_out=lo, wave_out=ro)
    fn = isw.sweep_lds_async if kind == 1 else isw.sweep_lds_matched_plain
    r = fn(buf, nbytes, D, 16, W, L, opts)
    p = oplan.wave_group(L, D, n_waves)
    assert r["issued_loads"] == p["issued"]
    assert (r["iters_min"], r["iters_max"]) == (p["iters_min"], p["iters_max"])
    words = host_words(buf)
    ws, wx = checksums.per_lane(words, 16, D, p["Q"], n_waves)
    gs, gx = decode_lanes(lo, n_waves)
    assert np.array_equal(gs, ws) and np.array_equal(gx, wx)
    rr = decode_recs(ro)
    os_, ox = checksums.per_wave(words, 16, D, p["Q"], n_waves)
    assert np.array_equal(rr["sum32"], os_) and np.array_equal(rr["xor32"], ox)
    assert (r["sum32"], r["xor32"]) == checksums.combine(ws, wx)


@pytest.mark.parametrize("kind_b", ["lds_async", "plain"])
@pytest.mark.parametrize("D,wa,wb", [(4, 4, 4), (8, 4, 4), (3, 1, 3),
                                     (5, 2, 0), (2, 0, 2), (16, 8, 8)])
def test_two_stream_matches_oracle(D, wa, wb, kind_b):
    grid = 3
    n_vec = 64 * 128
    nbytes = n_vec * 16
    buf = synth.random_bytes(nbytes, seed=D + 10 * wa + 100 * wb, device="cuda")
    L = 2 * 64 * D * 37 + 64
    na, nb = grid * wa, grid * wb
    ro = recs(na + nb)
    lo = lanes((na + nb) * 64)
    opts = isw.make_opts(grid_wgs=grid, wave_out=ro, lane_out=lo)
    kb = isw.KIND_LDS_ASYNC if kind_b == "lds_async" else isw.KIND_PLAIN
    ra, rb = isw.sweep_two_stream_kind(buf, nbytes, D, wa, wb, kb, L, opts)
    words = host_words(buf)
    (a0, an), (b0, bn) = checksums.two_stream_regions(n_vec)
    rr = decode_recs(ro)
    gs, gx = decode_lanes(lo, na + nb)
    La, Lb = L // 2, L - L // 2
    for (base, nv, Ls, nw, off, res) in ((a0, an, La, na, 0, ra),
                                         (b0, bn, Lb, nb, na, rb)):
        if nw == 0:
            assert res["issued_loads"] == 0
            continue
        p = oplan.wave_group(Ls, D, nw)
        assert res["issued_loads"] == p["issued"]
        ws, wx = checksums.per_lane(words, 16, D, p["Q"], nw, base=base, n_vec=nv)
        assert np.array_equal(gs[off:off + nw], ws)
        assert np.array_equal(gx[off:off + nw], wx)
        assert (res["sum32"], res["xor32"]) == checksums.combine(ws, wx)


@pytest.mark.parametrize("kind_b", ["lds_async", "plain"])
@pytest.mark.parametrize("D,wa,wb", [(4, 8, 8), (3, 2, 5), (5, 4, 0), (2, 0, 3), (16, 16, 1)])
def test_two_stream_split_matches_oracle(D, wa, wb, kind_b):
    """Split placement: stream A on half of the workgroups, stream B on the
    other half; per-lane sinks of both streams against the oracle with each
    stream's own wave count, and the global sinks equal to the same-workgroup
    run's (the sinks do not depend on which waves read the groups)."""
    grid = 32
    n_vec = 64 * 128
    nbytes = n_vec * 16
    buf = synth.random_bytes(nbytes, seed=7 + D + 10 * wa + 100 * wb, device="cuda")
    L = 2 * 64 * D * 300 + 64                  # 300 groups per stream: wraps its half
    na, nb = grid // 2 * wa, grid // 2 * wb
    ro = recs(na + nb)
    lo = lanes((na + nb) * 64)
    opts = isw.make_opts(grid_wgs=grid, wave_out=ro, lane_out=lo)
    kb = isw.KIND_LDS_ASYNC if kind_b == "lds_async" else isw.KIND_PLAIN
    ra, rb = isw.sweep_two_stream_split(buf, nbytes, D, wa, wb, kb, L, opts)
    words = host_words(buf)
    (a0, an), (b0, bn) = checksums.two_stream_regions(n_vec)
    gs, gx = decode_lanes(lo, na + nb)
    La, Lb = L // 2, L - L // 2
    for (base, nv, Ls, nw, off, res) in ((a0, an, La, na, 0, ra),
                                         (b0, bn, Lb, nb, na, rb)):
        if nw == 0:
            assert res["issued_loads"] == 0
            continue
        p = oplan.wave_group(Ls, D, nw)
        assert res["issued_loads"] == p["issued"] and res["waves"] == nw
        ws, wx = checksums.per_lane(words, 16, D, p["Q"], nw, base=base, n_vec=nv)
        assert np.array_equal(gs[off:off + nw], ws)
        assert np.array_equal(gx[off:off + nw], wx)
        assert (res["sum32"], res["xor32"]) == checksums.combine(ws, wx)
    sa, sb = isw.sweep_two_stream_kind(buf, nbytes, D, min(wa, 8), min(wb, 8), kb, L,
                                       isw.make_opts(grid_wgs=grid))
    for same, split_ in ((sa, ra), (sb, rb)):
        if split_["issued_loads"]:
            assert (same["sum32"], same["xor32"]) == (split_["sum32"], split_["xor32"])


def _random_two_stream_cases(n=24, seed=20261205):
    """Seeded random two-stream cells: mechanism of stream B, placement,
    depth, waves of each stream (either may be 0), grid, buffer size and
    target, and cache policy, drawn together."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        kind = ["lds_async", "plain"][int(rng.integers(2))]
        split = bool(rng.integers(2))
        D = int(rng.integers(1, 17))
        wmax = 16 if split else 8
        wa, wb = int(rng.integers(0, wmax + 1)), int(rng.integers(0, wmax + 1))
        if wa + wb == 0 or (kind == "lds_async" and wb * D > 160):
            continue
        grid = int(rng.choice([16, 32])) if split else int(rng.integers(1, 7))
        n_vec = 128 * int(rng.integers(1, 97))
        L = 2 * 64 * D * int(rng.integers(1, 400)) + int(rng.integers(0, 2 * 64 * D))
        out.append((kind, split, D, wa, wb, grid, n_vec, L, int(rng.integers(4))))
    return out


@pytest.mark.parametrize("kind_b,split,D,wa,wb,grid,n_vec,L,policy", _random_two_stream_cases())
def test_two_stream_random_cells_match_oracle(kind_b, split, D, wa, wb, grid, n_vec, L, policy):
    """Per-lane sinks of both streams against the oracle on random cells,
    in one workgroup or split across CUs."""
    print(f"two-stream case: {kind_b} split={split} D={D} wa={wa} wb={wb} grid={grid} "
          f"n_vec={n_vec} L={L} policy={policy}", flush=True)
    nbytes = n_vec * 16
    buf = synth.random_bytes(nbytes, seed=n_vec + D + 10 * wa + 100 * wb, device="cuda")
    per = grid // 2 if split else grid
    na, nb = per * wa, per * wb
    ro = recs(na + nb)
    lo = lanes((na + nb) * 64)
    opts = isw.make_opts(grid_wgs=grid, wave_out=ro, lane_out=lo, cache_policy=policy)
    kb = isw.KIND_LDS_ASYNC if kind_b == "lds_async" else isw.KIND_PLAIN
    fn = isw.sweep_two_stream_split if split else isw.sweep_two_stream_kind
    ra, rb = fn(buf, nbytes, D, wa, wb, kb, L, opts)
    words = host_words(buf)
    (a0, an), (b0, bn) = checksums.two_stream_regions(n_vec)
    gs, gx = decode_lanes(lo, na + nb)
    La, Lb = L // 2, L - L // 2
    for (base, nv, Ls, nw, off, res) in ((a0, an, La, na, 0, ra),
                                         (b0, bn, Lb, nb, na, rb)):
        if nw == 0:
            assert res["issued_loads"] == 0
            continue
        p = oplan.wave_group(Ls, D, nw)
        assert res["issued_loads"] == p["issued"] and res["waves"] == nw
        ws, wx = checksums.per_lane(words, 16, D, p["Q"], nw, base=base, n_vec=nv)
        assert np.array_equal(gs[off:off + nw], ws)
        assert np.array_equal(gx[off:off + nw], wx)
        assert (res["sum32"], res["xor32"]) == checksums.combine(ws, wx)


def test_two_stream_split_places_streams_on_different_cus():
    """At one workgroup per CU the two streams share no CU, and every XCD
    holds as many CUs of each stream (from the waves' HW_ID / XCC_ID)."""
    info = isw.sweep_device_info()
    nbytes = 64 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED + 5)
    n_wg = info["num_cus"] // 2
    for kb in (isw.KIND_PLAIN, isw.KIND_LDS_ASYNC):
        na, nb = n_wg * 8, n_wg * 4
        ro = recs(na + nb)
        isw.sweep_two_stream_split(buf, nbytes, 4, 8, 4, kb, nbytes // 16,
                                   isw.make_opts(wave_out=ro))
        rr = decode_recs(ro)
        hw = rr["hw_id"].astype(np.int64)
        xcc = rr["xcc_id"].astype(np.int64) & 0xF
        cu = xcc << 16 | ((hw >> 8) & 0xFF)
        cus_a, cus_b = set(cu[:na].tolist()), set(cu[na:].tolist())
        print(f"kind_b={kb}: {len(cus_a)} CUs run A, {len(cus_b)} run B, "
              f"{len(cus_a & cus_b)} both")
        assert not cus_a & cus_b
        assert len(cus_a) == len(cus_b) == n_wg
        per_xcd_a = np.bincount(xcc[:na], minlength=8) // 8
        per_xcd_b = np.bincount(xcc[na:], minlength=8) // 4
        assert np.array_equal(per_xcd_a, per_xcd_b)


def test_run_and_batched_equal_single_calls():
    nbytes = 4 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED + 1)
    cells = []
    for K in (1, 2, 3, 8):
        cells.append(isw.make_cell(buf, nbytes, K, 16, 8, nbytes // 16))
    cells.append(isw.make_cell(buf, nbytes, 4, 16, 4, nbytes // 16,
                               kind=isw.KIND_LDS_ASYNC))
    cells.append(isw.make_cell(buf, nbytes, 4, 16, 4, nbytes // 16,
                               kind=isw.KIND_LDS_MATCHED))
    run = isw.sweep_run(cells)
    bat, ms = isw.sweep_batched(cells)
    assert ms > 0
    words = splitmix.buffer_words(SEED + 1, nbytes)
    for c, a, b in zip(cells, run, bat):
        n_waves = a["waves"]
        p = oplan.wave_group(c.total_logical_loads, c.K, n_waves)
        want = checksums.combine(*checksums.per_wave(words, 16, c.K, p["Q"], n_waves))
        assert (a["sum32"], a["xor32"]) == want == (b["sum32"], b["xor32"])
        assert a["issued_bytes"] == b["issued_bytes"]
        assert a["gbps"] > 0 and b["gbps"] > 0


def _gpu_sum(kind, payload, n, w=8):
    dt = {"f32": isw.F32, "bf16": isw.BF16, "fp8_e4m3": isw.FP8_E4M3}[kind]
    return isw.sweep_reduce_fp(payload, n, dt, w)


def _oracle_sum(kind, payload_u8):
    a = payload_u8.cpu().numpy()
    if kind == "f32":
        return fpsum.exact_sum(fpsum.decode_f32(a.view(np.uint32)))
    if kind == "bf16":
        return fpsum.exact_sum(fpsum.decode_bf16(a.view(np.uint16)))
    return fpsum.exact_sum_e4m3(a)


def _bound(kind, payload_u8, n, res, w):
    a = payload_u8.cpu().numpy()
    x = {"f32": lambda: fpsum.decode_f32(a.view(np.uint32)),
         "bf16": lambda: fpsum.decode_bf16(a.view(np.uint16)),
         "fp8_e4m3": lambda: fpsum.decode_e4m3(a)}[kind]()
    terms = reduce_lane_terms(kind, n, res["waves"], w)
    return fpsum.sum2_bound(float(np.abs(x).sum()), terms, 8, res["grid_wgs"])


def fpsum_bytes(kind):
    return {"f32": 4, "bf16": 2, "fp8_e4m3": 1}[kind]


@pytest.mark.parametrize("w", [4, 8])
@pytest.mark.parametrize("kind", ["f32", "bf16", "fp8_e4m3"])
@pytest.mark.parametrize("n", [0, 1, 7, 1000, 4096 * 3 + 5, 8192 * 5 + 9, (1 << 20) + 3])
def test_reduce_matches_exact_sum(kind, n, w):
    payload = synth.normal_payload(kind, n, seed=n + 17, device="cuda")
    pad = torch.zeros(max(16, payload.numel() + 16), dtype=torch.uint8, device="cuda")
    pad[:payload.numel()] = payload
    got, res = _gpu_sum(kind, pad, n, w)
    want = _oracle_sum(kind, payload)
    err = abs(got - want)
    assert err <= _bound(kind, payload, n, res, w), (got, want)


def _negated(u8, kind):
    """Flip the sign bit of every element of a raw payload."""
    eb = fpsum_bytes(kind)
    b = u8.clone().view(-1, eb)
    b[:, eb - 1] ^= 0x80            # little endian: sign is in the last byte
    return b.view(-1)


@pytest.mark.parametrize("kind", ["f32", "bf16", "fp8_e4m3"])
def test_reduce_special_cases(kind):
    n = 64 * 1024 + 5
    dt = synth.DTYPES[kind]
    # constant payload: exact n * x
    x = torch.full((n,), 1.5, dtype=torch.float32, device="cuda").to(dt)
    for w in (4, 8):
        got, _ = _gpu_sum(kind, x.view(torch.uint8), n, w)
        assert got == n * 1.5
    # +v / -v pairs cancel exactly
    v = synth.normal_payload(kind, n, seed=3, device="cuda")
    both = torch.cat([v, _negated(v, kind)])
    for w in (4, 8):
        got, _ = _gpu_sum(kind, both, 2 * n, w)
        assert got == 0.0


def test_reduce_recovers_absorbed_terms():
    # every lane meets a large value first: plain FP32 summation would drop
    # the ones that follow; the compensated sum keeps them exactly
    n = 1 << 20
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    x[: n // 2: 4096] = 2.0**30
    x[n // 2:: 4096] = -(2.0**30)
    got, _ = _gpu_sum("f32", x.view(torch.uint8), n)
    want = _oracle_sum("f32", x.view(torch.uint8))
    assert got == want


def test_fp8_decode_every_finite_code():
    for code in list(range(0, 0x7F)) + list(range(0x80, 0xFF)):
        p = torch.full((16,), code, dtype=torch.uint8, device="cuda")
        got, _ = _gpu_sum("fp8_e4m3", p, 16, w=4)
        k, _nan = fpsum.e4m3_scaled_int(code)
        assert got == 16 * k * 2.0**-9, hex(code)


def test_host_validation_errors():
    buf = dev_bytes(1 << 20)
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plain(buf.data_ptr() + 4, (1 << 20) - 1024, 2, 16, 8, 1000)
    assert e.value.code == isw.EALIGN
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plain(buf, 1 << 20, 0, 16, 8, 1000)
    assert e.value.code == isw.EINVAL
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_lds_async(buf, 1 << 20, 4, 8, 4, 1000)
    assert e.value.code == isw.EINVAL
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_two_stream(buf, 1 << 20, 4, 0, 0, 1000)
    assert e.value.code == isw.EINVAL
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_two_stream_kind(buf, 1 << 20, 4, 2, 2, isw.KIND_LDS_MATCHED, 1 << 16)
    assert e.value.code == isw.EINVAL
    for wa, wb, grid in ((4, 4, 24), (17, 4, 16), (0, 0, 16)):
        with pytest.raises(isw.SweepError) as e:
            isw.sweep_two_stream_split(buf, 1 << 20, 4, wa, wb, isw.KIND_PLAIN, 1 << 16,
                                       isw.make_opts(grid_wgs=grid))
        assert e.value.code == isw.EINVAL
    # one wave per stream and 2^33 wave-groups each: iteration counts
    # beyond 32 bits; and a target whose issued bytes pass 64 bits
    for L in (1 << 40, 1 << 61):
        with pytest.raises(isw.SweepError) as e:
            isw.sweep_two_stream_kind(buf, 1 << 20, 1, 1, 1, isw.KIND_PLAIN, L,
                                      isw.make_opts(grid_wgs=1))
        assert e.value.code == isw.EINVAL
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plain(buf, 1 << 20, 1, 4, 4, 1 << 40, isw.make_opts(grid_wgs=1))
    assert e.value.code == isw.EINVAL
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_reduce_fp(buf, 10, 9)
    assert e.value.code == isw.EINVAL
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_fill_u32(buf.data_ptr() + 4, 64, 1)
    assert e.value.code == isw.EALIGN


def test_output_buffers_too_small_are_rejected():
    """A wave_out / lane_out smaller than the launch is refused before any
    kernel runs, and the buffers stay untouched."""
    nbytes = 1 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED)
    grid = 16                                   # 64 waves
    ro = recs(63)
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plain(buf, nbytes, 2, 16, 4, nbytes // 16,
                        isw.make_opts(grid_wgs=grid, wave_out=ro))
    assert e.value.code == isw.EINVAL
    lo = lanes(64 * 64 - 1)
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plain(buf, nbytes, 2, 16, 4, nbytes // 16,
                        isw.make_opts(grid_wgs=grid, lane_out=lo))
    assert e.value.code == isw.EINVAL
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_two_stream_kind(buf, nbytes, 4, 4, 4, isw.KIND_PLAIN, nbytes // 16,
                                  isw.make_opts(grid_wgs=grid, wave_out=recs(127)))
    assert e.value.code == isw.EINVAL
    torch.cuda.synchronize()
    assert not ro.any() and not lo.any()
    # a raw pointer needs its capacity stated
    with pytest.raises(ValueError):
        isw.make_opts(wave_out=ro.data_ptr())
    # exactly the launch's size is accepted
    r = isw.sweep_plain(buf, nbytes, 2, 16, 4, nbytes // 16,
                        isw.make_opts(grid_wgs=grid, wave_out=recs(64), lane_out=lanes(64 * 64)))
    assert r["waves"] == 64


@pytest.mark.parametrize("V,K,w,grid,n_vec,L", PLAIN_CASES[:6])
def test_plain_blocked_order_matches_oracle(V, K, w, grid, n_vec, L):
    nbytes = n_vec * V
    buf = synth.random_bytes(nbytes, seed=V * 7 + K, device="cuda")
    n_waves = grid * 4
    lo = lanes(n_waves * 64)
    opts = isw.make_opts(grid_wgs=grid, cache_policy=isw.CACHE_BYPASS_L1_NT,
                         lane_out=lo, order=isw.ORDER_BLOCKED)
    r = isw.sweep_plain(buf, nbytes, K, V, w, L, opts)
    p = oplan.wave_group(L, K, n_waves, order=oplan.BLOCKED)
    assert r["issued_loads"] == p["issued"]
    assert (r["iters_min"], r["iters_max"]) == (p["iters_min"], p["iters_max"])
    ws, wx = checksums.per_lane(host_words(buf), V, K, p["Q"], n_waves,
                                order=oplan.BLOCKED)
    gs, gx = decode_lanes(lo, n_waves)
    assert np.array_equal(gs, ws) and np.array_equal(gx, wx)


@pytest.mark.parametrize("V,K,w,grid,n_vec,L", PLAIN_CASES)
def test_plain_strided_layout_matches_oracle(V, K, w, grid, n_vec, L):
    """Strided layout: load j of group q reads segment j*Q + q."""
    nbytes = n_vec * V
    buf = synth.random_bytes(nbytes, seed=V * 11 + K, device="cuda")
    n_waves = grid * 4
    lo = lanes(n_waves * 64)
    ro = recs(n_waves)
    opts = isw.make_opts(grid_wgs=grid, cache_policy=isw.CACHE_BYPASS_L1_NT,
                         lane_out=lo, wave_out=ro, order=isw.ORDER_STRIDED)
    r = isw.sweep_plain(buf, nbytes, K, V, w, L, opts)
    p = oplan.wave_group(L, K, n_waves, order=oplan.STRIDED)
    assert r["issued_loads"] == p["issued"]
    ws, wx = checksums.per_lane(host_words(buf), V, K, p["Q"], n_waves,
                                order=oplan.STRIDED)
    gs, gx = decode_lanes(lo, n_waves)
    assert np.array_equal(gs, ws) and np.array_equal(gx, wx)
    # the global sinks are the adjacent layout's
    rr = isw.sweep_plain(buf, nbytes, K, V, w, L, isw.make_opts(grid_wgs=grid))
    assert (r["sum32"], r["xor32"]) == (rr["sum32"], rr["xor32"])


def test_lds_paths_reject_blocked_order():
    buf = dev_bytes(1 << 20)
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_lds_async(buf, 1 << 20, 4, 16, 4, 1000,
                            isw.make_opts(order=isw.ORDER_BLOCKED))
    assert e.value.code == isw.EINVAL


@pytest.mark.parametrize("policy", [0, 1, 2, 3])
@pytest.mark.parametrize("footprint,stride,warm,hops", [(8192, 128, 64, 200),
                                                       (1 << 20, 128, 100, 3000),
                                                       (4096, 4, 0, 5000)])
def test_chase_matches_oracle(footprint, stride, warm, hops, policy):
    from oracle import chase
    chain, start = synth.chase_chain(footprint, stride, seed=footprint + stride,
                                     device="cuda")
    samples = torch.zeros(min(hops, 4096), dtype=torch.int32, device="cuda")
    r = isw.sweep_chase(chain, footprint, start, warm, hops, policy, samples,
                        samples.numel())
    words = host_words(chain)
    assert r["final_index"] == chase.follow(words, start, warm + hops)
    assert r["ns_per_hop"] > 0 and r["shader_clock_hz"] > 1e8
    assert (samples.cpu().numpy() > 0).all()


def test_chase_rejects_bad_arguments():
    chain, start = synth.chase_chain(4096, 64, seed=1, device="cuda")
    for args in [(chain, 4096, 4096 // 4, 0, 10),      # start outside
                 (chain, 4096, start, 0, 0)]:           # no hops
        with pytest.raises(isw.SweepError) as e:
            isw.sweep_chase(*args)
        assert e.value.code == isw.EINVAL


def _xcd_of_active_wave(aw, mask):
    """The XCD of active wave ``aw``: active workgroups are numbered by
    (round of eight workgroups, rank of their XCD in the mask)."""
    bits = [x for x in range(8) if mask >> x & 1]
    return bits[(aw // 4) % len(bits)]


@pytest.mark.parametrize("policy", [1, 3])
@pytest.mark.parametrize("w", [4, 8])
@pytest.mark.parametrize("mask", [0x01, 0x80, 0x0F, 0x55, 0x77, 0xFF])
def test_xcd_subset_matches_oracle(mask, w, policy):
    """The active waves read the buffer's first issued vectors once: the
    global sinks equal the oracle's checksum of that prefix; every active
    wave ran on the XCD its workgroup index names."""
    nbytes = 64 << 20
    buf = synth.random_bytes(nbytes, seed=mask * 31 + w, device="cuda")
    n_cus = isw.sweep_device_info()["num_cus"]
    n_act = (n_cus * w // 32) * bin(mask).count("1") * 4      # workgroups per XCD x 4 waves
    ro = recs(n_act)
    print(f"xcd subset mask {mask:#04x}, {w} waves/CU, policy {policy}", flush=True)
    r = isw.sweep_xcd_subset(buf, nbytes, w, mask,
                             isw.make_opts(cache_policy=policy, wave_out=ro))
    groups = (nbytes // 16) // (n_act * 512)
    assert r["waves"] == n_act and r["issued_loads"] == n_act * groups * 512
    words = host_words(buf)
    assert (r["sum32"], r["xor32"]) == checksums.whole_buffer(words[: r["issued_loads"] * 4])
    rr = decode_recs(ro)
    got = rr["xcc_id"].astype(np.int64) & 0xF
    want = np.array([_xcd_of_active_wave(aw, mask) for aw in range(n_act)])
    assert np.array_equal(got, want), (got[:32].tolist(), want[:32].tolist())
    assert r["gbps"] > 0


@pytest.mark.parametrize("w", [4, 8])
@pytest.mark.parametrize("weights", [[1, 1, 1, 1, 1, 1, 1, 1],
                                     [1, 2, 0, 1, 3, 0.5, 1, 1],
                                     [0, 0, 0, 1, 0, 0, 0, 0],
                                     [13.5, 11.5, 13.5, 11.5, 13.5, 11.5, 13.5, 11.5]])
def test_xcd_split_matches_oracle(weights, w):
    """The weighted split reads each XCD's contiguous share once: the global
    sinks equal the oracle's checksum of the shares' prefix, and record i
    comes from the XCD of rank i / (waves per XCD) among those with a share."""
    nbytes = 64 << 20
    buf = synth.random_bytes(nbytes, seed=int(sum(weights) * 10) + w, device="cuda")
    n_cus = isw.sweep_device_info()["num_cus"]
    per_xcd = n_cus * w // 8          # workgroups per XCD x 4 waves
    total = (nbytes // 16) // 512
    tw = float(sum(weights))
    shares = [int(total * (v / tw)) for v in weights]
    bits = [x for x in range(8) if shares[x]]
    ro = recs(len(bits) * per_xcd)
    print(f"xcd split {weights} at {w} waves/CU", flush=True)
    r = isw.sweep_xcd_split(buf, nbytes, w, weights,
                            isw.make_opts(cache_policy=isw.CACHE_BYPASS_L1_NT, wave_out=ro))
    assert r["waves"] == len(bits) * per_xcd
    assert r["issued_loads"] == sum(shares) * 512
    words = host_words(buf)
    assert (r["sum32"], r["xor32"]) == checksums.whole_buffer(words[: r["issued_loads"] * 4])
    got = decode_recs(ro)["xcc_id"].astype(np.int64) & 0xF
    want = np.repeat(bits, per_xcd)
    assert np.array_equal(got, want), (got[::per_xcd].tolist(), bits)
    per_wave = [shares[x] / per_xcd for x in bits]
    assert r["iters_min"] == int(min(per_wave)) and r["iters_max"] == -int(-max(per_wave) // 1)


def _random_xcd_cases(n=12, seed=20261206):
    rng = np.random.default_rng(seed)
    masks = [int(m) for m in rng.integers(1, 256, size=n)]
    weights = []
    while len(weights) < n:
        wt = [0.0 if rng.random() < 0.25 else round(float(rng.uniform(0.05, 2.0)), 3)
              for _ in range(8)]
        if sum(wt) > 0:
            weights.append(wt)
    ws = [int(rng.choice([4, 8, 16])) for _ in range(n)]
    return list(zip(masks, weights, ws))


@pytest.mark.parametrize("mask,weights,w", _random_xcd_cases())
def test_xcd_reads_random_masks_and_weights(mask, weights, w):
    """Random XCD subsets and random per-XCD weights: each read covers its
    prefix once (global sinks against the oracle) and every wave ran on
    the XCD its number names."""
    nbytes = 64 << 20
    buf = synth.random_bytes(nbytes, seed=mask + 7 * w, device="cuda")
    words = host_words(buf)
    n_cus = isw.sweep_device_info()["num_cus"]
    print(f"xcd random: mask {mask:#04x}, weights {weights}, {w} waves/CU", flush=True)
    n_act = (n_cus * w // 32) * bin(mask).count("1") * 4
    ro = recs(max(n_act, n_cus * w // 8 * 8))
    r = isw.sweep_xcd_subset(buf, nbytes, w, mask, isw.make_opts(wave_out=ro))
    groups = (nbytes // 16) // (n_act * 512)
    assert r["waves"] == n_act and r["issued_loads"] == n_act * groups * 512
    assert (r["sum32"], r["xor32"]) == checksums.whole_buffer(words[: r["issued_loads"] * 4])
    got = decode_recs(ro)["xcc_id"][:n_act].astype(np.int64) & 0xF
    assert np.array_equal(got, [_xcd_of_active_wave(aw, mask) for aw in range(n_act)])
    per_xcd = n_cus * w // 8
    total = (nbytes // 16) // 512
    tw = float(sum(weights))
    shares = [int(total * (v / tw)) for v in weights]
    bits = [x for x in range(8) if shares[x]]
    r = isw.sweep_xcd_split(buf, nbytes, w, weights, isw.make_opts(wave_out=ro))
    assert r["waves"] == len(bits) * per_xcd and r["issued_loads"] == sum(shares) * 512
    assert (r["sum32"], r["xor32"]) == checksums.whole_buffer(words[: r["issued_loads"] * 4])
    got = decode_recs(ro)["xcc_id"][: r["waves"]].astype(np.int64) & 0xF
    assert np.array_equal(got, np.repeat(bits, per_xcd))


def test_xcd_split_rejects_bad_arguments():
    buf = dev_bytes(1 << 20)
    for wts in ([0] * 8, [1, -1, 1, 1, 1, 1, 1, 1], [float("nan")] + [1] * 7,
                [float("inf")] + [1] * 7):
        with pytest.raises(isw.SweepError) as e:
            isw.sweep_xcd_split(buf, 1 << 20, 4, wts)
        assert e.value.code == isw.EINVAL, wts
    with pytest.raises(ValueError):
        isw.sweep_xcd_split(buf, 1 << 20, 4, [1] * 7)


def test_xcd_subset_rejects_bad_arguments():
    buf = dev_bytes(1 << 20)
    for args, code in [((buf, 1 << 20, 4, 0), isw.EINVAL),        # empty mask
                       ((buf, 1 << 20, 4, 256), isw.EINVAL),      # beyond 8 XCDs
                       ((buf, 1 << 20, 6, 1), isw.EINVAL),        # waves not a multiple of 4
                       ((buf, 1000, 4, 1), isw.EALIGN),           # not whole segments
                       ((buf, 1 << 20, 32, 0xFF), isw.EINVAL)]:   # under one group per wave
        with pytest.raises(isw.SweepError) as e:
            isw.sweep_xcd_subset(*args)
        assert e.value.code == code, args


@pytest.mark.parametrize("policy", [0, 2, 3])
@pytest.mark.parametrize("n_walkers,footprint,warm,hops", [(1, 8192, 10, 300),
                                                          (8, 1 << 20, 100, 500),
                                                          (64, 1 << 20, 0, 700),
                                                          (37, 1 << 16, 512, 1000)])
def test_walkers_match_oracle(n_walkers, footprint, warm, hops, policy):
    """Every walker lands where the oracle's walk from its start lands, and
    reports a valid XCD; walkers wrap the cycle when warm + hops exceeds it."""
    from oracle import chase
    chain, starts = synth.chase_chain_starts(footprint, 128, footprint + n_walkers,
                                             n_walkers, device="cuda")
    print(f"walkers {n_walkers} over {footprint} B, warm {warm}, hops {hops}", flush=True)
    out = isw.sweep_chase_walkers(chain, footprint, starts, warm, hops, policy)
    words = host_words(chain)
    assert len(out) == n_walkers
    n_xcc = isw.sweep_device_info()["num_cus"] // 32
    for s0, r in zip(starts, out):
        assert r["final_index"] == chase.follow(words, s0, warm + hops)
        assert r["hops"] == hops and r["ns_per_hop"] > 0
        assert r["xcc_id"] < max(n_xcc, 1)
    if n_walkers >= 8:
        # workgroups are dealt to the XCDs in turn
        assert len({r["xcc_id"] for r in out}) == min(n_walkers, max(n_xcc, 1))


def test_walkers_reject_bad_arguments():
    chain, starts = synth.chase_chain_starts(4096, 64, 1, 4, device="cuda")
    for st, hops in [([], 10), (list(range(65)), 10), ([4096 // 4], 10), (starts, 0)]:
        with pytest.raises(isw.SweepError) as e:
            isw.sweep_chase_walkers(chain, 4096, st, 0, hops)
        assert e.value.code == isw.EINVAL


@pytest.mark.parametrize("V,K,n_vec,L", [(16, 4, 64, 64 * 4 * 3),      # one segment
                                         (4, 1, 256, 64 * 5),           # Q < waves
                                         (16, 16, 64, 64 * 16),         # one group
                                         (8, 3, 128, 64 * 3 * 1000)])   # deep wrap
def test_plain_degenerate_shapes(V, K, n_vec, L):
    nbytes = n_vec * V
    buf = synth.random_bytes(nbytes, seed=n_vec + K, device="cuda")
    info = isw.sweep_device_info()
    n_waves = info["num_cus"] * 8            # default grid at 8 waves/CU
    ro = recs(n_waves)
    r = isw.sweep_plain(buf, nbytes, K, V, 8, L, isw.make_opts(wave_out=ro))
    p = oplan.wave_group(L, K, n_waves)
    assert r["waves"] == n_waves and r["issued_loads"] == p["issued"]
    s, x = checksums.per_wave(host_words(buf), V, K, p["Q"], n_waves)
    rr = decode_recs(ro)
    assert np.array_equal(rr["sum32"], s) and np.array_equal(rr["xor32"], x)
    idle = np.array(p["iters"]) == 0
    assert (rr["sum32"][idle] == 0).all() and (rr["xor32"][idle] == 0).all()


def test_window_agrees_with_events():
    nbytes = 1 << 30
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, 5)
    isw.sweep_calibrate_clock(0.05)
    for w in (4, 32):
        r = isw.sweep_run([isw.make_cell(buf, nbytes, 4, 16, w, nbytes // 16)] * 3)[-1]
        ev_ns = r["event_ms"] * 1e6
        assert 0.85 < r["window_ns"] / ev_ns <= 1.02, (r["window_ns"], ev_ns)
        assert abs(r["gbps"] - r["issued_bytes"] / r["window_ns"]) < 1e-6
        # the same through a graph: the kernels' windows fill the replay
        g = isw.sweep_graph_create([isw.make_cell(buf, nbytes, 4, 16, w, nbytes // 16)] * 3)
        try:
            for _ in range(2):
                res, ms = isw.sweep_graph_launch(g)
            frac = sum(r["window_ns"] for r in res) / (ms * 1e6)
            assert 0.85 < frac <= 1.02, frac
        finally:
            isw.sweep_graph_destroy(g)


def test_sweep_drivers_run_small():
    from paper_2608_15764_amd import sweeps
    nbytes = 8 << 20
    buf = sweeps.device_buffer(nbytes, 11)
    out = sweeps.plain_k_sweep(buf, nbytes, nbytes // 16, isw.CACHE_BYPASS_L1_NT,
                               [4, 32], range(1, 5), passes=2)
    assert out["checksums_consistent"] and set(out["curves"]) == {4, 32}
    pc = sweeps.path_comparison(buf, nbytes, nbytes // 16, depths=(1, 4), waves_list=(1, 4), n=1)
    assert pc["checksums_equal_across_paths"] and pc[4][4]["ratio"] > 0
    # depths 1 and 4 both divide nbytes // 16 / 64: identical issued work
    assert pc["depth_set_mismatch"] == 0.0
    ts = sweeps.two_stream(buf, nbytes, nbytes // 16, depths=(4,), pairs=((4, 4), (1, 2)), n=1)
    assert set(ts) == {"D4_A4_B4", "D4_A1_B2"}
    tp = sweeps.two_stream(buf, nbytes, nbytes // 16, depths=(4,), pairs=((2, 2),), n=1,
                           kind_b=isw.KIND_PLAIN)
    assert tp["D4_A2_B2"]["co_b_gbps"] > 0
    tsp = sweeps.two_stream(buf, nbytes, nbytes // 16, depths=(4,), pairs=((4, 2),), n=1,
                            kind_b=isw.KIND_PLAIN, split=True)
    assert tsp["D4_A4_B2"]["co_a_gbps"] > 0 and tsp["D4_A4_B2"]["solo_b_gbps"] > 0
    al = sweeps.allocation_sweep([1 << 20, 4 << 20], Ks=(1, 2), waves_list=(8,), L=1 << 20, n=1)
    assert all(v["checksums_consistent"] for v in al.values())
    of = sweeps.order_footprint([1 << 20, 2 << 20], Ks=(1, 2), L=1 << 18, n=1)
    assert set(of[1 << 20]) == {"round_robin", "blocked", "strided"}
    man = sweeps.lds_counter_pass(nbytes=4 << 20, waves_list=(1,), depths=(2, 5), L=1 << 18,
                                  reps=2)
    assert len(man) == 8 and {m["path"] for m in man} == {"lds_async", "lds_matched"}
    assert all(m["issued_bytes"] > 0 and m["gbps"] > 0 for m in man)
    assert all("policy" not in m for m in man)
    man = sweeps.lds_counter_pass(nbytes=4 << 20, waves_list=(1,), depths=(2,), L=1 << 18,
                                  reps=2, policies=(isw.CACHE_DEFAULT, isw.CACHE_BYPASS_L1_NT))
    assert len(man) == 8 and {m["policy"] for m in man} == {"default", "bypass_l1_nt"}
    lad = sweeps.latency_ladder(footprints=[8 << 10, 1 << 20], hops=256, n_samples=128,
                                evict_bytes=16 << 20)
    assert lad[8 << 10]["default"]["mean_ns"] > 0
    ps = sweeps.precision_sum(payload_bytes=1 << 20, n=2)
    assert all(v["deterministic"] for v in ps.values())
    fixed = {"f32": 4, "bf16": 8, "fp8_e4m3": 4}
    ps2 = sweeps.precision_sum(payload_bytes=1 << 20, n=2, waves_fixed=fixed)
    for kind, w in fixed.items():
        assert ps2[kind]["waves_per_cu"] == w and ps2[kind]["tuning_gbps"] == {}
        assert ps2[kind]["sum"] == ps[kind]["sum"] or ps[kind]["waves_per_cu"] != w
    cs = sweeps.completion_spread(buf, nbytes, nbytes // 16, isw.CACHE_NT, [4, 16], K=2, reps=1)
    for v in cs.values():
        assert 0 <= v["end_p10"] <= v["end_p50"] <= v["end_p90"] <= 1
        assert v["xcd_last_end_max"] == pytest.approx(1.0) and v["last_start"] < 1
        assert len(v["xcd_mean_duration_ratio"]) == 8
    fi = sweeps.fixed_iteration_arm(buf, nbytes, Ks=(1, 2), waves_per_cu=8, n=1)
    assert fi["issued_bytes"][2] == 2 * fi["issued_bytes"][1]
    sg = sweeps.streaming_gate(buf, nbytes, launches=3)
    assert sg["best_gbps"] >= sg["median_gbps"] > 0


def test_new_bench_rows_run_small(tmp_path):
    """The rows added to the benchmark, on small inputs: the gate's verdict,
    the gap split, the regime map on several backends, coverage in the
    order/footprint and allocation rows, and the oracle-checked batch."""
    from oracle import checksums
    from paper_2608_15764_amd import stats, sweeps
    nbytes = 8 << 20
    buf = sweeps.device_buffer(nbytes, 13)
    sg = sweeps.streaming_gate(buf, nbytes, launches=3, latency_ns=360.0)
    assert sg["verdict"] in ("pass", "latency-bound", "fail")
    assert sg["littles_law_ceiling_gbps"] == pytest.approx(
        stats.littles_ceiling_gbps(sg["in_flight_bytes"], 360.0), abs=0.05)
    Ks, waves = [1, 2, 4], [4, 16]
    summ = sweeps.plain_k_sweep(buf, nbytes, nbytes // 16, isw.CACHE_BYPASS_L1_NT, waves, Ks,
                                passes=2)
    gap = sweeps.gap_breakdown(buf, nbytes, nbytes // 16, isw.CACHE_BYPASS_L1_NT, summ, 360.0,
                               waves, Ks)
    xw = sweeps.xcd_weighting(buf, nbytes, waves_list=(4,), rounds=1, n=1)
    assert len(xw[4]["rounds"]) == 2 and abs(sum(xw[4]["rounds"][1]["shares"]) - 1) < 1e-3
    man_path = tmp_path / "fabric_manifest.json"
    fb = sweeps.fabric_by_xcd(buf, nbytes, waves_list=(4,), n=1,
                              masks=(("one", (0x01,)), ("all", (0xFF,))), manifest=str(man_path))
    assert set(fb[4]["masks"]) == {"0x01", "0xff"}
    man = json.loads(man_path.read_text())
    assert [(m["mask"], m["warmup"]) for m in man] == [("0x01", True), ("0x01", False),
                                                       ("0xff", True), ("0xff", False)]
    assert man[3]["issued_bytes"] == fb[4]["masks"]["0xff"]["bytes"]
    assert all(m["misplaced_waves"] == 0 and m["gbps"] > 0 for m in fb[4]["masks"].values())
    prod = gap["ceiling_frac_of_peak"] * (1 - gap["tail_loss"]) * gap["residual_frac"]
    assert prod == pytest.approx(gap["kernel_frac"], rel=1e-3)
    assert set(gap["by_waves_per_cu"]) == set(waves)
    for row in gap["by_waves_per_cu"].values():
        for c in row["cells"].values():
            assert 0 < c["active_ceiling_gbps"] <= c["ceiling_gbps"] + 1e-6
    rm = sweeps.regime_map(waves_list=(4, 8), widths=(16,), Ks=range(1, 5),
                           backends=(("a", 4 << 20), ("b", 2 << 20)), work_bytes=8 << 20, n=1)
    assert set(rm["backends"]) == {"a", "b"}
    for b in rm["backends"].values():
        assert sum(b["counts"].values()) == 4 and b["launches_per_cell"] == 2
        fi = b["fixed_iters"]
        assert sum(fi["counts"].values()) == 4
        # K = 8 reads the fixed-work volume: 8 MiB (full grid), 4 MiB (half)
        n_cus = isw.sweep_device_info()["num_cus"]
        assert fi["iters"]["full_V16_w4"] == max(1, (8 << 20) // (16 * 8 * 64 * n_cus * 4))
        assert fi["iters"]["half_V16_w8"] == max(1, (4 << 20) // (16 * 8 * 64 * n_cus // 2 * 8))
    man = sweeps.order_counter_pass(sizes=(1 << 20,), Ks=(1, 2), L=1 << 17, reps=2,
                                    waves_per_cu=4)
    assert len(man) == 3 * 2 * 2 and sum(m["warmup"] for m in man) == 6
    assert {m["layout"] for m in man} == {"round_robin", "blocked", "strided"}
    assert all(m["issued_bytes"] == 16 * (1 << 17) for m in man)
    of = sweeps.order_footprint([1 << 20, 4 << 20], Ks=(1, 2), L=1 << 17, n=1)
    assert of[4 << 20]["blocked"]["coverage"][2]["coverage"] == 0.5
    assert of[4 << 20]["strided"]["coverage"][2]["coverage"] == 0.5
    assert of[1 << 20]["strided"]["checksums_consistent"]
    assert of[1 << 20]["round_robin"]["coverage"][1]["max_reads"] == 2
    seen = []

    def verify(checks):
        seen.extend(checks)
        want = checksums.range_sinks_many([c[:3] for c in checks], threads=4)
        return [w == (c[3], c[4]) for w, c in zip(want, checks)]

    space = {"vec_widths": [4, 16], "Ks": [3, 7], "waves_per_cu": [4, 12],
             "policies": [isw.CACHE_NT]}
    bt = sweeps.batched_autotuned(n_points=6, n=2, space=space, verify=verify, hi_log2=24)
    assert bt["matches_oracle"] and bt["points_checked"] == 12 == len(seen)
    assert bt["batched_aggregate_gbps"] > 0


def test_graph_replays_match_eager_runs():
    """Several graph launches with eager work and synchronisation between
    them; every replay must reproduce the eager sinks."""
    nbytes = 8 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED + 9)
    cells = [isw.make_cell(buf, nbytes, K, 16, w, nbytes // 16, cache_policy=pol)
             for K, w, pol in ((1, 4, 0), (2, 32, 3), (5, 16, 1), (16, 8, 2))]
    cells.append(isw.make_cell(buf, nbytes, 6, 16, 2, nbytes // 16, kind=isw.KIND_LDS_ASYNC))
    eager = [(r["sum32"], r["xor32"]) for r in isw.sweep_run(cells)]
    for rep in range(4):
        res, ms = isw.sweep_batched(cells)
        assert [(r["sum32"], r["xor32"]) for r in res] == eager, rep
        # eager work in between: a different cell set, then a sync
        isw.sweep_plain(buf, nbytes, 3, 8, 12, nbytes // 8)
        torch.cuda.synchronize()


def test_persistent_graph_replays():
    """A graph captured once: every replay reads the buffer's current
    contents, keeps its own scratch across other library calls, and times
    each kernel with its captured events."""
    nbytes = 8 << 20
    buf = dev_bytes(nbytes)
    other = dev_bytes(nbytes)
    isw.sweep_fill_u32(other, nbytes, SEED + 21)
    cells = [isw.make_cell(buf, nbytes, K, 16, w, nbytes // 16, cache_policy=pol)
             for K, w, pol in ((1, 4, 3), (3, 32, 0), (7, 16, 2), (16, 8, 1))]
    cells.append(isw.make_cell(buf, nbytes, 4, 16, 4, nbytes // 16, kind=isw.KIND_LDS_MATCHED))
    g = isw.sweep_graph_create(cells)
    try:
        for rep in range(4):
            seed = SEED + 30 + rep
            isw.sweep_fill_u32(buf, nbytes, seed)
            torch.cuda.synchronize()
            res, ms = isw.sweep_graph_launch(g)
            words = splitmix.buffer_words(seed, nbytes)
            for c, r in zip(cells, res):
                n_waves = r["waves"]
                p = oplan.wave_group(c.total_logical_loads, c.K, n_waves)
                want = checksums.combine(*checksums.per_wave(words, 16, c.K, p["Q"], n_waves))
                assert (r["sum32"], r["xor32"]) == want, (rep, c.K)
                assert r["issued_loads"] == p["issued"]
                assert r["window_ns"] > 0 and r["event_ms"] == 0
            assert 0 < sum(r["window_ns"] for r in res) <= ms * 1e6 * 1.02
            # other calls between replays reuse the library's shared scratch
            isw.sweep_run([isw.make_cell(other, nbytes, 2, 16, 32, nbytes // 16)] * 3)
            isw.sweep_batched([isw.make_cell(other, nbytes, 5, 8, 8, nbytes // 8)])
    finally:
        isw.sweep_graph_destroy(g)
    isw.sweep_graph_destroy(g)          # a destroyed handle is cleared, not freed twice


FUSED_POINTS = [  # (offset, bytes, L) inside one buffer: ragged, exact, wrapping
    (0, 1 << 20, (1 << 20) // 16),
    (1 << 20, 3 << 20, 3 * (1 << 20) // 16 + 64 * 7 * 5),
    (4 << 20, 64 << 10, 9 * (64 << 10) // 16),
    (5 << 20, 2 << 20, (2 << 20) // 16 - 64 * 3),
    (8 << 20, 7 << 20, (7 << 20) // 16),
]


def _fused_cells(base_ptr, K, w, pol):
    return [isw.make_cell(base_ptr + o, b, K, 16, w, L, cache_policy=pol)
            for o, b, L in FUSED_POINTS]


@pytest.mark.parametrize("K,w,pol", [(1, 32, 3), (7, 4, 0), (3, 16, 2), (16, 8, 1)])
def test_fused_batch_graph_matches_the_oracle(K, w, pol):
    """Points that share K, width, policy and occupancy run as one fused
    persistent launch: every point's sinks and issued loads equal the
    oracle's and the separate launches', on every replay (ragged sizes,
    a point read nine times over, a point smaller than one round of the
    grid)."""
    nbytes = 16 << 20
    seed = SEED + 40 + K
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, seed)
    words = splitmix.buffer_words(seed, nbytes)
    cells = _fused_cells(buf.data_ptr(), K, w, pol)
    alone = isw.sweep_run(cells)
    print(f"fused K={K} w={w} policy={pol}: {len(cells)} points", flush=True)
    with isw.sweep_graph_create(cells, isw.make_opts(fuse=True)) as g:
        for rep in range(3):
            res, ms = isw.sweep_graph_launch(g)
            assert ms > 0
            for (o, b, L), r, a in zip(FUSED_POINTS, res, alone):
                n_waves = r["waves"]
                p = oplan.wave_group(L, K, n_waves)
                want = checksums.combine(*checksums.per_wave(
                    words, 16, K, p["Q"], n_waves, base=o // 16, n_vec=b // 16))
                assert (r["sum32"], r["xor32"]) == want, (rep, o)
                assert (a["sum32"], a["xor32"]) == want
                assert r["issued_loads"] == p["issued"] == a["issued_loads"]
                assert r["window_ns"] > 0


@pytest.mark.parametrize("case", range(8))
def test_fused_batch_random_points_match_the_oracle(case):
    """Seeded random batches run as one fused launch: 3-12 points of one
    configuration (K, width, occupancy, policy drawn per case) at random
    offsets and sizes in one buffer, with ragged targets that may wrap the
    point's region several times; every point equals the oracle on every
    replay."""
    rng = np.random.default_rng(1000 + case)
    nbytes = 32 << 20
    seed = SEED + 70 + case
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, seed)
    words = splitmix.buffer_words(seed, nbytes)
    K = int(rng.integers(1, 17))
    V = int(rng.choice([4, 8, 16]))
    w = int(rng.choice([4, 8, 12, 16, 20, 24, 28]))
    pol = int(rng.integers(0, 4))
    seg = 64 * V
    pts = []
    for _ in range(int(rng.integers(3, 13))):
        size = seg * int(rng.integers(1, (4 << 20) // seg + 1))
        off = seg * int(rng.integers(0, (nbytes - size) // seg + 1))
        L = int(rng.integers(64 * K, 3 * size // V + 64 * K + 1))
        pts.append((off, size, L))
    cells = [isw.make_cell(buf.data_ptr() + o, b, K, V, w, L, cache_policy=pol)
             for o, b, L in pts]
    print(f"random fused batch {case}: K={K} V={V} w={w} policy={pol}, {len(pts)} points",
          flush=True)
    try:
        g = isw.sweep_graph_create(cells, isw.make_opts(fuse=True))
    except isw.SweepError as e:
        assert e.code == isw.EOCCUPANCY
        pytest.skip("configuration cannot reach its occupancy")
    with g:
        for rep in range(2):
            res, _ = isw.sweep_graph_launch(g)
            for (o, b, L), r in zip(pts, res):
                p = oplan.wave_group(L, K, r["waves"])
                want = checksums.combine(*checksums.per_wave(
                    words, V, K, p["Q"], r["waves"], base=o // V, n_vec=b // V))
                assert (r["sum32"], r["xor32"]) == want, (rep, o, b, L)
                assert r["issued_loads"] == p["issued"]


def test_fused_batch_groups_runs_of_equal_cells():
    """Only consecutive cells with the same kernel and launch shape fuse; a
    cell of another kind, order or configuration between them splits the
    runs, and every cell keeps its own result."""
    nbytes = 16 << 20
    seed = SEED + 60
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, seed)
    words = splitmix.buffer_words(seed, nbytes)
    base = buf.data_ptr()
    a = _fused_cells(base, 4, 16, 3)
    b = _fused_cells(base, 2, 8, 3)
    cells = a[:2] + [isw.make_cell(buf, 1 << 20, 4, 16, 4, 1 << 16, kind=isw.KIND_LDS_ASYNC,
                                   cache_policy=3)] + a[2:] + b \
        + [isw.make_cell(buf, 2 << 20, 4, 16, 16, 1 << 17, cache_policy=3,
                         order=isw.ORDER_BLOCKED)] + b[:1]
    want = [(r["sum32"], r["xor32"], r["issued_loads"]) for r in isw.sweep_run(cells)]
    res, _ = isw.sweep_batched(cells, isw.make_opts(fuse=True))
    assert [(r["sum32"], r["xor32"], r["issued_loads"]) for r in res] == want
    # and against the oracle for the plain round-robin cells
    for c, r in zip(cells, res):
        if c.kind != isw.KIND_PLAIN or c.order != isw.ORDER_ROUND_ROBIN:
            continue
        o = (c.buf - base) // 16
        p = oplan.wave_group(c.total_logical_loads, c.K, r["waves"])
        assert (r["sum32"], r["xor32"]) == checksums.combine(*checksums.per_wave(
            words, 16, c.K, p["Q"], r["waves"], base=o, n_vec=c.bytes // 16))


def test_graph_handle_as_context_manager():
    nbytes = 1 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED + 60)
    want = checksums.whole_buffer(splitmix.buffer_words(SEED + 60, nbytes))
    with isw.sweep_graph_create([isw.make_cell(buf, nbytes, 2, 16, 4, nbytes // 16)]) as g:
        res, _ = isw.sweep_graph_launch(g)
    assert (res[0]["sum32"], res[0]["xor32"]) == want and g.handle is None


def test_persistent_graph_rejects_bad_cells():
    nbytes = 1 << 20
    buf = dev_bytes(nbytes)
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_graph_create([isw.make_cell(buf, nbytes, 17, 16, 4, nbytes // 16)])
    assert e.value.code == isw.EINVAL
    with pytest.raises(isw.SweepError):
        isw.sweep_graph_create([])
    assert isw.lib.sweep_graph_destroy(None) == isw.OK


def test_concurrent_callers_get_their_own_results():
    """Calls from several host threads (ctypes releases the GIL) are
    serialised by the library; every caller gets the sinks of its own
    buffer, and errors stay with the thread that caused them."""
    import threading
    nbytes = 4 << 20
    bufs = [dev_bytes(nbytes) for _ in range(3)]
    for i, b in enumerate(bufs):
        isw.sweep_fill_u32(b, nbytes, SEED + 40 + i)
    torch.cuda.synchronize()
    want = [checksums.whole_buffer(splitmix.buffer_words(SEED + 40 + i, nbytes))
            for i in range(3)]
    g = isw.sweep_graph_create([isw.make_cell(bufs[2], nbytes, 2, 16, 8, nbytes // 16)])
    got, errs = {}, {}

    def plain(i):
        for rep in range(20):
            K = (1, 2, 4, 8)[rep % 4]             # whole passes: every K divides
            r = isw.sweep_plain(bufs[i], nbytes, K, 16, 8, nbytes // 16)
            got.setdefault(i, set()).add((r["sum32"], r["xor32"]))
        errs[i] = isw.lib.sweep_last_error()     # this thread never failed

    def graph():
        for _ in range(20):
            res, _ = isw.sweep_graph_launch(g)
            got.setdefault(2, set()).add((res[0]["sum32"], res[0]["xor32"]))

    def failing():
        for _ in range(20):
            try:
                isw.sweep_plain(bufs[0], nbytes, 17, 16, 8, nbytes // 16)
            except isw.SweepError as e:
                errs.setdefault("codes", set()).add(e.code)
        errs["msg"] = isw.lib.sweep_last_error()

    ts = [threading.Thread(target=plain, args=(0,)), threading.Thread(target=plain, args=(1,)),
          threading.Thread(target=graph), threading.Thread(target=failing)]
    try:
        for t in ts:
            t.start()
        for t in ts:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in ts)
    finally:
        isw.sweep_graph_destroy(g)
    for i in range(3):
        assert got[i] == {want[i]}, i
    assert errs["codes"] == {isw.EINVAL} and errs["msg"]
    assert errs[0] == b"" and errs[1] == b""


def test_entry_points_honour_the_callers_stream():
    """Every entry point runs on the stream it is given: work queued on a
    side stream (a fill, then the sweeps, without host synchronisation in
    between) sees the fill, and gives the default stream's results."""
    nbytes = 8 << 20
    side = torch.cuda.Stream()                 # default priority
    buf = dev_bytes(nbytes)
    torch.cuda.synchronize()
    isw.sweep_fill_u32(buf, nbytes, SEED + 50, stream=side)
    o = isw.make_opts(stream=side, cache_policy=isw.CACHE_NT)
    r = isw.sweep_plain(buf, nbytes, 4, 16, 8, nbytes // 16, o)
    want = checksums.whole_buffer(splitmix.buffer_words(SEED + 50, nbytes))
    assert (r["sum32"], r["xor32"]) == want
    # refill on the side stream, then a sweep, a graph replay, two streams
    isw.sweep_fill_u32(buf, nbytes, SEED + 51, stream=side)
    want = checksums.whole_buffer(splitmix.buffer_words(SEED + 51, nbytes))
    cells = [isw.make_cell(buf, nbytes, K, 16, 16, nbytes // 16) for K in (1, 2, 8)]
    assert all((x["sum32"], x["xor32"]) == want for x in isw.sweep_run(cells, o))
    g = isw.sweep_graph_create(cells)
    try:
        isw.sweep_fill_u32(buf, nbytes, SEED + 52, stream=side)
        res, _ = isw.sweep_graph_launch(g, stream=side)
    finally:
        isw.sweep_graph_destroy(g)
    want = checksums.whole_buffer(splitmix.buffer_words(SEED + 52, nbytes))
    assert all((x["sum32"], x["xor32"]) == want for x in res)
    isw.sweep_fill_u32(buf, nbytes, SEED + 53, stream=side)
    words = splitmix.buffer_words(SEED + 53, nbytes)
    a, b = isw.sweep_two_stream_kind(buf, nbytes, 4, 2, 2, isw.KIND_PLAIN, nbytes // 16, o)
    half = words.size // 2
    assert (a["sum32"], a["xor32"]) == checksums.whole_buffer(words[:half])
    assert (b["sum32"], b["xor32"]) == checksums.whole_buffer(words[half:])
    # a payload written on the side stream and summed there
    x = torch.full((1 << 20,), 0.5, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        x.fill_(0.25)
    s, _ = isw.sweep_reduce_fp(x, x.numel(), isw.F32, 8, o)
    assert s == 0.25 * x.numel()


def test_unpinned_occupancy_gives_the_same_sinks():
    """Residency pinning only pads LDS; the sinks do not depend on it."""
    nbytes = 4 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED + 70)
    want = checksums.whole_buffer(splitmix.buffer_words(SEED + 70, nbytes))
    for w in (4, 16, 32):
        a = isw.sweep_plain(buf, nbytes, 2, 16, w, nbytes // 16, isw.make_opts(pin_occupancy=True))
        b = isw.sweep_plain(buf, nbytes, 2, 16, w, nbytes // 16, isw.make_opts(pin_occupancy=False))
        assert (a["sum32"], a["xor32"]) == (b["sum32"], b["xor32"]) == want
        assert a["lds_bytes"] > 0 and b["lds_bytes"] == 0 and a["waves"] == b["waves"]


def test_graph_survives_library_shutdown():
    """A captured graph owns its scratch: sweep_shutdown() frees the library's
    shared scratch but leaves the graph replayable; the library initialises
    itself again on the next call."""
    nbytes = 2 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED + 80)
    want = checksums.whole_buffer(splitmix.buffer_words(SEED + 80, nbytes))
    with isw.sweep_graph_create([isw.make_cell(buf, nbytes, 4, 16, 8, nbytes // 16)]) as g:
        isw.sweep_shutdown()
        res, _ = isw.sweep_graph_launch(g)
        assert (res[0]["sum32"], res[0]["xor32"]) == want
    r = isw.sweep_plain(buf, nbytes, 2, 16, 8, nbytes // 16)
    assert (r["sum32"], r["xor32"]) == want
