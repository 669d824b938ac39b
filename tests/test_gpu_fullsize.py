"""Parity at the workloads' full sizes, in the launch configurations the
bench times: sampled per-wave checksums recomputed one by one by the oracle
from the generator seed, global checksums through closed forms, and the
invariants the method fixes (matched work across K, order independence)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_util import decode_recs, recs, reduce_lane_terms
from oracle import checksums, fpsum, plan as oplan, splitmix
from paper_2608_15764_amd import ilpsweep as isw
from paper_2608_15764_amd import sweeps
import synth

GIB = 1 << 30


def _sample(n, k=5, seed=0):
    rng = np.random.default_rng(seed)
    pick = {0, 1, n // 2, n - 1}
    pick.update(int(v) for v in rng.integers(0, n, k))
    return sorted(pick)


@pytest.fixture(scope="module")
def c2():
    nbytes = GIB
    seed = sweeps.SEED_BASE + 1
    buf = sweeps.device_buffer(nbytes, seed)
    whole = checksums.whole_buffer(splitmix.buffer_words(seed, nbytes))
    yield buf, nbytes, seed, whole
    del buf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("policy", [isw.CACHE_BYPASS_L1, isw.CACHE_BYPASS_L1_NT])
@pytest.mark.parametrize("w", [4, 16, 32])
def test_k_sweep_full_size(c2, w, policy):
    buf, nbytes, seed, whole = c2
    L = 1 << 26
    issued = []
    for K in range(1, 17):
        n_waves = 256 * w
        ro = recs(n_waves)
        try:
            r = isw.sweep_plain(buf, nbytes, K, 16, w, L,
                                isw.make_opts(cache_policy=policy, wave_out=ro))
        except isw.SweepError as e:
            assert e.code == isw.EOCCUPANCY
            continue
        p = oplan.wave_group(L, K, r["waves"])
        assert r["issued_loads"] == p["issued"]
        issued.append(r["issued_loads"])
        rr = decode_recs(ro)[: r["waves"]]
        for wave in _sample(r["waves"], seed=K * 100 + w):
            want = checksums.wave_from_seed(seed, 16, K, p["Q"], r["waves"], wave,
                                            buffer_bytes=nbytes)
            assert (rr["sum32"][wave], rr["xor32"][wave]) == want, (K, wave)
        if K & (K - 1) == 0:        # one full pass: the whole buffer
            assert (r["sum32"], r["xor32"]) == whole
        assert r["gbps"] > 0
    # matched issued logical loads across K (Section 4.2: <= 0.0246 %)
    assert oplan.kset_mismatch(issued) <= 0.0246 / 100


def test_bench_sweep_graph_full_size(c2):
    """The exact timed configuration of the bench: the 1 GiB K sweep at 4..32
    waves per CU, ascending then reversed, cache policy sc1+nt, captured into
    one graph and replayed.  Every cell's global sinks equal the oracle's
    checksum of the vectors it issues (a prefix of the buffer: 64*K*Q <=
    2**26 vectors, no wrap), on every replay."""
    buf, nbytes, seed, _whole = c2
    L = 1 << 26
    cells, meta = sweeps.plain_k_cells(buf, nbytes, L, isw.CACHE_BYPASS_L1_NT,
                                       [4 * w for w in range(1, 9)], range(1, 17))
    cells, meta, dropped = sweeps.drop_infeasible(cells, meta)
    assert len(cells) == 252 and len(dropped) == 4
    words = splitmix.buffer_words(seed, nbytes)
    prefix = {}
    g = isw.sweep_graph_create(cells)
    try:
        for rep in range(2):
            res, ms = isw.sweep_graph_launch(g)
            assert ms > 0
            for m, r in zip(meta, res):
                n_vec = r["issued_loads"]
                assert n_vec == oplan.wave_group(L, m["K"], r["waves"])["issued"]
                if n_vec not in prefix:
                    prefix[n_vec] = checksums.whole_buffer(words[: n_vec * 4])
                assert (r["sum32"], r["xor32"]) == prefix[n_vec], (rep, m)
                assert r["window_ns"] > 0 and r["event_ms"] == 0
    finally:
        isw.sweep_graph_destroy(g)


def test_orders_give_identical_results(c2):
    buf, nbytes, _seed, _whole = c2
    L = 1 << 26
    cells, meta = sweeps.plain_k_cells(buf, nbytes, L, isw.CACHE_BYPASS_L1, [16],
                                       range(1, 17))
    res = isw.sweep_run(cells)
    by = {}
    for m, r in zip(meta, res):
        by.setdefault(m["K"], set()).add((r["issued_loads"], r["sum32"], r["xor32"]))
    assert all(len(v) == 1 for v in by.values())


def test_residency_is_pinned(c2):
    """Every CU hosts exactly the requested workgroups (HW_ID / XCC_ID)."""
    buf, nbytes, _seed, _whole = c2
    info = isw.sweep_device_info()
    for w in (4, 8, 16, 32):
        n_waves = info["num_cus"] * w
        ro = recs(n_waves)
        isw.sweep_plain(buf, nbytes, 2, 16, w, 1 << 26, isw.make_opts(wave_out=ro))
        rr = decode_recs(ro)
        hw = rr["hw_id"].astype(np.int64)
        cu = (rr["xcc_id"].astype(np.int64) & 0xF) << 16 | ((hw >> 8) & 0xFF)
        wg = np.arange(n_waves) // 4
        per_cu = {}
        for c, g in zip(cu, wg):
            per_cu.setdefault(int(c), set()).add(int(g))
        counts = sorted(len(v) for v in per_cu.values())
        print(f"w={w}: {len(per_cu)} CUs, workgroups per CU {counts[0]}..{counts[-1]}")
        assert len(per_cu) == info["num_cus"]
        assert counts[0] == counts[-1] == w // 4


@pytest.mark.parametrize("V,K", [(4, 3), (8, 5), (16, 16)])
def test_vector_indices_past_2_to_32(V, K):
    """A 20 GiB buffer read in 4-, 8- and 16-byte vectors (the last at the
    largest K): vector indices exceed 2**32 (V = 4) and byte offsets exceed
    2**34; the work wraps past the end.  Sampled waves, including the last
    one, are recomputed from the seed."""
    size = 20 * GIB
    seed = sweeps.SEED_BASE + 2
    buf = sweeps.device_buffer(size, seed)
    n_vec = size // V
    L = n_vec + 64 * K * 12345 + 17           # more than one pass, ragged
    w = 8
    try:
        ro = recs(256 * w)
        r = isw.sweep_plain(buf, size, K, V, w, L,
                            isw.make_opts(cache_policy=isw.CACHE_BYPASS_L1_NT, wave_out=ro))
        p = oplan.wave_group(L, K, r["waves"])
        assert r["issued_loads"] == p["issued"] and p["issued"] > n_vec
        rr = decode_recs(ro)
        for wave in _sample(r["waves"], k=1, seed=V):
            want = checksums.wave_from_seed(seed, V, K, p["Q"], r["waves"], wave,
                                            buffer_bytes=size)
            assert (rr["sum32"][wave], rr["xor32"][wave]) == want, wave
    finally:
        del buf
        torch.cuda.empty_cache()


@pytest.mark.parametrize("size,V,K,w,L", [
    (GIB, 16, 7, 16, 1 << 26),                        # the order row at 1 GiB
    (128 << 20, 16, 8, 16, 1 << 26),                  # wrapped: K loads alias
    (20 * GIB, 4, 3, 8, 20 * GIB // 4 + 64 * 3 * 999 + 5),   # indices past 2**32
])
def test_strided_layout_full_size(size, V, K, w, L):
    """The strided layout in the order/footprint row's launch configuration,
    and past 2**32 vectors: sampled waves recomputed from the seed, and the
    cell's global sinks equal the round-robin cell's (both read the stream
    0 .. issued - 1 modulo the allocation)."""
    seed = sweeps.SEED_BASE + 3
    buf = sweeps.device_buffer(size, seed)
    try:
        print(f"strided {size} B, V={V} K={K} w={w} L={L}", flush=True)
        ro = recs(256 * w)
        r = isw.sweep_plain(buf, size, K, V, w, L,
                            isw.make_opts(cache_policy=isw.CACHE_BYPASS_L1_NT, wave_out=ro,
                                          order=isw.ORDER_STRIDED))
        p = oplan.wave_group(L, K, r["waves"], order=oplan.STRIDED)
        assert r["issued_loads"] == p["issued"]
        rr = decode_recs(ro)
        for wave in _sample(r["waves"], k=2 if size > GIB else 5, seed=K):
            want = checksums.wave_from_seed(seed, V, K, p["Q"], r["waves"], wave,
                                            buffer_bytes=size, order=oplan.STRIDED)
            assert (rr["sum32"][wave], rr["xor32"][wave]) == want, wave
        rb = isw.sweep_plain(buf, size, K, V, w, L,
                             isw.make_opts(cache_policy=isw.CACHE_BYPASS_L1_NT))
        assert (r["sum32"], r["xor32"]) == (rb["sum32"], rb["xor32"])
        assert r["issued_loads"] == rb["issued_loads"]
    finally:
        del buf
        torch.cuda.empty_cache()


def test_allocation_sweep_graph_full_size():
    """The allocation sweep as the bench runs it: one captured graph over
    allocation x occupancy x K x order, 16 GiB issued per cell.  512 MiB and
    2 GiB are whole numbers of passes (32 and 8), so every cell's sinks have
    a closed form: (passes x S mod 2**32, 0)."""
    seed = sweeps.SEED_BASE + 2
    sizes = [512 << 20, 2 * GIB]
    buf = sweeps.device_buffer(max(sizes), seed)
    L = 1 << 30
    try:
        cells, meta = [], []
        for size in sizes:
            c, m = sweeps.plain_k_cells(buf, size, L, isw.CACHE_BYPASS_L1, [16, 32],
                                        (1, 2, 4, 8))
            cells += c
            meta += [dict(x, bytes=size) for x in m]
        want = {}
        for size in sizes:
            S, _X = checksums.whole_buffer(splitmix.buffer_words(seed, size))
            want[size] = (((L * 16 // size) * S) & 0xFFFFFFFF, 0)
        with isw.sweep_graph_create(cells) as g:
            for rep in range(2):
                res, _ = isw.sweep_graph_launch(g)
                for m, r in zip(meta, res):
                    assert r["issued_loads"] == L
                    assert (r["sum32"], r["xor32"]) == want[m["bytes"]], (rep, m)
    finally:
        del buf
        torch.cuda.empty_cache()


@pytest.mark.parametrize("size", [512 << 20, 20 * GIB])
def test_allocation_sweep_full_size(size):
    seed = sweeps.SEED_BASE + 2
    buf = sweeps.device_buffer(size, seed)
    L = 1 << 30
    try:
        for K in (1, 2, 4, 8):
            w = 16
            ro = recs(256 * w)
            r = isw.sweep_plain(buf, size, K, 16, w, L,
                                isw.make_opts(cache_policy=isw.CACHE_BYPASS_L1, wave_out=ro))
            p = oplan.wave_group(L, K, r["waves"])
            assert r["issued_loads"] == p["issued"] == L
            rr = decode_recs(ro)
            for wave in _sample(r["waves"], k=2, seed=K):
                want = checksums.wave_from_seed(seed, 16, K, p["Q"], r["waves"], wave,
                                                buffer_bytes=size)
                assert (rr["sum32"][wave], rr["xor32"][wave]) == want
            if size == 512 << 20:
                # 16 GiB issued over 512 MiB: exactly 32 passes
                S, _X = checksums.whole_buffer(splitmix.buffer_words(seed, size))
                assert (r["sum32"], r["xor32"]) == ((32 * S) & 0xFFFFFFFF, 0)
    finally:
        del buf
        torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def c4():
    nbytes = 2 * GIB
    seed = sweeps.SEED_BASE + 3
    buf = sweeps.device_buffer(nbytes, seed)
    words = splitmix.buffer_words(seed, nbytes)
    yield buf, nbytes, seed, words
    del buf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", [isw.KIND_LDS_ASYNC, isw.KIND_LDS_MATCHED])
@pytest.mark.parametrize("D,W", [(1, 1), (4, 8), (16, 8), (16, 1)])
def test_lds_paths_full_size(c4, kind, D, W):
    buf, nbytes, seed, words = c4
    L = nbytes // 16
    ro = recs(256 * W)
    fn = isw.sweep_lds_async if kind == isw.KIND_LDS_ASYNC else isw.sweep_lds_matched_plain
    r = fn(buf, nbytes, D, 16, W, L, isw.make_opts(wave_out=ro))
    p = oplan.wave_group(L, D, r["waves"])
    assert r["issued_loads"] == p["issued"] == L
    assert (r["sum32"], r["xor32"]) == checksums.whole_buffer(words)
    rr = decode_recs(ro)
    for wave in _sample(r["waves"], k=2, seed=D):
        want = checksums.wave_from_seed(seed, 16, D, p["Q"], r["waves"], wave,
                                        buffer_bytes=nbytes)
        assert (rr["sum32"][wave], rr["xor32"][wave]) == want


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("kind_b", [isw.KIND_LDS_ASYNC, isw.KIND_PLAIN])
@pytest.mark.parametrize("D", [4, 8])
def test_two_stream_full_size(c4, D, kind_b, split):
    """The bench's two-stream launches (4 + 4 waves in one workgroup, or
    8 + 8 on different CUs): each stream's sinks are its whole half."""
    buf, nbytes, _seed, words = c4
    n_vec = nbytes // 16
    (a0, an), (b0, bn) = checksums.two_stream_regions(n_vec)
    if split:
        ra, rb = isw.sweep_two_stream_split(buf, nbytes, D, 8, 8, kind_b, n_vec)
    else:
        ra, rb = isw.sweep_two_stream_kind(buf, nbytes, D, 4, 4, kind_b, n_vec)
    assert (ra["sum32"], ra["xor32"]) == checksums.whole_buffer(words[a0 * 4:(a0 + an) * 4])
    assert (rb["sum32"], rb["xor32"]) == checksums.whole_buffer(words[b0 * 4:(b0 + bn) * 4])
    assert ra["issued_loads"] + rb["issued_loads"] == n_vec


def test_batched_points_full_size():
    sizes = sweeps.point_sizes(64)
    assert sizes[0] == 1 << 20 and sizes[-1] == 2 * GIB
    offs = np.concatenate([[0], np.cumsum(sizes)])
    seed = sweeps.SEED_BASE + 4
    big = sweeps.device_buffer(int(offs[-1]), seed)
    base = big.data_ptr()
    cells = [isw.make_cell(base + int(o), s, 4, 16, 16, s // 16,
                           cache_policy=isw.CACHE_BYPASS_L1_NT)
             for s, o in zip(sizes, offs[:-1])]
    res, ms = isw.sweep_batched(cells)
    run = isw.sweep_run(cells)
    assert ms > 0
    for i, (s, o) in enumerate(zip(sizes, offs[:-1])):
        assert res[i]["issued_bytes"] == s
        assert (res[i]["sum32"], res[i]["xor32"]) == (run[i]["sum32"], run[i]["xor32"])
    for i in (0, 1, 31, 62, 63):
        w = splitmix.words(seed, int(offs[i]) // 4, sizes[i] // 4)
        assert (res[i]["sum32"], res[i]["xor32"]) == checksums.whole_buffer(w), i
    del big
    torch.cuda.empty_cache()


def test_autotuned_batch_matches_oracle():
    """The autotuned batch over the tuner's whole space (V in {4, 8, 16},
    K = 1..16, 1..8 waves per SIMD, every cache policy): every point of the
    tuned graph, and of the untuned pass beside it, carries the sinks of
    exactly the words it read, its issued prefix 64 K floor(L / 64 K)
    vectors of its point, whatever K the tuner chose."""
    import os
    threads = max(1, min(16, os.cpu_count() or 1))
    seen = []

    def verify(checks):
        seen.extend(checks)
        want = checksums.range_sinks_many([c[:3] for c in checks], threads=threads)
        return [w == (c[3], c[4]) for w, c in zip(want, checks)]

    out = sweeps.batched_autotuned(n=2, verify=verify)
    print("tuned:", out["tuned"], flush=True)
    assert out["matches_oracle"], out["mismatched_points"]
    assert out["points_checked"] == 128 == len(seen)
    space = sweeps.DEFAULT_SPACE
    assert space["Ks"] == list(range(1, 17)) and space["vec_widths"] == [4, 8, 16]
    assert space["waves_per_cu"] == [4, 8, 12, 16, 20, 24, 28, 32]
    for p in out["points"]:
        V, K = p["vec_width"], p["K"]
        assert V in space["vec_widths"] and K in space["Ks"]
        assert p["waves_per_cu"] in space["waves_per_cu"]
        L = p["bytes"] // V
        assert p["issued_bytes"] == 64 * K * (L // (64 * K)) * V
    assert out["batched_aggregate_gbps"] > 0 and out["hbm_aggregate_gbps"] > 0
    torch.cuda.empty_cache()


def test_autotuner_picks_a_candidate():
    nbytes = 256 << 20
    buf = sweeps.device_buffer(nbytes, 9)
    cfg, g = isw.sweep_autotune(buf, nbytes, [16, 8], [1, 2, 4], [8, 32],
                                isw.CACHE_NT, 2)
    assert cfg["vec_width"] in (16, 8) and cfg["K"] in (1, 2, 4)
    assert cfg["waves_per_cu"] in (8, 32) and g > 0


@pytest.mark.parametrize("kind", ["f32", "bf16", "fp8_e4m3"])
def test_precision_sum_full_size(kind):
    payload_bytes = 4 * GIB
    eb = synth.ELEM_BYTES[kind]
    n = payload_bytes // eb
    p = synth.normal_payload(kind, n, sweeps.SEED_BASE + 5, device="cuda")
    dt = {"f32": isw.F32, "bf16": isw.BF16, "fp8_e4m3": isw.FP8_E4M3}[kind]
    s1, r = isw.sweep_reduce_fp(p, n, dt, 32)
    s2, _ = isw.sweep_reduce_fp(p, n, dt, 32)
    assert s1 == s2                              # deterministic
    s4, r4 = isw.sweep_reduce_fp(p, n, dt, 4)    # eight loads per lane
    assert s4 == isw.sweep_reduce_fp(p, n, dt, 4)[0]
    host = p.cpu().numpy()
    del p
    torch.cuda.empty_cache()
    # exact sums of the stored values and of their magnitudes (sign bit off)
    if kind == "fp8_e4m3":
        exact = fpsum.exact_sum_e4m3_hist(host)
        absx = fpsum.exact_sum_e4m3_hist(host & np.uint8(0x7F))
    elif kind == "bf16":
        bits = host.view(np.uint16)
        exact = fpsum.exact_sum_bf16_bits(bits)
        absx = fpsum.exact_sum_bf16_bits(bits & np.uint16(0x7FFF))
    else:
        bits = host.view(np.uint32)
        exact = fpsum.exact_sum_f32_bits(bits)
        absx = fpsum.exact_sum_f32_bits(bits & np.uint32(0x7FFFFFFF))
    for got, res, w in ((s1, r, 32), (s4, r4, 4)):
        err = abs(got - exact)
        print(f"{kind} at {w} waves/CU: gpu {got!r} exact {exact!r} |err| {err:.3e} "
              f"({res['gbps']:.0f} GB/s)")
        terms = reduce_lane_terms(kind, n, res["waves"], w)
        assert err <= fpsum.sum2_bound(absx, terms, 8, res["grid_wgs"])


def test_chase_full_size():
    """The latency ladder's largest footprint (2 GiB, 128-byte nodes): three
    runs of 8192 hops, each continuing the chain where the previous stopped,
    land where the oracle's walk of the same chain lands."""
    from oracle import chase
    footprint, stride = 2 * GIB, 128
    chain, start = synth.chase_chain(footprint, stride, seed=sweeps.SEED_BASE + 8,
                                     device="cuda")
    words = chain.view(torch.int32).cpu().numpy()
    try:
        idx = start
        for _ in range(3):
            r = isw.sweep_chase(chain, footprint, idx, 0, 8192, isw.CACHE_BYPASS_L1)
            want = chase.follow(words, idx, 8192)
            assert r["final_index"] == want
            assert 100 < r["ns_per_hop"] < 5000
            idx = r["final_index"]
    finally:
        del chain
        torch.cuda.empty_cache()


def test_walkers_full_size():
    """The per-XCD latency row's walkers at a cold footprint: 64 walkers
    spread along a 256 MiB chain, each landing where the oracle's walk from
    its start lands; one XCD per workgroup in turn."""
    from oracle import chase
    footprint = 256 << 20
    chain, starts = synth.chase_chain_starts(footprint, 128, sweeps.SEED_BASE + 9, 64,
                                             device="cuda")
    words = chain.view(torch.int32).cpu().numpy()
    try:
        out = isw.sweep_chase_walkers(chain, footprint, starts, 0, 2000, isw.CACHE_BYPASS_L1)
        for s0, r in zip(starts, out):
            assert r["final_index"] == chase.follow(words, s0, 2000)
            assert 50 < r["ns_per_hop"] < 5000
        assert len({r["xcc_id"] for r in out}) == 8
    finally:
        del chain
        torch.cuda.empty_cache()


@pytest.mark.parametrize("mask", [0x01, 0x0F, 0x77, 0xFF])
def test_xcd_subset_full_size(c2, mask):
    """The fabric row's read on the bench's 1 GiB buffer: the global sinks
    equal the oracle's checksum of the issued prefix, for one XCD, a group,
    three per group and all eight."""
    buf, nbytes, seed, _whole = c2
    r = isw.sweep_xcd_subset(buf, nbytes, 4, mask,
                             isw.make_opts(cache_policy=isw.CACHE_BYPASS_L1_NT))
    words = splitmix.words(seed, 0, r["issued_loads"] * 4)
    assert (r["sum32"], r["xor32"]) == checksums.whole_buffer(words)
    assert r["gbps"] > 0
