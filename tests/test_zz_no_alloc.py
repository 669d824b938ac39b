"""The allocation-free plain-load entry point (sweep_plain_noalloc) against
sweep_plain: the same sinks, plan and records, on two calls in a row with
the second smaller, through the C ABI."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import numpy as np

from gpu_util import decode_lanes, decode_recs, dev_bytes, lanes, recs
from paper_2608_15764_amd import ilpsweep as isw

SEED = 0x1D5EED00 + 21
SAME = ("target_loads", "issued_loads", "issued_bytes", "mismatch", "sum32", "xor32",
        "grid_wgs", "wg_threads", "waves", "iters_min", "iters_max", "vgprs",
        "lds_bytes", "scratch_bytes", "max_wgs_per_cu")


def _check_pair(buf, nbytes, K, V, w, L, policy, **kw):
    print(f"noalloc vs plain: {nbytes} B K={K} V={V} w={w} L={L} policy={policy}",
          flush=True)
    want = isw.sweep_plain(buf, nbytes, K, V, w, L, isw.make_opts(cache_policy=policy, **kw))
    got = isw.sweep_plain_noalloc(buf, nbytes, K, V, w, L,
                                  isw.make_opts(cache_policy=policy, **kw))
    for k in SAME:
        assert got[k] == want[k], (k, got[k], want[k])
    assert got["event_ms"] == 0.0
    assert got["window_ns"] > 0 and got["gbps"] > 0
    return got, want


def test_two_calls_in_a_row_second_smaller():
    nbytes = 256 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED)
    # the largest default grid (32 waves per CU), K that leaves a ragged end
    big, _ = _check_pair(buf, nbytes, 7, 16, 32, nbytes // 16, isw.CACHE_BYPASS_L1_NT)
    assert big["waves"] == isw.sweep_device_info()["num_cus"] * 32
    # then a smaller cell over a prefix, with wrap-around (3 passes)
    small_bytes = 4 << 20
    small, _ = _check_pair(buf, small_bytes, 3, 8, 8, 3 * small_bytes // 8,
                           isw.CACHE_DEFAULT)
    assert small["waves"] < big["waves"]
    # and the first one again: nothing left over changes it
    again, _ = _check_pair(buf, nbytes, 7, 16, 32, nbytes // 16, isw.CACHE_BYPASS_L1_NT)
    assert (again["sum32"], again["xor32"]) == (big["sum32"], big["xor32"])


def test_caller_records_and_lanes_match():
    nbytes = 8 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED + 1)
    grid = 64                                      # 256 waves
    ra, rb = recs(256), recs(256)
    la, lb = lanes(256 * 64), lanes(256 * 64)
    L = nbytes // 16 + 64 * 5 * 3
    a = isw.sweep_plain(buf, nbytes, 5, 16, 16, L,
                        isw.make_opts(grid_wgs=grid, wave_out=ra, lane_out=la))
    b = isw.sweep_plain_noalloc(buf, nbytes, 5, 16, 16, L,
                                isw.make_opts(grid_wgs=grid, wave_out=rb, lane_out=lb))
    assert (a["sum32"], a["xor32"]) == (b["sum32"], b["xor32"])
    da, db = decode_recs(ra), decode_recs(rb)
    assert np.array_equal(da["sum32"], db["sum32"]) and np.array_equal(da["xor32"], db["xor32"])
    sa, xa = decode_lanes(la, 256)
    sb, xb = decode_lanes(lb, 256)
    assert np.array_equal(sa, sb) and np.array_equal(xa, xb)
    # then a smaller launch through the static scratch again
    _check_pair(buf, 1 << 20, 2, 4, 4, (1 << 20) // 4, isw.CACHE_NT)


def test_rejects_what_sweep_plain_rejects_and_oversized_launches():
    buf = dev_bytes(1 << 20)
    for args in ((buf, 1 << 20, 0, 16, 8, 1000), (buf, 1 << 20, 2, 12, 8, 1000),
                 (buf.data_ptr() + 4, (1 << 20) - 1024, 2, 16, 8, 1000)):
        with pytest.raises(isw.SweepError) as e1:
            isw.sweep_plain(*args)
        with pytest.raises(isw.SweepError) as e2:
            isw.sweep_plain_noalloc(*args)
        assert e1.value.code == e2.value.code
    # more waves than the static scratch holds, and no caller records
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plain_noalloc(buf, 1 << 20, 1, 16, 4, 1 << 16,
                                isw.make_opts(grid_wgs=4097, pin_occupancy=False))
    assert e.value.code == isw.EINVAL and "static scratch" in str(e.value)
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plain_noalloc(buf, 1 << 20, 1, 16, 4, 1 << 16,
                                isw.make_opts(grid_wgs=16, wave_out=recs(63)))
    assert e.value.code == isw.EINVAL


def test_works_after_library_shutdown():
    nbytes = 2 << 20
    buf = dev_bytes(nbytes)
    isw.sweep_fill_u32(buf, nbytes, SEED + 2)
    torch.cuda.synchronize()
    before = isw.sweep_plain_noalloc(buf, nbytes, 4, 16, 8, nbytes // 16)
    isw.sweep_shutdown()
    after = isw.sweep_plain_noalloc(buf, nbytes, 4, 16, 8, nbytes // 16)
    assert (before["sum32"], before["xor32"]) == (after["sum32"], after["xor32"])
    _check_pair(buf, nbytes, 4, 16, 8, nbytes // 16, isw.CACHE_DEFAULT)
