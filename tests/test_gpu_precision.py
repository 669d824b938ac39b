"""The streaming sum on payloads that an uncompensated binary32 sum gets
badly wrong, so that the rigorous tolerance can fail (every payload type,
both load depths, several occupancies, and the 4 GiB size).

The payloads follow the launch's layout: lane l of wave w starts with
load 0 of wave-group w, i.e. vector w*NL*64 + l (NL = loads per lane per
group), and continues with groups w + n_waves, w + 2 n_waves, ...

* FP32 and BF16: the first element a lane reads is 2**24, every other
  element is 1.  2**24 + 1 is a tie that rounds back to 2**24, so a plain
  binary32 running sum drops every 1 after the first element: it misses
  every 1 in the payload.  Sum2 keeps each dropped 1 in its c part.
* FP8 e4m3: a lane sums 64 values (four vectors) exactly at a time.  The
  first three rounds of groups hold 448 (code 0x7E) everywhere, so a lane's
  running sum reaches at least 3 * 28672 > 2**16 in binary32; after that
  every chunk holds one 2**-9 (code 0x01) and zeros, a quarter of a unit in
  the last place of that running sum, which a plain sum drops.

In all three the compensated sum is exact: TwoSum is error-free, and the
c parts only ever hold counts of the small unit (1, or 2**-9) well inside
binary32's exact integer range, while the s parts hold multiples of the
large one.  The tests check that the kernel returns the exact sum, that
its error is within the rigorous bound, and that the plain sum's shortfall
(every small term) is over a hundred times that bound.
"""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_util import reduce_lane_terms
from oracle import fpsum
from paper_2608_15764_amd import ilpsweep as isw
from precision_payloads import EB, absorbed_payload

DT = {"f32": isw.F32, "bf16": isw.BF16, "fp8_e4m3": isw.FP8_E4M3}


def _check(kind, n_bytes, w, grid=0):
    n_cus = isw.sweep_device_info()["num_cus"]
    wgs = grid or n_cus * w // 4
    n_waves, loads = wgs * 4, (8 if w == 4 else 4)
    p, exact, short = absorbed_payload(kind, n_bytes, n_waves, loads)
    n = n_bytes // EB[kind]
    print(f"absorbed {kind} {n_bytes} B at {w} waves/CU, {wgs} workgroups", flush=True)
    got, res = isw.sweep_reduce_fp(p, n, DT[kind], w, isw.make_opts(grid_wgs=grid))
    assert res["waves"] == n_waves
    bound = fpsum.sum2_bound(float(exact), reduce_lane_terms(kind, n, n_waves, w), 8,
                             res["grid_wgs"])
    assert short > 100 * bound, (short, bound)
    assert abs(got - exact) <= bound, (got, exact, bound)
    assert got == exact, (got, exact)
    del p


@pytest.mark.parametrize("w", [4, 8, 32])
@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_absorbed_terms_recovered(kind, w):
    _check(kind, 256 << 20, w)


@pytest.mark.parametrize("w", [4, 8, 32])
def test_absorbed_fp8_chunks_recovered(w):
    # 32 workgroups, so that every lane sums far more than three rounds
    _check("fp8_e4m3", 64 << 20, w, grid=32)


@pytest.mark.parametrize("w", [4, 32])
@pytest.mark.parametrize("kind", ["f32", "bf16", "fp8_e4m3"])
def test_absorbed_terms_full_size(kind, w):
    _check(kind, 4 << 30, w)
    torch.cuda.empty_cache()
