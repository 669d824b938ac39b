"""CPU pins of the absorbed-term payloads the GPU precision tests use: in
the kernel's lane layout, the binary32 model of the compensated scheme sums
them exactly, and a plain binary32 sum in the same layout misses exactly the
shortfall the tests claim (no GPU)."""
import pytest

import fp_scheme as fs
from precision_payloads import absorbed_payload, kernel_lanes


@pytest.mark.parametrize("loads", [4, 8])
@pytest.mark.parametrize("kind", ["f32", "bf16", "fp8_e4m3"])
def test_payload_claims_hold_in_the_kernel_layout(kind, loads):
    n_waves = 8
    rounds = 6 if kind == "fp8_e4m3" else 3
    n_bytes = loads * 1024 * n_waves * rounds
    u, exact, short = absorbed_payload(kind, n_bytes, n_waves, loads, device="cpu")
    lanes = kernel_lanes(kind, u, n_waves, loads)
    assert fs.scheme(lanes) == exact
    assert exact - fs.scheme(lanes, compensated=False) == short
    assert short > 0
