"""Absorbed-term payloads for the streaming sum, and a CPU emulation of
which terms each lane of the kernel sums (test helpers).

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
large one.
"""
import numpy as np
import torch

EB = {"f32": 4, "bf16": 2, "fp8_e4m3": 1}
BIG_ROUNDS = 3


def absorbed_payload(kind, n_bytes, n_waves, loads, device="cuda"):
    """(uint8 payload, exact sum, plain binary32 shortfall); every element
    is non-negative, so the exact sum is also sum |x|."""
    group_bytes = loads * 64 * 16
    assert n_bytes % group_bytes == 0
    n_groups = n_bytes // group_bytes
    if kind in ("f32", "bf16"):
        assert n_groups >= 2 * n_waves
        dt = torch.float32 if kind == "f32" else torch.bfloat16
        per_vec = 16 // EB[kind]
        x = torch.ones(n_bytes // EB[kind], dtype=dt, device=device)
        x.view(n_groups, loads, 64, per_vec)[:n_waves, 0, :, 0] = 2.0**24
        n_big = n_waves * 64
        n_small = n_bytes // EB[kind] - n_big
        return x.view(torch.uint8), n_big * 2**24 + n_small, float(n_small)
    assert n_groups >= (BIG_ROUNDS + 1) * n_waves
    u = torch.zeros(n_bytes, dtype=torch.uint8, device=device)
    g = u.view(n_groups, loads, 64, 16)
    big = BIG_ROUNDS * n_waves
    g[:big] = 0x7E                              # 448
    g[big:, 0::4, :, 0] = 0x01                  # 2**-9, first vector of each chunk
    tiny = (n_groups - big) * (loads // 4) * 64
    exact = big * group_bytes * 448 + tiny * 2.0**-9
    return u, exact, tiny * 2.0**-9


def kernel_lanes(kind, payload_u8, n_waves, loads):
    """The terms every lane adds, in order, grouped as the scheme model
    takes them (a list over workgroups of 256 lanes).  FP8 lanes add the
    binary32 sum of each chunk of four vectors (exact for e4m3)."""
    b = payload_u8.cpu().numpy()
    n_groups = b.size // (loads * 1024)
    if kind == "f32":
        vals = b.view(np.float32)
    elif kind == "bf16":
        vals = (b.view(np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)
    else:
        vals = torch.from_numpy(b.copy()).view(torch.float8_e4m3fn).float().numpy()
    per = 16 // EB[kind]
    V = vals.reshape(n_groups, loads, 64, per)
    waves = []
    for wid in range(n_waves):
        lanes = []
        for lane in range(64):
            terms = []
            for g in range(wid, n_groups, n_waves):
                if kind == "fp8_e4m3":
                    for q in range(loads // 4):
                        chunk = V[g, 4 * q:4 * q + 4, lane].ravel()
                        terms.append(np.float32(np.add.reduce(chunk, dtype=np.float32)))
                else:
                    terms.extend(V[g, :, lane].ravel())
            lanes.append(terms)
        waves.append(lanes)
    return [[t for k in range(4) for t in waves[4 * w + k]] for w in range(n_waves // 4)]
