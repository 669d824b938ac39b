"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds none of the method's arithmetic: it only draws seeded
random data with torch's generators, on the CPU or on a GPU, and hands the
same bytes to both the HIP path and the CPU oracle.

Recipes
-------
``random_bytes``  uniform bytes (any 32-bit word pattern), for checksum
                  parity independent of the library's own seeded fill.
``normal_payload``  N(0, 1) samples drawn in FP32 and stored as FP32, BF16
                  (round to nearest even) or FP8 e4m3fn (clamped to +-448,
                  then round to nearest even), as raw little-endian bytes.
``chase_chain``   a pointer-chase chain: one node per ``stride`` bytes of a
                  ``footprint``-byte buffer, linked in a seeded random order
                  into a single cycle; each node's first 32-bit word holds
                  the word index of the next node.
"""
import torch

DTYPES = {"f32": torch.float32, "bf16": torch.bfloat16,
          "fp8_e4m3": torch.float8_e4m3fn}
ELEM_BYTES = {"f32": 4, "bf16": 2, "fp8_e4m3": 1}


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def random_bytes(nbytes, seed, device="cpu"):
    """uint8 tensor of ``nbytes`` uniform random bytes."""
    g = _gen(seed, device)
    return torch.randint(0, 256, (int(nbytes),), dtype=torch.uint8,
                         generator=g, device=device)


def normal_payload(kind, n, seed, device="cpu", chunk=1 << 26):
    """uint8 tensor holding ``n`` N(0,1) values stored as ``kind``."""
    dt = DTYPES[kind]
    eb = ELEM_BYTES[kind]
    out = torch.empty(int(n) * eb, dtype=torch.uint8, device=device)
    g = _gen(seed, device)
    view = out.view(dt) if n else None
    for s in range(0, int(n), chunk):
        c = min(chunk, int(n) - s)
        x = torch.randn(c, dtype=torch.float32, generator=g, device=device)
        if kind == "fp8_e4m3":
            x = x.clamp_(-448.0, 448.0)
        view[s:s + c] = x.to(dt)
    return out


def _chase_cycle(footprint, stride, seed, device):
    if footprint % stride or stride % 4:
        raise ValueError("footprint must be a multiple of stride, stride of 4")
    n = footprint // stride
    step = stride // 4
    g = _gen(seed, device)
    order = torch.randperm(n, generator=g, device=device, dtype=torch.int64)
    words = torch.zeros(footprint // 4, dtype=torch.int32, device=device)
    nxt = torch.roll(order, -1)
    words[order * step] = (nxt * step).to(torch.int32)
    return words.view(torch.uint8), order, step


def chase_chain(footprint, stride, seed, device="cpu"):
    """(uint8 tensor of ``footprint`` bytes, start word index): one cycle
    through every ``stride``-byte node in random order."""
    words, order, step = _chase_cycle(footprint, stride, seed, device)
    return words, int(order[0].item()) * step


def chase_chain_starts(footprint, stride, seed, n_starts, device="cpu"):
    """The same chain as ``chase_chain`` and ``n_starts`` word indices spread
    evenly along its cycle (start i is i * nodes / n_starts hops on)."""
    words, order, step = _chase_cycle(footprint, stride, seed, device)
    n = order.numel()
    if not 1 <= n_starts <= n:
        raise ValueError("n_starts must be 1..nodes")
    starts = [int(order[(i * n) // n_starts].item()) * step for i in range(n_starts)]
    return words, starts
