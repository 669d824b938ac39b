"""Helpers for the GPU tests: device buffers and wave-record decoding."""
import numpy as np
import torch

REC_DTYPE = np.dtype([("sum32", "<u4"), ("xor32", "<u4"), ("hw_id", "<u4"),
                      ("xcc_id", "<u4"), ("t0", "<u8"), ("t1", "<u8")])


def dev_bytes(n):
    return torch.empty(int(n), dtype=torch.uint8, device="cuda")


def recs(n_waves):
    return torch.zeros(int(n_waves) * REC_DTYPE.itemsize, dtype=torch.uint8,
                       device="cuda")


def decode_recs(t):
    return t.cpu().numpy().view(REC_DTYPE)


def lanes(n_threads):
    return torch.zeros(int(n_threads) * 2, dtype=torch.int32, device="cuda")


def decode_lanes(t, n_waves):
    a = t.cpu().numpy().view(np.uint32).reshape(n_waves, 64, 2)
    return a[..., 0], a[..., 1]


def host_words(buf):
    return buf.cpu().numpy().view(np.uint32)


def reduce_lane_terms(kind, n, waves, waves_per_cu):
    """Upper bound on the TwoSum terms one lane of the streaming sum adds:
    its share of the full wave-groups (8 loads per lane at 4 waves per CU,
    4 above; FP8 adds one term per four vectors), one remainder vector and
    the trailing elements."""
    per_vec = {"f32": 4, "bf16": 8, "fp8_e4m3": 16}[kind]
    eb = {"f32": 4, "bf16": 2, "fp8_e4m3": 1}[kind]
    loads = 8 if waves_per_cu == 4 else 4
    groups = (n * eb // 16) // (64 * loads)
    g_lane = -(-groups // waves) if waves else 0
    per_group = loads * per_vec if kind != "fp8_e4m3" else loads // 4
    return g_lane * per_group + per_vec + 16
