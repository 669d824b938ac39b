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
