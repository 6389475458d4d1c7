"""Shared helpers for the GPU tests: numpy <-> device tensors, seeded tables."""
import numpy as np

import datagen


def dev(a: np.ndarray):
    """Device copy of a uint32/uint64 numpy array (as int32/int64 bits)."""
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    elif a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).cuda()


def host_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def host_u64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def host_u8(t) -> np.ndarray:
    return t.cpu().numpy().astype(np.uint8)


def workload(n: int, seed: int):
    return datagen.unique_keys(n, seed), datagen.values(n, seed)
