"""Helpers for the GPU parity tests: device transfer and case labelling."""
import sys

import numpy as np


def say(*parts):
    """Print (and flush) what the next GPU step is, so a failing run names it."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t) -> np.ndarray:
    return t.cpu().numpy()


def first_mismatch(a: np.ndarray, b: np.ndarray):
    if a.size != b.size:
        return f"size {a.size} != {b.size}"
    idx = np.nonzero(a != b)[0]
    return None if idx.size == 0 else f"{idx.size} mismatches, first at {idx[0]}"
