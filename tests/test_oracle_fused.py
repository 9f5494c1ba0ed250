"""Pins for the oracle's fused consumer (CPU only): rows of base64-encoded
float32 decoded into bfloat16.

  - The float32 -> bfloat16 rounding against PyTorch's own CPU conversion (a
    library routine) for every non-NaN input: special values, every dropped
    half-word for an even and an odd kept half, and random bit patterns.
    NaN inputs (numpy's isnan) become the canonical quiet NaN 0x7FC0, the
    rule of PyTorch's scalar bfloat16 type; its vectorized CPU path writes
    0xFFFF instead, so NaN lanes are compared with the rule, not with it.
  - Whole rows against the standard-library decoder followed by the same
    PyTorch conversion; invalid rows against the pinned decoder's first
    invalid offset; rows of the wrong length.
"""
import base64

import numpy as np
import torch

import workloads

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"


def torch_bf16(bits: np.ndarray) -> np.ndarray:
    bits = np.ascontiguousarray(bits, dtype=np.uint32)
    f = torch.from_numpy(bits.view(np.float32))
    out = f.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16).copy()
    out[np.isnan(bits.view(np.float32))] = 0x7FC0
    return out


def test_rounding_matches_torch(oracle):
    specials = np.array([0, 0x80000000, 0x3F800000, 0xBF800000, 0x7F800000, 0xFF800000,
                         0x7F7FFFFF, 0xFF7FFFFF, 0x00000001, 0x807FFFFF, 0x7FC00000, 0xFFC00000,
                         0x7F800001, 0xFF800001, 0x7FFFFFFF, 0x3F808000, 0x3F818000, 0x3F807FFF,
                         0x3F808001, 0x7F7F8000, 0x7F7F7FFF], dtype=np.uint32)
    assert (oracle.f32_to_bf16(specials) == torch_bf16(specials)).all()
    # every dropped half-word, kept half even (0x3F80) and odd (0x3F81)
    low = np.arange(1 << 16, dtype=np.uint32)
    for hi in (0x3F80, 0x3F81, 0x7F7F, 0x0000, 0x807F):
        bits = (np.uint32(hi) << np.uint32(16)) | low
        assert (oracle.f32_to_bf16(bits) == torch_bf16(bits)).all(), hex(hi)
    rnd = workloads.random_bytes(workloads.SEED_BASE + 201, 4 * 100000).view(np.uint32)
    assert (oracle.f32_to_bf16(rnd) == torch_bf16(rnd)).all()


def _rows(seed, nrows, dim, flags=0):
    raw = workloads.random_bytes(seed, 4 * dim * nrows).reshape(nrows, 4 * dim)
    texts = [base64.b64encode(r.tobytes()) for r in raw]
    if flags & 1:
        texts = [t.rstrip(b"=") for t in texts]
    return raw, texts


def test_rows_match_stdlib_and_torch(oracle):
    for dim, flags in ((1, 0), (3, 1), (7, 0), (96, 0), (96, 1), (385, 0)):
        raw, texts = _rows(workloads.SEED_BASE + 202 + dim, 13, dim, flags)
        src = np.frombuffer(b"".join(texts), dtype=np.uint8)
        in_off = workloads.offsets(np.array([len(t) for t in texts], dtype=np.int64))
        dst, status = oracle.decode_f32_bf16_rows(src, in_off, dim, STD, flags)
        assert (status == -1).all()
        ref = torch_bf16(raw.reshape(-1).view(np.uint32)).reshape(13, dim)
        assert (dst == ref).all(), (dim, flags)


def test_invalid_and_wrong_length_rows(oracle):
    dim = 10
    raw, texts = _rows(workloads.SEED_BASE + 210, 7, dim)
    texts[1] = texts[1][:5] + b"*" + texts[1][6:]          # invalid byte at 5
    texts[2] = base64.b64encode(raw[2].tobytes()[:-4])     # valid, 4 bytes short
    texts[3] = texts[3][:-1]                               # truncated
    texts[4] = b""                                         # empty row
    texts[6] = base64.b64encode(raw[6].tobytes() + b"1234")  # valid, 4 bytes long
    src = np.frombuffer(b"".join(texts), dtype=np.uint8)
    in_off = workloads.offsets(np.array([len(t) for t in texts], dtype=np.int64))
    dst, status = oracle.decode_f32_bf16_rows(src, in_off, dim)
    assert status.tolist() == [-1, 5, -2, len(texts[3]), -2, -1, -2]
    assert status[3] == ~oracle.decode_raw(np.frombuffer(texts[3], dtype=np.uint8))
    ref = torch_bf16(raw.reshape(-1).view(np.uint32)).reshape(7, dim)
    assert (dst[0] == ref[0]).all() and (dst[5] == ref[5]).all()
