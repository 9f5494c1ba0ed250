"""GPU parity of the fused consumer (b64_decode_f32_bf16) against the oracle:
rows of base64 float32 decoded straight into bfloat16, bit for bit, with the
same per-row status (good, first invalid offset, wrong length)."""
import numpy as np
import pytest

import workloads
from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"
NOPAD = 1


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


def _rows(oracle, seed, nrows, dim, alpha, flags):
    raw = workloads.random_bytes(seed, 4 * dim * nrows)
    in_off = workloads.offsets(np.full(nrows, 4 * dim, dtype=np.int64))
    text, t_off, _ = oracle.encode_mode_list(raw, in_off, alpha, flags)
    return text, t_off


def _check(b64, oracle, text, t_off, dim, alpha, flags, label):
    import torch
    say("fused", label, "rows", t_off.size - 1, "dim", dim, "flags", flags)
    ref, ref_st = oracle.decode_f32_bf16_rows(text, t_off, dim, alpha, flags)
    src = to_dev(text) if text.size else torch.zeros(1, dtype=torch.uint8, device="cuda")
    out, st = b64.decode_f32_bf16(src, to_dev(t_off), dim, alpha, flags=flags)
    st = to_host(st)
    assert (st == ref_st).all(), (label, np.nonzero(st != ref_st)[0][:5])
    got = to_host(out.view(torch.int16)).view(np.uint16)
    good = ref_st == -1
    assert (got[good] == ref[good]).all(), (label, np.argwhere(got[good] != ref[good])[:5])


@pytest.mark.parametrize("dim", [1, 2, 3, 4, 5, 7, 96, 384, 1536, 3072])
@pytest.mark.parametrize("flags", [0, NOPAD])
def test_dims(b64, oracle, dim, flags):
    nrows = max(8, 200000 // (4 * dim))
    alpha = URL if flags else STD
    text, t_off = _rows(oracle, workloads.SEED_BASE + 220 + dim, nrows, dim, alpha, flags)
    _check(b64, oracle, text, t_off, dim, alpha, flags, f"dim {dim}")


def test_bad_rows(b64, oracle):
    dim = 96
    nrows = 400
    text, t_off = _rows(oracle, workloads.SEED_BASE + 240, nrows, dim, STD, 0)
    g = workloads.rng(workloads.SEED_BASE + 241)
    rows = [text[t_off[b]:t_off[b + 1]].copy() for b in range(nrows)]
    bad = workloads.non_alphabet_bytes(STD)
    for b in range(0, nrows, 7):
        kind = int(g.integers(0, 6))
        r = rows[b]
        if kind == 0:                                        # invalid byte anywhere
            r[int(g.integers(0, r.size))] = bad[int(g.integers(0, bad.size))]
        elif kind == 1:                                      # '=' in the body
            r[int(g.integers(0, r.size - 4))] = ord("=")
        elif kind == 2:                                      # truncated
            rows[b] = r[: r.size - int(g.integers(1, 8))]
        elif kind == 3:                                      # valid, 4 bytes short
            rows[b] = oracle.encode(workloads.random_bytes(b, 4 * dim - 4))
        elif kind == 4:                                      # valid, 4 bytes long
            rows[b] = oracle.encode(workloads.random_bytes(b, 4 * dim + 4))
        else:                                                # empty row
            rows[b] = r[:0]
    text = np.concatenate(rows)
    t_off = workloads.offsets(np.array([r.size for r in rows], dtype=np.int64))
    _check(b64, oracle, text, t_off, dim, STD, 0, "bad rows")


def test_embeddings_64k_rows(b64, oracle):
    """65,536 rows of 1,536 float32 (the bench workload: 512 MiB of text)."""
    dim, nrows = 1536, 65536
    text, t_off = _rows(oracle, workloads.SEED_BASE + 250, nrows, dim, STD, 0)
    _check(b64, oracle, text, t_off, dim, STD, 0, "64k x 1536")
