"""HIP-graph capture of the single-buffer entry points and the fused decode:
one graph holds b64_encode, b64_decode_async, b64_validate_async and
b64_decode_f32_bf16; it is replayed several times with new input contents
(valid and invalid, in turn) and eager work between the replays, and every
replay is checked against the oracle.  The status words hold garbage before
each replay (the captured decode and validation keep their running status in
a status slot of their own, and no memset nodes are recorded)."""
import numpy as np
import pytest

import workloads
from gpu_util import first_mismatch, say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


def test_single_and_fused_in_one_graph(b64, oracle):
    import torch
    n = 1_000_003
    dim, nrows = 96, 300
    xs = [workloads.random_bytes(workloads.SEED_BASE + 260 + k, n) for k in range(4)]
    texts = [oracle.encode(x) for x in xs]
    bad_pos = [None, 12345, None, len(texts[3]) - 2]
    for k, p in enumerate(bad_pos):
        if p is not None:
            texts[k] = texts[k].copy()
            texts[k][p] = ord("*")
    rows_raw = [workloads.random_bytes(workloads.SEED_BASE + 270 + k, 4 * dim * nrows) for k in range(4)]
    r_off = workloads.offsets(np.full(nrows, 4 * dim, dtype=np.int64))
    rows_txt = [oracle.encode_mode_list(r, r_off)[:2] for r in rows_raw]

    N = texts[0].size
    x_dev = torch.zeros(n, dtype=torch.uint8, device="cuda")
    enc_out = torch.zeros(N, dtype=torch.uint8, device="cuda")
    t_dev = torch.zeros(N, dtype=torch.uint8, device="cuda")
    dec_out = torch.zeros(n + 3, dtype=torch.uint8, device="cuda")
    st_dec = torch.zeros(2, dtype=torch.int64, device="cuda")
    st_val = torch.zeros(2, dtype=torch.int64, device="cuda")
    R = rows_txt[0][0].size
    r_dev = torch.zeros(R, dtype=torch.uint8, device="cuda")
    r_off_dev = to_dev(rows_txt[0][1])
    f_out = torch.zeros((nrows, dim), dtype=torch.bfloat16, device="cuda")
    f_st = torch.zeros(nrows, dtype=torch.int64, device="cuda")

    def work():
        b64.encode(x_dev, out=enc_out)
        b64.decode_async(t_dev, out=dec_out, status=st_dec)
        b64.validate_async(t_dev, status=st_val)
        b64.decode_f32_bf16(r_dev, r_off_dev, dim, dst=f_out, status=f_st, validate=False)

    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        work()                                                # warm up outside the capture
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    say("graph capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    for rep in range(8):
        k = rep % 4
        say("graph replay", rep, "case", k)
        x_dev.copy_(to_dev(xs[k]))
        t_dev.copy_(to_dev(texts[k]))
        r_dev.copy_(to_dev(rows_txt[k][0]))
        for t in (enc_out, dec_out, f_out):
            t.zero_()
        st_dec.fill_(123)
        st_val.fill_(456)
        f_st.fill_(789)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert first_mismatch(to_host(enc_out), oracle.encode(xs[k])) is None, rep
        want = [n, -1] if bad_pos[k] is None else [-1, bad_pos[k]]
        assert to_host(st_dec).tolist() == want, (rep, to_host(st_dec))
        assert to_host(st_val).tolist() == want, (rep, to_host(st_val))
        if bad_pos[k] is None:
            assert first_mismatch(to_host(dec_out)[:n], xs[k]) is None, rep
        ref, ref_st = oracle.decode_f32_bf16_rows(rows_txt[k][0], rows_txt[k][1], dim)
        assert (to_host(f_st) == ref_st).all(), rep
        assert (to_host(f_out.view(torch.int16)).view(np.uint16) == ref).all(), rep
