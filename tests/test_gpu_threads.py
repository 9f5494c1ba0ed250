"""Concurrent callers: four host threads, each on its own HIP stream, call
the library at once (encode, blocking and asynchronous decode, validation,
the whitespace-skipping decode with its per-thread workspace, a batch), many
times over.  Every result must equal the oracle's, as when each runs alone:
the library's per-thread status slots and workspaces, and its launch-shape
table behind a lock, keep the calls apart."""
import threading

import numpy as np
import pytest

import workloads
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"
NOPAD, SKIP_WS = 1, 2
ROUNDS = 25


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


def test_four_threads_four_streams(b64, oracle):
    import torch
    g = workloads.rng(workloads.SEED_BASE + 270)
    # per thread: (kind, input bytes, alphabet, flags), expected values from the oracle
    jobs = []
    x0 = workloads.random_bytes(workloads.SEED_BASE + 271, (3 << 20) + 1)
    t0 = oracle.encode(x0, STD)
    bad0, _ = workloads.plant_invalid(t0, workloads.SEED_BASE + 272, STD)
    jobs.append(("plain", x0, t0, bad0, ~oracle.decode_mode_raw(bad0, STD, 0), STD, 0))
    x1 = workloads.random_bytes(workloads.SEED_BASE + 273, (1 << 20) + 2)
    t1 = oracle.encode_mode(x1, URL, NOPAD)
    bad1, _ = workloads.plant_invalid(t1, workloads.SEED_BASE + 274, URL)
    jobs.append(("nopad", x1, t1, bad1, ~oracle.decode_mode_raw(bad1, URL, NOPAD), URL, NOPAD))
    x2 = workloads.random_bytes(workloads.SEED_BASE + 275, 2 << 20)
    t2 = workloads.sprinkle_ws(oracle.encode_mode(x2, STD, 0, workloads.MIME_LINE),
                               workloads.SEED_BASE + 276, 2000)
    bad2 = t2.copy()
    p2 = int(g.integers(0, bad2.size))
    while bad2[p2] in b" \t\r\n":
        p2 += 1
    bad2[p2] = ord("*")
    jobs.append(("ws", x2, t2, bad2, ~oracle.decode_mode_raw(bad2, STD, SKIP_WS), STD, SKIP_WS))
    lens = workloads.batch_lengths(workloads.SEED_BASE + 277, 500, 1, 20000)
    in_off = workloads.offsets(lens)
    x3 = workloads.random_bytes(workloads.SEED_BASE + 278, int(in_off[-1]))
    ref_dst, ref_off, ref_len = oracle.encode_mode_list(x3, in_off, STD, 0)
    jobs.append(("batch", x3, (ref_dst, ref_off, ref_len, in_off), None, None, STD, 0))

    errors = []

    def run(job):
        kind, x, t, bad, pos, alpha, flags = job
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                dx = to_dev(x)
                if kind == "batch":
                    ref_dst, ref_off, ref_len, in_off = t
                    d_off, d_ref = to_dev(in_off), to_dev(ref_dst)
                    for _ in range(ROUNDS):
                        dst, out_off, out_len = b64.encode_batch(dx, d_off, alpha)
                        assert torch.equal(dst[: ref_dst.size], d_ref)
                        dec, dout_off, dlen, dbad = b64.decode_batch(dst, out_off, alpha)
                        assert (dbad == -1).all().item()
                        assert (dlen.cpu().numpy() == np.diff(in_off)).all()
                        h, ho = dec.cpu().numpy(), dout_off.cpu().numpy()
                        for k in range(in_off.size - 1):
                            n_k = int(in_off[k + 1] - in_off[k])
                            assert (h[ho[k]: ho[k] + n_k] == x[in_off[k]: in_off[k + 1]]).all(), k
                    return
                dt, dbad_t = to_dev(t), to_dev(bad)
                for _ in range(ROUNDS):
                    if kind != "ws":
                        enc = b64.encode(dx, alpha, flags=flags)
                        assert torch.equal(enc, dt)
                    out, b = b64.decode(dt, alpha, flags=flags)
                    assert b is None and torch.equal(out, dx)
                    _, b = b64.decode(dbad_t, alpha, flags=flags)
                    assert b == pos, (kind, b, pos)
                    out2, st = b64.decode_async(dt, alpha, flags=flags)
                    s.synchronize()
                    assert st.cpu().tolist() == [x.size, -1] and torch.equal(out2[: x.size], dx)
                    assert b64.validate(dbad_t, alpha, flags=flags) == (None, pos)
        except BaseException as exc:      # reported by the main thread
            errors.append((kind, repr(exc)))

    say("threads", [j[0] for j in jobs], "rounds", ROUNDS)
    threads = [threading.Thread(target=run, args=(j,)) for j in jobs]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=100)
    assert not any(th.is_alive() for th in threads), "a caller thread did not finish"
    assert not errors, errors
