"""The serving loop: every request's result in the coalesced mix equals its
result alone (single-buffer entry points) and the oracle's, bit-exact; the
loop coalesces, overlaps launches and respects its HBM budget."""
import numpy as np
import pytest

import workloads
from gpu_util import first_mismatch, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


@pytest.mark.parametrize("budget,rate", [(1 << 30, 2e4), (96 << 10, 5e4)],
                         ids=["roomy", "tight_budget"])
def test_mix_equals_alone(b64, oracle, budget, rate):
    import torch
    from paper_1910_05109_amd import serve
    seed = workloads.SEED_BASE + 140
    count = 800
    sizes = workloads.serve_sizes(seed, count, median=2048, sigma=1.5)
    sizes = np.minimum(sizes, 40_000)
    is_dec, is_bad = workloads.serve_kinds(seed + 1, count, invalid_frac=0.05)
    arrival = workloads.serve_arrivals(seed + 2, count, rate)
    kinds = is_dec.astype(np.int64)
    enc_idx, dec_idx = np.nonzero(~is_dec)[0], np.nonzero(is_dec)[0]
    pos = np.zeros(count, dtype=np.int64)
    pos[enc_idx] = np.arange(enc_idx.size)
    pos[dec_idx] = np.arange(dec_idx.size)
    raw = workloads.random_bytes(seed + 3, int(sizes.sum()))
    roff = workloads.offsets(sizes)
    payload = [raw[roff[i]:roff[i + 1]] for i in range(count)]
    # decode requests carry the oracle's encoding, some spoiled by one byte
    g = workloads.rng(seed + 4)
    bad_bytes = workloads.non_alphabet_bytes(oracle.STD)
    for i in dec_idx:
        t = oracle.encode(payload[i])
        if is_bad[i] and t.size:
            t = t.copy()
            t[g.integers(0, t.size)] = bad_bytes[g.integers(0, bad_bytes.size)]
        payload[i] = t
    enc_data = np.concatenate([payload[i] for i in enc_idx])
    dec_data = np.concatenate([payload[i] for i in dec_idx])
    enc_pool = serve.make_pool(serve.ENC, to_dev(enc_data), sizes[enc_idx])
    dec_pool = serve.make_pool(serve.DEC, to_dev(dec_data), np.array([payload[i].size for i in dec_idx]))

    served = {}

    def on_retire(L, srv):
        pool = srv.pools[L.kind]
        base = int(pool.out_rel[L.first])
        n = int(pool.out_rel[L.first + L.count]) - base
        region = to_host(srv.arena[L.start: L.start + n])
        for k in range(L.first, L.first + L.count):
            served[(L.kind, k)] = region[int(pool.out_rel[k]) - base: int(pool.out_rel[k + 1]) - base]

    say("serve", budget, rate)
    srv = serve.Server(enc_pool, dec_pool, budget_bytes=budget, max_inflight=3, max_batch=64,
                       on_retire=on_retire)
    stats = srv.run(kinds, arrival, pos)
    torch.cuda.synchronize()
    summ = stats.summary()
    say("serve summary", summ)
    assert np.isfinite(stats.latency).all() and (stats.latency >= 0).all()
    assert summ["launches"] < count and summ["mean_batch"] > 1.0     # coalescing happened
    assert summ["peak_arena_used"] <= srv.arena_bytes <= max(budget, 1 << 20)
    enc_len, _ = srv.results(serve.ENC)
    dec_len, dec_bad = srv.results(serve.DEC)
    for i in range(count):
        k = pos[i]
        if kinds[i] == serve.ENC:
            alone = to_host(b64.encode(to_dev(payload[i]))) if payload[i].size else np.zeros(0, np.uint8)
            ref = oracle.encode(payload[i])
            assert enc_len[k] == ref.size
            mixed = served[(serve.ENC, k)][: ref.size]
            assert first_mismatch(mixed, ref) is None, i
            assert first_mismatch(alone, ref) is None, i
        else:
            ref, ref_bad = oracle.decode(payload[i])
            import torch as _t
            dt = to_dev(payload[i]) if payload[i].size else _t.empty(0, dtype=_t.uint8, device="cuda")
            alone, alone_bad = b64.decode(dt)
            assert alone_bad == ref_bad
            if ref_bad is None:
                assert dec_bad[k] == -1 and dec_len[k] == ref.size, i
                assert first_mismatch(served[(serve.DEC, k)][: ref.size], ref) is None, i
                assert first_mismatch(to_host(alone), ref) is None, i
            else:
                assert dec_bad[k] == ref_bad and dec_len[k] == -1, i
