"""GPU parity of every launch shape b64_tune_set accepts, for every operation,
against the oracle, bit-exact.

A launch shape is (lane chunks in flight per lane 1/2/4/8, workgroups per
compute unit, nontemporal loads and stores on/off); the header promises that
it never changes results.  Each operation runs under every unroll x
nontemporal pair with 1, 3, 8 and 64 workgroups per CU on edge inputs: every
length to 48 and the lengths around wave and round edges, sources and
destinations at every byte offset mod 4, inputs large enough for several
grid-stride rounds, invalid bytes and misplaced '=' at chunk edges and in the
final quanta, ragged batches with empty and one-byte buffers, rows of the
fused consumer with bad rows.  Expected values come from the oracle once per
module; each shape's outputs are compared with them on the device.
"""
import numpy as np
import pytest

import workloads
from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
NOPAD, SKIP_WS = 1, 2
SHAPES = [(u, bpc, nt) for u in (1, 2, 4, 8) for bpc in (1, 3, 8, 64) for nt in (0, 1)]
SHAPE_IDS = [f"u{u}-b{b}-nt{nt}" for u, b, nt in SHAPES]
SMALL_LENGTHS = list(range(0, 49)) + [95, 96, 97, 767, 768, 769, 3071, 3072, 3073, 12287, 12288,
                                      12289, 49151, 49152, 49153, 100003]
# large enough that every unroll takes the streaming grid (more than 16
# workgroups per CU would be needed to cover it in one round), with several
# grid-stride rounds at 1 and 3 workgroups per CU
BIG_N = (128 << 20) + 1
MIS_N = (5 << 20) + 2             # misaligned source and destination
GUARD = 64


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


class _Shape:
    """Set op's launch shape for the duration of a with-block."""

    def __init__(self, b64, op, shape):
        self.b64, self.op, self.shape = b64, op, shape

    def __enter__(self):
        self.old = self.b64.tune_shapes(self.op)
        self.b64.tune_set(self.op, *self.shape)          # every size bucket

    def __exit__(self, *exc):
        self.b64.tune_restore(self.op, self.old)


def _place(parts, misalign=True):
    """Offsets of `parts` packed with guard gaps (each start at a different
    offset mod 4 when `misalign`); returns (offsets, total)."""
    offs, pos = [], GUARD
    for i, p in enumerate(parts):
        pos = (pos + 7) // 8 * 8 + (i % 4 if misalign else 0)
        offs.append(pos)
        pos += len(p) + GUARD
    return offs, pos + GUARD


def _arena(parts, offs, total):
    a = np.zeros(total, dtype=np.uint8)
    for o, p in zip(offs, parts):
        a[o:o + len(p)] = p
    return a


def _spoil_cases(oracle, texts, seed):
    """Invalid copies of encodings: a byte outside the alphabet at a seeded
    position, at a 16-character chunk edge and in the final quantum, and '='
    at a chunk edge inside the body."""
    g = workloads.rng(seed)
    outside = workloads.non_alphabet_bytes(STD)
    out = []
    for t in texts:
        if t.size < 8:
            continue
        for where in ("seeded", "edge", "final", "pad_edge"):
            s = t.copy()
            if where == "seeded":
                p = int(g.integers(0, s.size))
            elif where == "edge":
                p = int(g.integers(0, max(s.size // 16, 1))) * 16
                p = min(p, s.size - 1)
            elif where == "final":
                p = s.size - 1 - int(g.integers(0, 4))
            else:
                p = max(0, (s.size - 8) // 16 * 16 - 16 * int(g.integers(0, 4)))
            s[p] = ord("=") if where == "pad_edge" else outside[int(g.integers(0, outside.size))]
            out.append(s)
    return out


@pytest.fixture(scope="module")
def single(oracle):
    """Inputs and expected results of the single-buffer operations."""
    import torch
    x = workloads.random_bytes(workloads.SEED_BASE + 300, BIG_N + 8)
    small = [x[:n] for n in SMALL_LENGTHS]
    enc_small = [oracle.encode(p) for p in small]
    src_offs, src_total = _place(small)
    out_offs, out_total = _place(enc_small)
    d = {"x": x, "dx": to_dev(x), "small": small, "src_offs": src_offs,
         "d_src_small": to_dev(_arena(small, src_offs, src_total)),
         "enc_offs": out_offs, "enc_total": out_total,
         "exp_enc_small": to_dev(_arena(enc_small, out_offs, out_total))}
    big_text = oracle.encode(x[:BIG_N])
    mis_text = oracle.encode(x[:MIS_N])
    d["big_text"], d["mis_text"] = to_dev(big_text), to_dev(mis_text)
    # decode / validate cases: the small encodings, their invalid copies, the
    # encodings cut short by 1..3 characters, and the big text with spoils
    texts = list(enc_small) + _spoil_cases(oracle, enc_small[4:], workloads.SEED_BASE + 301)
    texts += [t[:-k] for t in enc_small[8:20] for k in (1, 2, 3)]
    res = [oracle.decode(t) for t in texts]
    dec_parts = [r[0] if r[0] is not None else np.zeros(0, np.uint8) for r in res]
    t_offs, t_total = _place(texts)
    o_offs, o_total = _place([np.zeros(3 * (t.size // 4), np.uint8) for t in texts])
    d.update({"texts": texts, "t_offs": t_offs, "d_texts": to_dev(_arena(texts, t_offs, t_total)),
              "o_offs": o_offs, "o_total": o_total,
              "exp_dec": to_dev(_arena(dec_parts, o_offs, o_total)),
              "exp_status": np.array([[r[0].size, -1] if r[1] is None else [-1, r[1]] for r in res],
                                     dtype=np.int64)})
    # the big text spoiled near its middle (by a seeded byte) and '=' in a late chunk
    big_bad = []
    for seed, lo, hi in ((302, big_text.size // 3, 2 * big_text.size // 3),
                         (303, big_text.size - 4096, big_text.size - 8)):
        s, p = workloads.plant_invalid(big_text, workloads.SEED_BASE + seed, STD, lo, hi)
        big_bad.append((to_dev(s), p))
    s = big_text.copy()
    p = (big_text.size - 200) // 16 * 16
    s[p] = ord("=")
    big_bad.append((to_dev(s), int(~oracle.decode_raw(s))))
    d["big_bad"] = big_bad
    torch.cuda.synchronize()
    return d


SHAPE_PARAMS = pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)


@SHAPE_PARAMS
def test_encode_shapes(b64, single, shape):
    import torch
    d = single
    with _Shape(b64, "encode", shape):
        say("shape encode", shape)
        arena = torch.zeros(d["enc_total"], dtype=torch.uint8, device="cuda")
        for n, so, oo in zip(SMALL_LENGTHS, d["src_offs"], d["enc_offs"]):
            m = 4 * ((n + 2) // 3)
            b64.encode(d["d_src_small"][so:so + n], out=arena[oo:oo + m])
        assert torch.equal(arena, d["exp_enc_small"]), shape
        big = b64.encode(d["dx"][:BIG_N])
        assert torch.equal(big, d["big_text"]), shape
        M = d["mis_text"].numel()
        buf = torch.zeros(M + 8, dtype=torch.uint8, device="cuda")
        b64.encode(d["dx"][:MIS_N], out=buf[3:3 + M])
        assert torch.equal(buf[3:3 + M], d["mis_text"]) and not bool(buf[:3].any()), shape
        assert not bool(buf[3 + M:].any()), shape


@SHAPE_PARAMS
def test_encode_misaligned_source_shapes(b64, oracle, single, shape):
    """A source that starts 1..3 bytes past a 4-byte boundary."""
    import torch
    d = single
    with _Shape(b64, "encode", shape):
        for so in (1, 2, 3):
            say("shape encode misaligned source", shape, so)
            if ("mis_src", so) not in d:
                d[("mis_src", so)] = to_dev(oracle.encode(d["x"][so:so + MIS_N]))
            exp = d[("mis_src", so)]
            got = b64.encode(d["dx"][so:so + MIS_N])
            assert torch.equal(got, exp), (shape, so)


def _decode_all(b64, d, status, arena):
    for i, (t, to, oo) in enumerate(zip(d["texts"], d["t_offs"], d["o_offs"])):
        cap = 3 * (t.size // 4)
        b64.decode_async(d["d_texts"][to:to + t.size], out=arena[oo:oo + cap],
                         status=status[2 * i:2 * i + 2])


@SHAPE_PARAMS
def test_decode_shapes(b64, single, shape):
    import torch
    d = single
    ncase = len(d["texts"])
    with _Shape(b64, "decode", shape):
        say("shape decode", shape, ncase, "cases")
        arena = torch.zeros(d["o_total"], dtype=torch.uint8, device="cuda")
        status = torch.empty(2 * ncase, dtype=torch.int64, device="cuda")
        _decode_all(b64, d, status, arena)
        st = to_host(status).reshape(-1, 2)
        bad = np.nonzero((st != d["exp_status"]).any(axis=1))[0]
        assert bad.size == 0, (shape, bad[:5], st[bad[:5]], d["exp_status"][bad[:5]])
        # outputs of invalid inputs are unspecified: compare the valid ones
        valid = np.zeros(d["o_total"], dtype=bool)
        for (ln, fb), oo in zip(d["exp_status"], d["o_offs"]):
            if fb == -1:
                valid[oo:oo + ln] = True
        mask = to_dev(valid)
        assert torch.equal(arena[mask], d["exp_dec"][mask]), shape
        say("shape decode big", shape)
        out, bad_ = b64.decode(d["big_text"])
        assert bad_ is None and torch.equal(out, d["dx"][:BIG_N]), shape
        for s, p in d["big_bad"]:
            _, st2 = b64.decode_async(s)
            assert to_host(st2).tolist() == [-1, p], (shape, p)
        M = d["mis_text"].numel()
        tbuf = torch.zeros(M + 4, dtype=torch.uint8, device="cuda")
        tbuf[2:2 + M].copy_(d["mis_text"])
        obuf = torch.zeros(MIS_N + 8, dtype=torch.uint8, device="cuda")
        _, st3 = b64.decode_async(tbuf[2:2 + M], out=obuf[1:1 + 3 * (M // 4)])
        assert to_host(st3).tolist() == [MIS_N, -1], shape
        assert torch.equal(obuf[1:1 + MIS_N], d["dx"][:MIS_N]) and not bool(obuf[0]), shape


@SHAPE_PARAMS
def test_validate_shapes(b64, single, shape):
    import torch
    d = single
    ncase = len(d["texts"])
    with _Shape(b64, "validate", shape):
        say("shape validate", shape)
        status = torch.empty(2 * ncase, dtype=torch.int64, device="cuda")
        for i, (t, to) in enumerate(zip(d["texts"], d["t_offs"])):
            b64.validate_async(d["d_texts"][to:to + t.size], status=status[2 * i:2 * i + 2])
        st = to_host(status).reshape(-1, 2)
        bad = np.nonzero((st != d["exp_status"]).any(axis=1))[0]
        assert bad.size == 0, (shape, bad[:5], st[bad[:5]], d["exp_status"][bad[:5]])
        assert b64.validate(d["big_text"]) == (BIG_N, None), shape
        for s, p in d["big_bad"]:
            assert b64.validate(s) == (None, p), (shape, p)


@pytest.fixture(scope="module")
def batch(oracle):
    """A ragged batch: 4,000 buffers log-uniform in [1, 32 KiB) (the first
    twelve of lengths 0..11, some empty), then 24 of up to 4 MiB."""
    g = workloads.rng(workloads.SEED_BASE + 310)
    lens = np.concatenate([workloads.batch_lengths(workloads.SEED_BASE + 311, 4000, 1, 32 << 10),
                           workloads.batch_lengths(workloads.SEED_BASE + 312, 24, 1 << 16, 4 << 20)])
    lens[:12] = np.arange(12)
    lens[g.random(lens.size) < 0.03] = 0
    in_off = workloads.offsets(lens)
    src = workloads.random_bytes(workloads.SEED_BASE + 313, int(in_off[-1]))
    enc, enc_off, enc_len = oracle.encode_list(src, in_off)
    # decode input: the encodings, 2% of the buffers spoiled
    text = enc.copy()
    outside = workloads.non_alphabet_bytes(STD)
    for b in np.nonzero(g.random(lens.size) < 0.02)[0]:
        k = int(enc_off[b + 1] - enc_off[b])
        if k:
            p = int(enc_off[b] + g.integers(0, k))
            text[p] = ord("=") if g.random() < 0.3 else outside[int(g.integers(0, outside.size))]
    ref_dst, ref_off, ref_res = oracle.decode_list(text, enc_off)
    tlens = np.diff(enc_off)
    dcap_off = workloads.offsets(3 * (tlens // 4))
    exp_dec = np.zeros(max(int(dcap_off[-1]), 1), dtype=np.uint8)
    valid = np.zeros(exp_dec.size, dtype=bool)
    for b in np.nonzero(ref_res > 0)[0]:
        r = int(ref_res[b])
        exp_dec[dcap_off[b]:dcap_off[b] + r] = ref_dst[ref_off[b]:ref_off[b] + r]
        valid[dcap_off[b]:dcap_off[b] + r] = True
    return {"d_src": to_dev(src), "d_in_off": to_dev(in_off), "exp_enc": to_dev(enc),
            "enc_len": enc_len, "d_text": to_dev(text), "d_tin": to_dev(enc_off),
            "exp_dec": to_dev(exp_dec), "valid": to_dev(valid),
            "exp_len": np.where(ref_res >= 0, ref_res, -1),
            "exp_bad": np.where(ref_res >= 0, -1, ~ref_res)}


@SHAPE_PARAMS
def test_encode_batch_shapes(b64, batch, shape):
    import torch
    with _Shape(b64, "encode_batch", shape):
        say("shape encode_batch", shape)
        dst, out_off, out_len = b64.encode_batch(batch["d_src"], batch["d_in_off"], validate=False)
        n = batch["exp_enc"].numel()
        assert torch.equal(dst[:n], batch["exp_enc"]), shape
        assert np.array_equal(to_host(out_len), batch["enc_len"]), shape


@SHAPE_PARAMS
def test_decode_batch_shapes(b64, batch, shape):
    import torch
    with _Shape(b64, "decode_batch", shape):
        say("shape decode_batch", shape)
        dst, _, out_len, first_bad = b64.decode_batch(batch["d_text"], batch["d_tin"],
                                                      validate=False)
        ol, fb = to_host(out_len), to_host(first_bad)
        wrong = np.nonzero((ol != batch["exp_len"]) | (fb != batch["exp_bad"]))[0]
        assert wrong.size == 0, (shape, wrong[:5], ol[wrong[:5]], fb[wrong[:5]])
        v = batch["valid"]
        n = v.numel()
        assert torch.equal(dst[:n][v], batch["exp_dec"][v]), shape


@pytest.fixture(scope="module")
def wrap(oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 320, (128 << 20) + 2)
    cases = []
    for line_len in (4, 64, 76):
        for n in (1, 2, 3, 47, 48, 57, 58, 3073, 100003, x.size):
            cases.append((n, line_len, to_dev(oracle.encode_mode(x[:n], STD, 0, line_len))))
    return {"dx": to_dev(x), "cases": cases}


@SHAPE_PARAMS
def test_encode_wrap_shapes(b64, wrap, shape):
    import torch
    with _Shape(b64, "encode_wrap", shape):
        for n, line_len, exp in wrap["cases"]:
            say("shape encode_wrap", shape, n, line_len)
            got = b64.encode(wrap["dx"][:n], line_len=line_len)
            assert torch.equal(got, exp), (shape, n, line_len)


@pytest.fixture(scope="module")
def fused(oracle):
    """Rows of base64 float32: 2,000 rows of 1,536 with every 37th row
    spoiled (an invalid byte, a truncation, or a valid row of the wrong
    length), and 3,000 rows of 7."""
    out = []
    for dim, nrows, seed in ((1536, 2000, 330), (7, 3000, 331)):
        raw = workloads.random_bytes(workloads.SEED_BASE + seed, 4 * dim * nrows)
        in_off = workloads.offsets(np.full(nrows, 4 * dim, dtype=np.int64))
        text, t_off, _ = oracle.encode_list(raw, in_off)
        rows = [text[t_off[b]:t_off[b + 1]].copy() for b in range(nrows)]
        g = workloads.rng(workloads.SEED_BASE + seed + 10)
        outside = workloads.non_alphabet_bytes(STD)
        for b in range(0, nrows, 37):
            kind = int(g.integers(0, 3))
            if kind == 0:
                rows[b][int(g.integers(0, rows[b].size))] = outside[int(g.integers(0, outside.size))]
            elif kind == 1:
                rows[b] = rows[b][:-int(g.integers(1, 4))]
            else:
                rows[b] = oracle.encode(workloads.random_bytes(b, 4 * dim + 4))
        text = np.concatenate(rows)
        t_off = workloads.offsets(np.array([r.size for r in rows], dtype=np.int64))
        ref, ref_st = oracle.decode_f32_bf16_rows(text, t_off, dim)
        out.append((dim, to_dev(text), to_dev(t_off), ref, ref_st))
    return out


@SHAPE_PARAMS
def test_fused_shapes(b64, fused, shape):
    import torch
    with _Shape(b64, "decode_f32_bf16", shape):
        for dim, text, t_off, ref, ref_st in fused:
            say("shape fused", shape, dim)
            got, st = b64.decode_f32_bf16(text, t_off, dim, validate=False)
            st = to_host(st)
            assert (st == ref_st).all(), (shape, dim, np.nonzero(st != ref_st)[0][:5])
            g = to_host(got.view(torch.int16)).view(np.uint16)
            good = ref_st == -1
            assert (g[good] == ref[good]).all(), (shape, dim)


@pytest.fixture(scope="module")
def mime(oracle):
    """MIME text (76-character lines, CR LF) of 3 MiB: regular, and with
    whitespace runs sprinkled in; the oracle's decodes."""
    x = workloads.random_bytes(workloads.SEED_BASE + 340, 3 << 20)
    regular = oracle.encode_mode(x, STD, 0, workloads.MIME_LINE)
    sprinkled = workloads.sprinkle_ws(regular, workloads.SEED_BASE + 341, 2000, 5, 1, 1 << 15)
    bad = sprinkled.copy()
    bad[bad.size // 2] = ord("!")
    out = []
    for t in (regular, sprinkled, bad):
        r, fb = oracle.decode_mode(t, STD, SKIP_WS)
        out.append((to_dev(t), None if r is None else to_dev(r), fb, 0 if r is None else r.size))
    return out


@SHAPE_PARAMS
def test_decode_ws_shapes(b64, mime, shape):
    """Whitespace-skipping decode: the counted path, and (with the guess
    threshold at 0) the regular-line guess and its fallback."""
    import torch
    old_min = b64.tune_ws_guess_min(-1)
    try:
        with _Shape(b64, "decode_ws", shape):
            for guess_min in (old_min, 0):
                b64.tune_ws_guess_min(guess_min)
                for k, (t, ref, fb, rlen) in enumerate(mime):
                    say("shape decode_ws", shape, "text", k, "guess_min", guess_min)
                    out, st = b64.decode_async(t, flags=SKIP_WS)
                    if fb is None:
                        assert to_host(st).tolist() == [rlen, -1], (shape, k, guess_min)
                        assert torch.equal(out[:rlen], ref), (shape, k, guess_min)
                    else:
                        assert to_host(st).tolist() == [-1, fb], (shape, k, guess_min)
    finally:
        b64.tune_ws_guess_min(old_min)
