"""GPU parity of the variants (unpadded, CR LF line-wrapped encode,
whitespace-skipping decode / validate) against the oracle, bit-exact: the
same characters, the same decoded bytes, the same decoded length or first
invalid offset.  Inputs come from the seeded generators and the oracle's own
encoder; every expected value from the oracle."""
import numpy as np
import pytest

import workloads
from gpu_util import first_mismatch, say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"
NOPAD, SKIP_WS = 1, 2


def _alphabets():
    g = workloads.rng(workloads.SEED_BASE + 171)
    perm = bytes(g.permutation(np.frombuffer(STD, dtype=np.uint8)).tolist())
    pool = np.array([c for c in range(256) if c not in b"= \t\r\n"], dtype=np.uint8)
    hi = bytes(g.choice(pool, 64, replace=False).tolist())
    return {"std": STD, "url": URL, "perm": perm, "hi": hi}


@pytest.fixture(scope="module")
def b64():
    """The library, with the regular-line guess of the whitespace-skipping
    decode tried at every size (by default only texts of 14 MiB and more try
    it), so that the small texts here reach every path."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    old = b64.tune_ws_guess_min(0)
    yield b64
    b64.tune_ws_guess_min(old)


def _dev(a):
    import torch
    return to_dev(a) if a.size else torch.empty(0, dtype=torch.uint8, device="cuda")


def _enc(b64, oracle, x, alpha, flags, line_len, label):
    say("encode", label, "n =", x.size, "flags", flags, "line", line_len)
    ref = oracle.encode_mode(x, alpha, flags, line_len)
    got = to_host(b64.encode(_dev(x), alpha, flags=flags, line_len=line_len))
    assert got.size == ref.size and first_mismatch(got, ref) is None, (label, first_mismatch(got, ref))


def _dec(b64, oracle, text, alpha, flags, label, check_validate=True):
    say("decode", label, "n =", text.size, "flags", flags)
    ref_raw = oracle.decode_mode_raw(text, alpha, flags)
    out, bad = b64.decode(_dev(text), alpha, flags=flags)
    if ref_raw >= 0:
        ref, _ = oracle.decode_mode(text, alpha, flags)
        assert bad is None, (label, bad)
        got = to_host(out)
        assert first_mismatch(got, ref) is None, (label, first_mismatch(got, ref))
    else:
        assert bad == ~ref_raw, (label, bad, ~ref_raw)
    if check_validate:
        say("validate", label)
        length, vbad = b64.validate(_dev(text), alpha, flags=flags)
        assert (length if vbad is None else ~vbad) == ref_raw, (label, length, vbad, ref_raw)
    return ref_raw


# ---------------------------------------------------------------- unpadded --

@pytest.mark.parametrize("name", ["std", "url", "perm", "hi"])
def test_nopad_encode_decode_all_lengths(b64, oracle, name):
    alpha = _alphabets()[name]
    x = workloads.random_bytes(workloads.SEED_BASE + 172, 2100)
    step = 1 if name == "url" else 5
    for n in range(0, 2100, step):
        _enc(b64, oracle, x[:n], alpha, NOPAD, 0, f"{name} {n}")
        text = oracle.encode_mode(x[:n], alpha, NOPAD)
        _dec(b64, oracle, text, alpha, NOPAD, f"{name} {n}", check_validate=(n % 25 == 0))


def test_nopad_3mib_misaligned_and_invalid(b64, oracle):
    import torch
    x = workloads.random_bytes(workloads.SEED_BASE + 173, workloads.SINGLE_3MIB + 2)
    for n in (workloads.SINGLE_3MIB, workloads.SINGLE_3MIB + 1, workloads.SINGLE_3MIB + 2):
        _enc(b64, oracle, x[:n], URL, NOPAD, 0, f"3MiB+{n % 3}")
        text = oracle.encode_mode(x[:n], URL, NOPAD)
        assert _dec(b64, oracle, text, URL, NOPAD, f"3MiB+{n % 3}") == n
    # misaligned source and destination
    text = oracle.encode_mode(x[:100001], URL, NOPAD)
    for off in (1, 2, 3, 5):
        say("nopad misaligned", off)
        src = torch.zeros(text.size + 8, dtype=torch.uint8, device="cuda")
        src[off:off + text.size] = to_dev(text)
        dst = torch.zeros(100001 + 16, dtype=torch.uint8, device="cuda")
        out, bad = b64.decode(src[off:off + text.size], URL, out=dst[off:], flags=NOPAD)
        assert bad is None and first_mismatch(to_host(out), x[:100001]) is None
    # '=' anywhere, a non-alphabet byte, a length of 1 mod 4, a non-canonical end
    for pos in (0, 1, 2, 3, 4096, text.size - 1):
        t = text.copy()
        t[pos] = ord("=")
        _dec(b64, oracle, t, URL, NOPAD, f"= at {pos}")
    bad, pos = workloads.plant_invalid(text, workloads.SEED_BASE + 174, URL)
    _dec(b64, oracle, bad, URL, NOPAD, "invalid byte")
    _dec(b64, oracle, text[:-2] if text.size % 4 == 3 else text[:-1], URL, NOPAD, "1 mod 4")
    t = oracle.encode_mode(x[:100000], URL, NOPAD)          # 2 characters in the last quantum
    t[-1] = URL[1]                                           # nonzero low bits
    _dec(b64, oracle, t, URL, NOPAD, "non-canonical")


def test_nopad_brute_force_as_batch(b64, oracle):
    """Every string of length <= 6 over a symbol set that exercises '=', the
    canonical bits and invalid bytes, decoded as buffers of one batch."""
    import torch
    symbols = np.frombuffer(b"AQRE=*", dtype=np.uint8)
    for length in range(0, 7):
        rows = symbols[np.indices((6,) * length).reshape(length, -1).T] if length else \
            np.zeros((1, 0), dtype=np.uint8)
        say("nopad brute force", length, rows.shape[0])
        ref = oracle.decode_mode_rows(rows, STD, NOPAD)
        src = rows.reshape(-1)
        in_off = workloads.offsets(np.full(rows.shape[0], length, dtype=np.int64))
        dst, out_off, out_len, first_bad = b64.decode_batch(
            _dev(src) if src.size else torch.zeros(1, dtype=torch.uint8, device="cuda"),
            to_dev(in_off), STD, flags=NOPAD)
        got = np.where(to_host(first_bad) >= 0, ~to_host(first_bad), to_host(out_len))
        assert (got == ref).all(), (length, np.nonzero(got != ref)[0][:5])


def test_nopad_ragged_batch(b64, oracle):
    lens = workloads.batch_lengths(workloads.SEED_BASE + 175, 3000, 1, 5000)
    lens[::97] = 0                                           # some empty buffers
    in_off = workloads.offsets(lens)
    x = workloads.random_bytes(workloads.SEED_BASE + 176, int(in_off[-1]))
    say("nopad batch encode", lens.size)
    ref_dst, ref_off, ref_len = oracle.encode_mode_list(x, in_off, URL, NOPAD)
    dst, out_off, out_len = b64.encode_batch(_dev(x), to_dev(in_off), URL, flags=NOPAD)
    assert (to_host(out_off) == ref_off).all() and (to_host(out_len) == ref_len).all()
    assert first_mismatch(to_host(dst)[: ref_dst.size], ref_dst) is None
    # decode the packed encodings back, with invalid buffers mixed in
    text = ref_dst.copy()
    bad_bufs = workloads.pick_buffers(workloads.SEED_BASE + 177, lens.size, 0.05)
    for b in bad_bufs.tolist():
        if ref_len[b] > 0:
            text[ref_off[b] + (b * 7919) % ref_len[b]] = ord("=")
    say("nopad batch decode", lens.size)
    _, _, ref_res = oracle.decode_mode_list(text, ref_off, URL, NOPAD)
    _, _, out_len, first_bad = b64.decode_batch(_dev(text), to_dev(ref_off), URL, flags=NOPAD)
    got = np.where(to_host(first_bad) >= 0, ~to_host(first_bad), to_host(out_len))
    assert (got == ref_res).all(), np.nonzero(got != ref_res)[0][:5]


# -------------------------------------------------------------- line-wrapped --

@pytest.mark.parametrize("line_len", [4, 8, 12, 16, 64, 76, 1000])
def test_wrapped_encode_lengths(b64, oracle, line_len):
    x = workloads.random_bytes(workloads.SEED_BASE + 178, 5000)
    for n in list(range(0, 200)) + list(range(200, 5000, 97)):
        for flags in (0, NOPAD):
            _enc(b64, oracle, x[:n], STD, flags, line_len, f"L{line_len} n{n}")


def test_wrapped_encode_large_and_misaligned(b64, oracle):
    import torch
    x = workloads.random_bytes(workloads.SEED_BASE + 179, workloads.SINGLE_3MIB + 2)
    for n in (workloads.SINGLE_3MIB, workloads.SINGLE_3MIB + 1, workloads.SINGLE_3MIB + 2):
        for flags in (0, NOPAD):
            _enc(b64, oracle, x[:n], STD, flags, 76, f"3MiB+{n % 3}")
    ref = oracle.encode_mode(x[:77777], URL, 0, 64)
    for off in (1, 2, 3):
        say("wrap misaligned", off)
        src = torch.zeros(77777 + 8, dtype=torch.uint8, device="cuda")
        src[off:off + 77777] = to_dev(x[:77777])
        dst = torch.zeros(ref.size + 8, dtype=torch.uint8, device="cuda")
        out = b64.encode(src[off:off + 77777], URL, out=dst[off:], line_len=64)
        assert first_mismatch(to_host(out), ref) is None


# ------------------------------------------------------- whitespace skipping --

def _mime(oracle, x, alpha=STD, flags=0):
    return oracle.encode_mode(x, alpha, flags, workloads.MIME_LINE)


@pytest.mark.parametrize("flags", [SKIP_WS, SKIP_WS | NOPAD])
def test_skip_ws_mime_lengths(b64, oracle, flags):
    x = workloads.random_bytes(workloads.SEED_BASE + 180, 20000)
    for n in list(range(0, 150)) + list(range(150, 20000, 331)):
        text = _mime(oracle, x[:n], STD, flags & NOPAD)
        assert _dec(b64, oracle, text, STD, flags, f"mime {n}", check_validate=(n % 7 == 0)) == n


@pytest.mark.parametrize("name", ["std", "url", "hi"])
def test_skip_ws_sprinkled_and_long_runs(b64, oracle, name):
    alpha = _alphabets()[name]
    x = workloads.random_bytes(workloads.SEED_BASE + 181, 3 << 20)
    cases = [(1000, 50, 0), (100000, 2000, 0), (300000, 5000, 2), (3 << 20, 20000, 3)]
    for k, (n, runs, longs) in enumerate(cases):
        for flags in (SKIP_WS, SKIP_WS | NOPAD):
            text = workloads.sprinkle_ws(_mime(oracle, x[:n], alpha, flags & NOPAD),
                                         workloads.SEED_BASE + 182 + k, runs, 5, longs, 1 << 17)
            assert _dec(b64, oracle, text, alpha, flags, f"{name} sprinkled {n}") == n


def test_skip_ws_invalid_cases(b64, oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 183, 400000)
    base = workloads.sprinkle_ws(_mime(oracle, x), workloads.SEED_BASE + 184, 3000, 5, 1, 1 << 17)
    n = base.size
    g = workloads.rng(workloads.SEED_BASE + 185)
    # a non-alphabet byte (not whitespace, not '=') at seeded positions
    bad_bytes = workloads.non_alphabet_bytes(STD + b" \t\r\n")
    for k in range(12):
        t = base.copy()
        t[int(g.integers(0, n))] = bad_bytes[int(g.integers(0, bad_bytes.size))]
        _dec(b64, oracle, t, STD, SKIP_WS, f"invalid {k}", check_validate=(k % 3 == 0))
    # '=' at seeded positions (padded: misplaced pad; unpadded: invalid)
    for k in range(12):
        t = base.copy()
        t[int(g.integers(0, n))] = ord("=")
        for flags in (SKIP_WS, SKIP_WS | NOPAD):
            _dec(b64, oracle, t, STD, flags, f"= {k}", check_validate=False)
    # '=' followed by a long whitespace run and more data (slow path)
    t = np.concatenate([_mime(oracle, x[:3000]), np.full(1 << 18, ord(" "), dtype=np.uint8),
                        _mime(oracle, x[3000:6000])])
    _dec(b64, oracle, t, STD, SKIP_WS, "= then long run then data")
    # truncations and the end rules
    text = _mime(oracle, x[:100000])
    for cut in range(1, 8):
        _dec(b64, oracle, text[:-cut], STD, SKIP_WS, f"cut {cut}")
        _dec(b64, oracle, text[:-cut], STD, SKIP_WS | NOPAD, f"nopad cut {cut}")
    # degenerate inputs
    for s in (b"", b"\r\n", b"    \t\n", b"====", b"=", b"A", b"AA", b"AA=", b"AA==", b"AA==\r\n",
              b"AA==\r\nA", b"A\r\nA=\r\n=", b"QQ==", b"QR==", b"QRE=", b"AAAA\n\n\n\nAA"):
        t = np.frombuffer(s, dtype=np.uint8).copy()
        for flags in (SKIP_WS, SKIP_WS | NOPAD):
            _dec(b64, oracle, t, STD, flags, repr(s))


def test_skip_ws_long_runs_at_the_edges(b64, oracle):
    """Whitespace runs longer than a tile where the decoder searches for
    neighbouring significant characters: before and after the text, between
    the two '=' of the final quantum, and just before a tile end, where the
    tile's last quantum takes its values from after the run."""
    x = workloads.random_bytes(workloads.SEED_BASE + 193, 20000)
    sp = lambda k: np.full(k, ord(" "), dtype=np.uint8)
    for n in (3000, 3001, 3002):
        for flags in (SKIP_WS, SKIP_WS | NOPAD):
            text = _mime(oracle, x[:n], STD, flags & NOPAD)
            _dec(b64, oracle, np.concatenate([text, sp(100000)]), STD, flags, f"{n} then run")
            _dec(b64, oracle, np.concatenate([sp(100000), text]), STD, flags, f"run then {n}")
            for cut in (1, 2, 3):
                _dec(b64, oracle, np.concatenate([text[:-cut], sp(70000)]), STD, flags,
                     f"{n} cut {cut} then run", check_validate=False)
    for n in (3001, 3002):                       # "xx==" and "xxx=" split by a run
        text = _mime(oracle, x[:n])
        k = text.size - 1                        # the last '='
        for at in (k, k - 1, k - 2):
            t = np.concatenate([text[:at], sp(70000), text[at:]])
            _dec(b64, oracle, t, STD, SKIP_WS, f"{n} run at {at} of {text.size}")
    for d in (1, 2, 3, 5, 77):
        for flags in (SKIP_WS, SKIP_WS | NOPAD):
            t = _mime(oracle, x, STD, flags & NOPAD)
            t = np.concatenate([t[:2 * 4096 - d], sp(50000), t[2 * 4096 - d:]])
            _dec(b64, oracle, t, STD, flags, f"run before a tile end, d = {d}",
                 check_validate=(d == 1))


def _lines(text: np.ndarray, L: int, sep: bytes) -> np.ndarray:
    """`text` cut into lines of L characters joined by `sep`."""
    parts = []
    for i in range(0, text.size, L):
        if i:
            parts.append(np.frombuffer(sep, dtype=np.uint8))
        parts.append(text[i:i + L])
    return np.concatenate(parts) if parts else text[:0].copy()


def test_skip_ws_regular_lines_and_breaks(b64, oracle):
    """Text in regular lines takes the checked decode on guessed tile counts;
    any break in the regularity must fall back to the counted path with the
    same result.  Line layouts: 76 + CR LF, 64 + LF, 64 + CR LF, 10 + LF (not
    a multiple of 4), lines longer than the first 4 KiB looked at; breaks: one
    extra space, a missing separator, a doubled separator, in the first tile,
    the middle and the last tile; invalid bytes, '=' and truncation inside
    regular text; trailing separators and long trailing runs."""
    x = workloads.random_bytes(workloads.SEED_BASE + 194, 120_000)
    g = workloads.rng(workloads.SEED_BASE + 195)
    for flags in (SKIP_WS, SKIP_WS | NOPAD):
        plain = oracle.encode_mode(x, STD, flags & NOPAD)
        for L, sep in ((76, b"\r\n"), (64, b"\n"), (64, b"\r\n"), (10, b"\n"), (5000, b"\r\n")):
            t = _lines(plain, L, sep)
            _dec(b64, oracle, t, STD, flags, f"lines {L} {sep!r}", check_validate=False)
            _dec(b64, oracle, np.concatenate([t, np.frombuffer(sep, dtype=np.uint8)]), STD, flags,
                 f"lines {L} trailing sep", check_validate=False)
            for at in (300, t.size // 2, t.size - 700):
                for kind in ("space", "missing", "double"):
                    p = at
                    while p < t.size and t[p] in b" \t\r\n":
                        p += 1
                    if kind == "space":
                        u = np.concatenate([t[:p], np.frombuffer(b" ", np.uint8), t[p:]])
                    else:
                        q = int(np.nonzero(t[p:] == sep[-1])[0][0]) + p + 1 if (t[p:] == sep[-1]).any() else t.size
                        s0 = q - len(sep)
                        u = (np.concatenate([t[:s0], t[q:]]) if kind == "missing" else
                             np.concatenate([t[:q], np.frombuffer(sep, np.uint8), t[q:]]))
                    _dec(b64, oracle, u, STD, flags, f"lines {L} {kind} at {at}", check_validate=False)
        t = _lines(plain, 76, b"\r\n")
        for k in range(4):                     # invalid bytes and '=' in regular text
            u = t.copy()
            p = int(g.integers(0, u.size))
            while u[p] in b"\r\n":
                p += 1
            u[p] = ord("*") if k % 2 == 0 else ord("=")
            _dec(b64, oracle, u, STD, flags, f"lines 76 spoiled {k}", check_validate=False)
        for back in (50, 100, 1000, 3000):    # in the last tile, which k_ws_predict scans
            for c in (ord("*"), ord("=")):
                u = t.copy()
                p = u.size - back
                while u[p] in b"\r\n":
                    p += 1
                u[p] = c
                _dec(b64, oracle, u, STD, flags, f"lines 76 byte {c} at end-{back}",
                     check_validate=False)
        for cut in (1, 2, 3, 5):
            _dec(b64, oracle, t[:-cut], STD, flags, f"lines 76 cut {cut}", check_validate=False)
        _dec(b64, oracle, np.concatenate([t, np.full(70_000, ord(" "), np.uint8)]), STD, flags,
             "lines 76 then a long run", check_validate=False)


@pytest.mark.parametrize("n", [32_000_000, 72_000_000], ids=["tiles_8k", "tiles_16k"])
def test_skip_ws_regular_lines_mid_sizes(b64, oracle, n):
    """MIME text of 43.8 MB and 98.5 MB, which the decoder cuts into tiles of
    8 and 16 KiB (the other sizes test 4 and 32 KiB tiles): regular lines on
    the checked path, and breaks that send it to the counted path: a trailing
    separator, one extra space, an invalid byte and a '=' inside the text, an
    invalid byte in the last tile, a cut final quantum."""
    x = workloads.random_bytes(workloads.SEED_BASE + 196, n)
    t = _mime(oracle, x)
    assert (32 << 20) <= t.size < (64 << 20) if n < 50_000_000 else (64 << 20) <= t.size < (128 << 20)
    cases = [("regular", t), ("trailing sep", np.concatenate([t, np.frombuffer(b"\r\n", np.uint8)]))]
    mid = t.size // 2 + 1001
    cases.append(("space", np.concatenate([t[:mid], np.frombuffer(b" ", np.uint8), t[mid:]])))
    for label, p, c in (("invalid", t.size // 3 + 17, ord("*")), ("pad", 3 * t.size // 4 + 5, ord("=")),
                        ("invalid last tile", t.size - 100, ord("!"))):
        u = t.copy()
        while u[p] in b"\r\n":
            p += 1
        u[p] = c
        cases.append((label, u))
    cases.append(("cut", t[:-2]))
    # breaks that the sampled line ends do not see (the layout is restored a
    # few lines later): only the byte-by-byte check of the line decode can
    # find them, and the counted path must then give the oracle's result
    P = workloads.MIME_LINE + 2
    k = (t.size // P) // 2 + 7                  # a line in the middle, no sample on it
    cr = k * P + workloads.MIME_LINE            # its CR
    assert t[cr] == ord("\r") and t[cr + 1] == ord("\n")
    sp = (k + 3) * P + workloads.MIME_LINE      # three lines later
    cases.append(("resync", np.concatenate([t[:cr], t[cr + 1:sp], np.frombuffer(b" ", np.uint8), t[sp:]])))
    u = t.copy()
    u[cr] = ord("A")                            # a separator byte made significant ...
    u[cr + P + 5] = ord(" ")                    # ... and a character of the next line whitespace
    cases.append(("swap", u))
    for label, u in cases:
        _dec(b64, oracle, u, STD, SKIP_WS, f"mid size {n} {label}", check_validate=(label == "space"))


@pytest.mark.parametrize("name", ["url", "hi"])
def test_skip_ws_regular_lines_alphabets(b64, oracle, name):
    """The line decode's checks go through the alphabet's map: MIME text of a
    30 MB payload (41 MB, enough for the pipelined steps) in the URL-safe
    alphabet and in one of 64 arbitrary bytes, padded and unpadded, clean and
    with a byte outside the alphabet planted past the middle."""
    alpha = _alphabets()[name]
    x = workloads.random_bytes(workloads.SEED_BASE + 200, 30_000_000)
    outside = [c for c in range(256) if c not in alpha and c not in b"= \t\r\n"]
    for flags in (SKIP_WS, SKIP_WS | NOPAD):
        t = _mime(oracle, x, alpha, flags & NOPAD)
        assert _dec(b64, oracle, t, alpha, flags, f"{name} lines", check_validate=False) == x.size
        u = t.copy()
        p = 2 * t.size // 3 + 11
        while u[p] in b"\r\n":
            p += 1
        u[p] = outside[len(outside) // 2]
        _dec(b64, oracle, u, alpha, flags, f"{name} lines invalid at {p}", check_validate=False)


def test_skip_ws_default_guess_threshold(b64, oracle):
    """With the default threshold, regular lines below 14 MiB take the counted
    path and those above the guess: both give the oracle's bytes, clean and
    with an invalid byte, padded and unpadded."""
    old = b64.tune_ws_guess_min(-1)
    b64.tune_ws_guess_min(14 << 20)
    try:
        x = workloads.random_bytes(workloads.SEED_BASE + 201, 12_000_000)
        for n in (100_000, 3_000_000, 12_000_000):
            for flags in (SKIP_WS, SKIP_WS | NOPAD):
                t = _mime(oracle, x[:n], STD, flags & NOPAD)
                assert _dec(b64, oracle, t, STD, flags, f"default threshold {n}",
                            check_validate=False) == n
                u = t.copy()
                u[t.size // 2] = ord("*") if u[t.size // 2] not in b"\r\n" else u[t.size // 2]
                _dec(b64, oracle, u, STD, flags, f"default threshold {n} invalid", check_validate=False)
    finally:
        b64.tune_ws_guess_min(old)


def test_skip_ws_regular_lines_output_offsets(b64, oracle):
    """The line decode aligns its stores by the destination's address mod 128:
    a 98.5 MB MIME text (enough for several pipelined steps of the whole grid)
    decoded into outputs at offsets 0..127 (mod 128) gives the payload, and
    the bytes before and after the output stay untouched."""
    import torch
    n = 72_000_000
    x = workloads.random_bytes(workloads.SEED_BASE + 198, n)
    dx = to_dev(x)
    text = b64.encode(dx, STD, line_len=workloads.MIME_LINE)
    cap = b64.decoded_max_len(text.numel(), SKIP_WS)
    buf = torch.zeros(cap + 256, dtype=torch.uint8, device="cuda")
    for off in (1, 5, 17, 42, 64, 100, 127, 128):
        say("lines output offset", off)
        buf.zero_()
        out, st = b64.decode_async(text, STD, out=buf[off:], flags=SKIP_WS)
        assert to_host(st).tolist() == [n, -1], off
        assert torch.equal(buf[off:off + n], dx), off
        assert not buf[:off].any().item() and not buf[off + n:].any().item(), off


def test_skip_ws_async_status_and_graph(b64, oracle):
    import torch
    x = workloads.random_bytes(workloads.SEED_BASE + 186, 1 << 20)
    text = workloads.sprinkle_ws(_mime(oracle, x), workloads.SEED_BASE + 187, 500)
    bad_text = text.copy()
    bad_text[text.size // 2] = ord("*")
    ref_bad = ~oracle.decode_mode_raw(bad_text, STD, SKIP_WS)
    s_ok, s_bad = _dev(text), _dev(bad_text)
    say("skip_ws async")
    out, st = b64.decode_async(s_ok, STD, flags=SKIP_WS)
    assert to_host(st).tolist() == [x.size, -1]
    assert first_mismatch(to_host(out)[: x.size], x) is None
    vst = b64.validate_async(s_bad, STD, flags=SKIP_WS)
    assert to_host(vst).tolist() == [-1, ref_bad]
    # capture the five launches in a graph; replay with eager work between
    say("skip_ws graph capture")
    cap = b64.decoded_max_len(text.size, SKIP_WS)
    out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    ws = torch.empty(b64.workspace_size(text.size, SKIP_WS), dtype=torch.uint8, device="cuda")
    src = s_ok.clone()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b64.decode_async(src, STD, out=out, status=st, flags=SKIP_WS, workspace=ws)   # warm up
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b64.decode_async(src, STD, out=out, status=st, flags=SKIP_WS, workspace=ws)
    for rep in range(4):
        say("replay", rep)
        src.copy_(s_bad if rep % 2 else s_ok)
        out.zero_()
        st.fill_(7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        if rep % 2:
            assert to_host(st).tolist() == [-1, ref_bad]
        else:
            assert to_host(st).tolist() == [x.size, -1]
            assert first_mismatch(to_host(out)[: x.size], x) is None


def test_skip_ws_large(b64, oracle):
    """A 256 MiB payload as MIME text (about 354 MB): about 10,800 tiles of
    32 KiB."""
    x = workloads.random_bytes(workloads.SEED_BASE + 188, 256 << 20)
    text = _mime(oracle, x)
    say("skip_ws large", text.size)
    s = _dev(text)
    out, bad = b64.decode(s, STD, flags=SKIP_WS)
    assert bad is None and first_mismatch(to_host(out), x) is None
    length, vbad = b64.validate(s, STD, flags=SKIP_WS)
    assert length == x.size and vbad is None
    say("wrap encode large")
    enc = to_host(b64.encode(_dev(x), STD, line_len=workloads.MIME_LINE))
    assert first_mismatch(enc, text) is None


@pytest.mark.parametrize("shape", [(1, 1, 0), (2, 3, 1), (4, 8, 1), (8, 16, 0)])
def test_skip_ws_launch_shapes_and_misaligned_output(b64, oracle, shape):
    """Every launch shape of the whitespace-skipping decode (rounds in flight
    per wave 1, 2, 4 and 8 -> 2; workgroups per CU; nontemporal on and off)
    gives the oracle's bytes, also into an output at each offset mod 4."""
    import torch
    x = workloads.random_bytes(workloads.SEED_BASE + 189, 6 << 20)
    texts = [workloads.sprinkle_ws(_mime(oracle, x[:300001]), workloads.SEED_BASE + 190, 3000, 5, 1,
                                   1 << 15),
             _mime(oracle, x[:(6 << 20) - 1])]
    old = b64.tune_shapes("decode_ws")
    try:
        b64.tune_set("decode_ws", *shape)
        for k, text in enumerate(texts):
            ref, _ = oracle.decode_mode(text, STD, SKIP_WS)
            s = _dev(text)
            for off in range(4):
                say("ws shape", shape, "text", k, "n", text.size, "offset", off)
                cap = b64.decoded_max_len(text.size, SKIP_WS)
                buf = torch.zeros(cap + 8, dtype=torch.uint8, device="cuda")
                out, st = b64.decode_async(s, STD, out=buf[off:], flags=SKIP_WS)
                assert to_host(st).tolist() == [ref.size, -1], (shape, k, off)
                got = to_host(buf)
                assert first_mismatch(got[off:off + ref.size], ref) is None, (shape, k, off)
                assert not got[:off].any() and not got[off + ref.size:].any(), (shape, k, off)
    finally:
        b64.tune_restore("decode_ws", old)


def test_skip_ws_input_ends_on_a_tile_boundary(b64, oracle):
    """Inputs whose length is a whole number of decode tiles (4 KiB at these
    sizes): the tile holding the final quanta is full, and the decoder must
    still leave them to its edge path.  Whitespace pads the text to length."""
    import torch
    x = workloads.random_bytes(workloads.SEED_BASE + 191, 20000)
    for k in (1, 2, 3, 5):
        n = 4096 * k
        for flags in (SKIP_WS, SKIP_WS | NOPAD):
            for cut in (0, 1, 2, 40):
                text = _mime(oracle, x[: (3 * n * 76) // (4 * 78) - 8 - cut], STD, flags & NOPAD)
                assert text.size <= n
                text = np.concatenate([text, np.full(n - text.size, ord("\n"), dtype=np.uint8)])
                ref, _ = oracle.decode_mode(text, STD, flags)
                s = _dev(text)
                for off in range(4):
                    say("ws tile end", n, "flags", flags, "cut", cut, "offset", off)
                    cap = b64.decoded_max_len(text.size, flags)
                    buf = torch.zeros(cap + 8, dtype=torch.uint8, device="cuda")
                    _, st = b64.decode_async(s, STD, out=buf[off:], flags=flags)
                    assert to_host(st).tolist() == [ref.size, -1], (n, flags, cut, off)
                    got = to_host(buf)
                    assert first_mismatch(got[off:off + ref.size], ref) is None, (n, flags, cut, off)


def test_skip_ws_last_tile_of_a_few_bytes(b64, oracle):
    """MIME text whose last decode tile (4 KiB at these sizes) holds only 1 to
    3 bytes, so that the final quantum starts in the tile before it: the line
    decode still takes it (the mode word the decoder leaves in its workspace
    names the path that ran), with the oracle's result.  (Padded MIME text has
    an even length; a trailing LF gives the odd cases.)  A byte changed just
    before the last tile breaks the layout there, and the decoder must leave
    the line decode, again with the oracle's result."""
    import torch
    TS, LINES = 4096, 2                       # tile size at these lengths; mode word: line decode
    x = workloads.random_bytes(workloads.SEED_BASE + 197, 200_000)
    for flags in (SKIP_WS, SKIP_WS | NOPAD):
        nopad = bool(flags & NOPAD)
        want = {1: [], 2: [], 3: []}          # (payload length, trailing LF) by bytes in the last tile
        P = workloads.MIME_LINE + 2
        for k in range(100_000, 200_000):
            c = (4 * k + 2) // 3 if nopad else 4 * ((k + 2) // 3)
            size = c + 2 * ((c - 1) // workloads.MIME_LINE)
            jq = 4 * (c // 4) if nopad else c - 4          # the final quantum's first character
            at = (jq // workloads.MIME_LINE) * P + jq % workloads.MIME_LINE
            for lf in (0, 1):
                r = (size + lf) % TS
                # only texts whose final quantum starts before the last tile
                if r in want and len(want[r]) < 2 and at < size + lf - r:
                    want[r].append((k, lf))
            if all(len(v) == 2 for v in want.values()):
                break
        # (unpadded text has no such case with 3 bytes in the last tile)
        assert sum(len(v) for v in want.values()) >= 4, (flags, want)
        for r, ks in want.items():
            for k, lf in ks:
                text = _mime(oracle, x[:k], STD, flags & NOPAD)
                if lf:
                    text = np.concatenate([text, np.frombuffer(b"\n", np.uint8)])
                assert text.size % TS == r
                lb = text.size - r                # the last tile's first byte
                cases = [("regular", text)]
                for back in (1, 2, 3):
                    u = text.copy()
                    u[lb - back] = ord("A") if u[lb - back] in b"\r\n" else ord(" ")
                    cases.append((f"changed at tile end - {back}", u))
                for label, u in cases:
                    say("ws last tile of", r, "bytes, payload", k, "LF", lf, "flags", flags, label)
                    ref_raw = oracle.decode_mode_raw(u, STD, flags)
                    ntiles = -(-u.size // TS)
                    ws = torch.zeros(b64.workspace_size(u.size, flags), dtype=torch.uint8, device="cuda")
                    out = torch.zeros(b64.decoded_max_len(u.size, flags) + 8, dtype=torch.uint8,
                                      device="cuda")
                    _, st = b64.decode_async(_dev(u), STD, out=out, flags=flags, workspace=ws)
                    s = to_host(st).tolist()
                    if ref_raw >= 0:
                        ref, _ = oracle.decode_mode(u, STD, flags)
                        assert s == [ref.size, -1], (label, s)
                        assert first_mismatch(to_host(out)[:ref.size], ref) is None, label
                    else:
                        assert s == [-1, ~ref_raw], (label, s, ~ref_raw)
                    mode = int(to_host(ws.view(torch.int64))[ntiles + 2])
                    assert ((mode & 3) == LINES) == (label == "regular"), (label, mode)


def test_skip_ws_round_trip_many_tiles(b64, oracle):
    """A 1.3 GB payload as MIME text (about 1.78 GB, more than 49,152 tiles of
    32 KiB, so the tile scan takes two passes): the whitespace-skipping decode
    of the wrapped encoding gives the payload back (a property that holds at
    any size; both kernels are checked against the oracle at smaller sizes)."""
    import torch
    n = 1_300_000_000
    x = torch.from_numpy(workloads.random_bytes(workloads.SEED_BASE + 192, n)).cuda()
    say("ws round trip", n)
    text = b64.encode(x, STD, line_len=workloads.MIME_LINE)
    assert text.numel() > 49152 * 32768
    out, st = b64.decode_async(text, STD, flags=SKIP_WS)
    assert to_host(st).tolist() == [n, -1]
    assert torch.equal(out[:n], x)
    del x, text, out
    torch.cuda.empty_cache()


# ------------------------------------------ one-workgroup path for small texts --

class _WsSmall:
    """Sets the one-workgroup limit of the whitespace-skipping decode for a
    block of code (0: small texts take the multi-launch paths)."""

    def __init__(self, b64, max_chars):
        self.b64, self.max_chars = b64, max_chars

    def __enter__(self):
        self.old = self.b64.tune_ws_small_max(self.max_chars)

    def __exit__(self, *exc):
        self.b64.tune_ws_small_max(self.old)


def _ws_rows_on_gpu(b64, rows, flags):
    """decode_async and validate_async of every row of `rows` (one launch
    sequence per row, all enqueued, one synchronisation); returns the decode
    statuses [nrows, 2], the validate statuses and the outputs."""
    import torch
    nrows, L = rows.shape
    dev = torch.from_numpy(np.ascontiguousarray(rows).reshape(-1)).cuda() if rows.size else None
    cap = max(b64.decoded_max_len(L, flags), 1)
    out = torch.zeros((nrows, cap), dtype=torch.uint8, device="cuda")
    st = torch.full((nrows, 2), 7, dtype=torch.int64, device="cuda")
    vst = torch.full((nrows, 2), 7, dtype=torch.int64, device="cuda")
    empty = torch.empty(0, dtype=torch.uint8, device="cuda")
    for i in range(nrows):
        s = dev[i * L:(i + 1) * L] if L else empty
        b64.decode_async(s, STD, out=out[i], status=st[i], flags=flags)
        b64.validate_async(s, STD, status=vst[i], flags=flags)
    torch.cuda.synchronize()
    return to_host(st), to_host(vst), to_host(out)


def _check_rows(oracle, rows, flags, st, vst, out, label):
    want = oracle.decode_mode_rows(rows, STD, flags)
    for i in range(rows.shape[0]):
        w = int(want[i])
        exp = [w, -1] if w >= 0 else [-1, ~w]
        assert st[i].tolist() == exp, (label, bytes(rows[i]), st[i].tolist(), exp)
        assert vst[i].tolist() == exp, (label, "validate", bytes(rows[i]), vst[i].tolist(), exp)
        if w > 0:
            ref, _ = oracle.decode_mode(rows[i], STD, flags)
            assert first_mismatch(out[i][:w], ref) is None, (label, bytes(rows[i]))


@pytest.mark.parametrize("small", [True, False], ids=["one_workgroup", "multi_launch"])
@pytest.mark.parametrize("flags", [SKIP_WS, SKIP_WS | NOPAD], ids=["padded", "nopad"])
def test_skip_ws_brute_force_short(b64, oracle, small, flags):
    """Every string of up to 5 characters over A, B, Q, '=', space, LF and
    '*' (outside the alphabet): status, validate status and decoded bytes
    against the oracle, through the one-workgroup path and through the
    multi-launch paths.  A (value 0), Q (16) and B (1) make the canonical
    rules before '=' hold or fail."""
    import itertools
    sym = np.frombuffer(b"ABQ= \n*", dtype=np.uint8)
    with _WsSmall(b64, 65536 if small else 0):
        for L in range(0, 6):
            rows = (np.array(list(itertools.product(sym, repeat=L)), dtype=np.uint8) if L
                    else np.zeros((1, 0), dtype=np.uint8))
            say("brute force", "small" if small else "multi", flags, "L =", L, "rows", rows.shape[0])
            st, vst, out = _ws_rows_on_gpu(b64, rows, flags)
            _check_rows(oracle, rows, flags, st, vst, out, f"L={L}")


@pytest.mark.parametrize("small", [True, False], ids=["one_workgroup", "multi_launch"])
def test_skip_ws_random_short_strings(b64, oracle, small):
    """Random strings of 6 .. 80 characters over the same symbols, weighted
    towards valid text, and valid encodings with whitespace sprinkled in."""
    g = workloads.rng(workloads.SEED_BASE + 190)
    sym = np.frombuffer(b"ABQgw09+/= \n\r\t*", dtype=np.uint8)
    weights = np.array([8, 2, 4, 4, 4, 4, 4, 2, 2, 2, 3, 2, 1, 1, 1], dtype=np.float64)
    weights /= weights.sum()
    with _WsSmall(b64, 65536 if small else 0):
        for flags in (SKIP_WS, SKIP_WS | NOPAD):
            for L in (6, 7, 9, 13, 16, 17, 31, 64, 80):
                rows = g.choice(sym, size=(300, L), p=weights).astype(np.uint8)
                say("random", "small" if small else "multi", flags, "L =", L)
                st, vst, out = _ws_rows_on_gpu(b64, rows, flags)
                _check_rows(oracle, rows, flags, st, vst, out, f"random L={L}")


def test_skip_ws_one_workgroup_limits(b64, oracle):
    """Texts around the one-workgroup path's limit (65,536 characters) and
    its per-thread load counts (16,384, 32,768, 49,152), valid and with an
    invalid byte, a misplaced '=' or a cut at the end: the same results as
    the multi-launch paths and the oracle."""
    x = workloads.random_bytes(workloads.SEED_BASE + 191, 60000)
    g = workloads.rng(workloads.SEED_BASE + 192)
    for target in (16383, 16384, 16385, 32768, 49151, 49153, 65535, 65536, 65537):
        # MIME text of about `target` characters, padded out with spaces
        text = _mime(oracle, x[: target * 57 // 78])[:target]
        text = np.concatenate([text, np.full(max(target - text.size, 0), ord(" "), np.uint8)])
        cases = [("valid", text)]
        t = text.copy()
        t[int(g.integers(0, t.size))] = ord("*")
        cases.append(("invalid", t))
        t = text.copy()
        t[int(g.integers(0, t.size))] = ord("=")
        cases.append(("misplaced =", t))
        cases.append(("cut", text[:-3]))
        for label, tx in cases:
            for flags in (SKIP_WS, SKIP_WS | NOPAD):
                ref = oracle.decode_mode_raw(tx, STD, flags)
                for small in (True, False):
                    with _WsSmall(b64, 65536 if small else 0):
                        got = _dec(b64, oracle, tx, STD, flags, f"{target} {label} small={small}",
                                   check_validate=True)
                    assert got == ref
    with pytest.raises(Exception):
        b64.tune_ws_small_max(65537)
    assert b64.tune_ws_small_max(-1) == 65536
