"""CPU model of the whitespace-skipping decode's work split (no GPU).

The kernels cut the input into tiles of TS characters.  Tile t holds the
significant characters with indices prefix[t] .. prefix[t+1]-1 and decodes
the quanta whose first significant value lies in it: it skips
(4 - prefix[t] % 4) % 4 values that finish an earlier quantum and reads
rounds of 4096 characters into two value buffers used in turn.  Position 16
of the first buffer stands for quantum Q0 - h (h < 4 chosen so that every
16-value group stores at a 4-byte aligned output address); every 16 values
from position 16 on are emitted as 4 quanta, and the values after the last
whole group are copied to position 16 of the other buffer, where the next
round continues.  The last quantum is completed with up to three values
borrowed from later tiles.  Quanta before Q0 and at index >= qlimit are not
stored by the tile.

This model repeats that index arithmetic in Python, on random inputs with
whitespace runs of every length (empty tiles, runs longer than a tile), and
checks that every quantum below qlimit is written exactly once, by one tile,
from the right significant values.
"""
import numpy as np
import pytest

import workloads

WS = set(b" \t\r\n")
ROUND = 4096
BUF = 16 + ROUND + 48                # bytes of one value buffer


def tile_size(n):
    ts = ROUND
    while ts < 32768 and n // (2 * ts) >= 4096:
        ts *= 2
    return ts


def model(text: bytes, nopad: bool, ts: int, dmod: int = 0):
    n = len(text)
    sig = [i for i, c in enumerate(text) if c not in WS]
    ntiles = (n + ts - 1) // ts if n else 0
    prefix = [0]
    for t in range(ntiles):
        prefix.append(prefix[-1] + sum(1 for c in text[t * ts:(t + 1) * ts] if c not in WS))
    total = prefix[-1] if ntiles else 0
    assert total == len(sig)
    qlimit = total // 4 if nopad else (total // 4 - 1 if total >= 4 else 0)
    writes = {}                                   # quantum -> (tile, value indices)

    def end_of(t):
        return min(n, (t + 1) * ts)
    for t in range(ntiles):
        K0, C = prefix[t], prefix[t + 1] - prefix[t]
        skip = (4 - K0 % 4) % 4
        if C <= skip:
            continue
        Q0 = (K0 + skip) // 4
        if Q0 >= qlimit:
            continue
        h = (Q0 + 3 * dmod) & 3
        Qr = Q0 - h
        assert (3 * Qr + dmod) % 4 == 0
        base, end = t * ts, min(n, (t + 1) * ts)
        # a full tile whose quanta all lie below qlimit: the kernel's hot path
        # stores every whole group without checking qlimit, and holds back
        # only the first group's quanta before Q0
        hot = end_of(t) - t * ts == ts and Q0 + C // 4 + 1 <= qlimit
        W, Qb = 16 + 4 * h - skip, Qr            # position 16 stands for quantum Qb
        bufs, cur = [{}, {}], 0                    # stale entries stay, as in LDS
        g = K0                                     # significant index of the next value
        for p0 in range(base, end, ROUND):
            cb, nb = bufs[cur], bufs[cur ^ 1]
            chunk = [c for c in text[p0:min(end, p0 + ROUND)] if c not in WS]
            for v in chunk:
                assert 0 <= W < BUF
                cb[W] = g
                W += 1
                g += 1
            avail = W - 16
            nfull = max(0, avail >> 4)
            for tid in range(nfull):
                r = 16 + 16 * tid
                q = Qb + 4 * tid
                assert (3 * q + dmod) % 4 == 0        # aligned 12-byte store
                if hot:
                    assert q + 4 <= qlimit
                    assert q >= Q0 or (q == Q0 - h and q + 4 > Q0)
                for k in range(4):
                    if Q0 <= q + k < qlimit:
                        idx = [cb.get(r + 4 * k + j) for j in range(4)]
                        assert (q + k) not in writes
                        writes[q + k] = (t, idx)
            keep = avail - 16 * nfull
            assert keep < 16 and (keep >= 0 or nfull == 0)
            for tid in range(max(keep, 0)):
                nb[16 + tid] = cb.get(16 + 16 * nfull + tid)   # junk below W0 too
            W = 16 + keep if keep >= 0 else W
            Qb += 4 * nfull
            cur ^= 1
        left = W - 16
        if left > 0:
            cb = bufs[cur]
            rem = left & 3
            extra = []
            gg = K0 + C
            while len(extra) < (4 - rem if rem else 0) and gg < total:
                extra.append(gg)                   # the kernel finds it via tile_of + scan
                gg += 1
            nq = (left + 3) // 4
            for tid in range(nq):
                q = Qb + tid
                idx = []
                for k in range(4):
                    i = 4 * tid + k
                    idx.append(cb.get(16 + i) if i < left else (extra[i - left] if i - left < len(extra) else None))
                if Q0 <= q < qlimit:
                    assert None not in idx
                    assert q not in writes
                    writes[q] = (t, idx)
    # every quantum below qlimit written once, from values 4q..4q+3
    assert sorted(writes) == list(range(max(qlimit, 0)))
    for q, (t, idx) in writes.items():
        assert idx == [4 * q + j for j in range(4)], (q, t, idx)
        first = sig[4 * q]
        assert t * ts <= first < (t + 1) * ts       # the tile of the quantum's first value
    return len(writes)


def random_text(rng, n_sig, ws_rate, long_runs, tile):
    out = bytearray()
    for _ in range(n_sig):
        while rng.random() < ws_rate:
            out += bytes([int(rng.choice(list(WS)))])
        out += b"A"
    for _ in range(long_runs):
        pos = int(rng.integers(0, len(out) + 1))
        out[pos:pos] = b" " * int(rng.integers(tile // 2, 3 * tile))
    return bytes(out)


@pytest.mark.parametrize("nopad", [False, True])
def test_every_quantum_written_once(nopad):
    rng = np.random.default_rng(workloads.SEED_BASE + 91)
    for trial in range(16):
        n_sig = int(rng.integers(0, 20000))
        text = random_text(rng, n_sig, float(rng.choice([0.0, 0.02, 0.3, 0.9])),
                           int(rng.integers(0, 4)), ROUND)
        model(text, nopad, ROUND, trial % 4)
        model(text, nopad, 2 * ROUND, (trial + 1) % 4)


def test_mime_lines_and_tile_sizes():
    # 76-character lines with CR LF, the workload's shape, several tile sizes
    for n_sig in (0, 1, 3, 4, 5, 76, 4095, 4096, 4097, 30001):
        lines = [b"A" * 76] * (n_sig // 76) + ([b"A" * (n_sig % 76)] if n_sig % 76 else [])
        text = b"\r\n".join(lines)
        for ts in (ROUND, 4 * ROUND):
            for nopad in (False, True):
                for dmod in range(4):
                    model(text, nopad, ts, dmod)


def test_tile_size_rule():
    assert tile_size(0) == 4096
    assert tile_size(10 ** 6) == 4096
    assert tile_size(64 << 20) == 16384
    assert tile_size(1431655764) == 32768


def test_last_tile_full():
    # inputs that end exactly on a tile boundary, so the tile holding the
    # final quanta is full: the hot-path condition must turn it away
    rng = np.random.default_rng(workloads.SEED_BASE + 92)
    for ts in (ROUND, 2 * ROUND):
        for k in (1, 2, 3):
            for trial in range(6):
                n = k * ts
                n_ws = int(rng.integers(0, 64))
                body = bytearray(b"A" * (n - n_ws))
                for _ in range(n_ws):
                    pos = int(rng.integers(0, len(body) + 1))
                    body[pos:pos] = b"\n"
                text = bytes(body[:n])
                assert len(text) == n
                for nopad in (False, True):
                    model(text, nopad, ts, trial % 4)


# ---------------------------------------------------------------------------
# Guessed prefix sums for text in regular lines (k_ws_predict): lines of L
# significant characters, each followed by s whitespace bytes, P = L + s.

def lined_before(p: int, L: int, P: int) -> int:
    """The kernel's closed form, its quotient taken from a double division
    and corrected, as on the GPU."""
    q = int(float(p) / float(P))
    r = p - q * P
    if r < 0:
        q, r = q - 1, r + P
    elif r >= P:
        q, r = q + 1, r - P
    return q * L + min(r, L)


@pytest.mark.parametrize("L,sep", [(4, 1), (10, 1), (64, 1), (64, 2), (76, 2), (1000, 2)])
def test_lined_before_counts_significant_characters(L, sep):
    g = workloads.rng(900 + L + sep)
    nlines = 3000 // max(1, L // 16) + 5
    sig = np.ones(nlines * (L + sep), dtype=bool)
    for k in range(nlines):
        sig[k * (L + sep) + L: (k + 1) * (L + sep)] = False
    sig = sig[: sig.size - int(g.integers(0, L + sep))]          # a shorter last line
    before = np.concatenate([[0], np.cumsum(sig)])
    for p in list(range(0, min(sig.size + 1, 700))) + g.integers(0, sig.size + 1, 500).tolist():
        assert lined_before(p, L, L + sep) == before[p], (p, L, sep)
    # the guess of every tile: never past its position, at most a tile per tile
    for ts in (4096, 32768):
        pre = [lined_before(t * ts, L, L + sep) for t in range(sig.size // ts + 2)]
        assert all(0 <= b - a <= ts for a, b in zip(pre, pre[1:]))
        assert all(v <= t * ts for t, v in enumerate(pre))


def test_lined_before_quotient_at_large_positions():
    """The double-division quotient, after its correction, is the integer
    floor for positions far past 2^32 (inputs of hundreds of GB)."""
    g = workloads.rng(905)
    for P in (5, 11, 66, 78, 1002, 4097):
        L = P - 2
        ps = np.concatenate([g.integers(0, 1 << 40, 2000), (np.arange(1, 200) * P) << 20,
                             ((np.arange(1, 200) * P) << 20) - 1])
        for p in ps.tolist():
            q, r = divmod(p, P)
            assert lined_before(p, L, P) == q * L + min(r, L), (p, P)


def lines_model(text: bytes, L: int, s: int, qlimit: int, h: int, S: int, D: int = 4):
    """The work split of the line decode (the kernel for text in lines of L
    significant characters, L a multiple of 4 and at least 16, each followed
    by s separator bytes): group g covers quanta 4g - h .. 4g - h + 3; step k
    takes groups kS .. kS + S - 1.  Returns {quantum: 4 characters} as the
    kernel reads them, after checking every load against the text's end and
    the incremental positions against the closed form."""
    n, P = len(text), L + s
    G = (qlimit + h + 3) // 4
    g_lo, g_full = (h + 3) // 4, (qlimit + h) // 4
    g_read = (lined_before(n - 19, L, P) + 4 * h) // 16
    g_hi = min(g_full, g_read)
    k_lo = (g_lo + S - 1) // S
    k_hi = max(g_hi // S, k_lo)
    nmain = (k_hi - k_lo) - (k_hi - k_lo) % D
    got = {}

    def pos(j):
        return (j // L) * P + j % L

    def vector_group(g, p, c):
        assert g_lo <= g < g_hi and 0 <= p and p + 20 <= n      # the 16 + 4 bytes loaded
        w = text[p:p + 20]
        rem = L - c
        chars = w[:16] if rem > 12 else w[:rem] + w[rem + s:16 + s]
        if rem <= 16:
            assert all(b in WS for b in w[rem:rem + s])         # the separator the kernel checks
        for k in range(4):
            qq = 4 * g - h + k
            assert 0 <= qq < qlimit and qq not in got
            got[qq] = chars[4 * k:4 * k + 4]

    def edge_group(g):
        for k in range(4):
            qq = 4 * g - h + k
            if 0 <= qq < qlimit:
                p = pos(4 * qq)
                assert p + 4 <= n and qq not in got
                got[qq] = text[p:p + 4]

    def one(g):
        if g_lo <= g < g_hi:
            j = 16 * g - 4 * h
            vector_group(g, pos(j), j % L)
        elif g < G:
            edge_group(g)

    for lane in range(S):
        for k in range(k_lo):
            one(k * S + lane)
        if nmain > 0:
            dj = 16 * S
            dl, dc = divmod(dj, L)
            dp = dl * P + dc
            j0 = 16 * (k_lo * S + lane) - 4 * h
            pn, cn = pos(j0), j0 % L
            for i in range(nmain):
                g = (k_lo + i) * S + lane
                assert (pn, cn) == (pos(16 * g - 4 * h), (16 * g - 4 * h) % L)
                vector_group(g, pn, cn)
                pn, cn = pn + dp, cn + dc
                if cn >= L:
                    cn, pn = cn - L, pn + s
        k = k_lo + nmain
        while k * S < G:
            one(k * S + lane)
            k += 1
    return got


@pytest.mark.parametrize("L,s", [(76, 2), (64, 1), (16, 2), (20, 1), (1000, 2)])
def test_line_decode_split(L, s):
    """Every quantum below qlimit is read exactly once, from its own four
    characters, with every load inside the text, for several destination
    alignments (h), grid sizes and text lengths, the final quantum padded
    and trailing separators included."""
    g = workloads.rng(workloads.SEED_BASE + 197)
    alpha = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
    sep = b"\r\n"[2 - s:]
    for trial in range(12):
        n_sig = int(g.integers(300, 6000)) * 4
        body = bytes(alpha[int(c)] for c in g.integers(0, 64, n_sig))
        lines = [body[i:i + L] for i in range(0, n_sig, L)]
        text = sep.join(lines) + (sep if trial % 3 == 0 else b"")
        total = n_sig
        qlimit = total // 4 - 1
        h = int(g.integers(0, 128))
        S = int(g.choice([64, 128, 256, 512]))
        got = lines_model(text, L, s, qlimit, h, S)
        assert sorted(got) == list(range(qlimit))
        for qq, chars in got.items():
            assert chars == body[4 * qq:4 * qq + 4], (L, s, trial, qq)


def test_line_decode_eligibility_is_safe():
    """When the guess picks the line decode (L a multiple of 4, at least 16,
    and at most 64 bytes from the separator before the final quantum, as far
    as the guessed total goes, to the last tile), the bytes the line decode
    checks (every character of a quantum below qlimit and the separator after
    every line end it passes) and the bytes k_ws_predict checks itself (that
    stretch before the last tile, against the layout) cover all of the text
    before the last tile.  So either they all fit the layout and the guessed
    total is the true one, or one of them does not and the kernel falls back.
    Regular texts followed by whitespace runs of every size around a tile,
    texts whose last tile holds 1 to 3 bytes, some with an extra space
    inside, and tiles of 4 KiB."""
    g = workloads.rng(workloads.SEED_BASE + 199)
    alpha = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
    picked = fell_back = short_last = 0
    ts = 4096
    for trial in range(400):
        L = int(g.choice([16, 20, 64, 76]))
        s = int(g.integers(1, 3))
        sep = b"\r\n"[2 - s:]
        n_sig = int(g.integers(1500, 4000)) * 4
        if trial % 4 == 1:                      # a last tile of 1 to 3 bytes
            while (n_sig + s * ((n_sig - 1) // L)) % ts not in (1, 2, 3):
                n_sig += 4
        body = bytes(alpha[int(c)] for c in g.integers(0, 64, n_sig))
        text = sep.join(body[i:i + L] for i in range(0, n_sig, L))
        if trial % 4 != 1:
            text += b" " * int(g.choice([0, 1, 2, 3, 100, 4000, 4093, 4096, 5000, 9000, 20000]))
        if trial % 3 == 0:                      # a break in the layout
            at = int(g.integers(0, len(text) // 2)) if trial % 2 else len(text) - int(g.integers(1, 80))
            text = text[:at] + b" " + text[at:]
        n, P = len(text), L + s
        ntiles = (n + ts - 1) // ts
        if ntiles < 2:
            continue
        lb = (ntiles - 1) * ts
        total = lined_before(lb, L, P) + sum(1 for c in text[lb:] if c not in WS)
        ql = total // 4 - 1
        jq = 4 * ql
        at_q = (jq // L) * P + jq % L
        frm = at_q - s
        if lb - frm > 64:
            continue
        picked += 1
        short_last += frm < lb
        checked = {}
        for j in range(4 * ql):
            p = (j // L) * P + j % L
            checked[p] = "char"
            if j % L == L - 1:
                for k in range(s):
                    checked[p + 1 + k] = "sep"
        for p in range(max(frm, 0), lb):        # k_ws_predict's own check
            checked[p] = "char" if p % P < L else "sep"
        assert all(p in checked for p in range(lb)), (L, s, trial)
        fits = all(p < n and ((text[p] in WS) == (kind == "sep")) for p, kind in checked.items())
        true_total = sum(1 for c in text if c not in WS)
        if fits:
            assert total == true_total, (L, s, trial)
        else:
            fell_back += 1
    assert picked > 100 and fell_back > 0 and short_last > 20, (picked, fell_back, short_last)
