"""CPU model of the batched kernels' work partition (no GPU).

The batched kernels cut the packed input into equal tiles, deal the tiles to
waves grid-stride, and let each wave walk the buffers a tile touches.  This
test re-traces that index arithmetic on the host for many layouts, tile sizes
and grid sizes and checks, before any launch, that:
  - every group (encode) / quantum (decode) of every buffer is handled exactly
    once, by a lane chunk or by a lane that takes one unit outside the chunk
    grid (the tile holding the unit's first byte);
  - each tile's share of a buffer's chunk grid starts on a 128-byte output
    line (encode: when the output is 4-byte aligned; decode: always), so that
    every store instruction of a round covers whole lines;
  - every read stays inside its buffer and every write inside its output
    capacity;
  - exactly one wave writes each encode out_len, and exactly one lane runs the
    tail path of each non-empty decode buffer.
"""
import numpy as np
import pytest

import workloads

WAVES_PER_BLOCK = 4
XCDS = 8


def logical_block(b, G):
    if G % XCDS:
        return b
    return (b % XCDS) * (G // XCDS) + b // XCDS


def first_buffer(in_off, nbuf, pos):
    l, r = 0, nbuf
    while l < r:
        mid = (l + r) >> 1
        if in_off[mid + 1] < pos:
            l = mid + 1
        else:
            r = mid
    return l


LINE = 128
ENC_ALIGN, DEC_ALIGN = LINE // 16, LINE // 4


def grid_cut(u, h, nch, P):
    """First chunk of a tile's share: the first chunk at or after unit u,
    rounded up to a multiple of P, at most nch."""
    j = 0 if u <= h else (u - h + 3) >> 2
    j = (j + P - 1) // P * P
    return min(j, nch)


def tiles(in_off, nbuf, tile, grid):
    """(lo, hi, b0, last) of every tile, in the order the waves take them."""
    W = grid * WAVES_PER_BLOCK
    base, end = int(in_off[0]), int(in_off[nbuf])
    ntiles = (end - base + tile - 1) // tile if end > base else 1
    for blk in range(grid):
        for wv in range(WAVES_PER_BLOCK):
            w = logical_block(blk, grid) * WAVES_PER_BLOCK + wv
            k = 0
            while w + k * W < ntiles:
                t = w + k * W
                lo = base + t * tile
                last = t == ntiles - 1
                hi = end if last else lo + tile
                assert hi <= end
                yield lo, hi, first_buffer(in_off, nbuf, lo), last
                k += 1


def trace_encode(in_off, out_off, nbuf, grid, tile, dst_base=0):
    seen = [np.zeros((int(in_off[b + 1] - in_off[b]) + 2) // 3, dtype=np.int64) for b in range(nbuf)]
    owners = np.zeros(nbuf, dtype=np.int64)
    for lo, hi, b0, last in tiles(in_off, nbuf, tile, grid):
        for b in range(b0, nbuf):
            s, e = int(in_off[b]), int(in_off[b + 1])
            if s >= hi and not (last and s == hi):
                break
            length = e - s
            ngroups, nfull = (length + 2) // 3, length // 3
            if s >= lo:
                owners[b] += 1
            g_lo = 0 if s >= lo else (lo - s + 2) // 3
            g_hi = 0 if hi <= s else (hi - s + 2) // 3
            g_hi = min(g_hi, ngroups)
            if g_lo >= g_hi:
                continue
            oa = dst_base + int(out_off[b])
            h = 0 if oa & 3 else ((LINE - (oa & (LINE - 1))) & (LINE - 1)) >> 2
            h = min(h, nfull)
            nch = (nfull - h) >> 2
            j_lo, j_hi = grid_cut(g_lo, h, nch, ENC_ALIGN), grid_cut(g_hi, h, nch, ENC_ALIGN)
            nchunk = j_hi - j_lo
            c_first = h + 4 * j_lo
            assert nchunk >= 0
            if nchunk:
                seen[b][c_first: c_first + 4 * nchunk] += 1
                # reads [s + 3 c_first, + 12 nchunk), writes 16 per chunk, on lines
                assert s + 3 * c_first + 12 * nchunk <= e
                assert 4 * c_first + 16 * nchunk <= 4 * ngroups
                if oa % 4 == 0:
                    assert (oa + 4 * c_first) % LINE == 0
            pre_hi = min(g_hi, h)
            npre = max(pre_hi - g_lo, 0)
            post_lo = max(g_lo, h + 4 * nch)
            nleft = npre + max(g_hi - post_lo, 0)
            assert nleft <= 35
            for i in range(nleft):
                g = g_lo + i if i < npre else post_lo + (i - npre)
                assert g < g_hi
                rem = length - 3 * g
                assert rem > 0 and 3 * g + min(rem, 3) <= length
                seen[b][g] += 1
    for b in range(nbuf):
        assert (seen[b] == 1).all(), (b, seen[b])
    assert (owners == 1).all(), np.nonzero(owners != 1)


def trace_decode(in_off, nbuf, grid, tile, dst_base=0):
    out_off = workloads.offsets(3 * (np.diff(in_off) // 4))
    seen = [np.zeros((int(in_off[b + 1] - in_off[b]) + 3) // 4, dtype=np.int64) for b in range(nbuf)]
    tails = np.zeros(nbuf, dtype=np.int64)
    empty_owner = np.zeros(nbuf, dtype=np.int64)
    for lo, hi, b0, last in tiles(in_off, nbuf, tile, grid):
        for b in range(b0, nbuf):
            s, e = int(in_off[b]), int(in_off[b + 1])
            if s >= hi and not (last and s == hi):
                break
            length = e - s
            if length == 0:
                if s >= lo:
                    empty_owner[b] += 1
                continue
            nq, nbody = (length + 3) >> 2, (length - 1) >> 2
            q_lo = 0 if s >= lo else (lo - s + 3) >> 2
            q_hi = min(0 if hi <= s else (hi - s + 3) >> 2, nq)
            if q_lo >= q_hi:
                continue
            oa = dst_base + int(out_off[b])
            h = min((-oa * 43) & (LINE - 1), nbody)
            nch = (nbody - h) >> 2
            j_lo, j_hi = grid_cut(q_lo, h, nch, DEC_ALIGN), grid_cut(q_hi, h, nch, DEC_ALIGN)
            nchunk = j_hi - j_lo
            c_first = h + 4 * j_lo
            assert nchunk >= 0
            if nchunk:
                seen[b][c_first: c_first + 4 * nchunk] += 1
                assert 4 * c_first + 16 * nchunk <= 4 * nbody < length
                assert 3 * c_first + 12 * nchunk <= 3 * (length // 4)
                assert (oa + 3 * c_first) % LINE == 0
            pre_hi = min(q_hi, h)
            npre = max(pre_hi - q_lo, 0)
            post_lo = max(q_lo, h + 4 * nch)
            nleft = npre + max(q_hi - post_lo, 0)
            assert nleft <= 131
            for i in range(nleft):
                q = q_lo + i if i < npre else post_lo + (i - npre)
                assert q < q_hi
                seen[b][q] += 1
                if q < nbody:
                    assert 4 * q + 4 <= length and 3 * q + 3 <= 3 * (length // 4)
                else:
                    assert q == nq - 1
                    tails[b] += 1
    for b in range(nbuf):
        assert (seen[b] == 1).all(), (b, seen[b])
        n = int(in_off[b + 1] - in_off[b])
        assert tails[b] == (1 if n else 0)
        assert empty_owner[b] == (0 if n else 1)


def _layouts():
    g = workloads.rng(77)
    yield np.array([0, 0], dtype=np.int64)                         # one empty buffer
    yield np.array([5, 5, 5, 5], dtype=np.int64)                   # all empty, offset base
    yield np.array([0, 1 << 20], dtype=np.int64)                   # one big buffer
    yield workloads.offsets(np.arange(0, 40, dtype=np.int64)) + 3  # every tiny length
    for k in range(6):
        nbuf = int(g.integers(1, 400))
        lens = g.integers(0, 20_000, size=nbuf)
        lens[g.random(nbuf) < 0.2] = 0
        yield workloads.offsets(lens.astype(np.int64)) + int(g.integers(0, 17))
    lens = workloads.batch_lengths(78, 300)
    yield workloads.offsets(lens)


# the kernels use 32 wave rounds per tile (24576 bytes for encode, 32768
# characters for decode); smaller tiles exercise more tile boundaries here
@pytest.mark.parametrize("grid,tile", [(1, 24576), (2, 768), (3, 1536), (8, 24576), (16, 768),
                                       (40, 3072)])
def test_encode_partition(grid, tile):
    for in_off in _layouts():
        nbuf = in_off.size - 1
        out_off = workloads.offsets(4 * ((np.diff(in_off) + 2) // 3))
        for dst_base in (0, 1, 4, 8, 12):
            trace_encode(in_off, out_off, nbuf, grid, tile, dst_base)


@pytest.mark.parametrize("grid,tile", [(1, 32768), (2, 1024), (3, 2048), (8, 32768), (16, 1024),
                                       (40, 4096)])
def test_decode_partition(grid, tile):
    for in_off in _layouts():
        for dst_base in (0, 1, 2, 3):
            trace_decode(in_off, in_off.size - 1, grid, tile, dst_base)


def test_single_buffer_heads_align_outputs():
    """Single-buffer kernels set aside `head` groups / quanta so that chunk
    outputs start on a 128-byte line, and never more than the body holds."""
    for addr in range(0, 512):
        ehead = 0 if addr & 3 else ((128 - (addr & 127)) & 127) >> 2
        assert ehead < 32
        if addr % 4 == 0:
            assert (addr + 4 * ehead) % 128 == 0
        dhead = (-addr * 43) & 127
        assert (addr + 3 * dhead) % 128 == 0 and dhead < 128
