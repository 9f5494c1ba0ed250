// b64_batch.hip -- batched ragged encode / decode kernels and their launchers.
//
// Buffers are packed back to back: buffer b is src[in_off[b] .. in_off[b+1]).
// The packed input [in_off[0], in_off[nbuf]) is cut into equal tiles of 32
// wave rounds (24 KiB of bytes for encode, 32 KiB of characters for decode),
// and tiles are dealt to waves grid-stride: wave w takes tiles w, w+W, w+2W...
// At any moment the waves of the grid therefore stream through one compact
// window of memory, as the single-buffer kernels do, instead of each walking
// a distant span of its own (which costs DRAM row locality: about a fifth of
// the bandwidth on MI355X).  A tile covers the groups (encode) or quanta
// (decode) whose first byte lies in it, buffer after buffer, with consecutive
// lanes on consecutive chunks of a per-buffer grid aligned for the stores;
// the grid is cut between tiles at output line starts rather than exactly at
// the tile boundary (grid_cut).  The 64 lanes of a wave look up the first
// buffer of 64 of its tiles at once (one binary search per lane over in_off),
// so the lookup costs one search latency per 64 tiles.  No work queue and no
// atomics beyond the first-invalid minimum.
//
// Ownership: the tile holding a buffer's first byte writes its encode out_len
// (and the out_len of an empty decode buffer); the tile holding a buffer's
// last quantum runs the decode tail path; buffers that start at the very end
// of the packed input (empty ones) belong to the last tile.
#include "b64_launch.h"

namespace b64hip {
namespace {

constexpr int64_t kTileRounds = 32;
constexpr int64_t kEncTile = kTileRounds * 64 * 12;   // input bytes per encode tile
constexpr int64_t kDecTile = kTileRounds * 64 * 16;   // input characters per decode tile

// First buffer b with in_off[b+1] >= pos: buffers that end before pos hold no
// work at or after it.
__device__ int64_t first_buffer(const int64_t *__restrict__ in_off, int64_t nbuf, int64_t pos)
{
    int64_t l = 0, r = nbuf;
    while (l < r) {
        const int64_t mid = (l + r) >> 1;
        if (in_off[mid + 1] < pos) l = mid + 1;
        else r = mid;
    }
    return l;
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Tiles of this wave and the first buffer of each.
struct TileWalk {
    int64_t base, end, tile_bytes, ntiles, W, w;

    __device__ TileWalk(const int64_t *__restrict__ in_off, int64_t nbuf, int64_t tile)
    {
        W = (int64_t)gridDim.x * kWaves;
        // the wave index is uniform across the wave; say so, so that it and
        // everything derived from it live in scalar registers
        w = logical_block() * kWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        base = in_off[0];
        end = in_off[nbuf];
        tile_bytes = tile;
        ntiles = end > base ? (end - base + tile - 1) / tile : 1;
    }
    // Lane l finds the first buffer of the wave's tile k0 + l.
    __device__ int64_t lookup(const int64_t *__restrict__ in_off, int64_t nbuf, int64_t k0,
                              int lane) const
    {
        const int64_t t = w + (k0 + lane) * W;
        return first_buffer(in_off, nbuf, t < ntiles ? base + t * tile_bytes : end);
    }
};

// A buffer's chunk grid: chunk j covers units (groups or quanta) h + 4j ..
// h + 4j + 3, j < nch.  A tile owns the chunks from grid_cut(its first unit)
// up to grid_cut(the next tile's first unit): the first chunk at or after
// unit u, rounded up to a multiple of P and capped at nch.  Neighbouring
// tiles compute the same cut, so every chunk has one owner, and every tile's
// share starts P chunks apart -- on a 128-byte output line.
__device__ __forceinline__ int64_t grid_cut(int64_t u, int64_t h, int64_t nch, int64_t P)
{
    int64_t j = u <= h ? 0 : (u - h + 3) >> 2;
    j = (j + P - 1) / P * P;
    return j < nch ? j : nch;
}

// Chunks between two line starts: 8 of 16 output bytes (encode), 32 of 12
// (decode: 384 bytes, three lines).
constexpr int64_t kEncAlign = kLine / 16, kDecAlign = kLine / 4;

// Encode the groups whose first byte lies in [lo, hi), starting at buffer b0.
// Per buffer the chunk grid starts `h` groups in (h < 32) and tiles cut it at
// line starts (grid_cut), so that whenever the buffer's output is 4-byte
// aligned every store instruction of a round (64 chunks, 1 KiB) covers whole
// 128-byte lines, as in the single-buffer kernel; a span that starts inside a
// line leaves two partial lines, whose halves reach memory separately under
// nontemporal stores.  The groups outside the grid -- the h before it and the
// at most three whole groups and one partial group after it -- go to the
// lanes in turn, each to the tile holding its first byte.
template <int U, bool NT>
__device__ void encode_tile(const uint8_t *__restrict__ src, const int64_t *__restrict__ in_off,
                            int64_t nbuf, uint8_t *__restrict__ dst,
                            const int64_t *__restrict__ out_off, int64_t *__restrict__ out_len,
                            const uint8_t *a, int64_t lo, int64_t hi, int64_t b0, bool last, int lane,
                            bool pad)
{
    if (b0 >= nbuf) return;
    // offsets of the next buffer, loaded one iteration ahead
    int64_t nx_s = in_off[b0], nx_e = in_off[b0 + 1], nx_o = out_off[b0];
    for (int64_t b = b0; b < nbuf; ++b) {
        const int64_t s = nx_s, e = nx_e, ob_off = nx_o;
        if (b + 1 < nbuf) {
            nx_s = e;
            nx_e = in_off[b + 2];
            nx_o = out_off[b + 1];
        }
        if (s >= hi && !(last && s == hi)) break;
        const int64_t len = e - s;
        const int64_t ngroups = (len + 2) / 3, nfull = len / 3;
        if (s >= lo && lane == 0) out_len[b] = pad ? 4 * ngroups : (4 * len + 2) / 3;
        const int64_t g_lo = s >= lo ? 0 : (lo - s + 2) / 3;
        int64_t g_hi = hi <= s ? 0 : (hi - s + 2) / 3;
        if (g_hi > ngroups) g_hi = ngroups;
        if (g_lo >= g_hi) continue;
        uint8_t *ob = dst + ob_off;
        const uint64_t oa = (uint64_t)(uintptr_t)ob;
        int64_t h = (oa & 3) ? 0 : (int64_t)((((uint64_t)kLine - (oa & (kLine - 1))) & (kLine - 1)) >> 2);
        if (h > nfull) h = nfull;
        const int64_t nch = (nfull - h) >> 2;
        const int64_t j_lo = grid_cut(g_lo, h, nch, kEncAlign), j_hi = grid_cut(g_hi, h, nch, kEncAlign);
        const int64_t nchunk = j_hi - j_lo;
        const int64_t c_first = h + 4 * j_lo;   // first chunked group
        const uint8_t *sp = src + s + 3 * c_first;
        uint8_t *dp = ob + 4 * c_first;
        // rounds of 64*U chunks; all but the last are complete
        const int64_t nround = nchunk / (64 * U);
        enc_stream<U, NT>(sp, dp, lane, 64, 64 * U, nround, a);
        enc_round_tail<U, NT>(sp, dp, lane + nround * 64 * U, 64, a, nchunk);
        // groups outside the grid: [g_lo, min(g_hi, h)) and [max(g_lo, h + 4*nch), g_hi)
        const int64_t pre_hi = g_hi < h ? g_hi : h;
        const int64_t npre = pre_hi > g_lo ? pre_hi - g_lo : 0;
        const int64_t post_lo = g_lo > h + 4 * nch ? g_lo : h + 4 * nch;
        const int64_t nleft = npre + (g_hi > post_lo ? g_hi - post_lo : 0);
        for (int64_t i = lane; i < nleft; i += 64) {
            const int64_t g = i < npre ? g_lo + i : post_lo + (i - npre);
            const int64_t rem = len - 3 * g;
            enc_scalar(src + s + 3 * g, rem < 3 ? rem : 3, ob + 4 * g, a, pad);
        }
    }
}

template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_encode_batch(
    const uint8_t *__restrict__ src, const int64_t *__restrict__ in_off, int64_t nbuf,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off, int64_t *__restrict__ out_len,
    EncTab tab, uint32_t flags)
{
    const bool pad = !(flags & kFlagNoPad);
    __shared__ uint32_t s_tab[16];
    stage_enc_table(s_tab, tab);
    const uint8_t *a = (const uint8_t *)s_tab;
    const int lane = threadIdx.x & 63;
    const TileWalk tw(in_off, nbuf, kEncTile);
    int64_t b_lane = 0;
    for (int64_t k = 0; tw.w + k * tw.W < tw.ntiles; ++k) {
        if ((k & 63) == 0) b_lane = tw.lookup(in_off, nbuf, k, lane);
        const int64_t tile = tw.w + k * tw.W;
        const int64_t b0 = readlane64(b_lane, (int)(k & 63));
        const int64_t lo = tw.base + tile * tw.tile_bytes;
        const bool last = tile == tw.ntiles - 1;
        const int64_t hi = last ? tw.end : lo + tw.tile_bytes;
        encode_tile<U, NT>(src, in_off, nbuf, dst, out_off, out_len, a, lo, hi, b0, last, lane, pad);
    }
}

// Decode the quanta whose first character lies in [lo, hi), starting at
// buffer b0.  The body of a buffer is its quanta but the last.  Per buffer the
// chunk grid starts `h` body quanta in (h < 128, 3h = -out mod 128) and tiles
// cut it at line starts (grid_cut), so that every store instruction of a
// round (64 chunks, 768 bytes) covers whole 128-byte lines; chunks of four
// body quanta go to lanes, and the quanta outside the grid -- the h before
// it, the at most three body quanta after it and the last quantum (through
// dec_tail_fast) -- to the lanes in turn, each to the tile holding its first
// character.
template <int U, bool NT>
__device__ void decode_tile(const uint8_t *__restrict__ src, const int64_t *__restrict__ in_off,
                            int64_t nbuf, uint8_t *__restrict__ dst,
                            const int64_t *__restrict__ out_off, int64_t *__restrict__ out_len,
                            int64_t *__restrict__ first_bad, const uint8_t *m, int64_t lo,
                            int64_t hi, int64_t b0, bool last, int lane, bool nopad)
{
    if (b0 >= nbuf) return;
    // offsets of the next buffer, loaded one iteration ahead
    int64_t nx_s = in_off[b0], nx_e = in_off[b0 + 1], nx_o = out_off[b0];
    for (int64_t b = b0; b < nbuf; ++b) {
        const int64_t s = nx_s, e = nx_e, ob_off = nx_o;
        if (b + 1 < nbuf) {
            nx_s = e;
            nx_e = in_off[b + 2];
            nx_o = out_off[b + 1];
        }
        if (s >= hi && !(last && s == hi)) break;
        const int64_t len = e - s;
        if (len == 0) {
            if (s >= lo && lane == 0) out_len[b] = 0;
            continue;
        }
        const int64_t nq = (len + 3) >> 2;           // quanta, the last maybe partial
        const int64_t nbody = (len - 1) >> 2;        // all quanta but the last
        const int64_t q_lo = s >= lo ? 0 : (lo - s + 3) >> 2;
        int64_t q_hi = hi <= s ? 0 : (hi - s + 3) >> 2;
        if (q_hi > nq) q_hi = nq;
        if (q_lo >= q_hi) continue;
        uint8_t *ob = dst + ob_off;
        int64_t h = (int64_t)(((0 - (uint64_t)(uintptr_t)ob) * 43u) & (uint64_t)(kLine - 1));
        if (h > nbody) h = nbody;
        const int64_t nch = (nbody - h) >> 2;
        const int64_t j_lo = grid_cut(q_lo, h, nch, kDecAlign), j_hi = grid_cut(q_hi, h, nch, kDecAlign);
        const int64_t nchunk = j_hi - j_lo;
        const int64_t c_first = h + 4 * j_lo;   // first chunked quantum
        const uint8_t *sp = src + s + 4 * c_first;
        uint8_t *dp = ob + 3 * c_first;
        uint32_t err = 0;
        // rounds of 64*U chunks; all but the last are complete
        const int64_t nround = nchunk / (64 * U);
        dec_stream<U, NT>(sp, dp, lane, 64, 64 * U, nround, m, err);
        dec_round_tail<U, NT>(sp, dp, lane + nround * 64 * U, 64, m, err, nchunk);
        if (__ballot(err & 0x80)) {
            if (err & 0x80) {
                for (int64_t k = lane; k < nchunk; k += 64) {
                    const int64_t bad = dec_check_inner(sp + 16 * k, 16, m, nopad);
                    if (bad >= 0) {
                        atomic_min_i64(first_bad + b, 4 * c_first + 16 * k + bad);
                        break;
                    }
                }
            }
        }
        // quanta outside the grid: [q_lo, min(q_hi, h)) and [max(q_lo, h + 4*nch), q_hi)
        const int64_t pre_hi = q_hi < h ? q_hi : h;
        const int64_t npre = pre_hi > q_lo ? pre_hi - q_lo : 0;
        const int64_t post_lo = q_lo > h + 4 * nch ? q_lo : h + 4 * nch;
        const int64_t nleft = npre + (q_hi > post_lo ? q_hi - post_lo : 0);
        for (int64_t i = lane; i < nleft; i += 64) {
            const int64_t q = i < npre ? q_lo + i : post_lo + (i - npre);
            const uint8_t *qp = src + s + 4 * q;
            uint8_t *qo = ob + 3 * q;
            if (q < nbody) {
                uint32_t qerr = 0;
                const uint32_t v = dec_quantum(*(const u32a1 *)qp, m, qerr);
                qo[0] = (uint8_t)(v >> 16);
                qo[1] = (uint8_t)(v >> 8);
                qo[2] = (uint8_t)v;
                if (qerr & 0x80) {
                    const int64_t bad = dec_check_inner(qp, 4, m, nopad);
                    if (bad >= 0) atomic_min_i64(first_bad + b, 4 * q + bad);
                }
            } else {
                int64_t ol = 0;
                const int64_t bad = dec_tail_fast(qp, len - 4 * q, len, qo, m, &ol, nopad);
                if (bad >= 0) atomic_min_i64(first_bad + b, 4 * q + bad);
                else out_len[b] = ol;
            }
        }
    }
}

template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_decode_batch(
    const uint8_t *__restrict__ src, const int64_t *__restrict__ in_off, int64_t nbuf,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off, int64_t *__restrict__ out_len,
    int64_t *__restrict__ first_bad, DecMap map, uint32_t flags)
{
    const bool nopad = (flags & kFlagNoPad) != 0;
    __shared__ uint32_t s_map[64];
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;
    const int lane = threadIdx.x & 63;
    const TileWalk tw(in_off, nbuf, kDecTile);
    int64_t b_lane = 0;
    for (int64_t k = 0; tw.w + k * tw.W < tw.ntiles; ++k) {
        if ((k & 63) == 0) b_lane = tw.lookup(in_off, nbuf, k, lane);
        const int64_t tile = tw.w + k * tw.W;
        const int64_t b0 = readlane64(b_lane, (int)(k & 63));
        const int64_t lo = tw.base + tile * tw.tile_bytes;
        const bool last = tile == tw.ntiles - 1;
        const int64_t hi = last ? tw.end : lo + tw.tile_bytes;
        decode_tile<U, NT>(src, in_off, nbuf, dst, out_off, out_len, first_bad, m, lo, hi, b0,
                           last, lane, nopad);
    }
}

}  // namespace

hipError_t launch_encode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                               uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                               const EncTab &tab, uint32_t flags, Shape sh, int cus, hipStream_t stream)
{
    const int64_t grid = (int64_t)cus * sh.bpc;
    B64_DISPATCH(k_encode_batch, sh, grid, stream, src, in_off, nbuf, dst, out_off, out_len, tab,
                 flags);
    return hipGetLastError();
}

hipError_t launch_decode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                               uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                               int64_t *first_bad, const DecMap &map, uint32_t flags, Shape sh,
                               int cus, hipStream_t stream)
{
    const int64_t grid = (int64_t)cus * sh.bpc;
    B64_DISPATCH(k_decode_batch, sh, grid, stream, src, in_off, nbuf, dst, out_off, out_len,
                 first_bad, map, flags);
    return hipGetLastError();
}

}  // namespace b64hip
