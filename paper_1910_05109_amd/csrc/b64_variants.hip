// b64_variants.hip -- line-wrapped encode and whitespace-skipping decode.
//
// The paper's codec handles base64 as one unbroken string; MIME email, which
// the paper names as a main carrier of base64 (Section "Introduction"), breaks
// it into lines separated by CR LF.  These kernels add the two MIME-style
// variants on top of the same per-lane arithmetic (enc_chunk, the 256-entry
// LDS map):
//
// Wrapped encode (k_encode_wrap).  Character j of the unwrapped encoding goes
// to position j + 2*floor(j / L) and a CR LF precedes every line after the
// first.  Lane chunks are the plain kernel's (12 bytes -> 16 characters); a
// lane tracks the line and column of its chunk incrementally, so no 64-bit
// division runs per chunk, and stores each group of four characters (L is a
// multiple of 4, so a line never splits a group) plus a CR LF where a line
// starts.
//
// Whitespace-skipping decode.  The significant characters (all but space,
// tab, CR, LF) form the encoding; their positions in the input depend on
// every whitespace byte before them, so decoding is a stream compaction.
// After a status reset (k_ws_init), kernels with no inter-block waiting:
//   k_ws_count   per tile of TS characters: the number of significant
//                characters, and (atomic minima) the first invalid character
//                and the first '='.
//   k_ws_scan    one block: inclusive prefix sums of the tile counts.
//   k_ws_decode  per tile, one wave: rounds of 1024 characters are compacted
//                into an LDS buffer (characters read back transposed, a
//                ballot and a masked bit count per row of 64 give each its
//                position) and the whole quanta whose first value lies in the
//                tile are decoded; the last one may borrow up to three values
//                from the following tiles.
//   k_ws_finish  one block: the '=' and end-of-input rules over the sequence
//                of significant characters, the final quantum, the status.
// Text in regular lines (MIME, PEM) skips the counting pass: k_ws_predict
// guesses the prefix sums from the first line and picks a path in the mode
// word.  For lines whose length is a multiple of 4 (16 or more), k_ws_lines
// reads every quantum at its closed-form position and checks each byte
// against the layout; other line lengths take k_ws_decode<.., true>, which
// decodes on the guessed sums and checks every tile's count (the tiles with
// no quantum of their own are only counted).  A failed check sets the mode word back to
// the counted path, and k_ws_count, k_ws_scan and k_ws_decode then run as
// above (every launch returns at once unless the mode word names its path).  Tiles are dealt grid-stride (to blocks in
// k_ws_count, to waves in k_ws_decode), so the grid streams through one
// window of memory.
#include "b64_launch.h"

namespace b64hip {
namespace {

typedef uint16_t u16a1 __attribute__((aligned(1)));

// ------------------------------------------------------------ wrapped encode --

// Characters [j0, j0+4k) of the unwrapped encoding, given as k words of four,
// stored for lines of L; (line, col) are those of character j0 (col a
// multiple of 4, col < L).
__device__ __forceinline__ void store_wrapped(uint8_t *dst, int64_t j0, int64_t line, int64_t col,
                                              int64_t L, const uint32_t *w, int k)
{
    for (int g = 0; g < k; ++g) {
        const int64_t j = j0 + 4 * g;
        const int64_t pos = j + 2 * line;
        if (col == 0 && j > 0) *(u16a1 *)(dst + pos - 2) = (uint16_t)('\r' | ('\n' << 8));
        *(u32a1 *)(dst + pos) = w[g];
        col += 4;
        if (col == L) {
            col = 0;
            ++line;
        }
    }
}

// The r <= 11 input bytes after the chunks, fetched early by enc_tail_load,
// encoded from registers and stored for lines of L; j0 is the index of their
// first character in the unwrapped encoding.  L is a multiple of 4, so each
// group (the padded or, with !pad, cut last one included) lands whole in one
// line; the line and column of j0 come from one division and are stepped per
// group.
__device__ __forceinline__ void enc_tail_wrap(const EncTailIn &ti, int r, int64_t j0, uint8_t *dst,
                                              int64_t L, const uint8_t *tab, bool pad)
{
    if (r <= 0) return;
    // shift the window right by off bytes: t[0..2] hold the r bytes in order
    const int q = ti.off >> 2;
    const uint32_t k = (uint32_t)(ti.off & 3);
    const uint32_t x0 = __builtin_amdgcn_alignbyte(ti.w[1], ti.w[0], k);
    const uint32_t x1 = __builtin_amdgcn_alignbyte(ti.w[2], ti.w[1], k);
    const uint32_t x2 = __builtin_amdgcn_alignbyte(0u, ti.w[2], k);
    const uint32_t t[3] = {q == 0 ? x0 : q == 1 ? x1 : q == 2 ? x2 : 0u,
                           q == 0 ? x1 : q == 1 ? x2 : 0u, q == 0 ? x2 : 0u};
    int64_t line = j0 / L, col = j0 - line * L;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int i = 3 * g;
        if (i >= r) break;
        const int kk = r - i < 3 ? r - i : 3;              // input bytes of the group
        const uint32_t s1 = (t[i >> 2] >> (8 * (i & 3))) & 0xFF;
        const uint32_t s2 = kk > 1 ? (t[(i + 1) >> 2] >> (8 * ((i + 1) & 3))) & 0xFF : 0u;
        const uint32_t s3 = kk > 2 ? (t[(i + 2) >> 2] >> (8 * ((i + 2) & 3))) & 0xFF : 0u;
        uint32_t v = enc_group(s2 | (s1 << 8) | (s3 << 16) | (s2 << 24), tab);
        int nc = kk + 1;                                   // characters that carry bits
        if (kk == 3) nc = 4;
        else if (pad) {
            v = kk == 1 ? (v & 0xFFFFu) | (kPad << 16) | (kPad << 24) : (v & 0xFFFFFFu) | (kPad << 24);
            nc = 4;
        }
        const int64_t j = j0 + 4 * g;
        uint8_t *o = dst + j + 2 * line;                   // j + 2 * floor(j / L)
        if (col == 0 && j > 0) *(u16a1 *)(o - 2) = (uint16_t)('\r' | ('\n' << 8));
        if (nc == 4) {
            *(u32a1 *)o = v;
        } else {
            o[0] = (uint8_t)v;
            o[1] = (uint8_t)(v >> 8);
            if (nc == 3) o[2] = (uint8_t)(v >> 16);
        }
        col += 4;
        if (col == L) {
            col = 0;
            ++line;
        }
    }
}

// Stores the chunks of one lane, in increasing order c, c+T, c+2T, ...:
// tracks the line and column of the next chunk's first character and steps
// them by T chunks (16T characters) per call.
// Lines of L in [16, 2^31) (at most one line starts inside a chunk): a lane
// tracks the output position of its chunk's first character (64 bits) and
// its column (32 bits), stepped by T chunks per call: pos += 16T + 2*(lines
// crossed).
struct WideSink {
    uint8_t *dst;
    int64_t pos, dpos;              // dpos = 16T + 2*((16T) / L)
    int32_t col, dcol, L;           // dcol = (16T) % L
    template <bool NT>
    __device__ __forceinline__ void put(int64_t c, u32x4 o)
    {
        constexpr uint32_t kCrLf = '\r' | ('\n' << 8);
        const int32_t a = col == 0 ? 0 : L - col;      // characters before the next line start
        const bool brk = col == 0 ? c > 0 : a < 16;
        const int k = brk ? a >> 2 : 4;                // dword of the break; 4: none
        const uint32_t w[5] = {o.x, o.y, o.z, o.w, 0u};
        uint32_t x[5];
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            // the dword shifted by the two inserted bytes: bytes 2,3 of w[d-1], bytes 0,1 of w[d]
            const uint32_t shifted = d == 0 ? (w[0] << 16) : __builtin_amdgcn_alignbyte(w[d], w[d - 1], 2);
            x[d] = d < k ? w[d] : (d == k ? (kCrLf | (w[d] << 16)) : shifted);
        }
        uint8_t *q = dst + pos - (brk && a == 0 ? 2 : 0);
        store16<NT>(q, u32x4{x[0], x[1], x[2], x[3]});
        if (brk) *(u16a1 *)(q + 16) = (uint16_t)x[4];
        col += dcol;
        const bool wrap = col >= L;
        col -= wrap ? L : 0;
        pos += dpos + (wrap ? 2 : 0);
    }
};

// Shorter lines (or longer than 2^31): lane by lane per group of four.
struct WrapSink {
    uint8_t *dst;
    int64_t L, line, col, dline, dcol;
    template <bool NT>
    __device__ __forceinline__ void put(int64_t c, u32x4 o)
    {
        const uint32_t w[4] = {o.x, o.y, o.z, o.w};
        store_wrapped(dst, 16 * c, line, col, L, w, 4);
        line += dline;
        col += dcol;
        if (col >= L) {
            col -= L;
            ++line;
        }
    }
};

// enc_stream's software-pipelined rounds (the loads of round r+1 issued
// before round r is stored) with the stores done by a WrapSink.
template <int U, bool NT, typename Sink>
__device__ __forceinline__ void enc_stream_wrap(const uint8_t *s0, int64_t c0, int64_t stride,
                                                int64_t rstep, int64_t nrounds, const uint8_t *tab,
                                                Sink &sink)
{
    if (nrounds <= 0) return;
    u32x3 A[U], B[U];
    enc_load<U, NT>(A, s0, c0, stride);
    int64_t r = 0;
    for (; r + 2 < nrounds; r += 2) {
        enc_load<U, NT>(B, s0, c0 + rstep, stride);
#pragma unroll
        for (int j = 0; j < U; ++j) sink.template put<NT>(c0 + j * stride, enc_chunk(A[j], tab));
        enc_load<U, NT>(A, s0, c0 + 2 * rstep, stride);
#pragma unroll
        for (int j = 0; j < U; ++j) sink.template put<NT>(c0 + rstep + j * stride, enc_chunk(B[j], tab));
        c0 += 2 * rstep;
    }
    if (r + 1 < nrounds) {
        enc_load<U, NT>(B, s0, c0 + rstep, stride);
#pragma unroll
        for (int j = 0; j < U; ++j) sink.template put<NT>(c0 + j * stride, enc_chunk(A[j], tab));
#pragma unroll
        for (int j = 0; j < U; ++j) sink.template put<NT>(c0 + rstep + j * stride, enc_chunk(B[j], tab));
    } else {
#pragma unroll
        for (int j = 0; j < U; ++j) sink.template put<NT>(c0 + j * stride, enc_chunk(A[j], tab));
    }
}

// Lane chunk c (input [12c, 12c+12), characters [16c, 16c+16)) for chunks
// c = t, t+T, ... < nch: complete rounds of U per lane through
// enc_stream_wrap, then a partial round with clamped loads; the last thread
// encodes what follows the chunks.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_encode_wrap(const uint8_t *__restrict__ src, int64_t n,
                                                          uint8_t *__restrict__ dst, EncTab tab,
                                                          uint32_t flags, int64_t L)
{
    const int64_t nch = n / 12;
    const int64_t T = (int64_t)gridDim.x * kThreads;
    const int64_t t = logical_block() * kThreads + threadIdx.x;
    // the bytes after the chunks: loaded now, encoded last (from registers)
    EncTailIn tin;
    if (t == kThreads - 1) tin = enc_tail_load(src + 12 * nch, (int)(n - 12 * nch), 12 * nch, n);

    __shared__ uint32_t s_tab[16];
    stage_enc_table(s_tab, tab);
    const uint8_t *a = (const uint8_t *)s_tab;

    const int64_t nfull = nch / (U * T);
    const int64_t c0 = t + nfull * U * T;
    // complete rounds, then the partial round with clamped loads
    auto run = [&](auto &sink) {
        enc_stream_wrap<U, NT>(src, t, T, U * T, nfull, a, sink);
        if (c0 < nch) {
            u32x3 in[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t c = c0 + j * T;
                in[j] = load12<NT>(src + 12 * (c < nch ? c : nch - 1));
            }
            for (int j = 0; j < U; ++j) {
                if (c0 + j * T >= nch) break;
                sink.template put<NT>(c0 + j * T, enc_chunk(in[j], a));
            }
        }
    };
    // the output position (or line) and column of this thread's first
    // character, and their steps per T chunks
    if (L >= 16 && L < ((int64_t)1 << 31)) {
        const int64_t line0 = (16 * t) / L, dline = (16 * T) / L;
        WideSink sink{dst, 16 * t + 2 * line0, 16 * T + 2 * dline, (int32_t)((16 * t) % L),
                      (int32_t)((16 * T) % L), (int32_t)L};
        run(sink);
    } else {
        WrapSink sink{dst, L, (16 * t) / L, (16 * t) % L, (16 * T) / L, (16 * T) % L};
        run(sink);
    }
    if (t == kThreads - 1)
        enc_tail_wrap(tin, (int)(n - 12 * nch), 16 * nch, dst, L, a, !(flags & kFlagNoPad));
}

// ------------------------------------------------ whitespace-skipping decode --

// Map codes: 0..63 alphabet values, kWsCode for the four ignored bytes,
// kPadCode for '=' in padded mode, kBadCode for everything else.  Bit 6 marks
// whitespace, bit 7 an invalid character or '='.
constexpr uint32_t kWsCode = 0x40, kBadCode = 0x80, kPadCode = 0x81;
constexpr int kWsBlock = 256;            // threads per block of the tile kernels
constexpr int64_t kRound = kWsBlock * 16;   // characters per block round
constexpr int kMaxRounds = 8;            // rounds per tile at most (tiles of 4 .. 32 KiB)

// The mode word in the decode workspace: kModeCounted, the counted path
// (k_ws_count, k_ws_scan, k_ws_decode) runs; kModeChecked, k_ws_decode<.., true>
// runs on guessed prefix sums; kModeLines | s << 2 | L << 4,
// k_ws_lines runs for lines of L significant characters and s separator
// bytes.  A failed check sets it back to kModeCounted.
constexpr int64_t kModeCounted = 0, kModeChecked = 1, kModeLines = 2;

__device__ __forceinline__ bool is_sig(uint32_t code) { return !(code & kWsCode); }

// Four codes of a dword of characters, packed as bytes.
__device__ __forceinline__ uint32_t codes4(uint32_t q, const uint8_t *map)
{
    return (uint32_t)map[q & 0xFF] | ((uint32_t)map[(q >> 8) & 0xFF] << 8) |
           ((uint32_t)map[(q >> 16) & 0xFF] << 16) | ((uint32_t)map[q >> 24] << 24);
}

// Codes of the last r (1 .. 15) characters of an input, given the 16 bytes
// that end the input (b), as the codes of a 16-character chunk that starts r
// characters before the end: b is shifted down by 16 - r bytes, and the
// positions from r on read as whitespace.
__device__ __forceinline__ u32x4 ws_codes_window(u32x4 b, int r, const uint8_t *map)
{
    const int sh = 16 - r, q = sh >> 2;
    const uint32_t k = (uint32_t)(sh & 3);
    const uint32_t x0 = __builtin_amdgcn_alignbyte(b.y, b.x, k);
    const uint32_t x1 = __builtin_amdgcn_alignbyte(b.z, b.y, k);
    const uint32_t x2 = __builtin_amdgcn_alignbyte(b.w, b.z, k);
    const uint32_t x3 = __builtin_amdgcn_alignbyte(0u, b.w, k);
    const uint32_t t[4] = {q == 0 ? x0 : q == 1 ? x1 : q == 2 ? x2 : x3,
                           q == 0 ? x1 : q == 1 ? x2 : q == 2 ? x3 : 0u,
                           q == 0 ? x2 : q == 1 ? x3 : 0u, q == 0 ? x3 : 0u};
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int keep = r - 4 * i;
        const uint32_t msk = keep >= 4 ? 0xFFFFFFFFu : keep <= 0 ? 0u : (1u << (8 * keep)) - 1u;
        w[i] = (codes4(t[i], map) & msk) | (0x40404040u & ~msk);
    }
    return u32x4{w[0], w[1], w[2], w[3]};
}

// The 16 characters at p as packed codes; characters at or past n read as
// whitespace.  A partial chunk of an input of 16 bytes or more is one load of
// the 16 bytes that end at n (byte loads would each wait for the one before).
template <bool NT>
__device__ __forceinline__ u32x4 ws_codes(const uint8_t *src, int64_t n, int64_t p,
                                          const uint8_t *map)
{
    u32x4 c;
    if (p + 16 <= n) {
        const u32x4 q = load16<NT>(src + p);
        c.x = codes4(q.x, map);
        c.y = codes4(q.y, map);
        c.z = codes4(q.z, map);
        c.w = codes4(q.w, map);
    } else if (n >= 16) {
        c = ws_codes_window(load16<NT>(src + n - 16), (int)(n - p), map);
    } else {
        uint32_t w[4] = {0, 0, 0, 0};
        for (int j = 0; j < 16; ++j) {
            const uint32_t code = p + j < n ? (uint32_t)map[src[p + j]] : kWsCode;
            w[j >> 2] |= code << (8 * (j & 3));
        }
        c.x = w[0];
        c.y = w[1];
        c.z = w[2];
        c.w = w[3];
    }
    return c;
}

__device__ __forceinline__ int sig_count(u32x4 c)
{
    // significant = bit 6 clear
    return 16 - __builtin_popcount(c.x & 0x40404040u) - __builtin_popcount(c.y & 0x40404040u) -
           __builtin_popcount(c.z & 0x40404040u) - __builtin_popcount(c.w & 0x40404040u);
}

__host__ __device__ __forceinline__ int64_t ws_tiles(int64_t n, int64_t TS) { return n > 0 ? (n + TS - 1) / TS : 0; }

// Codes of a full 16-character load.
__device__ __forceinline__ u32x4 codes16(u32x4 q, const uint8_t *map)
{
    u32x4 c;
    c.x = codes4(q.x, map);
    c.y = codes4(q.y, map);
    c.z = codes4(q.z, map);
    c.w = codes4(q.w, map);
    return c;
}

// k_ws_count: tile `tile` covers characters [tile*TS, min(n, (tile+1)*TS)),
// TS = R rounds of kRound; prefix[tile+1] receives its number of significant
// characters.  A full tile issues all R loads of a thread before it looks at
// any.  Invalid characters go to *first_bad, '=' (padded mode) to
// *first_pad, both by atomic minimum; both must hold kNoError before the
// launch.  It does nothing when the checked decode has succeeded (*mode 1).
template <int R, bool NT>
__global__ __launch_bounds__(kWsBlock) void k_ws_count(const uint8_t *__restrict__ src, int64_t n,
                                                       DecMap map, int64_t *__restrict__ prefix,
                                                       int64_t *__restrict__ first_pad,
                                                       int64_t *__restrict__ first_bad,
                                                       const int64_t *__restrict__ mode)
{
    constexpr int64_t TS = R * kRound;
    __shared__ uint32_t s_map[64];
    __shared__ int s_sum;
    if (*mode != kModeCounted) return;
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;
    const int64_t ntiles = ws_tiles(n, TS);
    for (int64_t tile = logical_block(); tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * TS, end = base + TS < n ? base + TS : n;
        int cnt = 0;
        uint32_t err = 0;
        if (end - base == TS) {
            u32x4 q[R];
#pragma unroll
            for (int r = 0; r < R; ++r) q[r] = load16<NT>(src + base + r * kRound + 16 * threadIdx.x);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const u32x4 c = codes16(q[r], m);
                cnt += sig_count(c);
                err |= c.x | c.y | c.z | c.w;
            }
        } else {
            for (int64_t p = base + 16 * threadIdx.x; p < end; p += kRound) {
                const u32x4 c = ws_codes<NT>(src, end, p, m);
                cnt += sig_count(c);
                err |= c.x | c.y | c.z | c.w;
            }
        }
        // err ORs packed codes: bit 7 of any byte flags an invalid character or '='
        if (__ballot(err & 0x80808080u)) {
            if (err & 0x80808080u) {
                bool bad_found = false, pad_found = false;
                for (int64_t p = base + 16 * threadIdx.x; p < end && !(bad_found && pad_found); p += kRound) {
                    for (int64_t i = p; i < p + 16 && i < end; ++i) {
                        const uint32_t code = m[src[i]];
                        if (code == kBadCode && !bad_found) {
                            atomic_min_i64(first_bad, i);
                            bad_found = true;
                        } else if (code == kPadCode && !pad_found) {
                            atomic_min_i64(first_pad, i);
                            pad_found = true;
                        }
                    }
                }
            }
        }
        if (threadIdx.x == 0) s_sum = 0;
        __syncthreads();
        // sum over the block: wave sums, then one LDS atomic per wave
        int x = cnt;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
        if ((threadIdx.x & 63) == 0) atomicAdd(&s_sum, x);
        __syncthreads();
        if (threadIdx.x == 0) prefix[tile + 1] = s_sum;
        __syncthreads();
    }
}

// k_ws_scan: prefix[0] = 0 and prefix[1..ntiles] turned into inclusive sums,
// by one block, kScanRows rows of kScanThreads counts per pass.  Thread t
// holds entry t of every row, so every load and store of the block is
// contiguous.  A row is scanned in 32 bits (a tile count is at most 32 KiB,
// so a row sums to less than 2^31): an inclusive scan within each wave, the
// exclusive sums of the waves' totals, then a 64-bit exclusive scan of the row
// totals carried across passes.
constexpr int kScanThreads = 1024, kScanRows = 48;

// Inclusive sum over the 64 lanes of a wave with DPP: shifts by 1, 2, 4, 8
// within rows of 16 lanes, then the last lane of rows 0 and 2 added to rows 1
// and 3, and the last lane of row 1 to rows 2 and 3.
__device__ __forceinline__ int wave_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return x;
}

__global__ __launch_bounds__(kScanThreads) void k_ws_scan(int64_t *__restrict__ prefix, int64_t ntiles,
                                                          const int64_t *__restrict__ mode)
{
    constexpr int kW = kScanThreads / 64;
    __shared__ int s_wave[kScanRows][kW];        // wave totals, then their exclusive sums
    __shared__ int64_t s_row[kScanRows];          // rows' exclusive offsets
    __shared__ int64_t s_carry;
    if (*mode != kModeCounted) return;            // the guessed sums were exact
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        prefix[0] = 0;
        s_carry = 0;
    }
    for (int64_t base = 1; base <= ntiles; base += (int64_t)kScanRows * kScanThreads) {
        int x[kScanRows];
#pragma unroll
        for (int i = 0; i < kScanRows; ++i) {
            const int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;
            x[i] = idx <= ntiles ? (int)prefix[idx] : 0;
        }
#pragma unroll
        for (int i = 0; i < kScanRows; ++i) {
            x[i] = wave_incl_scan(x[i]);
            if (lane == 63) s_wave[i][wv] = x[i];
        }
        __syncthreads();
        if (wv == 0) {
            // lane i < kScanRows: row i's wave prefixes and total
            int64_t total = 0;
            if (lane < kScanRows) {
                int acc = 0;
#pragma unroll
                for (int k = 0; k < kW; ++k) {
                    const int t = s_wave[lane][k];
                    s_wave[lane][k] = acc;
                    acc += t;
                }
                total = acc;
            }
            // exclusive scan of the row totals over the lanes, after the carry
            int64_t y = total;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int64_t z = __shfl_up(y, d, 64);
                if (lane >= d) y += z;
            }
            const int64_t carry = s_carry;
            if (lane < kScanRows) s_row[lane] = carry + y - total;
            const int64_t all = __shfl(y, 63, 64);
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) s_carry = carry + all;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kScanRows; ++i) {
            const int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;
            if (idx <= ntiles) prefix[idx] = s_row[i] + s_wave[i][wv] + x[i];
        }
        __syncthreads();
    }
}

// Index of the tile that holds significant character g (0 <= g < total):
// the last u with prefix[u] <= g.
__device__ int64_t tile_of(const int64_t *prefix, int64_t ntiles, int64_t g)
{
    int64_t lo = 0, hi = ntiles;          // prefix[lo] <= g < prefix[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The scans below are wave-cooperative: every lane of the wave calls them
// with the same arguments and gets the same result.  A step tests 1,024
// characters, 16 per lane, so a long whitespace run costs one load latency
// per KiB instead of one per character.
//
// First significant character in [lo, hi), or hi.
__device__ int64_t wave_first_sig(const uint8_t *src, int64_t lo, int64_t hi, const uint8_t *m)
{
    const int lane = threadIdx.x & 63;
    {   // the next 64 characters first, one per lane: the usual distance
        const bool sig = lo + lane < hi && is_sig(m[src[lo + lane]]);
        const uint64_t b = __builtin_amdgcn_ballot_w64(sig);
        if (b) return lo + __builtin_ctzll(b);
        lo += 64;
    }
    for (int64_t p = lo; p < hi; p += 64 * 16) {
        const int64_t q = p + 16 * lane;
        int best = 16;
#pragma unroll
        for (int j = 15; j >= 0; --j)
            if (q + j < hi && is_sig(m[src[q + j]])) best = j;
        const uint64_t b = __builtin_amdgcn_ballot_w64(best < 16);
        if (b) return readlane_i64(q + best, __builtin_ctzll(b));
    }
    return hi;
}

// Last significant character in [lo, hi), or lo - 1.
__device__ int64_t wave_last_sig(const uint8_t *src, int64_t lo, int64_t hi, const uint8_t *m)
{
    const int lane = threadIdx.x & 63;
    {   // the previous 64 characters first, one per lane
        const int64_t i = hi - 64 + lane;
        const bool sig = i >= lo && is_sig(m[src[i]]);
        const uint64_t b = __builtin_amdgcn_ballot_w64(sig);
        if (b) return hi - 64 + (63 - __builtin_clzll(b));
        hi -= 64;
    }
    for (int64_t e = hi; e > lo; e -= 64 * 16) {
        const int64_t s = e - 64 * 16 > lo ? e - 64 * 16 : lo;
        const int64_t q = s + 16 * lane;
        int best = -1;
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (q + j < e && is_sig(m[src[q + j]])) best = j;
        const uint64_t b = __builtin_amdgcn_ballot_w64(best >= 0);
        if (b) return readlane_i64(q + best, 63 - __builtin_clzll(b));
    }
    return lo - 1;
}

// Position of the first significant character at or after pos, or n
// (wave-cooperative); tiles without one are stepped over by the prefix sums.
__device__ int64_t next_sig(const uint8_t *src, int64_t n, int64_t pos, const uint8_t *m,
                            const int64_t *prefix, int64_t ntiles, int64_t TS)
{
    const int64_t total = prefix[ntiles];
    while (pos < n) {
        const int64_t u = pos / TS, end = (u + 1) * TS < n ? (u + 1) * TS : n;
        const int64_t p = wave_first_sig(src, pos, end, m);
        if (p < end) return p;
        const int64_t g = prefix[u + 1];     // index of the next significant character
        if (g >= total) return n;
        pos = tile_of(prefix, ntiles, g) * TS;
    }
    return n;
}

// Position of the last significant character before pos, or -1
// (wave-cooperative).
__device__ int64_t prev_sig(const uint8_t *src, int64_t n, int64_t pos, const uint8_t *m,
                            const int64_t *prefix, int64_t ntiles, int64_t TS)
{
    while (pos > 0) {
        const int64_t u = (pos - 1) / TS, start = u * TS;
        const int64_t p = wave_last_sig(src, start, pos, m);
        if (p >= start) return p;
        const int64_t g = prefix[u] - 1;     // index of the previous significant character
        if (g < 0) return -1;
        const int64_t v = tile_of(prefix, ntiles, g);
        pos = (v + 1) * TS < n ? (v + 1) * TS : n;
    }
    return -1;
}

// Three bytes of the quantum of values w = v0 | v1<<8 | v2<<16 | v3<<24
// (each below 64), as b0 | b1<<8 | b2<<16: the closed form of Section
// "Base64" as v0<<18 | v1<<12 | v2<<6 | v3, its two 12-bit halves v0*64 + v1
// and v2*64 + v3 being byte dot products.  (Values of 64 and more, which
// only invalid input yields, give unspecified bytes.)
__device__ __forceinline__ uint32_t ws_quantum(uint32_t w)
{
    const uint32_t a = __builtin_amdgcn_udot4(w, 0x00000140u, 0u, false);   // v0*64 + v1
    const uint32_t b = __builtin_amdgcn_udot4(w, 0x01400000u, 0u, false);   // v2*64 + v3
    return __builtin_amdgcn_perm(0u, (a << 12) | b, 0x0C000102u);           // v.b2 v.b1 v.b0 0
}

__device__ __forceinline__ void store3(uint8_t *o, uint32_t b)
{
    o[0] = (uint8_t)b;
    o[1] = (uint8_t)(b >> 8);
    o[2] = (uint8_t)(b >> 16);
}

// k_ws_decode works per wave: a wave decodes a whole tile in rounds of
// kWaveRound characters.  Its value buffer takes a round's significant values
// after those the previous round left over (fewer than 16, moved to position
// 16), groups of 16 are read back from position 16 on (16-byte aligned
// loads), and positions 0..15 take at most three values that belong to a
// quantum of an earlier tile (never read).
constexpr int kWaveRound = 1024;
constexpr int kWsTrash = 16 + kWaveRound + 16;   // 64 bytes, one per lane: whitespace writes
constexpr int kWsBuf = kWsTrash + 64;

// The first `need` (<= 3) significant values at or after position `from`
// (the end of a tile), packed as bytes; fewer if the input ends first
// (wave-cooperative).  Fast path (`fast`: the next tile holds at least `need`
// significant characters): its first 16 characters, loaded ahead by lane 0 as
// `head`, hold them; else a scan.
__device__ uint32_t borrow_values(const uint8_t *src, int64_t n, const uint8_t *m,
                                  const int64_t *prefix, int64_t ntiles, int64_t TS, int64_t from,
                                  int need, bool fast, u32x4 head)
{
    uint32_t extra = 0;
    int got = 0;
    if (fast) {
        if ((threadIdx.x & 63) == 0) {
            const uint32_t hw[4] = {head.x, head.y, head.z, head.w};
            for (int j = 0; j < 16 && got < need; ++j) {
                const uint32_t code = m[(hw[j >> 2] >> (8 * (j & 3))) & 0xFF];
                if (is_sig(code)) extra |= code << (8 * got++);
            }
        }
        got = __builtin_amdgcn_readfirstlane(got);
        extra = (uint32_t)__builtin_amdgcn_readfirstlane((int)extra);
        if (got == need) return extra;
        extra = 0;
        got = 0;
    }
    for (int64_t p = from; got < need; ++p) {
        p = next_sig(src, n, p, m, prefix, ntiles, TS);
        if (p >= n) break;
        extra |= (uint32_t)m[src[p]] << (8 * got++);
    }
    return extra;
}

// Per-wave state of k_ws_decode.  W is the next write position in the value
// buffer and Qb the quantum that buffer position 16 stands for; Q0 and qlimit
// bound the quanta the tile stores.  held/held_k: a group of four quanta that
// the hot path leaves for later (the first group of a tile, whose first h
// quanta are not the tile's), as output bytes and the index of its first
// quantum relative to Q0 (held_k = 1 when there is none).
struct WsState {
    int W;
    int64_t Qb, Q0, qlimit;
    uint32_t held[4];
    int held_k;
    uint32_t err;   // (checked decode) OR of the values read back: bit 7 of a byte flags '=' or an invalid byte
    int cnt;        // (checked decode) significant characters seen in the tile
};

// One round of k_ws_decode: the wave's characters [p0, p0 + kWaveRound), of
// which those at or past `end` count as whitespace (HOT: none are); `raw`
// holds the lane's 16 characters p0 + 16*lane ...
//
// HOT rounds belong to full tiles whose quanta all lie below qlimit.  There
// every round issues exactly one vector store instruction (lanes without a
// whole group of the tile's own quanta are masked off), so that the compiler
// can count the vector memory operations issued after a prefetched load
// exactly and wait for that load alone, not for the stores as well (loads
// and stores share one in-order counter).  The group of the tile's first
// round whose first quanta belong to the tile before is kept in S.held and
// stored after the rounds.
//
// Compaction: the lane puts its 16 characters in the wave's staging area and
// the wave reads them back transposed, row j being characters 64j .. 64j+63
// with lane l on character 64j + l.  Characters of a row are in lane order,
// so a ballot of "significant" over the row and a masked bit count below the
// lane (mbcnt) give each character its position among the row's significant
// values, and rows follow each other.  Per character: an LDS read of the
// staged byte, one of the map, a compare, two mbcnt and an add, and one byte
// write; a row's writes land on consecutive bytes.  A wave's LDS operations
// complete in order, so the wave needs no barrier between its phases, only
// fences that keep the compiler from moving LDS accesses across them.
// `vb` is the block's array of value buffers and `wo` this wave's offset in
// it: positions are kept as offsets into the whole array, so the array's
// address folds into the LDS instructions' constant offsets.
template <bool HOT, bool NT, bool CHECK>
__device__ __forceinline__ void ws_round(u32x4 raw, int64_t p0, int64_t end, uint8_t *st,
                                         const uint8_t *m, uint8_t *vb, int wo,
                                         uint8_t *__restrict__ dst, WsState &S)
{
    const int lane = threadIdx.x & 63;
    *(u32x4 *)(st + 16 * lane) = raw;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the running write offset lives in a vector register, where the masked
    // bit count can add it at no cost; whitespace lanes write to their own
    // trash byte
    int at0;
    asm volatile("v_mov_b32 %0, %1" : "=v"(at0) : "s"(wo + S.W));
    const int start = at0, trash = wo + kWsTrash + lane;
    // all 32 reads first: the writes below could alias them as far as the
    // compiler knows
    uint32_t code[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) code[j] = st[64 * j + lane];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        code[j] = m[code[j]];
        if (!HOT && p0 + 64 * j + lane >= end) code[j] = kWsCode;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const bool sig = code[j] != kWsCode;
        const uint64_t b = __builtin_amdgcn_ballot_w64(sig);
        const int at = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)b, (uint32_t)at0));
        vb[sig ? at : trash] = (uint8_t)code[j];
        at0 += (int)__builtin_popcountll(b);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint8_t *const cb = vb + wo;
    const int got = __builtin_amdgcn_readfirstlane(at0 - start);
    const int rb = S.W + got;
    if (CHECK) S.cnt += got;
    const int avail = rb - 16;
    const int nfull = avail > 0 ? avail >> 4 : 0;   // at most 64 (rb <= 31 + 1024)
    const int64_t lo64 = S.Q0 - S.Qb, hi64 = S.qlimit - S.Qb;
    const int lo = (int)lo64, hi = hi64 < (1 << 20) ? (int)hi64 : (1 << 20);
    uint8_t *const o = dst + 3 * S.Qb;
    if (HOT) {
        // quanta Qb + 4*lane .. +3; every lane computes, whole groups of the
        // tile's own quanta are stored, with one store instruction
        const int k0 = 4 * lane;
        const u32x4 v = *(const u32x4 *)(cb + 16 + 16 * lane);
        if (CHECK) S.err |= v.x | v.y | v.z | v.w;
        const uint32_t b0 = ws_quantum(v.x), b1 = ws_quantum(v.y), b2 = ws_quantum(v.z),
                       b3 = ws_quantum(v.w);
        u32x3 w;
        w.x = b0 | (b1 << 24);
        w.y = (b1 >> 8) | (b2 << 16);
        w.z = (b2 >> 16) | (b3 << 8);
        // a single masked store, the address and data computed outside it;
        // an ordinary store, so that the two halves of a line shared with the
        // next round meet in L2 before it is written back
        uint8_t *const to = o + 3 * k0;
        if (lane < nfull && k0 >= lo) store12<false>(to, w);
        if (lane < nfull && k0 < lo) {                  // lane 0 of the first round only
            S.held[0] = b0;
            S.held[1] = b1;
            S.held[2] = b2;
            S.held[3] = b3;
            S.held_k = k0 - lo;
        }
    } else if (lane < nfull) {
        const int g = lane;
        const u32x4 v = *(const u32x4 *)(cb + 16 + 16 * g);
        if (CHECK) S.err |= v.x | v.y | v.z | v.w;
        const uint32_t b0 = ws_quantum(v.x), b1 = ws_quantum(v.y), b2 = ws_quantum(v.z),
                       b3 = ws_quantum(v.w);
        // quanta Qb + 4g .. +3; those before Q0 or at qlimit and past are not stored
        const int k0 = 4 * g;
        if (k0 >= lo && k0 + 4 <= hi) {
            u32x3 w;
            w.x = b0 | (b1 << 24);
            w.y = (b1 >> 8) | (b2 << 16);
            w.z = (b2 >> 16) | (b3 << 8);
            store12<NT>(o + 3 * k0, w);
        } else {
            const uint32_t bb[4] = {b0, b1, b2, b3};
            for (int k = 0; k < 4; ++k)
                if (k0 + k >= lo && k0 + k < hi) store3(o + 3 * (k0 + k), bb[k]);
        }
    }
    // the values after the last whole group move to position 16 (none while
    // the write position is still below 16: positions below 16 are never
    // read); all lanes read before any writes
    const int keep = avail - 16 * nfull;
    uint32_t carry = 0;
    if (lane < keep) carry = cb[16 + 16 * nfull + lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < keep) cb[16 + lane] = (uint8_t)carry;
    S.W = keep >= 0 ? 16 + keep : rb;
    S.Qb += 4 * nfull;
}

// The indexes (0..15) of the first invalid character and the first '=' among
// the 16 packed codes of a chunk, as bad | pad << 8, 0xFF for none.  Only
// bytes with bit 7 set are looked at, lowest first.
__device__ __forceinline__ uint32_t ws_firsts16(u32x4 cw)
{
    uint32_t bad = 0xFFu, pad = 0xFFu;
    const uint32_t w[4] = {cw.x, cw.y, cw.z, cw.w};
#pragma unroll
    for (int d = 3; d >= 0; --d) {
        for (uint32_t hi = w[d] & 0x80808080u; hi; hi &= hi - 1) {
            const uint32_t b = (uint32_t)__builtin_ctz(hi) >> 3;
            const uint32_t code = (w[d] >> (8 * b)) & 0xFFu;
            const uint32_t i = 4 * (uint32_t)d + b;
            if (code == kBadCode && i < bad) bad = i;
            else if (code == kPadCode && i < pad) pad = i;
        }
    }
    return bad | pad << 8;
}

// The first invalid character and the first '=' (padded mode) of the tile
// [base, end), by atomic minimum, as k_ws_count records them; each lane scans
// its own 16 characters of every 1,024 (wave-cooperative).
__device__ void ws_rescan(const uint8_t *src, int64_t base, int64_t end, const uint8_t *m,
                          int64_t *first_pad, int64_t *first_bad)
{
    const int lane = threadIdx.x & 63;
    bool bad_found = false, pad_found = false;
    // a rare path: rolled loops, so that it adds no registers to the decode
#pragma unroll 1
    for (int64_t p = base + 16 * lane; p < end && !(bad_found && pad_found); p += kWaveRound) {
#pragma unroll 1
        for (int64_t i = p; i < p + 16 && i < end; ++i) {
            const uint32_t code = m[src[i]];
            if (code == kBadCode && !bad_found) {
                atomic_min_i64(first_bad, i);
                bad_found = true;
            } else if (code == kPadCode && !pad_found) {
                atomic_min_i64(first_pad, i);
                pad_found = true;
            }
        }
    }
}

// The checked decode's work on a tile with no quantum of its own: count its
// significant characters against the guessed count C (when check_count) and
// record its first invalid character and '=' (wave-cooperative).  Inlined: a
// call left 8 bytes of stack per lane in the checked decode and was no faster.
__device__ __forceinline__ void ws_check_tile(const uint8_t *src, int64_t base, int64_t end, const uint8_t *m,
                              bool check_count, int64_t C, int64_t *mode, int64_t *first_pad,
                              int64_t *first_bad)
{
    const int lane = threadIdx.x & 63;
    int cnt = 0;
    uint32_t err = 0;
#pragma unroll 4
    for (int64_t p = base + 16 * lane; p < end; p += kWaveRound) {
        const u32x4 c = ws_codes<false>(src, end, p, m);
        cnt += sig_count(c);
        err |= c.x | c.y | c.z | c.w;
    }
    err = (err | (err >> 8) | (err >> 16) | (err >> 24)) & 0xFFu;   // bit 7 of any code
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    if (check_count && cnt != C && lane == 0)
        __hip_atomic_store(mode, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__ballot(err & 0x80u)) ws_rescan(src, base, end, m, first_pad, first_bad);
}

// k_ws_decode: tile `tile` decodes the quanta whose first significant value
// lies in it, except quanta at index >= qlimit (the final quantum, left to
// k_ws_finish).  Quantum q covers significant values [4q, 4q+4) and writes
// dst[3q, 3q+3).  Buffer position 16 of the first round stands for quantum
// Qr = Q0 - h, with h < 4 chosen so that 3*Qr + dst is a multiple of 4: every
// group of 16 values read back then stores its 12 bytes at a 4-byte aligned
// address (the h quanta before Q0 belong to earlier tiles and are not
// stored).  Tiles are dealt to waves grid-stride (the launch sizes the grid
// to the workgroups that are resident at once, so every wave starts at once);
// a wave keeps the loads of its next D rounds in flight.
//
// CHECK: the checked decode that runs on k_ws_predict's guessed prefix sums
// (*mode == kModeChecked; it returns at once otherwise).  Every tile it decodes, but the
// last, compares the significant characters it saw with its guessed count,
// and clears *mode on a difference or on any '=' or invalid character (the
// counting path then finds them).  Tiles with no quantum of their own are
// only counted and scanned (ws_check_tile), and the last tile is
// k_ws_predict's.  When every count holds, the
// guessed sums are the exact ones, so its output is the output of the plain
// decode on exact sums.  Without CHECK the kernel runs only when *mode is 0
// (no guess, or a check failed).
template <int D, bool NT, bool CHECK>
__global__ __launch_bounds__(kWsBlock) void k_ws_decode(const uint8_t *__restrict__ src, int64_t n,
                                                        uint8_t *__restrict__ dst, DecMap map,
                                                        const int64_t *__restrict__ prefix,
                                                        int64_t TS, uint32_t flags,
                                                        int64_t *__restrict__ mode,
                                                        int64_t *__restrict__ first_pad,
                                                        int64_t *__restrict__ first_bad)
{
    __shared__ uint32_t s_map[64];
    __shared__ __align__(16) uint8_t stage[kWsBlock / 64][kWaveRound];
    __shared__ __align__(16) uint8_t vbuf[kWsBlock / 64 * kWsBuf];
    if (*mode != (CHECK ? kModeChecked : kModeCounted)) return;    // uniform
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;
    const int64_t ntiles = ws_tiles(n, TS);
    if (ntiles == 0) return;
    const int64_t total = prefix[ntiles];
    const bool nopad = (flags & kFlagNoPad) != 0;
    const int64_t qlimit = nopad ? total / 4 : (total >= 4 ? total / 4 - 1 : 0);
    const int64_t dmod = (int64_t)((uint64_t)(uintptr_t)dst & 3);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint8_t *const st = stage[wv];
    const int wo = wv * kWsBuf;                   // this wave's value buffer
    uint8_t *const cb = vbuf + wo;
    const int64_t nwaves = (int64_t)gridDim.x * (kWsBlock / 64);
    if (CHECK) {
        // the checked decode ORs every group it reads back, stale ones too:
        // start from zeros, so that only this launch's values are seen
        for (int i = 16 * lane; i < kWsBuf; i += 16 * 64) *(u32x4 *)(cb + i) = u32x4{0u, 0u, 0u, 0u};
    }

    for (int64_t tile = logical_block() * (kWsBlock / 64) + wv; tile < ntiles; tile += nwaves) {
        const int64_t base = tile * TS, end = base + TS < n ? base + TS : n;
        const int64_t K0 = prefix[tile], C = prefix[tile + 1] - K0;
        const int64_t skip = (4 - (K0 & 3)) & 3;
        const int64_t Q0 = (K0 + skip) >> 2;
        if (C <= skip || Q0 >= qlimit) {            // wave-uniform: no quantum of its own
            // checked: such a tile (but the last, which k_ws_predict scanned)
            // is counted against its guess and scanned for '=' and invalid
            // characters here, as k_ws_count would
            if (CHECK && tile + 1 < ntiles)
                ws_check_tile(src, base, end, m, true, C, mode, first_pad, first_bad);
            continue;
        }
        const int64_t h = (Q0 + 3 * dmod) & 3;
        // what the last quantum may borrow from the next tile, fetched early
        const bool has_next = tile + 1 < ntiles;
        const int64_t next_end = has_next ? prefix[tile + 2] : total;
        const bool head_ok = has_next && base + TS + 16 <= n;
        u32x4 head = u32x4{0u, 0u, 0u, 0u};
        if (lane == 0 && head_ok) head = load16<false>(src + base + TS);
        WsState S{16 + 4 * (int)h - (int)skip, Q0 - h, Q0, qlimit, {0u, 0u, 0u, 0u}, 1, 0u, 0};
        const uint8_t *const s0 = src + base + 16 * lane;
        // a full tile whose quanta (at most Q0 + C/4) all lie below qlimit
        const bool hot = end - base == TS && Q0 + C / 4 + 1 <= qlimit;
        if (hot) {
            // TS/kWaveRound rounds, a multiple of D; the loads of the next D
            // rounds in flight (the last ones repeat the last round, unused)
            // (each load is issued after the round that frees its registers;
            // the last D rounds load nothing)
            const int nr = (int)(TS / kWaveRound);
            u32x4 q[D];
#pragma unroll
            for (int d = 0; d < D; ++d) q[d] = load16<NT>(s0 + d * kWaveRound);
            int r = 0;
            for (; r < nr - D; r += D) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    ws_round<true, NT, CHECK>(q[d], base + (int64_t)(r + d) * kWaveRound, end, st, m, vbuf, wo,
                                       dst, S);
                    q[d] = load16<NT>(s0 + (int64_t)(r + d + D) * kWaveRound);
                }
            }
#pragma unroll
            for (int d = 0; d < D; ++d)
                ws_round<true, NT, CHECK>(q[d], base + (int64_t)(r + d) * kWaveRound, end, st, m, vbuf, wo, dst, S);
            // the first group's quanta that are the tile's own
            if (S.held_k <= 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k >= -S.held_k) store3(dst + 3 * (Q0 + S.held_k + k), S.held[k]);
            }
        } else {
            for (int64_t p0 = base; p0 < end; p0 += kWaveRound) {
                u32x4 raw;
                if (p0 + kWaveRound <= end) {
                    raw = load16<NT>(s0 + (p0 - base));
                } else {
                    uint32_t w[4] = {0, 0, 0, 0};
                    for (int j = 0; j < 16; ++j) {
                        const int64_t i = p0 + 16 * lane + j;
                        if (i < end) w[j >> 2] |= (uint32_t)src[i] << (8 * (j & 3));
                    }
                    raw = u32x4{w[0], w[1], w[2], w[3]};
                }
                ws_round<false, NT, CHECK>(raw, p0, end, st, m, vbuf, wo, dst, S);
            }
        }
        // fewer than 16 values left: whole quanta, then one quantum that may
        // take up to three values from later tiles
        const int left = S.W - 16;
        if (left > 0) {
            const int rem = left & 3;
            uint32_t extra = 0;
            if (rem)
                extra = borrow_values(src, n, m, prefix, ntiles, TS, end, 4 - rem,
                                      head_ok && next_end - (K0 + C) >= 4 - rem, head);
            const int nq = (left + 3) >> 2;
            if (lane < nq) {
                const int64_t qq = S.Qb + lane;
                uint32_t w = 0;
                for (int k = 0; k < 4; ++k) {
                    const int idx = 4 * lane + k;
                    const uint32_t v = idx < left ? cb[16 + idx] : (extra >> (8 * (idx - left))) & 0xFF;
                    w |= v << (8 * k);
                }
                if (CHECK) S.err |= w;
                if (qq >= Q0 && qq < qlimit) store3(dst + 3 * qq, ws_quantum(w));
            }
        }
        if (CHECK && tile + 1 < ntiles) {
            const bool fail = S.cnt != C || __ballot(S.err & 0x80808080u) != 0;
            if (fail && lane == 0)
                __hip_atomic_store(mode, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// k_ws_finish (one block): the '=' and end rules over the significant
// characters, the final quantum, and the public status (*out_len = length or
// -1, *first_bad = -1 or the first invalid offset).  *first_bad holds the raw
// minimum from k_ws_count, *first_pad the first '=' (padded mode).  The rules
// run on wave 0, every lane with the same values, so that its searches for
// neighbouring significant characters are wave-cooperative; lane 0 writes.
__global__ __launch_bounds__(kWsBlock) void k_ws_finish(const uint8_t *__restrict__ src, int64_t n,
                                                        uint8_t *__restrict__ dst, DecMap map,
                                                        int64_t TS, const int64_t *__restrict__ prefix,
                                                        const int64_t *__restrict__ first_pad,
                                                        int64_t *__restrict__ out_len,
                                                        int64_t *__restrict__ first_bad,
                                                        uint32_t flags, int write_output)
{
    __shared__ uint32_t s_map[64];
    __shared__ int64_t s_a, s_cnt;
    __shared__ int s_slow;
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;
    const int64_t ntiles = ws_tiles(n, TS);
    const int64_t total = ntiles ? prefix[ntiles] : 0;
    const bool nopad = (flags & kFlagNoPad) != 0;
    const int tid = threadIdx.x;

    // padded mode with a '=': its index among the significant characters
    // decides the rules.  Fast case: at most one significant character
    // follows it (a valid input has that form).
    int64_t a = -1, after = 0;
    if (tid < 64) {
        if (!nopad && *first_pad != kNoError) {
            a = *first_pad;
            int64_t p = a;
            while (after < 2) {
                p = next_sig(src, n, p + 1, m, prefix, ntiles, TS);
                if (p >= n) break;
                ++after;
            }
        }
        if (tid == 0) {
            s_slow = after >= 2;
            s_cnt = 0;
            s_a = a;
        }
    }
    __syncthreads();
    if (s_slow) {       // count the significant characters before the '=' in its tile
        const int64_t aa = s_a, start = aa / TS * TS;
        int64_t cnt = 0;
        for (int64_t i = start + tid; i < aa; i += kWsBlock) cnt += is_sig(m[src[i]]);
        atomicAdd((unsigned long long *)&s_cnt, (unsigned long long)cnt);
    }
    __syncthreads();
    if (tid >= 64) return;

    int64_t bad = *first_bad;                 // kNoError when none
    int64_t len = 0;
    // the last up to four significant characters (positions, latest last)
    const int r = (int)(total & 3);
    const int nlast = nopad ? r : (total >= 4 ? 4 : 0);
    int64_t lp[4] = {-1, -1, -1, -1};
    {
        int64_t p = n;
        for (int k = nlast - 1; k >= 0; --k) {
            p = prev_sig(src, n, p, m, prefix, ntiles, TS);
            lp[k] = p;
        }
    }
    if (nopad) {
        if (r == 1) bad = bad < n ? bad : n;
        else if (r >= 2 && (m[src[lp[r - 1]]] & (r == 2 ? 15u : 3u))) bad = bad < n ? bad : n;
        len = 3 * (total >> 2) + (r ? r - 1 : 0);
    } else if (a < 0) {
        if (r != 0) bad = bad < n ? bad : n;
        len = 3 * (total >> 2);
    } else {
        const int64_t i = s_slow ? prefix[a / TS] + s_cnt : total - 1 - after;
        const int pq = (int)(i & 3);
        int64_t e = kNoError;
        if (pq < 2) {
            e = a;
        } else {
            const int64_t pv = prev_sig(src, n, a, m, prefix, ntiles, TS);
            const uint32_t prev = m[src[pv]];
            if (pq == 2) {
                if (prev & 15) {
                    e = a;
                } else {
                    const int64_t nx = next_sig(src, n, a + 1, m, prefix, ntiles, TS);
                    if (nx >= n) e = n;
                    else if (src[nx] != kPad) e = nx;
                    else {
                        const int64_t nx2 = next_sig(src, n, nx + 1, m, prefix, ntiles, TS);
                        e = nx2 < n ? nx2 : kNoError;
                    }
                }
            } else {
                if (prev & 3) {
                    e = a;
                } else {
                    const int64_t nx = next_sig(src, n, a + 1, m, prefix, ntiles, TS);
                    e = nx < n ? nx : kNoError;
                }
            }
        }
        bad = bad < e ? bad : e;
        len = 3 * (total >> 2) - (total - i);
    }
    if (bad != kNoError) {
        if (tid == 0) {
            *out_len = -1;
            *first_bad = bad;
        }
        return;
    }
    if (write_output && nlast > 0) {
        // the final quantum: 4 characters (padded) or r (unpadded); its data
        // values give (number of data values - 1) bytes
        uint32_t w = 0;
        int nd = 0;
        for (int k = 0; k < nlast; ++k) {
            const uint8_t ch = src[lp[k]];
            if (ch == kPad && !nopad) break;
            w |= (uint32_t)m[ch] << (8 * k);
            ++nd;
        }
        const uint32_t b = ws_quantum(w);
        uint8_t *o = dst + 3 * (nopad ? (total >> 2) : (total >> 2) - 1);
        if (tid == 0)
            for (int k = 0; k < nd - 1; ++k) o[k] = (uint8_t)(b >> (8 * k));
    }
    if (tid == 0) {
        *out_len = len;
        *first_bad = -1;
    }
}

__global__ void k_ws_init(int64_t *first_bad, int64_t *first_pad, int64_t *mode)
{
    if (threadIdx.x == 0) {
        *first_bad = kNoError;
        *first_pad = kNoError;
        *mode = 0;
    }
}

// Significant characters before position p of text laid out in lines of L
// significant characters, each followed by s whitespace bytes (P = L + s).
// The quotient comes from a double division (exact for p < 2^53) and is then
// corrected, which is cheaper on the GPU than a 64-bit integer division.
__device__ __forceinline__ int64_t lined_before(int64_t p, int64_t L, int64_t P)
{
    int64_t q = (int64_t)((double)p / (double)P);
    int64_t r = p - q * P;
    if (r < 0) {
        --q;
        r += P;
    } else if (r >= P) {
        ++q;
        r -= P;
    }
    return q * L + (r < L ? r : L);
}

// k_ws_predict: guessed tile prefix sums for text laid out in lines, as MIME
// and PEM bodies are: lines of L significant characters, each followed by the
// same s = 1 or 2 whitespace bytes (LF or CR LF), the last line shorter.
// Every block takes L and s from the first line and writes the guess for its
// share of the tiles, prefix[t] = lined_before(t*TS); block 0 checks one line
// end per thread spread over the input, counts the last tile into
// prefix[ntiles], records the last tile's first invalid byte and '=' as
// k_ws_count would (the checked decode leaves that tile to it), and, if the
// checks hold, sets *mode to kModeLines (L a multiple of 4, at least 16, and
// the final quantum at or past the last tile, as far as the guess tells) or
// else to kModeChecked; block 0 first resets the status, as k_ws_init does.
// Otherwise *mode stays kModeCounted and k_ws_count and k_ws_scan overwrite
// the guess.  The guess has
// prefix[t] <= t*TS and at most TS per tile, so the checked decode that uses
// it stays inside its buffers however wrong it is.
__global__ __launch_bounds__(kWsBlock) void k_ws_predict(const uint8_t *__restrict__ src, int64_t n,
                                                         DecMap map, int64_t *__restrict__ prefix,
                                                         int64_t TS, uint32_t flags,
                                                         int64_t *__restrict__ mode,
                                                         int64_t *__restrict__ first_pad,
                                                         int64_t *__restrict__ first_bad)
{
    __shared__ uint32_t s_map[64];
    __shared__ int s_first, s_ok, s_cnt;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) {          // the status reset of k_ws_init
        *first_bad = kNoError;
        *first_pad = kNoError;
        *mode = 0;
    }
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;
    const int64_t ntiles = ws_tiles(n, TS);
    if (tid == 0) {
        s_first = INT_MAX;
        s_ok = 1;
        s_cnt = 0;
    }
    __syncthreads();
    if (ntiles < 2) return;
    // block 0: the last tile's significant characters, and each thread's
    // first invalid character and '=' in it (loaded first, to overlap the
    // line search)
    const int64_t lb = (ntiles - 1) * TS;
    int my_bad = INT_MAX, my_pad = INT_MAX;      // offsets from lb
    if (blockIdx.x == 0) {
        // all of a thread's loads first (the tile is at most kMaxRounds rounds)
        u32x4 q[kMaxRounds];
#pragma unroll
        for (int k = 0; k < kMaxRounds; ++k) {
            const int64_t p = lb + 16 * tid + (int64_t)k * kRound;
            q[k] = p + 16 <= n ? load16<false>(src + p) : u32x4{0u, 0u, 0u, 0u};
        }
        int c = 0;
#pragma unroll
        for (int k = 0; k < kMaxRounds; ++k) {
            const int64_t p = lb + 16 * tid + (int64_t)k * kRound;
            if (p < n) {
                const u32x4 cw = p + 16 <= n ? codes16(q[k], m) : ws_codes<false>(src, n, p, m);
                c += sig_count(cw);
                if ((cw.x | cw.y | cw.z | cw.w) & 0x80808080u) {
                    // rounds go in increasing position: the first found is the lane's first
                    const uint32_t f = ws_firsts16(cw);
                    const int off = (int)(p - lb);
                    if (my_bad == INT_MAX && (f & 0xFFu) != 0xFFu) my_bad = off + (int)(f & 0xFFu);
                    if (my_pad == INT_MAX && (f >> 8) != 0xFFu) my_pad = off + (int)(f >> 8);
                }
            }
        }
        atomicAdd(&s_cnt, c);
    }
    // the first whitespace byte of the first 4 KiB: 16 bytes per thread
    const int64_t look = n < 4096 ? n : 4096;
    {
        const int64_t p = 16 * (int64_t)tid;
        int first = INT_MAX;
        if (p + 16 <= look) {
            const u32x4 c = codes16(load16<false>(src + p), m);
            const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (int j = 15; j >= 0; --j)
                if (!is_sig((w[j >> 2] >> (8 * (j & 3))) & 0xFFu)) first = (int)p + j;
        } else {
            for (int64_t i = p + 15; i >= p; --i)
                if (i < look && !is_sig(m[src[i]])) first = (int)i;
        }
        if (first != INT_MAX) atomicMin(&s_first, first);
    }
    __syncthreads();
    // the last tile's first invalid character and '=', as k_ws_count records
    // them (after the barrier, so after the reset above)
    if (my_bad != INT_MAX) atomic_min_i64(first_bad, lb + my_bad);
    if (my_pad != INT_MAX) atomic_min_i64(first_pad, lb + my_pad);
    const int64_t L = s_first;                   // the first line's length (uniform)
    if (L == INT_MAX || L < 4 || L + 3 > look) return;
    const bool w1 = !is_sig(m[src[L + 1]]), w2 = !is_sig(m[src[L + 2]]);   // src[L] is whitespace
    const int64_t sep = !w1 ? 1 : (!w2 ? 2 : 3);
    if (sep > 2) return;
    const int64_t P = L + sep;
    for (int64_t t = (int64_t)blockIdx.x * kWsBlock + tid; t < ntiles; t += (int64_t)gridDim.x * kWsBlock)
        prefix[t] = lined_before(t * TS, L, P);
    if (blockIdx.x != 0) return;
    const int64_t total = lined_before(lb, L, P) + s_cnt;
    // the final quantum's first character, where the layout puts it
    const int64_t ql = (flags & kFlagNoPad) ? total / 4 : (total >= 4 ? total / 4 - 1 : 0);
    const int64_t jq = 4 * ql;
    const int64_t at = (jq / L) * P + jq % L;
    // The line decode checks the layout up to the separator before the final
    // quantum, and this kernel counted the last tile, so the prefix sums are
    // exact when the layout also holds from that separator to the last tile.
    // That stretch is empty unless the last tile is only a few bytes long
    // (the final quantum then starts in the tile before it); up to 64 bytes of
    // it are checked here, one per lane of wave 0, with their loads issued
    // beside the line-end samples': whitespace exactly at separator
    // positions.  Neither the line decode nor the last tile's scan looks at
    // these bytes for '=' or invalid characters (the final quantum's '=' may
    // lie here), so they are recorded here as k_ws_count records them (true
    // positions, so also right when the samples below send the decode to the
    // counted path).
    const int64_t from = at - sep;
    bool lines = L % 4 == 0 && L >= 16 && lb - from <= 64;
    const bool gap = lines && from < lb;
    bool off = false;
    if (gap && tid < 64) {
        const int64_t x = from + tid;
        if (x >= 0 && x < lb) {
            const uint32_t code = m[src[x]];
            off = is_sig(code) != (x % P < L);
            if (code == kBadCode) atomic_min_i64(first_bad, x);
            else if (code == kPadCode) atomic_min_i64(first_pad, x);
        }
    }
    {   // line k's separator, and the characters on either side of it
        const int64_t k = (n / P) * tid / kWsBlock;
        const int64_t q = k * P + L;
        if (q + sep < n) {
            const uint32_t before = src[q - 1], s0 = src[q], s1 = src[q + 1], after = src[q + sep];
            const bool ok = is_sig(m[before]) && !is_sig(m[s0]) && (sep == 1 || !is_sig(m[s1])) &&
                            is_sig(m[after]);
            if (!ok) s_ok = 0;
        }
    }
    __syncthreads();
    if (!s_ok || tid >= 64) return;              // wave 0 decides the path
    if (gap && __ballot(off)) lines = false;
    if (tid == 0) {
        prefix[ntiles] = total;
        *mode = lines ? (kModeLines | sep << 2 | L << 4) : kModeChecked;
    }
}

// k_ws_lines: the decode of text in regular lines (*mode = kModeLines | s << 2
// | L << 4, L a multiple of 4 and at least 16) straight from the layout, with
// no compaction: significant character j lies at (j div L)*P + j mod L, so a
// quantum is four adjacent bytes of one line.  A lane takes a group of four
// quanta (16 characters -> 12 bytes): one 16-byte load at the group's
// position and the dword after it; when a line ends inside the group, the
// characters past the separator are shifted down over it (v_alignbyte).  The
// kernel checks what the layout claims, byte by byte: every character of a
// quantum below qlimit decodes to a value (no whitespace, '=' or invalid
// byte), and the s bytes after every line end it passes are whitespace.
// k_ws_predict chose this path only when these bytes, with those it checked
// itself from the separator before quantum qlimit up to the last tile, are
// all of the text before the last tile, which k_ws_predict counted exactly:
// when no check fails, every guessed prefix sum is exact, the output is the
// plain decode's, and k_ws_finish adds the final quantum.  Any failure sets
// *mode to kModeCounted, and the counted path decodes everything again.
//
// Group g covers quanta 4g - h .. 4g - h + 3 and writes 12 bytes at
// dst + 12g - 3h; h < 128 makes that 128-byte aligned for g a multiple of 32,
// so a wave's 64 stores fill six whole cache lines.  Step k of the grid
// (S lanes) takes groups kS .. kS + S - 1, lane-contiguous.  Steps whose
// groups all have four quanta below qlimit and 20 readable bytes run
// pipelined, D steps of loads in flight; a lane tracks its position
// incrementally (no division per group).  The first and last steps take
// each group through a guarded path.
template <int D, bool NT>
__global__ __launch_bounds__(kWsBlock) void k_ws_lines(const uint8_t *__restrict__ src, int64_t n,
                                                       uint8_t *__restrict__ dst, DecMap map,
                                                       const int64_t *__restrict__ prefix, int64_t TS,
                                                       uint32_t flags, int64_t *__restrict__ mode)
{
    __shared__ uint32_t s_map[64];
    const int64_t md = *mode;
    if ((md & 3) != kModeLines) return;          // uniform
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;
    const int64_t L = md >> 4, s = (md >> 2) & 3, P = L + s;
    const int64_t ntiles = ws_tiles(n, TS);
    const int64_t total = prefix[ntiles];
    const bool nopad = (flags & kFlagNoPad) != 0;
    const int64_t qlimit = nopad ? total / 4 : (total >= 4 ? total / 4 - 1 : 0);
    const int64_t h = (((int64_t)(uintptr_t)dst & 127) * 43) & 127;   // 3h = dst (mod 128)
    const int64_t G = (qlimit + h + 3) / 4;       // groups with a quantum below qlimit
    const int64_t g_lo = (h + 3) / 4;             // first group with no quantum below 0
    const int64_t g_full = (qlimit + h) / 4;      // groups below it: four quanta below qlimit
    // groups below g_read: bytes [position, position + 20) lie in the text
    // (position <= x exactly when lined_before(x + 1) > 16g - 4h)
    const int64_t g_read = (lined_before(n - 19, L, P) + 4 * h) / 16;
    const int64_t g_hi = g_full < g_read ? g_full : g_read;
    const int64_t S = (int64_t)gridDim.x * kWsBlock;
    const int64_t gid = logical_block() * kWsBlock + threadIdx.x;
    const int64_t k_lo = (g_lo + S - 1) / S;
    const int64_t k_hi = g_hi / S > k_lo ? g_hi / S : k_lo;
    const int64_t nmain = (k_hi - k_lo) - (k_hi - k_lo) % D;
    bool bad = false;
    uint32_t err = 0;

    // the group whose 20 bytes from its position are q and t (column c):
    // its 12 bytes; a separator that is not whitespace sets bit 7 of err
    const int Li = (int)L;
    const uint32_t sb = (uint32_t)s;
    const bool two = s == 2;
    auto group = [&](u32x4 q, uint32_t t, int c, uint8_t *o) {
        const int rem = Li - c;                    // characters to the line end: 4, 8, ...
        u32x4 v;
        v.x = q.x;
        v.y = rem <= 4 ? __builtin_amdgcn_alignbyte(q.z, q.y, sb) : q.y;
        v.z = rem <= 8 ? __builtin_amdgcn_alignbyte(q.w, q.z, sb) : q.z;
        v.w = rem <= 12 ? __builtin_amdgcn_alignbyte(t, q.w, sb) : q.w;
        uint32_t sw = t;                           // the dword that starts with the separator
        sw = rem <= 12 ? q.w : sw;
        sw = rem <= 8 ? q.z : sw;
        sw = rem <= 4 ? q.y : sw;
        const uint32_t c0 = m[sw & 0xFF], c1 = m[(sw >> 8) & 0xFF];
        const bool sep_bad = (c0 != kWsCode) | (two & (c1 != kWsCode));
        err |= (uint32_t)((rem <= 16) & sep_bad) << 7;
        store12<NT>(o, dec_chunk(v, m, err));
    };
    // any group, each quantum on its own, every byte read checked against n
    auto edge = [&](int64_t g) {
        for (int k = 0; k < 4; ++k) {
            const int64_t qq = 4 * g - h + k;
            if (qq < 0 || qq >= qlimit) continue;
            const int64_t j = 4 * qq, l = j / L, c = j - l * L, p = l * P + c;
            if (p + 4 > n) {
                bad = true;
                continue;
            }
            const uint32_t w = (uint32_t)src[p] | ((uint32_t)src[p + 1] << 8) |
                               ((uint32_t)src[p + 2] << 16) | ((uint32_t)src[p + 3] << 24);
            const uint32_t v = dec_quantum(w, m, err);
            uint8_t *const o = dst + 3 * qq;
            o[0] = (uint8_t)(v >> 16);
            o[1] = (uint8_t)(v >> 8);
            o[2] = (uint8_t)v;
            if (c + 4 == L) {
                if (p + 4 + s > n) bad = true;
                else if (m[src[p + 4]] != kWsCode || (s == 2 && m[src[p + 5]] != kWsCode)) bad = true;
            }
        }
    };
    // a group of an edge step: the vector path if it qualifies
    auto one = [&](int64_t g) {
        if (g >= g_lo && g < g_hi) {
            const int64_t j = 16 * g - 4 * h, l = j / L, c = j - l * L, p = l * P + c;
            group(load16<NT>(src + p), *(const u32a1 *)(src + p + 16), (int)c, dst + 3 * (j / 4));
        } else if (g < G) {
            edge(g);
        }
    };

    for (int64_t k = 0; k < k_lo; ++k) one(k * S + gid);
    if (nmain > 0) {
        // position (pn, cn) of the next step's group to load; each step moves
        // it by 16 S characters: dl lines and dc columns, one more line (s
        // more bytes) when the column passes L
        const int64_t dj = 16 * S, dl = dj / L, dp = dl * P + (dj - dl * L);
        const int dc = (int)(dj - dl * L);
        const int64_t j0 = 16 * (k_lo * S + gid) - 4 * h, l0 = j0 / L;
        int cn = (int)(j0 - l0 * L);
        int64_t pn = l0 * P + cn;
        uint8_t *o = dst + 3 * (j0 / 4);
        const int64_t dout = 12 * S;
        u32x4 q[D];
        uint32_t t[D];
        int cq[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            q[d] = load16<NT>(src + pn);
            t[d] = *(const u32a1 *)(src + pn + 16);
            cq[d] = cn;
            pn += dp;
            cn += dc;
            if (cn >= Li) {
                cn -= Li;
                pn += s;
            }
        }
        for (int64_t i = 0; i < nmain - D; i += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                group(q[d], t[d], cq[d], o);
                o += dout;
                q[d] = load16<NT>(src + pn);
                t[d] = *(const u32a1 *)(src + pn + 16);
                cq[d] = cn;
                pn += dp;
                cn += dc;
                if (cn >= Li) {
                    cn -= Li;
                    pn += s;
                }
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            group(q[d], t[d], cq[d], o);
            o += dout;
        }
    }
    for (int64_t k = k_lo + nmain; k * S < G; ++k) one(k * S + gid);
    if (__ballot(bad || (err & 0xC0u) != 0) && (threadIdx.x & 63) == 0)
        __hip_atomic_store(mode, kModeCounted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------ small texts, one workgroup --

// k_ws_small: a text of at most kWsSmallMax characters decoded (or, !write,
// validated) by one workgroup in one launch, where the counted path takes
// five.  The text is read in rows of kSmallThreads lane chunks of 16
// characters: thread t owns chunk t of every row (characters 16*(1024r + t)
// onward), so every load of the workgroup is contiguous.  A thread counts
// the significant characters of each of its chunks; a workgroup scan per row
// gives each chunk the index of its first significant character, and the
// thread writes the codes at their indices into an LDS array (chunks of
// neighbouring lanes write neighbouring ranges).  The first invalid byte and
// the first '=' (padded mode) are workgroup minima.  The '=' and
// end-of-input rules then run on the array, as k_ws_finish runs them on the
// prefix sums: the index E of the first '=', the value before it, and the
// significant characters after it, whose offsets the threads that own them
// report.  Then the quanta are decoded from the array, 3 bytes each (the last
// one: the bytes its data values carry).  Nothing is shared between
// workgroups, and every wait is a barrier of this one workgroup.
constexpr int kSmallThreads = 1024;
constexpr int kSmallPer = 4;                    // rows (16-character loads per thread) at most
static_assert(kWsSmallMax == (int64_t)kSmallThreads * 16 * kSmallPer, "one workgroup's characters");

__global__ __launch_bounds__(kSmallThreads) void k_ws_small(const uint8_t *__restrict__ src, int64_t n,
                                                            uint8_t *__restrict__ dst, DecMap map,
                                                            int64_t *__restrict__ out_len,
                                                            int64_t *__restrict__ first_bad,
                                                            uint32_t flags, int write)
{
    __shared__ uint32_t s_map[64];
    __shared__ __align__(16) uint8_t vals[kWsSmallMax + 16];   // codes of the significant characters
    __shared__ int s_wsum[kSmallPer][kSmallThreads / 64];
    __shared__ uint32_t s_bad;                   // offset of the first invalid byte
    __shared__ unsigned long long s_pad;         // first '=': offset << 32 | its index E
    __shared__ uint32_t s_after[2];              // offsets of significant characters E+1, E+2
    __shared__ int64_t s_len, s_err;
    const int tid = threadIdx.x;
    const bool nopad = (flags & kFlagNoPad) != 0;
    const int K = (int)((n + 16 * kSmallThreads - 1) / (16 * kSmallThreads));   // rows, 0 .. kSmallPer
    // the bulk loads first; the map is staged while they are in flight
    u32x4 raw[kSmallPer];
#pragma unroll
    for (int j = 0; j < kSmallPer; ++j) {
        const int p = 16 * (j * kSmallThreads + tid);
        if (j < K && p + 16 <= n) raw[j] = load16<false>(src + p);
        else if (j < K && p < n && n >= 16) raw[j] = load16<false>(src + n - 16);   // the last bytes
    }
    if (tid == 0) {
        s_bad = 0xFFFFFFFFu;
        s_pad = ~0ull;
        s_after[0] = s_after[1] = 0xFFFFFFFFu;
    }
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;

    const int lane = tid & 63, wv = tid >> 6;
    u32x4 c[kSmallPer];
    int cnt[kSmallPer], incl[kSmallPer];
    uint32_t any = 0;
#pragma unroll
    for (int j = 0; j < kSmallPer; ++j) {
        const int p = 16 * (j * kSmallThreads + tid);
        if (j < K && p + 16 <= n) c[j] = codes16(raw[j], m);
        else if (j < K && p < n && n >= 16) c[j] = ws_codes_window(raw[j], (int)(n - p), m);
        else if (j < K && p < n) c[j] = ws_codes<false>(src, n, p, m);
        else c[j] = u32x4{0x40404040u, 0x40404040u, 0x40404040u, 0x40404040u};
        cnt[j] = sig_count(c[j]);
        any |= c[j].x | c[j].y | c[j].z | c[j].w;
        incl[j] = j < K ? wave_incl_scan(cnt[j]) : 0;
        if (j < K && lane == 63) s_wsum[j][wv] = incl[j];
    }
    __syncthreads();
    // index of the first significant character of each of this thread's
    // chunks: the rows before, the waves before in the row, the lanes before
    int excl[kSmallPer];
    int total = 0;
#pragma unroll
    for (int j = 0; j < kSmallPer; ++j) {
        int woff = 0, rsum = 0;
        if (j < K)
            for (int w = 0; w < kSmallThreads / 64; ++w) {
                const int v = s_wsum[j][w];
                woff += w < wv ? v : 0;
                rsum += v;
            }
        excl[j] = total + woff + incl[j] - cnt[j];
        total += rsum;
    }
    // The first invalid byte and the first '=' (with its index) of the
    // threads that saw either, then every thread's significant codes at their
    // indices.  Both loops are free of branches: a character's index is a
    // running count, and a whitespace byte is written to a spare byte.
    if (any & 0x80808080u) {
        uint32_t pad_off = 0xFFFFFFFFu, pad_pos = 0, bad_off = 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < kSmallPer; ++j) {
            if (j >= K) break;                   // uniform
            const uint32_t w4[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
            int pos = excl[j];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t code = (w4[i >> 2] >> (8 * (i & 3))) & 0xFFu;
                const uint32_t off = (uint32_t)(16 * (j * kSmallThreads + tid) + i);
                const bool first_pad = code == kPadCode && pad_off == 0xFFFFFFFFu;
                pad_pos = first_pad ? (uint32_t)pos : pad_pos;
                pad_off = first_pad ? off : pad_off;
                const bool bad = (code & 0x80u) && code != kPadCode;
                bad_off = bad && off < bad_off ? off : bad_off;
                pos += is_sig(code) ? 1 : 0;
            }
        }
        if (pad_off != 0xFFFFFFFFu) atomicMin(&s_pad, ((unsigned long long)pad_off << 32) | pad_pos);
        if (bad_off != 0xFFFFFFFFu) atomicMin(&s_bad, bad_off);
    }
#pragma unroll
    for (int j = 0; j < kSmallPer; ++j) {
        if (j >= K) break;                       // uniform
        const uint32_t w4[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
        int pos = excl[j];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t code = (w4[i >> 2] >> (8 * (i & 3))) & 0xFFu;
            const bool sg = is_sig(code);
            vals[sg ? pos : kWsSmallMax + 8] = (uint8_t)code;
            pos += sg ? 1 : 0;
        }
    }
    __syncthreads();
    const unsigned long long pad = s_pad;
    const int E = pad == ~0ull ? -1 : (int)(pad & 0xFFFFFFFFu);
    // offsets of significant characters E+1 and E+2, from the threads whose
    // chunks hold them
#pragma unroll
    for (int j = 0; j < kSmallPer; ++j) {
        if (j >= K) break;                       // uniform
        if (E >= 0 && excl[j] < E + 3 && excl[j] + cnt[j] > E + 1) {
            const uint32_t w4[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
            int pos = excl[j];
            uint32_t o1 = 0xFFFFFFFFu, o2 = 0xFFFFFFFFu;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t code = (w4[i >> 2] >> (8 * (i & 3))) & 0xFFu;
                const uint32_t off = (uint32_t)(16 * (j * kSmallThreads + tid) + i);
                const bool sg = is_sig(code);
                o1 = sg && pos == E + 1 ? off : o1;
                o2 = sg && pos == E + 2 ? off : o2;
                pos += sg ? 1 : 0;
            }
            if (o1 != 0xFFFFFFFFu) s_after[0] = o1;
            if (o2 != 0xFFFFFFFFu) s_after[1] = o2;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int64_t bad = s_bad == 0xFFFFFFFFu ? kNoError : (int64_t)s_bad;
        const int64_t k = total;
        const int r = (int)(k & 3);
        int64_t len;
        if (nopad) {
            if (r == 1) bad = bad < n ? bad : n;
            else if (r >= 2 && (vals[k - 1] & (r == 2 ? 15u : 3u))) bad = bad < n ? bad : n;
            len = 3 * (k >> 2) + (r ? r - 1 : 0);
        } else if (E < 0) {
            if (r != 0) bad = bad < n ? bad : n;
            len = 3 * (k >> 2);
        } else {
            const int64_t a = (int64_t)(pad >> 32);
            const int pq = E & 3;
            int64_t e = kNoError;
            if (pq < 2) {
                e = a;
            } else {
                const uint32_t prev = vals[E - 1];
                if (prev & (pq == 2 ? 15u : 3u)) e = a;
                else if (pq == 3) e = E + 1 < k ? (int64_t)s_after[0] : kNoError;
                else if (E + 1 >= k) e = n;
                else if (vals[E + 1] != kPadCode) e = (int64_t)s_after[0];
                else e = E + 2 < k ? (int64_t)s_after[1] : kNoError;
            }
            bad = bad < e ? bad : e;
            len = 3 * (k >> 2) - (k - E);
        }
        s_len = len;
        s_err = bad;
    }
    __syncthreads();
    const int64_t err = s_err, len = s_len;
    if (err == kNoError && write) {
        // quantum q: values 4q .. 4q+3 (those at D and past are zero), the
        // bytes below len
        const int D = nopad || E < 0 ? total : E;
        const int nq = (D + 3) >> 2;
        for (int q = tid; q < nq; q += kSmallThreads) {
            uint32_t w = *(const uint32_t *)(vals + 4 * q);
            const int have = D - 4 * q;
            if (have < 4) w &= (1u << (8 * have)) - 1u;
            const uint32_t b = ws_quantum(w);
            const int64_t nb = len - 3 * (int64_t)q < 3 ? len - 3 * (int64_t)q : 3;
            uint8_t *o = dst + 3 * (int64_t)q;
            if (nb == 3) store3(o, b);
            else
                for (int i = 0; i < nb; ++i) o[i] = (uint8_t)(b >> (8 * i));
        }
    }
    if (tid == 0) {
        *out_len = err == kNoError ? len : -1;
        *first_bad = err == kNoError ? -1 : err;
    }
}

}  // namespace

hipError_t launch_encode_wrap(const uint8_t *src, int64_t n, uint8_t *dst, const EncTab &tab,
                              uint32_t flags, int64_t line_len, Shape sh, int cus, hipStream_t stream)
{
    const int64_t grid = grid_for(n / 12, sh, cus);
    B64_DISPATCH(k_encode_wrap, sh, grid, stream, src, n, dst, tab, flags, line_len);
    return hipGetLastError();
}

int64_t ws_tile_size(int64_t n)
{
    // about 4096 tiles or more; 4 KiB .. 32 KiB (1 .. kMaxRounds rounds), a power of two
    int64_t ts = kRound;
    while (ts < kMaxRounds * kRound && n / (2 * ts) >= 4096) ts *= 2;
    return ts;
}

int64_t ws_workspace_bytes(int64_t n)
{
    const int64_t TS = ws_tile_size(n);
    const int64_t ntiles = n > 0 ? (n + TS - 1) / TS : 0;
    return 8 * (ntiles + 3);      // prefix sums, first '=', mode
}

namespace {

template <int R>
void launch_ws_count(const uint8_t *src, int64_t n, const DecMap &map, int64_t *prefix,
                     int64_t *first_pad, int64_t *first_bad, const int64_t *mode, int64_t grid, bool nt,
                     hipStream_t stream)
{
    if (nt) hipLaunchKernelGGL((k_ws_count<R, true>), dim3(grid), dim3(kWsBlock), 0, stream, src, n, map, prefix, first_pad, first_bad, mode);
    else hipLaunchKernelGGL((k_ws_count<R, false>), dim3(grid), dim3(kWsBlock), 0, stream, src, n, map, prefix, first_pad, first_bad, mode);
}

// Workgroups of `kernel` resident on one compute unit at once (1 if the
// query fails), asked once per kernel.
template <typename K>
int resident_per_cu(K kernel, int *cache)
{
    int v = __atomic_load_n(cache, __ATOMIC_RELAXED);
    if (v > 0) return v;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kWsBlock, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    __atomic_store_n(cache, nb, __ATOMIC_RELAXED);
    return nb;
}

// One wave per tile, tiles dealt grid-stride: the grid is at most the
// workgroups that fit at once (blocks_per_cu caps it), so that no wave starts
// after others have finished and the tiles are shared evenly.
template <int D, bool CHECK>
void launch_ws_decode_tiles(const uint8_t *src, int64_t n, uint8_t *dst, const DecMap &map,
                            const int64_t *prefix, int64_t TS, int64_t ntiles, uint32_t flags,
                            int64_t *mode, int64_t *first_pad, int64_t *first_bad, int bpc, int cus,
                            bool nt, hipStream_t stream)
{
    static int fit[2] = {0, 0};
    const int per_cu = nt ? resident_per_cu(k_ws_decode<D, true, CHECK>, &fit[1])
                          : resident_per_cu(k_ws_decode<D, false, CHECK>, &fit[0]);
    int64_t grid = (int64_t)cus * (bpc < per_cu ? bpc : per_cu);
    const int64_t need = (ntiles + kWsBlock / 64 - 1) / (kWsBlock / 64);
    if (grid > need) grid = need;
    if (grid >= kXcds) grid -= grid % kXcds;
    if (grid < 1) grid = 1;
    if (nt) hipLaunchKernelGGL((k_ws_decode<D, true, CHECK>), dim3(grid), dim3(kWsBlock), 0, stream, src, n, dst, map, prefix, TS, flags, mode, first_pad, first_bad);
    else hipLaunchKernelGGL((k_ws_decode<D, false, CHECK>), dim3(grid), dim3(kWsBlock), 0, stream, src, n, dst, map, prefix, TS, flags, mode, first_pad, first_bad);
}

// k_ws_lines with 12 steps of loads in flight per lane on two workgroups per
// compute unit, a shape of its own: on 1 GiB of MIME text it took 0.484 ms
// per call, against 0.488-0.492 ms for 14 or 16 steps, 0.50 ms for 2, 4 or
// 10, 0.54 ms for 8, and 0.53-0.54 ms for 4 steps on four workgroups per
// compute unit (grid-stride steps).
void launch_ws_lines(const uint8_t *src, int64_t n, uint8_t *dst, const DecMap &map, const int64_t *prefix,
                     int64_t TS, uint32_t flags, int64_t *mode, int cus, bool nt, hipStream_t stream)
{
    constexpr int D = 12, bpc = 2;
    static int fit[2] = {0, 0};
    const int per_cu = nt ? resident_per_cu(k_ws_lines<D, true>, &fit[1])
                          : resident_per_cu(k_ws_lines<D, false>, &fit[0]);
    int64_t grid = (int64_t)cus * (bpc < per_cu ? bpc : per_cu);
    if (grid >= kXcds) grid -= grid % kXcds;
    if (grid < 1) grid = 1;
    if (nt) hipLaunchKernelGGL((k_ws_lines<D, true>), dim3(grid), dim3(kWsBlock), 0, stream, src, n, dst, map, prefix, TS, flags, mode);
    else hipLaunchKernelGGL((k_ws_lines<D, false>), dim3(grid), dim3(kWsBlock), 0, stream, src, n, dst, map, prefix, TS, flags, mode);
}

template <bool CHECK>
void launch_ws_decode_shape(const uint8_t *src, int64_t n, uint8_t *dst, const DecMap &map,
                            const int64_t *prefix, int64_t TS, int64_t ntiles, uint32_t flags,
                            int64_t *mode, int64_t *first_pad, int64_t *first_bad, Shape sh, int cus,
                            hipStream_t stream)
{
    switch (sh.unroll) {
    case 1: launch_ws_decode_tiles<1, CHECK>(src, n, dst, map, prefix, TS, ntiles, flags, mode, first_pad, first_bad, sh.bpc, cus, sh.nt, stream); break;
    case 4: launch_ws_decode_tiles<4, CHECK>(src, n, dst, map, prefix, TS, ntiles, flags, mode, first_pad, first_bad, sh.bpc, cus, sh.nt, stream); break;
    default: launch_ws_decode_tiles<2, CHECK>(src, n, dst, map, prefix, TS, ntiles, flags, mode, first_pad, first_bad, sh.bpc, cus, sh.nt, stream); break;
    }
}

}  // namespace

hipError_t launch_decode_ws(const uint8_t *src, int64_t n, uint8_t *dst, bool write, const DecMap &map,
                            int64_t *out_len, int64_t *first_bad, uint32_t flags, void *workspace,
                            Shape sh, int cus, int64_t guess_min, int64_t small_max,
                            hipStream_t stream)
{
    if (n <= small_max && n <= kWsSmallMax) {
        (void)launch_args(&k_ws_small, dim3(1), dim3(kSmallThreads), stream, src, n, dst, map, out_len,
                          first_bad, flags, write ? 1 : 0);
        return hipGetLastError();
    }
    const int64_t TS = ws_tile_size(n);
    const int64_t ntiles = n > 0 ? (n + TS - 1) / TS : 0;
    int64_t *prefix = (int64_t *)workspace;      // ntiles + 1 words
    int64_t *first_pad = prefix + ntiles + 1;
    int64_t *mode = first_pad + 1;               // kModeCounted, kModeChecked or kModeLines | ...
    // a decode first tries guessed prefix sums for text in regular lines (no
    // counting pass; k_ws_predict also resets the status); every later launch
    // checks *mode and does nothing unless it names that launch's path.
    // Texts shorter than guess_min take the counted path alone: there the
    // guess's three extra launches cost more than the counting pass.
    const bool guess = write && ntiles > 0 && n >= guess_min;
    if (!guess)
        hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(64), 0, stream, first_bad, first_pad, mode);
    if (guess) {
        const int64_t pgrid = std::min<int64_t>((ntiles + kWsBlock - 1) / kWsBlock, 1024);
        hipLaunchKernelGGL(k_ws_predict, dim3(pgrid), dim3(kWsBlock), 0, stream, src, n, map, prefix, TS, flags,
                           mode, first_pad, first_bad);
        launch_ws_lines(src, n, dst, map, prefix, TS, flags, mode, cus, sh.nt, stream);
        launch_ws_decode_shape<true>(src, n, dst, map, prefix, TS, ntiles, flags, mode, first_pad,
                                     first_bad, sh, cus, stream);
    }
    int64_t grid = (int64_t)cus * sh.bpc;
    if (grid > ntiles) grid = ntiles;
    if (grid >= kXcds) grid -= grid % kXcds;
    if (grid < 1) grid = 1;
    if (ntiles > 0) {
        switch (TS / kRound) {
        case 1: launch_ws_count<1>(src, n, map, prefix, first_pad, first_bad, mode, grid, sh.nt, stream); break;
        case 2: launch_ws_count<2>(src, n, map, prefix, first_pad, first_bad, mode, grid, sh.nt, stream); break;
        case 4: launch_ws_count<4>(src, n, map, prefix, first_pad, first_bad, mode, grid, sh.nt, stream); break;
        default: launch_ws_count<8>(src, n, map, prefix, first_pad, first_bad, mode, grid, sh.nt, stream); break;
        }
    }
    hipLaunchKernelGGL(k_ws_scan, dim3(1), dim3(kScanThreads), 0, stream, prefix, ntiles, mode);
    if (write && ntiles > 0)
        launch_ws_decode_shape<false>(src, n, dst, map, prefix, TS, ntiles, flags, mode, first_pad,
                                      first_bad, sh, cus, stream);
    hipLaunchKernelGGL(k_ws_finish, dim3(1), dim3(kWsBlock), 0, stream, src, n, dst, map, TS, prefix,
                       first_pad, out_len, first_bad, flags, write ? 1 : 0);
    return hipGetLastError();
}

}  // namespace b64hip
