// b64_validate.hip -- read-only validation of one base64 buffer and its launcher.
//
// The decoder's validation (Section "Decoding": every character goes through
// the look-up table whose special value marks characters outside the
// alphabet, the results ORed into one error word tested once) without the
// packing and the stores: the kernel reads the N characters and writes
// nothing but the status words, so it moves N bytes where decode moves 1.75N.
// It reports exactly what b64_decode would: the decoded length of a valid
// input, or the first invalid offset.
#include "b64_launch.h"

namespace b64hip {
namespace {

// OR of the map entries of four characters (bit 7 set iff one is invalid).
__device__ __forceinline__ uint32_t val_quantum(uint32_t q, const uint8_t *map)
{
    return (uint32_t)map[q & 0xFF] | map[(q >> 8) & 0xFF] | map[(q >> 16) & 0xFF] | map[q >> 24];
}

__device__ __forceinline__ uint32_t val_chunk(u32x4 in, const uint8_t *map)
{
    return val_quantum(in.x, map) | val_quantum(in.y, map) | val_quantum(in.z, map) |
           val_quantum(in.w, map);
}

// `nrounds` complete rounds of lane chunks c0 + r*rstep + j*stride, the loads
// of round r+1 issued before round r is looked up.
template <int U, bool NT>
__device__ __forceinline__ uint32_t val_stream(const uint8_t *s0, int64_t c0, int64_t stride,
                                               int64_t rstep, int64_t nrounds, const uint8_t *map)
{
    uint32_t err = 0;
    if (nrounds <= 0) return 0;
    u32x4 A[U], B[U];
#pragma unroll
    for (int j = 0; j < U; ++j) A[j] = load16<NT>(s0 + 16 * (c0 + j * stride));
    int64_t r = 0;
    for (; r + 2 < nrounds; r += 2) {
#pragma unroll
        for (int j = 0; j < U; ++j) B[j] = load16<NT>(s0 + 16 * (c0 + rstep + j * stride));
#pragma unroll
        for (int j = 0; j < U; ++j) err |= val_chunk(A[j], map);
#pragma unroll
        for (int j = 0; j < U; ++j) A[j] = load16<NT>(s0 + 16 * (c0 + 2 * rstep + j * stride));
#pragma unroll
        for (int j = 0; j < U; ++j) err |= val_chunk(B[j], map);
        c0 += 2 * rstep;
    }
    if (r + 1 < nrounds) {
#pragma unroll
        for (int j = 0; j < U; ++j) B[j] = load16<NT>(s0 + 16 * (c0 + rstep + j * stride));
#pragma unroll
        for (int j = 0; j < U; ++j) err |= val_chunk(A[j], map) | val_chunk(B[j], map);
    } else {
#pragma unroll
        for (int j = 0; j < U; ++j) err |= val_chunk(A[j], map);
    }
    return err;
}

// The body is every quantum but the last; lane chunk c covers characters
// [16c, 16c+16).  The last thread validates the characters after the chunks
// (at most three body quanta and the last quantum) as the end of the input
// and, when they are valid, reports the decoded length.  The result goes to
// `sink` (raw or slot form, see DecSink).  kFlagNoPad selects the unpadded
// rules.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_validate(const uint8_t *__restrict__ src, int64_t n,
                                                       EncTab alpha, DecSink sink, uint32_t flags)
{
    const bool nopad = (flags & kFlagNoPad) != 0;
    const int64_t nbq = n >= 1 ? (n - 1) >> 2 : 0;
    const int64_t nch = nbq >> 2;
    const int64_t T = (int64_t)gridDim.x * kThreads;
    const int64_t t = logical_block() * kThreads + threadIdx.x;
    const int64_t rstep = U * T;
    const bool single = nch < rstep;                // one round, all but the last lanes' chunks
    const int64_t q0 = 4 * nch;                     // first quantum after the chunks
    // Loads that need no map go first, overlapping the staging of the map:
    // when the input takes a single round, that round's chunks, then the tail.
    u32x4 first[U];
    if (single && nch > 0) {
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t c = t + j * T;
            first[j] = load16<NT>(src + 16 * (c < nch ? c : nch - 1));
        }
    }
    TailIn tin = {{0u, 0u, 0u}, 0u};
    if (t == kThreads - 1) tin = tail_load(src + 4 * q0, n - 4 * q0);

    __shared__ uint32_t s_map[64];
    stage_dec_map_alpha(s_map, alpha);
    const uint8_t *m = (const uint8_t *)s_map;
    SinkLane lane;
    uint32_t err = 0;
    if (single) {
        if (nch > 0) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (t + j * T < nch) err |= val_chunk(first[j], m);
        }
    } else {
        const int64_t nfull = full_rounds(nch, rstep);
        err = val_stream<U, NT>(src, t, T, rstep, nfull, m);
        for (int64_t c = t + nfull * rstep; c < nch; c += T)
            err |= val_chunk(load16<NT>(src + 16 * c), m);
    }
    if (__ballot(err & 0x80)) {
        if (err & 0x80) {
            for (int64_t c = t; c < nch; c += T) {
                const int64_t bad = dec_check_inner(src + 16 * c, 16, m, nopad);
                if (bad >= 0) {
                    sink_bad(sink, lane, 16 * c + bad);
                    break;   // later chunks of this lane have larger offsets
                }
            }
        }
    }
    if (t == kThreads - 1) {
        int64_t len = 0;
        const int64_t bad = dec_tail_regs(tin, src + 4 * q0, n - 4 * q0, n, nullptr, m, &len, nopad);
        if (bad >= 0) sink_bad(sink, lane, 4 * q0 + bad);
        else sink_len(sink, lane, len, n);
    }
    sink_finish(sink, lane, logical_block() == 0, n);
}

}  // namespace

hipError_t launch_validate(const uint8_t *src, int64_t n, const EncTab &alpha, const DecSink &sink,
                           uint32_t flags, Shape sh, int cus, hipStream_t stream)
{
    const int64_t nbq = n >= 1 ? (n - 1) >> 2 : 0;
    const int64_t grid = grid_for(nbq >> 2, sh, cus);
    B64_DISPATCH(k_validate, sh, grid, stream, src, n, alpha, sink, flags);
    return hipGetLastError();
}

}  // namespace b64hip
