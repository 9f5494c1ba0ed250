// b64_single.hip -- single-buffer encode / decode kernels and their launchers.
#include "b64_launch.h"

namespace b64hip {

// Status slots of the single-launch decode and validation (the slot form of
// DecSink): kStatusSlots x kSlotWords int64 (4.1 MiB) per device, zero when
// the code object is loaded and put back to zero by every call that uses one.
// Kernels reach them through the address passed in DecSink only.
__device__ __align__(256) int64_t g_status_slots[kStatusSlots * kSlotWords];

namespace {

// Device address of g_status_slots per device (each device holds its own
// copy of the array), looked up once.
int64_t *g_slots_base[64];

// Single buffer.  `head` whole groups are set aside so that the chunk outputs
// start on a 128-byte line (when dst is 4-byte aligned); then lane chunk c
// covers input [3*head + 12c, +12) and output [4*head + 16c, +16), grid-stride
// with U chunks in flight per lane.  Threads t < head encode one head group
// each; the last thread encodes the at most three whole groups and the
// partial group left after the chunks (padded, or cut short under
// kFlagNoPad).  Loads that need no table are issued before the table is
// staged, so that their latency overlaps the staging: when the input takes a
// single round, that round's chunks, then the head groups and the tail.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_encode(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, EncTab tab,
                                                     uint32_t flags)
{
    const int64_t ng = n / 3;
    const uint64_t da = (uint64_t)(uintptr_t)dst;
    int64_t head = (da & 3) ? 0 : (int64_t)((((uint64_t)kLine - (da & (kLine - 1))) & (kLine - 1)) >> 2);
    if (head > ng) head = ng;
    const int64_t nch = (ng - head) >> 2;
    const uint8_t *s0 = src + 3 * head;
    uint8_t *d0 = dst + 4 * head;
    const int64_t T = (int64_t)gridDim.x * kThreads;
    const int64_t t = logical_block() * kThreads + threadIdx.x;
    const int64_t rstep = U * T;
    const bool single = nch < rstep;                // one round, all but the last lanes' chunks
    const int64_t g = head + 4 * nch;               // first group of the tail
    u32x3 first[U];
    if (single) enc_round_load<U, NT>(first, s0, t, T, nch);
    EncTailIn hin, tin;
    if (t < head) hin = enc_tail_load(src + 3 * t, 3, 3 * t, n);
    if (t == kThreads - 1) tin = enc_tail_load(src + 3 * g, (int)(n - 3 * g), 3 * g, n);

    __shared__ uint32_t s_tab[16];
    stage_enc_table(s_tab, tab);
    const uint8_t *a = (const uint8_t *)s_tab;
    if (single) {
        enc_round_store<U, NT>(first, d0, t, T, a, nch);
    } else {
        const int64_t nfull = full_rounds(nch, rstep);
        enc_stream<U, NT>(s0, d0, t, T, rstep, nfull, a);
        enc_round_tail<U, NT>(s0, d0, t + nfull * rstep, T, a, nch);
    }
    if (t < head) enc_tail_regs(hin, 3, dst + 4 * t, a);
    if (t == kThreads - 1) enc_tail_regs(tin, (int)(n - 3 * g), dst + 4 * g, a, !(flags & kFlagNoPad));
}

// Single buffer.  The body is every quantum but the last (nbq quanta).
// `head` body quanta are set aside so that the chunk outputs start on a
// 128-byte line (3*head = -dst mod 128; 43 is the inverse of 3 mod 128); then
// lane chunk c covers characters [4*head + 16c, +16) and bytes
// [3*head + 12c, +12).  Threads t < head decode one head quantum each; the
// last thread decodes the tail: the (at most three) body quanta left after
// the chunks and the last quantum.
// The result goes to `sink` (raw or slot form, see DecSink).  Under
// kFlagNoPad '=' is invalid everywhere and the last quantum may have 2 or 3
// characters; the body is the same.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_decode(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, EncTab alpha,
                                                     DecSink sink, uint32_t flags)
{
    const bool nopad = (flags & kFlagNoPad) != 0;
    const int64_t nbq = n >= 1 ? (n - 1) >> 2 : 0;
    const uint64_t da = (uint64_t)(uintptr_t)dst;
    int64_t head = (int64_t)(((0 - da) * 43u) & (uint64_t)(kLine - 1));
    if (head > nbq) head = nbq;
    const int64_t nch = (nbq - head) >> 2;
    const uint8_t *s0 = src + 4 * head;
    uint8_t *d0 = dst + 3 * head;
    const int64_t T = (int64_t)gridDim.x * kThreads;
    const int64_t t = logical_block() * kThreads + threadIdx.x;
    const int64_t rstep = U * T;
    const bool single = nch < rstep;                // one round, all but the last lanes' chunks
    const int64_t q = head + 4 * nch;               // first quantum of the tail
    // Loads that need no map are issued before the map is staged, so that
    // their latency overlaps the staging: when the input takes a single round,
    // that round's chunks, then the head quantum and the tail.
    u32x4 first[U];
    if (single) dec_round_load<U, NT>(first, s0, t, T, nch);
    uint32_t hq = 0;
    if (t < head) hq = *(const u32a1 *)(src + 4 * t);
    TailIn tin = {{0u, 0u, 0u}, 0u};
    if (t == kThreads - 1) tin = tail_load(src + 4 * q, n - 4 * q);

    __shared__ uint32_t s_map[64];
    stage_dec_map_alpha(s_map, alpha);
    const uint8_t *m = (const uint8_t *)s_map;
    uint32_t err = 0;
    SinkLane lane;
    if (single) {
        if (nch > 0) dec_round_store<U, NT>(first, d0, t, T, m, err, nch);
    } else {
        const int64_t nfull = full_rounds(nch, rstep);
        dec_stream<U, NT>(s0, d0, t, T, rstep, nfull, m, err);
        dec_round_tail<U, NT>(s0, d0, t + nfull * rstep, T, m, err, nch);
    }
    // One test per lane for its whole share (bit 7 is set only by kBad).
    if (__ballot(err & 0x80)) {
        if (err & 0x80) {
            for (int64_t c = t; c < nch; c += T) {
                const int64_t bad = dec_check_inner(s0 + 16 * c, 16, m, nopad);
                if (bad >= 0) {
                    sink_bad(sink, lane, 4 * head + 16 * c + bad);
                    break;   // later chunks of this lane have larger offsets
                }
            }
        }
    }
    if (t < head) {
        uint32_t qerr = 0;
        const uint32_t v = dec_quantum(hq, m, qerr);
        dst[3 * t] = (uint8_t)(v >> 16);
        dst[3 * t + 1] = (uint8_t)(v >> 8);
        dst[3 * t + 2] = (uint8_t)v;
        if (qerr & 0x80) {
            const int64_t bad = dec_check_inner(src + 4 * t, 4, m, nopad);
            if (bad >= 0) sink_bad(sink, lane, 4 * t + bad);
        }
    }
    if (t == kThreads - 1) {
        int64_t len = 0;
        const int64_t bad =
            dec_tail_regs(tin, src + 4 * q, n - 4 * q, n, dst + 3 * q, m, &len, nopad);
        if (bad >= 0) sink_bad(sink, lane, 4 * q + bad);
        else sink_len(sink, lane, len, n);
    }
    sink_finish(sink, lane, logical_block() == 0, n);
}

__global__ void k_fill_i64(int64_t *p, int64_t count, int64_t value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// After a decode: first_bad == kNoError becomes -1 (valid); otherwise the
// buffer is invalid and its out_len becomes -1.
__global__ void k_finish_status(int64_t *out_len, int64_t *first_bad, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        if (first_bad[i] == kNoError) first_bad[i] = -1;
        else out_len[i] = -1;
    }
}

}  // namespace

int64_t grid_for(int64_t nch, Shape sh, int cus)
{
    const int64_t per_block = (int64_t)kThreads * sh.unroll;
    const int64_t need = (nch + per_block - 1) / per_block;
    // An input that `bpc` blocks per CU cover in one round gets exactly the
    // blocks it needs, so that all its loads are in flight at once; larger
    // inputs stream through `bpc` blocks per CU.  (Small inputs are tuned to
    // many blocks per CU, large ones to few.)
    int64_t grid = need <= (int64_t)cus * sh.bpc ? need : (int64_t)cus * sh.bpc;
    if (grid >= kXcds) grid -= grid % kXcds;   // a whole number of blocks per XCD
    return grid < 1 ? 1 : grid;
}

hipError_t launch_encode(const uint8_t *src, int64_t n, uint8_t *dst, const EncTab &tab, uint32_t flags,
                         Shape sh, int cus, hipStream_t stream)
{
    const int64_t grid = grid_for(n / 12, sh, cus);
    B64_DISPATCH(k_encode, sh, grid, stream, src, n, dst, tab, flags);
    return hipGetLastError();
}

hipError_t launch_decode(const uint8_t *src, int64_t n, uint8_t *dst, const EncTab &alpha,
                         const DecSink &sink, uint32_t flags, Shape sh, int cus, hipStream_t stream)
{
    const int64_t nbq = n >= 1 ? (n - 1) >> 2 : 0;
    const int64_t grid = grid_for(nbq >> 2, sh, cus);
    B64_DISPATCH(k_decode, sh, grid, stream, src, n, dst, alpha, sink, flags);
    return hipGetLastError();
}

hipError_t status_slot_addr(int idx, int64_t **out)
{
    if (idx < 0 || idx >= kStatusSlots) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    int64_t *base = __atomic_load_n(&g_slots_base[dev], __ATOMIC_ACQUIRE);
    if (!base) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_status_slots));
        if (e != hipSuccess) return e;
        base = (int64_t *)p;
        __atomic_store_n(&g_slots_base[dev], base, __ATOMIC_RELEASE);
    }
    *out = base + (int64_t)kSlotWords * idx;
    return hipSuccess;
}

hipError_t launch_fill(int64_t *p, int64_t count, int64_t value, hipStream_t stream)
{
    const int64_t blocks = (count + kThreads - 1) / kThreads;
    (void)launch_args(&k_fill_i64, dim3(blocks), dim3(kThreads), stream, p, count, value);
    return hipGetLastError();
}

hipError_t launch_finish(int64_t *out_len, int64_t *first_bad, int64_t count, hipStream_t stream)
{
    const int64_t blocks = (count + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_finish_status, dim3(blocks), dim3(kThreads), 0, stream, out_len,
                       first_bad, count);
    return hipGetLastError();
}

}  // namespace b64hip
