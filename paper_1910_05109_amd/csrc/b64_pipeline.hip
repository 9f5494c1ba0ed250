// b64_pipeline.hip -- host-memory encode / decode through a chunked
// host -> device -> host pipeline (the GPU reading of the paper's advice, in
// Section "Experiments", to process large inputs in parts that fit on chip
// rather than streaming whole buffers through memory).
//
// A pipeline owns `depth` slots, each with pinned host staging and device
// buffers sized for one chunk, and three HIP streams, one per stage.  Chunk k
// goes to slot k mod depth: the host copies it into pinned memory (split
// across `host_threads` threads), then the H2D copy runs on the first stream,
// the codec kernels on the second and the D2H copy on the third, chained by
// events, and the host collects the result when it comes back to that slot.
// Up to `depth` chunks are in flight, so host copies, PCIe transfers in both
// directions and kernels overlap; with one copy per direction at a time, each
// transfer has the link's full bandwidth in its direction.  Every codec step runs in
// the library's kernels; the pipeline only moves bytes.  When the caller's
// source or destination is already pinned host memory, the copies go straight
// between it and the device and the staging copy on that side is skipped: the
// host-side copies are what bound the pipeline on pageable memory (every byte
// crosses host memory twice more than the DMA itself).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "b64_launch.h"
#include "b64hip.h"

struct b64_pipeline {
    struct Slot {
        hipEvent_t loaded = nullptr, coded = nullptr, done = nullptr;   // after H2D, kernels, D2H
        uint8_t *h_in = nullptr, *h_out = nullptr;    // pinned
        uint8_t *d_in = nullptr, *d_out = nullptr;
        int64_t *d_status = nullptr, *h_status = nullptr;
        bool busy = false;
        int64_t in_off = 0, in_len = 0, out_off = 0, out_len = 0;
    };
    int device = 0;
    int64_t chunk = 0;          // input bytes (encode) or characters (decode) per slot
    int host_threads = 1;
    // one stream per stage: chunks cross each stage in order, one at a time,
    // so host-to-device and device-to-host copies each get the whole link in
    // their direction and the two directions overlap
    hipStream_t s_in = nullptr, s_code = nullptr, s_out = nullptr;
    std::vector<Slot> slots;
};

namespace {

thread_local char p_err[256];

int64_t p_fail(int64_t code, const char *msg)
{
    snprintf(p_err, sizeof p_err, "%s", msg);
    return code;
}

int64_t p_hip(hipError_t e, const char *where)
{
    snprintf(p_err, sizeof p_err, "%s: %s", where, hipGetErrorString(e));
    return B64_EHIP;
}

// memcpy split across up to `threads` threads (large copies only).
void par_copy(uint8_t *dst, const uint8_t *src, int64_t n, int threads)
{
    const int64_t min_part = 4 << 20;
    int64_t parts = std::min<int64_t>(threads, (n + min_part - 1) / min_part);
    if (parts <= 1) {
        if (n) memcpy(dst, src, (size_t)n);
        return;
    }
    const int64_t per = (n + parts - 1) / parts;
    std::vector<std::thread> ws;
    for (int64_t p = 1; p < parts; ++p) {
        const int64_t a = p * per, b = std::min(n, a + per);
        if (a < b) ws.emplace_back([=] { memcpy(dst + a, src + a, (size_t)(b - a)); });
    }
    memcpy(dst, src, (size_t)std::min(n, per));
    for (auto &w : ws) w.join();
}

// Whether [ptr, ptr + n) lies in pinned host memory (hipHostMalloc'd or
// registered), so that DMA can use it as it is.  A failed query (pageable
// memory) leaves an error that the next HIP call would report; it is cleared.
bool pinned(const void *ptr, int64_t n)
{
    if (!ptr || n <= 0) return false;
    for (const void *q : {ptr, (const void *)((const uint8_t *)ptr + n - 1)}) {
        hipPointerAttribute_t a;
        const hipError_t e = hipPointerGetAttributes(&a, q);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        if (a.type != hipMemoryTypeHost) return false;
    }
    return true;
}

// Stage 1 of a chunk: its input to the device on s_in, then s_code waits for
// it (the caller launches the kernels on s_code next).
hipError_t load_chunk(b64_pipeline *p, b64_pipeline::Slot &s, const uint8_t *h_in)
{
    hipError_t e;
    if ((e = hipMemcpyAsync(s.d_in, h_in, s.in_len, hipMemcpyHostToDevice, p->s_in)) != hipSuccess ||
        (e = hipEventRecord(s.loaded, p->s_in)) != hipSuccess)
        return e;
    return hipStreamWaitEvent(p->s_code, s.loaded, 0);
}

// Stage 3, after the kernels: out_len bytes of output (and the two status
// words first, when h_status is given) back to the host on s_out; s.done
// fires when they are there.
hipError_t store_chunk(b64_pipeline *p, b64_pipeline::Slot &s, uint8_t *h_out, int64_t out_len,
                       int64_t *h_status)
{
    hipError_t e;
    if ((e = hipEventRecord(s.coded, p->s_code)) != hipSuccess ||
        (e = hipStreamWaitEvent(p->s_out, s.coded, 0)) != hipSuccess)
        return e;
    if (h_status &&
        (e = hipMemcpyAsync(h_status, s.d_status, 2 * sizeof(int64_t), hipMemcpyDeviceToHost,
                            p->s_out)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(h_out, s.d_out, out_len, hipMemcpyDeviceToHost, p->s_out)) != hipSuccess)
        return e;
    return hipEventRecord(s.done, p->s_out);
}

// An error after chunks were enqueued: let every copy and kernel in flight
// finish (they may read the caller's source or write its destination, which
// the caller may free once the call returns), and forget the slots' chunks,
// so that the next call starts from empty slots.
int64_t p_abort(b64_pipeline *p, int64_t code)
{
    for (hipStream_t st : {p->s_in, p->s_code, p->s_out}) (void)hipStreamSynchronize(st);
    (void)hipGetLastError();
    for (auto &s : p->slots) s.busy = false;
    return code;
}

void release(b64_pipeline *p)
{
    for (hipStream_t st : {p->s_in, p->s_code, p->s_out})
        if (st) (void)hipStreamSynchronize(st);
    for (auto &s : p->slots) {
        for (hipEvent_t ev : {s.loaded, s.coded, s.done})
            if (ev) (void)hipEventDestroy(ev);
        if (s.h_in) (void)hipHostFree(s.h_in);
        if (s.h_out) (void)hipHostFree(s.h_out);
        if (s.h_status) (void)hipHostFree(s.h_status);
        if (s.d_in) (void)hipFree(s.d_in);
        if (s.d_out) (void)hipFree(s.d_out);
        if (s.d_status) (void)hipFree(s.d_status);
    }
    for (hipStream_t st : {p->s_in, p->s_code, p->s_out})
        if (st) (void)hipStreamDestroy(st);
    delete p;
}

}  // namespace

extern "C" {

const char *b64_pipeline_last_error(void) { return p_err; }

b64_pipeline *b64_pipeline_create(int64_t chunk_bytes, int depth, int host_threads)
{
    if (chunk_bytes < 48 || depth < 1 || depth > 16 || host_threads < 1 || host_threads > 64) {
        p_fail(B64_EARG, "chunk_bytes >= 48, 1 <= depth <= 16, 1 <= host_threads <= 64");
        return nullptr;
    }
    b64_pipeline *p = new b64_pipeline;
    // a multiple of 3*4*128 bytes: encode chunks end on a group, decode chunks
    // on a quantum, and both sides stay 128-byte aligned
    p->chunk = (chunk_bytes + 1535) / 1536 * 1536;
    p->host_threads = host_threads;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        p_hip(e, "device query");
        delete p;
        return nullptr;
    }
    // More than three chunks in flight measured slower on MI355X (1 GiB,
    // pinned buffers: 29 ms at depth 2 or 3, 40 to 65 ms at depth 4 to 6,
    // for any chunk size from 8 to 128 MiB): with copies queued further
    // ahead, the two copy directions stop overlapping.
    p->slots.resize(std::min(depth, 3));
    // input and output capacity of a slot: a chunk of bytes encodes to 4/3 as
    // many characters, and decoding a chunk of characters writes 3/4 as many
    const int64_t cap = p->chunk / 3 * 4;
    for (hipStream_t *st : {&p->s_in, &p->s_code, &p->s_out}) {
        if ((e = hipStreamCreateWithFlags(st, hipStreamNonBlocking)) != hipSuccess) {
            p_hip(e, "pipeline streams");
            release(p);
            return nullptr;
        }
    }
    for (auto &s : p->slots) {
        if ((e = hipEventCreateWithFlags(&s.loaded, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s.coded, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipHostMalloc((void **)&s.h_in, cap, hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc((void **)&s.h_out, cap, hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc((void **)&s.h_status, 2 * sizeof(int64_t), hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipMalloc((void **)&s.d_in, cap)) != hipSuccess ||
            (e = hipMalloc((void **)&s.d_out, cap)) != hipSuccess ||
            (e = hipMalloc((void **)&s.d_status, 2 * sizeof(int64_t))) != hipSuccess) {
            p_hip(e, "pipeline allocation");
            release(p);
            return nullptr;
        }
    }
    return p;
}

void b64_pipeline_destroy(b64_pipeline *p)
{
    if (p) release(p);
}

int64_t b64_pipeline_encode(b64_pipeline *p, const uint8_t *src, int64_t n, uint8_t *dst,
                            const char *alphabet)
{
    if (!p || n < 0 || (n > 0 && (!src || !dst))) return p_fail(B64_EARG, "bad argument");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return p_hip(e, "set device");
    const int depth = (int)p->slots.size();
    const int64_t nchunks = (n + p->chunk - 1) / p->chunk;
    const bool src_pinned = pinned(src, n), dst_pinned = pinned(dst, 4 * ((n + 2) / 3));
    for (int64_t k = 0; k < nchunks + depth; ++k) {
        b64_pipeline::Slot &s = p->slots[k % depth];
        if (s.busy) {   // collect this slot's previous chunk
            if ((e = hipEventSynchronize(s.done)) != hipSuccess) return p_abort(p, p_hip(e, "pipeline wait"));
            if (!dst_pinned) par_copy(dst + s.out_off, s.h_out, s.out_len, p->host_threads);
            s.busy = false;
        }
        if (k >= nchunks) continue;
        s.in_off = k * p->chunk;
        s.in_len = std::min(p->chunk, n - s.in_off);
        s.out_off = s.in_off / 3 * 4;
        s.out_len = (s.in_len + 2) / 3 * 4;
        if (!src_pinned) par_copy(s.h_in, src + s.in_off, s.in_len, p->host_threads);
        const uint8_t *h_in = src_pinned ? src + s.in_off : s.h_in;
        if ((e = load_chunk(p, s, h_in)) != hipSuccess) return p_abort(p, p_hip(e, "pipeline H2D"));
        const int64_t r = b64_encode(s.d_in, s.in_len, s.d_out, alphabet, p->s_code);
        if (r < 0) return p_abort(p, r);
        uint8_t *h_out = dst_pinned ? dst + s.out_off : s.h_out;
        if ((e = store_chunk(p, s, h_out, s.out_len, nullptr)) != hipSuccess)
            return p_abort(p, p_hip(e, "pipeline D2H"));
        s.busy = true;
    }
    return 4 * ((n + 2) / 3);
}

// Decode in chunks of whole quanta.  Chunk k is decoded as a standalone input;
// since every earlier chunk ended in the data state, its first invalid offset
// is the input's, shifted by the chunk's start.  A chunk other than the last
// that is valid only because it ends with padding makes the next character
// the first invalid one.
int64_t b64_pipeline_decode(b64_pipeline *p, const uint8_t *src, int64_t n, uint8_t *dst,
                            const char *alphabet)
{
    if (!p || n < 0 || (n > 0 && (!src || !dst))) return p_fail(B64_EARG, "bad argument");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return p_hip(e, "set device");
    const int depth = (int)p->slots.size();
    const int64_t nchunks = n ? (n + p->chunk - 1) / p->chunk : 1;
    const bool src_pinned = pinned(src, n), dst_pinned = pinned(dst, 3 * (n / 4));
    int64_t first_bad = -1, total = 0;
    for (int64_t k = 0; k < nchunks + depth; ++k) {
        b64_pipeline::Slot &s = p->slots[k % depth];
        if (s.busy) {
            if ((e = hipEventSynchronize(s.done)) != hipSuccess) return p_abort(p, p_hip(e, "pipeline wait"));
            s.busy = false;
            const int64_t len = s.h_status[0], bad = s.h_status[1];
            const bool last = s.in_off + s.in_len == n;
            int64_t off = -1;
            if (bad >= 0) off = s.in_off + bad;
            else if (!last && len != s.in_len / 4 * 3) off = s.in_off + s.in_len;
            if (off >= 0) {
                if (first_bad < 0 || off < first_bad) first_bad = off;
            } else if (first_bad < 0) {
                if (!dst_pinned) par_copy(dst + s.out_off, s.h_out, len, p->host_threads);
                total += len;
            }
        }
        if (k >= nchunks || first_bad >= 0) continue;
        s.in_off = k * p->chunk;
        s.in_len = std::min(p->chunk, n - s.in_off);
        s.out_off = s.in_off / 4 * 3;
        if (!src_pinned) par_copy(s.h_in, src + s.in_off, s.in_len, p->host_threads);
        const uint8_t *h_in = src_pinned ? src + s.in_off : s.h_in;
        if ((e = load_chunk(p, s, h_in)) != hipSuccess) return p_abort(p, p_hip(e, "pipeline H2D"));
        const int64_t r = b64_decode_async(s.d_in, s.in_len, s.d_out, s.d_status, s.d_status + 1,
                                           alphabet, p->s_code);
        if (r < 0) return p_abort(p, r);
        uint8_t *h_out = dst_pinned ? dst + s.out_off : s.h_out;
        if ((e = store_chunk(p, s, h_out, s.in_len / 4 * 3, s.h_status)) != hipSuccess)
            return p_abort(p, p_hip(e, "pipeline D2H"));
        s.busy = true;
    }
    return first_bad >= 0 ? ~first_bad : total;
}

}  // extern "C"
