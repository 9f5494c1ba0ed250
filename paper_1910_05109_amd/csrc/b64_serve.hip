// b64_serve.hip -- a continuous-batching request server over the batched
// codec (host code; every codec step runs in the batch kernels).
//
// Requests (encode or decode) arrive over time with their payloads in host
// memory.  One scheduler thread (the caller's, inside b64_server_run) loops:
//
//   1. it notes every launch whose work has finished (a HIP event per launch,
//      polled); the launch's requests are then done -- their results are in
//      pinned host memory -- and their latency is that moment minus their
//      arrival.  Device arena space is given back in launch order;
//   2. it admits every request whose arrival time has passed: the request
//      joins the queue of its kind;
//   3. while fewer than `depth` launches are in flight, it takes the queued
//      requests of one kind (the kinds alternate), as many as `max_batch`
//      requests and `max_batch_bytes` payload bytes allow and the device arena
//      (the HBM budget) can hold -- payloads and outputs -- and enqueues on the
//      next of `nstreams` streams (round robin): ONE copy of the payloads
//      into the arena, ONE batched encode / decode kernel (plus, for a
//      decode, a one-block kernel that hands its first invalid offsets to the
//      host), and ONE copy of the outputs back.  The copies of launches up to
//      1 MiB of payload are kernels that read or write the mapped host pools,
//      larger ones are DMA (hipMemcpyAsync); b64_server_set_staging can make
//      them all one or the other.
//
// The pools' offsets are copied to device memory once, before serving, and
// the kernels read them there.  The pools and each slot's status words are
// pinned host memory mapped into the device's address space: the kernels
// write the lengths straight to the status words.  The decode's first
// invalid offsets, which the kernel merges with device-scope atomics (not
// used on host memory), go to a per-slot device array kept at "no error";
// the one-block kernel after the decode copies the launch's entries to the
// status words and resets them.  The host turns the raw statuses into the
// public form when the launch is done.
//
// Requests that arrive while others are on the GPU join the next launch;
// launches on different streams run at the same time on the device (a copy
// of one overlaps the kernel of another).
//
// Optionally (b64_server_set_zero_copy_max), a launch whose payload is at
// most `zc_max` bytes moves no bytes by DMA and takes no arena space: its
// kernel reads the payloads from, and writes the outputs to, the mapped
// pools over PCIe.  For small launches the copies cost more than the kernel:
// on MI355X one request of 1 KB / 64 KB / 1 MB took 18.5 / 31 / 51 us
// zero-copy against 26 / 51 / 92 us with DMA copies around the same kernel.
//
// Requests of one kind are packed in arrival order in the pools when the run
// starts (the payloads as a network stack would have left them), so a batch
// is a contiguous range of its pool and moves with one copy each way.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <vector>

#include "b64_launch.h"
#include "b64hip.h"

using namespace b64hip;

namespace b64hip {
// Payload bytes of a launch at most which it runs zero-copy, by default: none.
// The serving model keeps every launch's buffers in device memory, admitted
// under the HBM budget; zero-copy is for callers whose payloads start in host
// memory and who would rather not stage them.  Mixing the two ways at high
// rates measured worse than either alone on MI355X (launches of up to 4 MiB
// zero-copy beside staged ones fell below an offered 10^6 requests/s).
constexpr int64_t kZeroCopyDefault = 0;
// Staged launches with payloads up to this size copy by kernels by default
// (B64_STAGE_AUTO): for small launches a copy kernel answers sooner than a
// DMA copy and never meets the runtime's DMA stalls; large launches, at high
// request rates, need both copy directions at once, which DMA gives and
// copy kernels, one direction per launch, did not (28 GB/s of base64 at 10^6
// requests/s against 33-38 GB/s).
constexpr int64_t kKernelCopyAuto = 1 << 20;
}  // namespace b64hip

struct b64_server {
    int device = 0;
    int64_t budget = 0;          // bytes of device arena
    uint8_t *arena = nullptr;
    int nstreams = 0, depth = 0;
    int64_t max_batch = 0, max_batch_bytes = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> ev_start, ev_end;     // one pair per in-flight slot
    // per in-flight slot: its launch's first invalid offsets and lengths
    // (2 * max_batch words, pinned and mapped: the kernels write them there)
    std::vector<int64_t *> stat_out;
    std::vector<int64_t *> stat_out_dev;          // stat_out as the device sees it
    std::vector<int64_t *> bad_dev;               // zero-copy decodes: first invalid offsets
    int64_t zc_max = kZeroCopyDefault;
    // staged launches with at most this many payload bytes copy with kernels,
    // larger ones by DMA (b64_server_set_staging)
    int64_t kcopy_max = kKernelCopyAuto;
    hipEvent_t ref = nullptr;
};

namespace {

thread_local char s_err[256];

int64_t s_fail(int64_t code, const char *msg)
{
    snprintf(s_err, sizeof s_err, "%s", msg);
    return code;
}

int64_t s_hip(hipError_t e, const char *where)
{
    snprintf(s_err, sizeof s_err, "%s: %s", where, hipGetErrorString(e));
    return B64_EHIP;
}

constexpr int64_t kAlign = 256;

int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// The device arena as a ring: allocations are given back in the order they
// were made, so the live region is one span (possibly wrapped); an allocation
// that does not fit before the end skips the tail, which stays held until the
// allocation is given back.
struct Ring {
    int64_t size = 0, head = 0, used = 0, live = 0;

    bool alloc(int64_t n, int64_t *start, int64_t *held)
    {
        if (n > size) return false;
        const int64_t tail = size - head;
        int64_t waste = 0, at = head;
        if (n > tail) {
            waste = tail;
            at = 0;
        }
        if (used + waste + n > size) return false;
        head = at + n;
        used += waste + n;
        ++live;
        *start = at;
        *held = waste + n;
        return true;
    }
    void release(int64_t held)
    {
        used -= held;
        if (--live == 0) head = used = 0;
    }
};

// Requests of one kind, packed in arrival order in pinned host memory.
struct Pool {
    int kind = 0;
    std::vector<int64_t> req;            // request index of each entry
    uint8_t *in = nullptr, *out = nullptr;
    int64_t *in_off = nullptr;           // entries + 1 (relative to `in`)
    int64_t *out_off = nullptr;          // entries + 1 (relative to `out`)
    int64_t *len = nullptr, *bad = nullptr;
    // for zero-copy launches: the payload pools as the device sees them, and
    // the offsets copied to device memory before serving (the kernels look
    // them up before they can load a payload byte; over PCIe each lookup is
    // a round trip)
    const uint8_t *d_in = nullptr;
    uint8_t *d_out = nullptr;
    int64_t *d_in_off = nullptr, *d_out_off = nullptr;
    int64_t ready = 0, next = 0;         // admitted prefix, first not yet launched

    int64_t n() const { return (int64_t)req.size(); }
    // arena bytes of entries [f, f + c) when staged: payload, then outputs
    // (offsets and statuses live outside the arena)
    int64_t need(int64_t f, int64_t c) const
    {
        return align_up(in_off[f + c] - in_off[f]) + align_up(out_off[f + c] - out_off[f]);
    }
    void free_host()
    {
        for (void *p : {(void *)in, (void *)out, (void *)in_off, (void *)out_off, (void *)len,
                        (void *)bad})
            if (p) (void)hipHostFree(p);
        for (void *p : {(void *)d_in_off, (void *)d_out_off})
            if (p) (void)hipFree(p);
        in = out = nullptr;
        in_off = out_off = len = bad = nullptr;
        d_in_off = d_out_off = nullptr;
    }
};

struct Launch {
    int kind = 0, slot = 0;
    int64_t first = 0, count = 0, held = 0;     // held < 0: zero-copy, no arena space
    bool done = false;
};

// n bytes from src to dst (any alignment): each thread loads four 16-byte
// chunks, a grid apart, before it stores them, so that four loads per thread
// are in flight (over PCIe a load is a round trip); the last partial chunk
// goes byte by byte.  The staged launches' payloads go into the arena and
// their outputs out of it this way, between device memory and the mapped
// host pools.
__global__ __launch_bounds__(kThreads) void k_copy_bytes(uint8_t *__restrict__ dst,
                                                         const uint8_t *__restrict__ src, int64_t n)
{
    const int64_t T = (int64_t)gridDim.x * kThreads;
    const int64_t full = n >> 4;
    for (int64_t i0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; i0 < full; i0 += 4 * T) {
        u32x4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = i0 + j * T;
            v[j] = load16<true>(src + 16 * (i < full ? i : i0));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = i0 + j * T;
            if (i < full) store16<true>(dst + 16 * i, v[j]);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (n & 15)) dst[16 * full + threadIdx.x] = src[16 * full + threadIdx.x];
}

hipError_t copy_bytes(uint8_t *dst, const uint8_t *src, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t per = (int64_t)kThreads * 4 * 16;          // four chunks per thread
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 16384));
    return launch_args(&k_copy_bytes, dim3((unsigned)g), dim3(kThreads), st, dst, src, n);
}

// Entries [0, c) of a zero-copy decode's first invalid offsets: to the host
// (mapped) array, and the device array back to "no error" for the slot's
// next launch.
__global__ __launch_bounds__(kThreads) void k_status_out(int64_t *__restrict__ host, int64_t *__restrict__ dev,
                                                         int64_t c)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < c; i += (int64_t)gridDim.x * kThreads) {
        host[i] = dev[i];
        dev[i] = kNoError;
    }
}

int64_t now_ns(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() -
                                                                 t0)
        .count();
}

// Pinned host memory, mapped into the device's address space.
hipError_t host_alloc(void **p, int64_t bytes)
{
    return hipHostMalloc(p, (size_t)std::max<int64_t>(bytes, 64), hipHostMallocMapped);
}

// The device's address of mapped host memory.
template <class T>
hipError_t dev_view(T *h, T **d)
{
    void *v = nullptr;
    const hipError_t e = hipHostGetDevicePointer(&v, (void *)h, 0);
    *d = (T *)v;
    return e;
}

// The HIP runtime sets up a stream's DMA copy queues on first use, and the
// hipMemcpyAsync that does it blocks the calling thread for milliseconds
// (5-8 ms measured on MI355X, on the first host-to-device and device-to-host
// copies of each stream).  The scheduler thread must not stall with requests
// waiting, so every stream makes copies of both directions, small and large,
// once here, at creation.
hipError_t warm_copies(b64_server *s)
{
    const int64_t big = std::min<int64_t>(1 << 20, s->budget);
    uint8_t *h = nullptr;
    hipError_t e = host_alloc((void **)&h, big);
    if (e != hipSuccess) return e;
    memset(h, 0, (size_t)big);
    for (hipStream_t st : s->streams) {
        for (const int64_t bytes : {(int64_t)64, big}) {
            if (e == hipSuccess) e = hipMemcpyAsync(s->arena, h, (size_t)bytes, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(h, s->arena, (size_t)bytes, hipMemcpyDeviceToHost, st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    (void)hipHostFree(h);
    return e;
}

}  // namespace

extern "C" {

const char *b64_server_last_error(void) { return s_err; }

b64_server *b64_server_create(int64_t budget_bytes, int nstreams, int depth, int64_t max_batch,
                              int64_t max_batch_bytes)
{
    if (budget_bytes < (1 << 20)) return s_fail(0, "budget_bytes must be at least 1 MiB"), nullptr;
    if (nstreams < 1 || nstreams > 16) return s_fail(0, "nstreams must be 1..16"), nullptr;
    if (depth < nstreams || depth > 64) return s_fail(0, "depth must be nstreams..64"), nullptr;
    if (max_batch < 1 || max_batch_bytes < 1) return s_fail(0, "batch limits must be positive"), nullptr;
    b64_server *s = new b64_server;
    s->budget = align_up(budget_bytes);
    s->nstreams = nstreams;
    s->depth = depth;
    s->max_batch = max_batch;
    s->max_batch_bytes = max_batch_bytes;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc((void **)&s->arena, (size_t)s->budget);
    for (int i = 0; e == hipSuccess && i < nstreams; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    for (int i = 0; e == hipSuccess && i < depth; ++i) {
        hipEvent_t a = nullptr, b = nullptr;
        e = hipEventCreate(&a);
        if (e == hipSuccess) s->ev_start.push_back(a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e == hipSuccess) s->ev_end.push_back(b);
        int64_t *so = nullptr, *sod = nullptr, *bd = nullptr;
        if (e == hipSuccess) e = host_alloc((void **)&so, 8 * (2 * max_batch));
        if (e == hipSuccess) s->stat_out.push_back(so);
        if (e == hipSuccess) e = dev_view(so, &sod);
        if (e == hipSuccess) s->stat_out_dev.push_back(sod);
        if (e == hipSuccess) e = hipMalloc((void **)&bd, (size_t)(8 * max_batch));
        if (e == hipSuccess) s->bad_dev.push_back(bd);
        if (e == hipSuccess) e = launch_fill(bd, max_batch, kNoError, s->streams[0]);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->streams[0]);
    if (e == hipSuccess) e = hipEventCreate(&s->ref);
    if (e == hipSuccess) e = warm_copies(s);
    if (e != hipSuccess) {
        s_hip(e, "server creation");
        b64_server_destroy(s);
        return nullptr;
    }
    return s;
}

int64_t b64_server_set_staging(b64_server *s, int mode)
{
    if (!s) return s_fail(B64_EARG, "null server");
    const int64_t old = s->kcopy_max == 0 ? B64_STAGE_DMA
                        : s->kcopy_max == INT64_MAX ? B64_STAGE_KERNELS : B64_STAGE_AUTO;
    switch (mode) {
    case B64_STAGE_AUTO: s->kcopy_max = kKernelCopyAuto; break;
    case B64_STAGE_KERNELS: s->kcopy_max = INT64_MAX; break;
    case B64_STAGE_DMA: s->kcopy_max = 0; break;
    case -1: break;
    default: return s_fail(B64_EARG, "mode must be B64_STAGE_AUTO, B64_STAGE_KERNELS, B64_STAGE_DMA or -1");
    }
    return old;
}

int64_t b64_server_set_zero_copy_max(b64_server *s, int64_t bytes)
{
    if (!s) return s_fail(B64_EARG, "null server");
    const int64_t old = s->zc_max;
    if (bytes >= 0) s->zc_max = bytes;
    else if (bytes != -1) return s_fail(B64_EARG, "bytes must be >= 0, or -1 to read");
    return old;
}

void b64_server_destroy(b64_server *s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : s->ev_start) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : s->ev_end) (void)hipEventDestroy(ev);
    if (s->ref) (void)hipEventDestroy(s->ref);
    for (int64_t *p : s->stat_out) (void)hipHostFree(p);
    for (int64_t *p : s->bad_dev) (void)hipFree(p);
    if (s->arena) (void)hipFree(s->arena);
    delete s;
}

int64_t b64_server_run(b64_server *s, int64_t nreq, const int32_t *kind, const int64_t *arrival_ns,
                       const uint8_t *src, const int64_t *in_off, uint8_t *dst,
                       const int64_t *out_off, int64_t *out_len, int64_t *first_bad,
                       int64_t *done_ns, const char *alphabet, int64_t *stats)
{
    if (!s) return s_fail(B64_EARG, "null server");
    if (nreq < 0) return s_fail(B64_EARG, "negative request count");
    if (nreq > 0 && (!kind || !arrival_ns || !src || !in_off || !dst || !out_off || !out_len ||
                     !first_bad || !done_ns))
        return s_fail(B64_EARG, "null pointer");
    if (!stats) return s_fail(B64_EARG, "null stats");
    if (!alphabet) return s_fail(B64_EARG, "null alphabet");
    // the batched entry points check the alphabet; check it here as well, so
    // that a bad one fails before anything is enqueued
    {
        bool seen[256] = {false};
        for (int v = 0; v < 64; ++v) {
            const uint8_t c = (uint8_t)alphabet[v];
            if (c == '=' || seen[c]) return s_fail(B64_EARG, "alphabet must be 64 distinct bytes without '='");
            seen[c] = true;
        }
    }
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return s_hip(e, "set device");

    // ---- untimed set-up: pack each kind's payloads in pinned pools
    Pool pool[2];
    pool[0].kind = B64_SERVE_ENCODE;
    pool[1].kind = B64_SERVE_DECODE;
    for (int64_t i = 0; i < nreq; ++i) {
        if (kind[i] != B64_SERVE_ENCODE && kind[i] != B64_SERVE_DECODE)
            return s_fail(B64_EARG, "request kind must be B64_SERVE_ENCODE or B64_SERVE_DECODE");
        if (in_off[i + 1] < in_off[i] || in_off[i] < 0) return s_fail(B64_EARG, "in_off must be non-decreasing");
        if (i > 0 && arrival_ns[i] < arrival_ns[i - 1]) return s_fail(B64_EARG, "arrivals must be non-decreasing");
        pool[kind[i]].req.push_back(i);
    }
    auto cleanup = [&]() {
        pool[0].free_host();
        pool[1].free_host();
    };
    for (Pool &p : pool) {
        const int64_t m = p.n();
        int64_t in_bytes = 0, out_bytes = 0;
        for (int64_t k = 0; k < m; ++k) {
            const int64_t len = in_off[p.req[k] + 1] - in_off[p.req[k]];
            in_bytes += len;
            out_bytes += p.kind == B64_SERVE_ENCODE ? b64_encoded_len(len) : b64_decoded_max_len(len);
        }
        if ((e = host_alloc((void **)&p.in, in_bytes)) != hipSuccess ||
            (e = host_alloc((void **)&p.out, out_bytes)) != hipSuccess ||
            (e = host_alloc((void **)&p.in_off, 8 * (m + 1))) != hipSuccess ||
            (e = host_alloc((void **)&p.out_off, 8 * (m + 1))) != hipSuccess ||
            (e = host_alloc((void **)&p.len, 8 * m)) != hipSuccess ||
            (e = host_alloc((void **)&p.bad, 8 * m)) != hipSuccess) {
            cleanup();
            return s_hip(e, "pinned pools");
        }
        p.in_off[0] = p.out_off[0] = 0;
        for (int64_t k = 0; k < m; ++k) {
            const int64_t i = p.req[k], len = in_off[i + 1] - in_off[i];
            memcpy(p.in + p.in_off[k], src + in_off[i], (size_t)len);
            p.in_off[k + 1] = p.in_off[k] + len;
            p.out_off[k + 1] = p.out_off[k] + (p.kind == B64_SERVE_ENCODE ? b64_encoded_len(len)
                                                                           : b64_decoded_max_len(len));
            p.len[k] = -1;
            p.bad[k] = -1;
        }
        for (int64_t k = 0; k < m; ++k)
            if (p.need(k, 1) > s->budget && (in_off[p.req[k] + 1] - in_off[p.req[k]]) > s->zc_max) {
                cleanup();
                return s_fail(B64_EARG, "a request does not fit in the HBM budget");
            }
        uint8_t *din = nullptr;
        const size_t ob = (size_t)(8 * (m + 1));
        if ((e = dev_view(p.in, &din)) != hipSuccess || (e = dev_view(p.out, &p.d_out)) != hipSuccess ||
            (e = hipMalloc((void **)&p.d_in_off, ob)) != hipSuccess ||
            (e = hipMalloc((void **)&p.d_out_off, ob)) != hipSuccess ||
            (e = hipMemcpy(p.d_in_off, p.in_off, ob, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p.d_out_off, p.out_off, ob, hipMemcpyHostToDevice)) != hipSuccess) {
            cleanup();
            return s_hip(e, "pool device views");
        }
        p.d_in = din;
    }

    // ---- the timed loop
    Ring ring;
    ring.size = s->budget;
    std::deque<Launch> fifo;
    std::vector<int> free_slots;
    for (int i = s->depth - 1; i >= 0; --i) free_slots.push_back(i);
    std::vector<std::pair<float, float>> spans;      // device start / end of each launch, ms
    int64_t launches = 0, zc_launches = 0, peak_used = 0, max_inflight = 0, retired = 0, next_arrival = 0;
    int turn = 0, next_stream = 0;
    int64_t err = 0;
    e = hipEventRecord(s->ref, s->streams[0]);
    if (e != hipSuccess) {
        cleanup();
        return s_hip(e, "reference event");
    }
    const auto t0 = std::chrono::steady_clock::now();

    int cus = 0;
    e = device_cus(&cus);
    if (e != hipSuccess) {
        cleanup();
        return s_hip(e, "device query");
    }
    const EncTab tab = make_enc(alphabet);
    const DecMap map = make_dec(alphabet);
    const Shape enc_shape = op_shape(2, -1), dec_shape = op_shape(3, -1);

    // Enqueue entries [f, f + c) of pool p on the next stream.  The kernels
    // take the entries' offsets from their device copy and write the lengths
    // (and, through k_status_out, the first invalid offsets) straight to the
    // slot's mapped status words.  Staged (held >= 0): the payload is copied
    // into the arena, the kernel writes the outputs there, and they are
    // copied back.  Zero-copy (held < 0): the kernel reads the payload from,
    // and writes the outputs to, the mapped pools.
    auto launch = [&](Pool &p, int64_t f, int64_t c, int64_t start, int64_t held, int slot) -> int64_t {
        hipStream_t st = s->streams[next_stream];
        next_stream = (next_stream + 1) % s->nstreams;
        const bool dec = p.kind == B64_SERVE_DECODE, zc = held < 0;
        const int64_t nin = p.in_off[f + c] - p.in_off[f], nout = p.out_off[f + c] - p.out_off[f];
        // entry k's bytes are at base + (pool offset of entry f + k)
        const uint8_t *src_base = p.d_in;
        uint8_t *dst_base = p.d_out;
        uint8_t *d_in = nullptr, *d_out = nullptr;
        if (!zc) {
            d_in = s->arena + start;
            d_out = d_in + align_up(nin);
            src_base = d_in - p.in_off[f];
            dst_base = d_out - p.out_off[f];
        }
        int64_t *hs = s->stat_out_dev[slot];      // first invalid offsets, then lengths
        hipError_t x = hipEventRecord(s->ev_start[slot], st);
        if (x == hipSuccess && !zc)
            x = nin > s->kcopy_max ? hipMemcpyAsync(d_in, p.in + p.in_off[f], (size_t)nin, hipMemcpyHostToDevice, st)
                                   : copy_bytes(d_in, p.d_in + p.in_off[f], nin, st);
        if (x == hipSuccess)
            x = dec ? launch_decode_batch(src_base, p.d_in_off + f, c, dst_base, p.d_out_off + f, hs + c,
                                          s->bad_dev[slot], map, 0, dec_shape, cus, st)
                    : launch_encode_batch(src_base, p.d_in_off + f, c, dst_base, p.d_out_off + f, hs + c,
                                          tab, 0, enc_shape, cus, st);
        if (x == hipSuccess && dec) {
            const int64_t g = std::min<int64_t>((c + kThreads - 1) / kThreads, 32);
            x = launch_args(&k_status_out, dim3((unsigned)g), dim3(kThreads), st, hs, s->bad_dev[slot], c);
        }
        if (x == hipSuccess && !zc)
            x = nin > s->kcopy_max ? hipMemcpyAsync(p.out + p.out_off[f], d_out, (size_t)nout, hipMemcpyDeviceToHost, st)
                                   : copy_bytes(p.d_out + p.out_off[f], d_out, nout, st);
        if (x == hipSuccess) x = hipEventRecord(s->ev_end[slot], st);
        if (x != hipSuccess) return s_hip(x, zc ? "zero-copy launch" : "staged launch");
        Launch L;
        L.kind = p.kind;
        L.slot = slot;
        L.first = f;
        L.count = c;
        L.held = held;
        fifo.push_back(L);
        ++launches;
        zc_launches += zc ? 1 : 0;
        max_inflight = std::max<int64_t>(max_inflight, (int64_t)fifo.size());
        return 0;
    };

    while (retired < nreq && !err) {
        bool progress = false;
        // 1. launches that have finished
        for (Launch &L : fifo) {
            if (L.done) continue;
            const hipError_t q = hipEventQuery(s->ev_end[L.slot]);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                err = s_hip(q, "event query");
                break;
            }
            const int64_t t = now_ns(t0);
            Pool &p = pool[L.kind];
            // the kernel's raw status: first invalid offset kNoError for a
            // valid decode (whose length the kernel wrote), else the offset
            const int64_t *bad = s->stat_out[L.slot], *len = bad + L.count;
            for (int64_t k = 0; k < L.count; ++k) {
                const int64_t e_ = L.first + k;
                done_ns[p.req[e_]] = t;
                if (p.kind == B64_SERVE_DECODE && bad[k] != kNoError) {
                    p.bad[e_] = bad[k];
                    p.len[e_] = -1;
                } else {
                    p.bad[e_] = -1;
                    p.len[e_] = len[k];
                }
            }
            float a = 0.f, b = 0.f;
            if (hipEventElapsedTime(&a, s->ref, s->ev_start[L.slot]) == hipSuccess &&
                hipEventElapsedTime(&b, s->ref, s->ev_end[L.slot]) == hipSuccess)
                spans.emplace_back(a, b);
            L.done = true;
            retired += L.count;
            progress = true;
        }
        while (!fifo.empty() && fifo.front().done) {
            if (fifo.front().held >= 0) ring.release(fifo.front().held);
            free_slots.push_back(fifo.front().slot);
            fifo.pop_front();
        }
        // 2. arrivals
        const int64_t t = now_ns(t0);
        while (next_arrival < nreq && arrival_ns[next_arrival] <= t) {
            ++pool[kind[next_arrival]].ready;
            ++next_arrival;
            progress = true;
        }
        // 3. launches of queued requests, the kinds in turn
        for (int pass = 0; pass < 2 && !err; ++pass) {
            Pool &p = pool[(turn + pass) & 1];
            if (free_slots.empty()) break;
            int64_t c = std::min<int64_t>(p.ready - p.next, s->max_batch);
            if (c <= 0) continue;
            while (c > 1 && p.in_off[p.next + c] - p.in_off[p.next] > s->max_batch_bytes) c = (c + 1) / 2;
            // zero-copy once the payload is small enough, else arena space;
            // halved until one of them fits
            int64_t start = 0, held = -1;        // held < 0: zero-copy
            while (c > 0) {
                if (p.in_off[p.next + c] - p.in_off[p.next] <= s->zc_max) break;
                if (ring.alloc(p.need(p.next, c), &start, &held)) break;
                c /= 2;
            }
            if (c == 0) continue;               // waits for earlier launches to give space back
            const int slot = free_slots.back();
            free_slots.pop_back();
            err = launch(p, p.next, c, start, held, slot);
            if (err) break;
            peak_used = std::max(peak_used, ring.used);
            p.next += c;
            progress = true;
        }
        turn ^= 1;
        if (!progress) {
            // nothing to do: wait for the next arrival if nothing is in flight
            if (fifo.empty() && next_arrival < nreq) {
                const int64_t wait = arrival_ns[next_arrival] - now_ns(t0);
                if (wait > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(wait - 100000));
            } else {
                std::this_thread::yield();
            }
        }
    }
    const int64_t wall = now_ns(t0);
    for (hipStream_t st : s->streams) {
        const hipError_t x = hipStreamSynchronize(st);
        if (x != hipSuccess && !err) err = s_hip(x, "stream synchronize");
    }
    if (err) {
        // a decode whose status hand-over never ran leaves its entries in the
        // slot's device array: set them all back to "no error" for the next run
        for (int64_t *bd : s->bad_dev) (void)launch_fill(bd, s->max_batch, kNoError, s->streams[0]);
        (void)hipStreamSynchronize(s->streams[0]);
        (void)hipGetLastError();
        cleanup();
        return err;
    }
    // ---- untimed: results to the caller's arrays
    for (const Pool &p : pool) {
        for (int64_t k = 0; k < p.n(); ++k) {
            const int64_t i = p.req[k];
            const int64_t len = p.len[k];
            out_len[i] = len;
            first_bad[i] = p.kind == B64_SERVE_ENCODE ? -1 : p.bad[k];
            if (len > 0) memcpy(dst + out_off[i], p.out + p.out_off[k], (size_t)len);
        }
    }
    // launches that were running on the device at the same time
    int64_t concurrent = 0, overlapped = 0;
    {
        std::vector<std::pair<float, int>> ev;
        for (auto &sp : spans) {
            ev.emplace_back(sp.first, +1);
            ev.emplace_back(sp.second, -1);
        }
        std::sort(ev.begin(), ev.end(),
                  [](const std::pair<float, int> &a, const std::pair<float, int> &b) {
                      return a.first < b.first || (a.first == b.first && a.second < b.second);
                  });
        int64_t cur = 0;
        for (auto &x : ev) concurrent = std::max(concurrent, cur += x.second);
        // sorted by start, launch k overlaps an earlier one when it starts
        // before the latest end so far, and a later one when the next launch
        // starts before it ends
        std::vector<std::pair<float, float>> sorted = spans;
        std::sort(sorted.begin(), sorted.end());
        float reach = -1.f;
        for (size_t k = 0; k < sorted.size(); ++k) {
            const bool with_earlier = k > 0 && sorted[k].first < reach;
            const bool with_later = k + 1 < sorted.size() && sorted[k + 1].first < sorted[k].second;
            overlapped += (with_earlier || with_later) ? 1 : 0;
            reach = std::max(reach, sorted[k].second);
        }
    }
    stats[B64_STAT_LAUNCHES] = launches;
    stats[B64_STAT_WALL_NS] = wall;
    stats[B64_STAT_PEAK_ARENA] = peak_used;
    stats[B64_STAT_MAX_INFLIGHT] = max_inflight;
    stats[B64_STAT_MAX_CONCURRENT] = concurrent;
    stats[B64_STAT_OVERLAPPED] = overlapped;
    stats[B64_STAT_ARENA] = s->budget;
    stats[B64_STAT_ZERO_COPY] = zc_launches;
    cleanup();
    return 0;
}

}  // extern "C"
