// b64_fused.hip -- decode fused into its consumer.
//
// The paper ends by proposing to run its decoder inside the code that
// consumes the data (Section "Conclusion": inside vectorized parsers), so
// that the decoded bytes are used where they are produced.  This kernel does
// that for a common GPU consumer: rows of base64 that each encode `dim`
// little-endian float32 values (embedding vectors carried in JSON, for
// instance) are decoded and converted to bfloat16 in registers, and only the
// bfloat16 row reaches memory: N characters read and 3N/8 bytes written,
// against N + 3N/4 + 3N/4 + 3N/8 for decoding to bytes and converting them in
// a second pass.
//
// One wave per row, rows dealt to waves grid-stride.  A lane chunk of 16
// characters decodes to 12 bytes, exactly three floats, so lane chunk k of a
// row yields floats 3k..3k+2: dec_chunk, then the rounding below; the even
// lane of each pair takes its neighbour's three values and stores the pair's
// 12 bytes with one store.  A lane keeps two passes of U chunks in flight
// (the next pass loaded before this one is decoded).  Validation is the decoder's own (the OR of map values
// tested once per row with a wave ballot, a rescan for the first invalid
// offset); the row's last quanta are decoded on registers by lanes 0..3.
#include "b64_launch.h"

namespace b64hip {
namespace {

// float32 bits -> bfloat16 bits, round to nearest with ties to even; every
// NaN becomes the quiet NaN 0x7FC0.
__device__ __forceinline__ uint32_t bf16_rne(uint32_t u)
{
    const uint32_t r = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    return (u & 0x7FFFFFFFu) > 0x7F800000u ? 0x7FC0u : r;
}

__device__ __forceinline__ int64_t wave_min(int64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int64_t o = __shfl_xor(v, d, 64);
        v = o < v ? o : v;
    }
    return v;
}

// Three bytes of a quantum value as b0 | b1<<8 | b2<<16 in output order.
__device__ __forceinline__ uint32_t quantum_bytes(uint32_t v)
{
    return __builtin_amdgcn_perm(0u, v, 0x0C000102u);
}

// Row b: characters src[in_off[b] .. in_off[b+1]), output dst[b*dim .. +dim).
// status[b] = -1 (good), the first invalid offset, or -2 (valid base64 whose
// decoded length is not 4*dim).  Chunks whose floats lie past dim are not
// stored, so a row of the wrong length never writes outside its own row.
// The body is every quantum but the last; lane chunks cover its first
// 4*nch quanta, lanes 1..3 take the (at most three) body quanta left, lane 0
// the final quantum, and lane 0 assembles and stores the floats they hold.
// Everything runs on registers; the next row's offsets are loaded while this
// row is decoded.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_decode_f32_bf16(
    const uint8_t *__restrict__ src, const int64_t *__restrict__ in_off, int64_t nrows, int64_t dim,
    uint16_t *__restrict__ dst, int64_t *__restrict__ status, DecMap map, uint32_t flags)
{
    __shared__ uint32_t s_map[64];
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;
    const bool nopad = (flags & kFlagNoPad) != 0;
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * kWaves;
    const int64_t w = logical_block() * kWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));

    int64_t s = 0, e = 0;
    if (w < nrows) {
        s = in_off[w];
        e = in_off[w + 1];
    }
    for (int64_t b = w; b < nrows; b += W) {
        const int64_t len = e - s;
        const uint8_t *row = src + s;
        uint16_t *out = dst + b * dim;
        if (b + W < nrows) {                                   // next row's offsets, early
            s = in_off[b + W];
            e = in_off[b + W + 1];
        }
        const int64_t nbq = len >= 1 ? (len - 1) >> 2 : 0;   // body quanta
        const int64_t nch = nbq >> 2;                         // lane chunks
        const int nl = (int)(nbq - 4 * nch);                  // body quanta left, 0..3
        const int r = (int)(len - 4 * nbq);                   // final quantum, 0..4
        // the leftover and final quanta, loaded with the chunks
        uint32_t tq = 0;
        if (lane >= 1 && lane <= nl) {
            tq = *(const u32a1 *)(row + 4 * (4 * nch + lane - 1));
        } else if (lane == 0 && r > 0) {
            if (len >= 4) {
                tq = *(const u32a1 *)(row + len - 4) >> (8 * (4 - r));
            } else {
                for (int i = 0; i < r; ++i) tq |= (uint32_t)row[i] << (8 * i);
            }
        }
        uint32_t err = 0;
        // U lane chunks per pass (chunks k0 + 64j), two passes in flight: the
        // loads of the next pass are issued before this one is decoded
        auto load = [&](u32x4 (&in)[U], int64_t k0) {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t k = k0 + 64 * j;
                in[j] = load16<NT>(row + 16 * (k < nch ? k : nch - 1));
            }
        };
        auto work = [&](const u32x4 (&in)[U], int64_t k0) {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t k = k0 + 64 * j;
                const u32x3 f = dec_chunk(in[j], m, err);
                const uint32_t h0 = bf16_rne(f.x), h1 = bf16_rne(f.y), h2 = bf16_rne(f.z);
                // lanes 2i and 2i+1 hold chunks k and k+1: the even lane takes its
                // neighbour's three values (DPP quad_perm [1,0,3,2]) and stores the
                // pair's 12 bytes at once.  (k has the parity of the lane; an odd
                // lane's chunk is valid exactly when its even neighbour's pair is,
                // so odd lanes never store on their own.)
                const uint32_t n01 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(h0 | (h1 << 16)), 0xB1, 0xF, 0xF, false);
                const uint32_t n2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)h2, 0xB1, 0xF, 0xF, false);
                if ((lane & 1) == 0) {
                    if (k + 1 < nch && 3 * k + 6 <= dim) {
                        u32x3 o;
                        o.x = h0 | (h1 << 16);
                        o.y = h2 | (n01 << 16);
                        o.z = (n01 >> 16) | (n2 << 16);
                        store12<false>((uint8_t *)(out + 3 * k), o);
                    } else if (k < nch && 3 * k + 3 <= dim) {
                        uint16_t *o = out + 3 * k;
                        o[0] = (uint16_t)h0;
                        o[1] = (uint16_t)h1;
                        o[2] = (uint16_t)h2;
                    }
                }
            }
        };
        {
            u32x4 A[U], B[U];
            int64_t k0 = lane;
            if (k0 < nch) load(A, k0);
            while (k0 < nch) {
                const int64_t k1 = k0 + 64 * U;
                if (k1 < nch) load(B, k1);
                work(A, k0);
                if (k1 >= nch) break;
                const int64_t k2 = k1 + 64 * U;
                if (k2 < nch) load(A, k2);
                work(B, k1);
                k0 = k2;
            }
        }
        int64_t bad = kNoError;
        if (__ballot(err & 0x80)) {
            if (err & 0x80) {
                for (int64_t k = lane; k < nch; k += 64) {
                    const int64_t off = dec_check_inner(row + 16 * k, 16, m, nopad);
                    if (off >= 0) {
                        bad = 16 * k + off;
                        break;
                    }
                }
            }
        }
        // leftover body quanta (lanes 1..nl) and the final quantum (lane 0)
        uint32_t g = 0;                                       // output bytes of the lane's quantum
        int nd = 0;
        if (lane >= 1 && lane <= nl) {
            uint32_t qerr = 0;
            g = quantum_bytes(dec_quantum(tq, m, qerr));
            if (qerr & 0x80) {
                const int64_t qi = 4 * nch + lane - 1;
                const int64_t off = dec_check_inner(row + 4 * qi, 4, m, nopad);
                if (off >= 0) bad = bad < 4 * qi + off ? bad : 4 * qi + off;
            }
        } else if (lane == 0 && r > 0) {
            uint32_t v = 0;
            const int off = final_quantum(tq, r, m, nopad, &nd, &v);
            if (off >= 0) bad = bad < 4 * nbq + off ? bad : 4 * nbq + off;
            else g = quantum_bytes(v);
        }
        bad = wave_min(bad);
        const uint32_t g1 = (uint32_t)__shfl(g, 1, 64), g2 = (uint32_t)__shfl(g, 2, 64),
                       g3 = (uint32_t)__shfl(g, 3, 64);
        if (lane == 0) {
            const int64_t dlen = 3 * nbq + (nd > 0 ? nd - 1 : 0);
            const bool good = bad == kNoError && dlen == 4 * dim;
            if (good && dim > 3 * nch) {
                // the tail bytes: nl groups of 3, then the final quantum's nd-1
                uint64_t lo = 0, hi = 0;
                const uint32_t grp[4] = {g1, g2, g3, 0u};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t x = i < nl ? grp[i] : (i == nl ? g : 0u);
                    const int sh = 24 * i;                     // bit position of the group
                    if (i <= nl) {
                        if (sh < 64) lo |= (uint64_t)x << sh;
                        if (sh + 24 > 64) hi |= sh >= 64 ? (uint64_t)x << (sh - 64) : (uint64_t)x >> (64 - sh);
                    }
                }
                const uint32_t fl[3] = {(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi};
#pragma unroll
                for (int t = 0; t < 3; ++t)
                    if (3 * nch + t < dim) out[3 * nch + t] = (uint16_t)bf16_rne(fl[t]);
            }
            status[b] = bad != kNoError ? bad : (dlen == 4 * dim ? -1 : -2);
        }
    }
}

}  // namespace

hipError_t launch_decode_f32_bf16(const uint8_t *src, const int64_t *in_off, int64_t nrows,
                                  int64_t dim, uint16_t *dst, int64_t *status, const DecMap &map,
                                  uint32_t flags, Shape sh, int cus, hipStream_t stream)
{
    int64_t grid = (int64_t)cus * sh.bpc;
    const int64_t need = (nrows + kWaves - 1) / kWaves;
    if (grid > need) grid = need;
    if (grid >= kXcds) grid -= grid % kXcds;
    if (grid < 1) grid = 1;
    B64_DISPATCH(k_decode_f32_bf16, sh, grid, stream, src, in_off, nrows, dim, dst, status, map, flags);
    return hipGetLastError();
}

}  // namespace b64hip
