// Time-scrunching corner turn: the input's s-sample sums written
// channel-major as byte or 16-bit samples for the tiled and tree kernels.
#include "dedisp_device.h"

namespace dedisp {

namespace {

// Time-scrunching corner turn (Section 2.1): scratch sample t' of a live
// channel is the sum of input samples s*t' .. s*t'+s-1 (s = b.scrunch),
// written channel-major as one byte (OB = 1) or one 16-bit word (OB = 2)
// per scrunched sample.  A workgroup covers SC channels (32 input words of a
// row) and ST scrunched samples; lanes 0..31 of a wave read consecutive
// words of one row.  Requires row_bytes % 4 == 0, 4-byte aligned rows and
// 3*s (2-bit) or 255*s (8-bit) below the format's value bound.
template <int NBITS, int OB>
__global__ __launch_bounds__(256) void k_scrunch(BeamDesc b)
{
    constexpr int SC = NBITS == 2 ? 512 : 128;     // channels per workgroup
    constexpr int ST = NBITS == 2 ? 32 : 64;       // scrunched samples per workgroup
    constexpr int RB = ST * OB;                    // tile bytes per channel row
    static_assert(NBITS == 2 || OB == 2, "8-bit sums need 16 bits");
    const int s = b.scrunch;
    const long long ns = b.nsamps / s;             // whole scrunched samples
    // consecutive time tiles write consecutive pieces of the same scratch
    // lines: one XCD takes a contiguous range of them (its L2 merges the pieces)
    const long long tp0 = (long long)xcd_remap((int)blockIdx.x, (int)gridDim.x) * ST;
    const int c0 = blockIdx.y * SC;
    const int w = threadIdx.x & 31;                // input word within the row segment
    const int cw = c0 + w * (32 / NBITS);          // first channel of that word
    constexpr int PPR = RB / 16;                   // 16-byte pieces per channel row
    const long long byte0 = tp0 * OB;
    if constexpr (NBITS == 2) {
        // Lane (w, qg) sums the 16 channels of input word w for the four
        // consecutive scrunched samples 4qg .. 4qg+3, packs them per channel
        // into one (bytes) or two (16 bits) dwords, and writes the dword
        // tile channel-major.  Rows are NCOL + 1 dwords and dword column x of
        // row ch sits at x ^ (ch/16 mod NCOL): the 32 lanes writing one
        // channel offset each (rows 16 apart) then spread over the LDS banks.
        constexpr int NCOL = RB / 4;               // dwords per channel row: 8 or 16
        constexpr int LPW = NCOL + 1;
        __shared__ uint32_t tile[SC * LPW];
        const int qg = threadIdx.x >> 5;           // 0..7
        uint32_t W[16 * OB];
#pragma unroll
        for (int e = 0; e < 16 * OB; ++e) W[e] = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long long tp = tp0 + 4 * qg + i;
            uint32_t g[4] = {0u, 0u, 0u, 0u};      // byte k of g[j]: channel 4k + j of the word
            if (tp < ns && cw < b.nchans)
                // a lane's s input rows are read four at a time (independent
                // loads in flight together; s is a power of two >= 2)
                for (int r = 0; r < s; r += 4) {
                    uint32_t v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        v[u] = r + u < s ? *reinterpret_cast<const uint32_t*>(row_ptr(b, tp * s + r + u) + cw / 4) : 0u;
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) g[jj] += (v[u] >> (2 * jj)) & 0x03030303u;
                }
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const uint32_t val = (g[jj] >> (8 * k)) & 0xFFu;
                    if constexpr (OB == 1) W[4 * k + jj] |= val << (8 * i);
                    else W[2 * (4 * k + jj) + (i >> 1)] |= val << (16 * (i & 1));
                }
        }
        const int sw = w & (NCOL - 1);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            uint32_t* row = tile + (16 * w + c) * LPW;
            if constexpr (OB == 1) {
                row[qg ^ sw] = W[c];
            } else {
                row[(2 * qg) ^ sw] = W[2 * c];
                row[(2 * qg + 1) ^ sw] = W[2 * c + 1];
            }
        }
        __syncthreads();
        // 16-byte pieces to each live channel's scratch row; samples past
        // the last whole scrunched sample hold zeros
        // scratch rows first: a load inside the store loop would make every
        // store wait for the one before it
        constexpr int NIT = SC * PPR / 256;
        static_assert(SC * PPR % 256 == 0, "whole items per thread");
        int rows[NIT];
#pragma unroll
        for (int n = 0; n < NIT; ++n) {
            const int c = c0 + (threadIdx.x + 256 * n) / PPR;
            rows[n] = c < b.nchans ? (b.chanmap ? b.chanmap[c] : c) : -1;
        }
#pragma unroll
        for (int n = 0; n < NIT; ++n) {
            const int it = threadIdx.x + 256 * n;
            const int c = it / PPR;
            const int p = it % PPR;
            const int row = rows[n];
            if (row < 0) continue;
            const uint32_t* src = tile + c * LPW;
            const int csw = (c >> 4) & (NCOL - 1);
            const u32x4 val = {src[(4 * p) ^ csw], src[(4 * p + 1) ^ csw], src[(4 * p + 2) ^ csw],
                               src[(4 * p + 3) ^ csw]};
            *reinterpret_cast<u32x4*>(b.xc + (long long)row * b.pitch + byte0 + 16 * p) = val;
        }
    } else {
        constexpr int LP = RB + 16;                // LDS row pitch in bytes
        __shared__ __attribute__((aligned(16))) uint8_t tile[SC * LP];
        for (int q = threadIdx.x >> 5; q < ST; q += 8) {
            const long long tp = tp0 + q;
            uint32_t lo = 0u, hi = 0u;             // 16-bit lanes: channels (0, 2) and (1, 3) of the word
            if (tp < ns && cw < b.nchans)
                for (int r = 0; r < s; r += 4) {
                    uint32_t v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        v[u] = r + u < s ? *reinterpret_cast<const uint32_t*>(row_ptr(b, tp * s + r + u) + cw) : 0u;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        lo += v[u] & 0x00FF00FFu;
                        hi += (v[u] >> 8) & 0x00FF00FFu;
                    }
                }
            uint16_t* t16 = reinterpret_cast<uint16_t*>(tile);
            t16[(4 * w + 0) * (LP / 2) + q] = (uint16_t)(lo & 0xFFFFu);
            t16[(4 * w + 1) * (LP / 2) + q] = (uint16_t)(hi & 0xFFFFu);
            t16[(4 * w + 2) * (LP / 2) + q] = (uint16_t)(lo >> 16);
            t16[(4 * w + 3) * (LP / 2) + q] = (uint16_t)(hi >> 16);
        }
        __syncthreads();
        constexpr int NIT = SC * PPR / 256;
        static_assert(SC * PPR % 256 == 0, "whole items per thread");
        int rows[NIT];
#pragma unroll
        for (int n = 0; n < NIT; ++n) {
            const int c = c0 + (threadIdx.x + 256 * n) / PPR;
            rows[n] = c < b.nchans ? (b.chanmap ? b.chanmap[c] : c) : -1;
        }
#pragma unroll
        for (int n = 0; n < NIT; ++n) {
            const int it = threadIdx.x + 256 * n;
            const int c = it / PPR;
            const int p = it % PPR;
            if (rows[n] < 0) continue;
            *reinterpret_cast<u32x4*>(b.xc + (long long)rows[n] * b.pitch + byte0 + 16 * p) =
                *reinterpret_cast<const u32x4*>(tile + (size_t)c * LP + 16 * p);
        }
    }
    if (b.pad_row >= 0 && blockIdx.y == 0 && threadIdx.x < PPR * (b.nact - b.pad_row)) {
        const int r = b.pad_row + threadIdx.x / PPR;
        const int p = threadIdx.x % PPR;
        *reinterpret_cast<u32x4*>(b.xc + (long long)r * b.pitch + byte0 + 16 * p) =
            u32x4{0u, 0u, 0u, 0u};
    }
}

}  // namespace

hipError_t launch_scrunch(const BeamDesc& d, int nbits, int fmt, hipStream_t st)
{
    BeamDesc arg = d;
    void* args[] = {&arg};
    const long long sc = nbits == 2 ? 512 : 128, stl = nbits == 2 ? 32 : 64;
    const long long ns = d.nsamps / d.scrunch;
    const long long gx = (ns + stl - 1) / stl;
    const long long gy = (d.nchans + sc - 1) / sc;
    if (gx <= 0 || gx > 0x7fffffffLL || gy > 65535) return hipErrorInvalidValue;
    const void* fn = nullptr;
    // 2-bit sums as bytes: byte-lane (s <= 8) or 8-bit-code (s <= 85) scratch
    if (nbits == 2 && (fmt == kFmtByteS || fmt == kFmtByte) && 3 * d.scrunch <= 255)
        fn = reinterpret_cast<const void*>(&k_scrunch<2, 1>);
    else if (nbits == 2 && fmt == kFmtHalf) fn = reinterpret_cast<const void*>(&k_scrunch<2, 2>);
    else if (nbits == 8 && fmt == kFmtHalf) fn = reinterpret_cast<const void*>(&k_scrunch<8, 2>);
    if (!fn) return hipErrorInvalidValue;
    return hipLaunchKernel(fn, dim3((unsigned)gx, (unsigned)gy), dim3(256), args, 0, st);
}

}  // namespace dedisp
