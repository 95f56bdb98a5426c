// gfx950 kernels for the direct incoherent dedispersion transform
// (Barsdell et al. 2012, Section 2.1, eq. direct):
//
//     out[d][t] = sum_c in[t + delay[d][c]][c]
//
// LDS-tiled kernel.  A workgroup owns one time tile of 256*M output samples
// and a block of DB = NW*DPW neighbouring trial DMs.  For each chunk of CC
// channels it stages, per channel, the window of input samples that the
// whole DM block needs ([tile start + smallest delay, ... + largest delay +
// tile length)) into LDS, decoded to one byte per sample and laid out
// channel-major with time contiguous.  That window is then read by all DB
// DMs of the block: the temporal reuse the paper discusses in Section 2.2,
// which on gfx950 pays because LDS is large and the kernel is bound by
// integer adds, not by HBM.
//
// Each lane owns 4*M consecutive output samples of DPW DMs.  For one
// (DM, channel) pair the delay is wave-uniform, so a lane reads M+1
// consecutive 32-bit LDS words starting at its word offset plus delay/4 and
// realigns them by delay%4 bytes with one v_alignbyte (2-bit data) or spreads
// them into 16-bit lanes with v_perm (8-bit data).  Lanes are M words apart
// with M odd, so the 64 lanes of a wave hit distinct LDS banks.
//
// The sums use bit-level parallelism (Section 2.3): 2-bit codes are added
// four at a time in the 8-bit lanes of a 32-bit register, which is exact for
// up to (2^8-1)/(2^2-1) = 85 channels, then flushed into 32-bit
// accumulators; 8-bit codes are added two at a time in 16-bit lanes, exact
// for up to 257 channels.  Every result is an exact integer sum.
//
// Untiled kernel: one thread per 4 outputs of one DM, reading the input
// straight from global memory.  Used when a DM block's delay spread is too
// large for LDS (e.g. a DM list with huge gaps).
//
// Persistent kernel: a grid sized to the machine pulls (beam, tile, DM block)
// work items from a global counter; beams may differ in channel count, bit
// depth, length, DM list and tile shape.  Used for batches and for several
// stream pushes in one launch.
#include "dedisp_internal.h"

namespace dedisp {

namespace {

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Address of input row r in the two-segment virtual input.
__device__ __forceinline__ const uint8_t* row_ptr(const BeamDesc& b, long long r)
{
    return r < b.n0 ? b.in0 + r * (long long)b.row_bytes
                    : b.in1 + (r - b.n0) * (long long)b.row_bytes;
}

// Map the hardware workgroup index to a logical one so that the workgroups
// dispatched to one XCD (round-robin over 8 XCDs) get a contiguous range of
// logical indices, i.e. all DM blocks of the same few time tiles: they read
// the same input rows, which then stay in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int i, int n)
{
    constexpr int kXcds = 8;
    const int per = n / kXcds, rem = n % kXcds;
    const int x = i % kXcds, k = i / kXcds;
    return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Input staging.  Chunk k of a tile covers channel groups [G*k, G*k+G) (4
// channels per group).  For group g the LDS holds rw words per channel; word
// p = samples (t0 + base[g] + 4p) .. +3 of that channel, one byte each.
// Thread x stages words p = x + i*NT (i < PI) of every group of the chunk.
// Loading (global -> registers) and storing (registers -> LDS) are separate
// so the loads of chunk k+1 can be in flight while chunk k is summed.
// Rows past the end of the input are clamped to the last row: only outputs
// t >= nout, which are never stored, read them.
template <int NBITS, int G, int PI>
struct Staging {
    // 2-bit: one 32-bit word per item (byte k = row r+k, 4 channels per byte).
    // 8-bit: four words per item (word k = row r+k, 4 channels per word).
    static constexpr int W = NBITS == 2 ? 1 : 4;
    uint32_t v[PI][G][W];

    // FAST: the tile's whole window lies in one input segment and before the
    // last row, so row r is at seg + (r - seg_row0) * row_bytes.
    template <int NT, bool FAST>
    __device__ __forceinline__ void load(const BeamDesc& b, const int32_t* basep, long long t0,
                                         int col0, int ngroups, int pi, const uint8_t* seg,
                                         long long seg_row0)
    {
        const int rw = b.rw;
        const long long last = b.nsamps - 1;
        const long long rb = b.row_bytes;
#pragma unroll
        for (int i = 0; i < PI; ++i) {
            const int p = threadIdx.x + i * NT;
            const long long p4 = 4LL * p;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                // words p >= rw are outside the window: never stored, never read
                if (i >= pi || p >= rw || g >= ngroups) continue;
                const long long r = t0 + (long long)basep[g] + p4;
                if constexpr (FAST) {
                    const uint8_t* q = seg + (r - seg_row0) * rb + (NBITS == 2 ? col0 + g : 4 * (col0 + g));
                    if constexpr (NBITS == 2) {
                        uint32_t word = 0;
#pragma unroll
                        for (int k = 0; k < 4; ++k) word |= (uint32_t)q[k * rb] << (8 * k);
                        v[i][g][0] = word;
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            v[i][g][k] = *reinterpret_cast<const uint32_t*>(q + k * rb);
                    }
                } else if constexpr (NBITS == 2) {
                    uint32_t word = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint8_t* row = row_ptr(b, r + k < last ? r + k : last);
                        word |= (uint32_t)row[col0 + g] << (8 * k);
                    }
                    v[i][g][0] = word;
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint8_t* row = row_ptr(b, r + k < last ? r + k : last);
                        v[i][g][k] = *reinterpret_cast<const uint32_t*>(row + 4 * (col0 + g));
                    }
                }
            }
        }
    }

    template <int NT>
    __device__ __forceinline__ void load_any(bool fast, const BeamDesc& b, const int32_t* basep,
                                             long long t0, int col0, int ngroups, int pi,
                                             const uint8_t* seg, long long seg_row0)
    {
        if (fast) load<NT, true>(b, basep, t0, col0, ngroups, pi, seg, seg_row0);
        else load<NT, false>(b, basep, t0, col0, ngroups, pi, seg, seg_row0);
    }

    template <int NT>
    __device__ __forceinline__ void store(uint32_t* lds, int rw, int ngroups, int pi) const
    {
#pragma unroll
        for (int i = 0; i < PI; ++i) {
            const int p = threadIdx.x + i * NT;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (i >= pi || p >= rw || g >= ngroups) continue;
                uint32_t* dst = lds + (size_t)(g * 4) * rw + p;
                if constexpr (NBITS == 2) {
                    // channel q of the group is bits [2q, 2q+1] of every byte
                    const uint32_t word = v[i][g][0];
#pragma unroll
                    for (int q = 0; q < 4; ++q) dst[(size_t)q * rw] = (word >> (2 * q)) & 0x03030303u;
                } else {
                    // 4x4 byte transpose: channel q gets byte q of rows r..r+3
                    const uint32_t a01 = __builtin_amdgcn_perm(v[i][g][1], v[i][g][0], 0x05010400u);
                    const uint32_t a23 = __builtin_amdgcn_perm(v[i][g][3], v[i][g][2], 0x05010400u);
                    const uint32_t b01 = __builtin_amdgcn_perm(v[i][g][1], v[i][g][0], 0x07030602u);
                    const uint32_t b23 = __builtin_amdgcn_perm(v[i][g][3], v[i][g][2], 0x07030602u);
                    dst[0] = __builtin_amdgcn_perm(a23, a01, 0x05040100u);
                    dst[(size_t)rw] = __builtin_amdgcn_perm(a23, a01, 0x07060302u);
                    dst[(size_t)2 * rw] = __builtin_amdgcn_perm(b23, b01, 0x05040100u);
                    dst[(size_t)3 * rw] = __builtin_amdgcn_perm(b23, b01, 0x07060302u);
                }
            }
        }
    }
};

// One (time tile, DM block) work item.
template <int NBITS, int NW, int DPW, int M, int CC, int PI>
__device__ __forceinline__ void tile_body(const BeamDesc& b, int tile, int block, uint32_t* lds)
{
    static_assert(M % 2 == 1, "lanes must be an odd number of LDS words apart");
    static_assert(CC % 4 == 0, "chunks are whole 4-channel groups");
    static_assert(NBITS == 8 || CC <= 84, "2-bit lanes hold at most 85 codes");
    constexpr int NT = NW * 64;
    constexpr int T = 256 * M;
    constexpr int DB = NW * DPW;
    constexpr int G = CC / 4;
    constexpr int NSW = NBITS == 2 ? 1 : 2;
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    tile = wave_uniform(tile);
    block = wave_uniform(block);
    const long long t0 = (long long)tile * T;
    const int nchans = b.nchans;
    const int rw = b.rw;
    const int pi = (rw + NT - 1) / NT;
    // Rows this tile can touch: [t0, t0 + 4*rw + max_delay).
    const long long hi_row = t0 + 4LL * rw + (b.nsamps - b.nout);
    const bool fast = hi_row <= b.nsamps && (hi_row <= b.n0 || t0 >= b.n0);
    const uint8_t* seg = t0 >= b.n0 ? b.in1 : b.in0;
    const long long seg_row0 = t0 >= b.n0 ? b.n0 : 0;
    const int32_t* basep = b.base + (size_t)block * (size_t)(nchans >> 2);
    // rel row of DM k of this wave: rel[(block*DB + wave*DPW + k)*nchans + c]
    const int rel_row0 = wave_uniform((block * DB + wave * DPW) * nchans);

    uint32_t acc[DPW][M][4];
    uint32_t sw[DPW][M][NSW];
#pragma unroll
    for (int k = 0; k < DPW; ++k)
#pragma unroll
        for (int j = 0; j < M; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[k][j][e] = 0u;
#pragma unroll
            for (int h = 0; h < NSW; ++h) sw[k][j][h] = 0u;
        }

    Staging<NBITS, G, PI> stg;
    stg.template load_any<NT>(fast, b, basep, t0, 0, min(G, nchans >> 2), pi, seg, seg_row0);

    int since_flush = 0;
    for (int c0 = 0; c0 < nchans; c0 += CC) {
        const int ncur = min(CC, nchans - c0);
        __syncthreads();
        stg.template store<NT>(lds, rw, ncur >> 2, pi);
        __syncthreads();
        if (c0 + CC < nchans)
            stg.template load_any<NT>(fast, b, basep + ((c0 + CC) >> 2), t0, (c0 + CC) >> 2,
                                      min(G, (nchans - c0 - CC) >> 2), pi, seg, seg_row0);

        const uint32_t* lrow = lds + lane * M;
        // delays of 4 channels x DPW DMs, fetched one step ahead
        int4 rnext[DPW];
#pragma unroll
        for (int k = 0; k < DPW; ++k)
            rnext[k] = *reinterpret_cast<const int4*>(b.rel + rel_row0 + k * nchans + c0);
        for (int c = 0; c < ncur; c += 4) {
            int4 rcur[DPW];
#pragma unroll
            for (int k = 0; k < DPW; ++k) rcur[k] = rnext[k];
            if (c + 4 < ncur) {
#pragma unroll
                for (int k = 0; k < DPW; ++k)
                    rnext[k] = *reinterpret_cast<const int4*>(b.rel + rel_row0 + k * nchans + c0 + c + 4);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t* row = lrow + (size_t)(c + q) * rw;
#pragma unroll
                for (int k = 0; k < DPW; ++k) {
                    const int r = q == 0 ? rcur[k].x : q == 1 ? rcur[k].y : q == 2 ? rcur[k].z : rcur[k].w;
                    const uint32_t* src = row + (r >> 2);
                    const uint32_t s = (uint32_t)(r & 3);
                    uint32_t w[M + 1];
#pragma unroll
                    for (int j = 0; j <= M; ++j) w[j] = src[j];
                    if constexpr (NBITS == 2) {
#pragma unroll
                        for (int j = 0; j < M; ++j)
                            sw[k][j][0] += __builtin_amdgcn_alignbyte(w[j + 1], w[j], s);
                    } else {
                        // bytes s, s+1 -> 16-bit lanes of `lo`; s+2, s+3 -> `hi`
                        const uint32_t sel_lo = s | 0x0C00u | ((s + 1u) << 16) | 0x0C000000u;
                        const uint32_t sel_hi = sel_lo + 0x00020002u;
#pragma unroll
                        for (int j = 0; j < M; ++j) {
                            sw[k][j][0] += __builtin_amdgcn_perm(w[j + 1], w[j], sel_lo);
                            sw[k][j][1] += __builtin_amdgcn_perm(w[j + 1], w[j], sel_hi);
                        }
                    }
                }
            }
        }

        if (++since_flush == b.flush_every || c0 + CC >= nchans) {
            since_flush = 0;
#pragma unroll
            for (int k = 0; k < DPW; ++k)
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    if constexpr (NBITS == 2) {
                        const uint32_t v = sw[k][j][0];
                        acc[k][j][0] += v & 0xFFu;
                        acc[k][j][1] += (v >> 8) & 0xFFu;
                        acc[k][j][2] += (v >> 16) & 0xFFu;
                        acc[k][j][3] += v >> 24;
                    } else {
                        const uint32_t lo = sw[k][j][0], hi = sw[k][j][1];
                        acc[k][j][0] += lo & 0xFFFFu;
                        acc[k][j][1] += lo >> 16;
                        acc[k][j][2] += hi & 0xFFFFu;
                        acc[k][j][3] += hi >> 16;
                    }
#pragma unroll
                    for (int h = 0; h < NSW; ++h) sw[k][j][h] = 0u;
                }
        }
    }

    const bool vec = ((b.out_stride & 3) == 0) &&
                     ((reinterpret_cast<uintptr_t>(b.out) & 15) == 0);
#pragma unroll
    for (int k = 0; k < DPW; ++k) {
        const int d = block * DB + wave * DPW + k;
        if (d >= b.ndm) continue;
        uint32_t* orow = b.out + (size_t)d * (size_t)b.out_stride;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const long long t = t0 + 4LL * (lane * M + j);
            if (vec && t + 3 < b.nout) {
                *reinterpret_cast<uint4*>(orow + t) =
                    make_uint4(acc[k][j][0], acc[k][j][1], acc[k][j][2], acc[k][j][3]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (t + e < b.nout) orow[t + e] = acc[k][j][e];
            }
        }
    }
}

template <int NBITS, int NW, int DPW, int M, int CC, int PI>
__global__ __launch_bounds__(NW * 64) void k_tiled(BeamDesc b)
{
    extern __shared__ uint32_t lds_dyn[];
    const int n = b.ntiles * b.nblocks;
    const int logical = xcd_remap((int)blockIdx.x, n);
    tile_body<NBITS, NW, DPW, M, CC, PI>(b, logical / b.nblocks, logical % b.nblocks, lds_dyn);
}

template <int NBITS>
__device__ __forceinline__ uint32_t sample_at(const BeamDesc& b, long long r, int c)
{
    const uint8_t* row = row_ptr(b, r);
    if constexpr (NBITS == 8) return row[c];
    else return (row[c >> 2] >> (2 * (c & 3))) & 3u;
}

template <int NBITS>
__global__ __launch_bounds__(256) void k_untiled(BeamDesc b)
{
    const long long t = ((long long)blockIdx.x * 256 + threadIdx.x) * 4;
    if (t >= b.nout) return;
    for (int d = blockIdx.y; d < b.ndm; d += gridDim.y) {
        const int32_t* dl = b.table + (size_t)d * b.nchans;
        uint32_t a[4] = {0u, 0u, 0u, 0u};
        for (int c = 0; c < b.nchans; ++c) {
            const int off = dl[c];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < b.nout) a[e] += sample_at<NBITS>(b, t + e + off, c);
        }
        uint32_t* orow = b.out + (size_t)d * (size_t)b.out_stride;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (t + e < b.nout) orow[t + e] = a[e];
    }
}

// ---------------------------------------------------------------- shapes

// (nbits, waves, DMs per wave, words per lane, channels per chunk, staging
// slabs).  A slab is one staged word per thread per channel group, so a shape
// fits a DM block whose window is at most slabs*waves*64 words long.
#define DEDISP_SHAPES(X)        \
    X(2, 4, 4, 5, 32, 2)        \
    X(2, 4, 4, 5, 64, 2)        \
    X(2, 4, 8, 3, 32, 2)        \
    X(2, 4, 8, 5, 32, 2)        \
    X(2, 4, 4, 3, 32, 2)        \
    X(2, 4, 2, 7, 32, 3)        \
    X(2, 8, 4, 5, 64, 1)        \
    X(2, 8, 2, 5, 64, 1)        \
    X(8, 4, 4, 5, 16, 2)        \
    X(8, 4, 4, 5, 32, 2)        \
    X(8, 4, 8, 3, 16, 2)        \
    X(8, 4, 4, 3, 32, 2)        \
    X(8, 8, 4, 3, 32, 1)        \
    X(8, 8, 4, 5, 16, 1)

struct ShapeEntry {
    Shape s;
    const void* fn;
};

#define DEDISP_ENTRY(NB, NW, DPW, M, CC, PI) \
    {Shape{0, NB, NW, DPW, M, CC, PI}, reinterpret_cast<const void*>(&k_tiled<NB, NW, DPW, M, CC, PI>)},

const ShapeEntry kShapes[] = {
    DEDISP_SHAPES(DEDISP_ENTRY)
    {Shape{1, 2, 4, 1, 1, 0, 0}, reinterpret_cast<const void*>(&k_untiled<2>)},
    {Shape{1, 8, 4, 1, 1, 0, 0}, reinterpret_cast<const void*>(&k_untiled<8>)},
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// Persistent kernel: the shapes with kPersistentWaves waves.
template <int NBITS, int NW, int DPW, int M, int CC, int PI>
__device__ __forceinline__ bool run_if(int shape_id, int want, const BeamDesc& b, int tile,
                                       int block, uint32_t* lds)
{
    if constexpr (NW == kPersistentWaves) {
        if (shape_id == want) {
            tile_body<NBITS, NW, DPW, M, CC, PI>(b, tile, block, lds);
            return true;
        }
    }
    return false;
}

__global__ __launch_bounds__(kPersistentWaves * 64) void k_persistent(
    const BeamDesc* __restrict__ descs, int nbeams, long long total, unsigned int* counters)
{
    extern __shared__ uint32_t lds_dyn[];
    __shared__ unsigned int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(&counters[0], 1u);
        __syncthreads();
        const long long item = (long long)wave_uniform((int)s_item);
        if (item >= total) break;
        int bi = 0;
        while (bi + 1 < nbeams && descs[bi + 1].work_begin <= item) ++bi;
        const BeamDesc& b = descs[bi];
        const long long local = item - b.work_begin;
        const int tile = (int)(local / b.nblocks);
        const int block = (int)(local % b.nblocks);
        int id = 0;
        bool done = false;
#define DEDISP_RUN(NB, NW, DPW, M, CC, PI) \
    if (!done) done = run_if<NB, NW, DPW, M, CC, PI>(b.shape, id, b, tile, block, lds_dyn); \
    ++id;
        DEDISP_SHAPES(DEDISP_RUN)
#undef DEDISP_RUN
        (void)done;
    }
    // The last workgroup to finish re-arms the counters for the next launch.
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int finished = atomicAdd(&counters[1], 1u);
        if (finished == gridDim.x - 1) {
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
            __threadfence();
        }
    }
}

bool g_attr_done[kNumShapes + 1] = {};

hipError_t ensure_lds_attr(int idx, const void* fn)
{
    if (g_attr_done[idx]) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kMaxLdsBytes);
    if (e == hipSuccess) g_attr_done[idx] = true;
    return e;
}

}  // namespace

int shape_count() { return kNumShapes; }
const Shape& shape_at(int i) { return kShapes[i].s; }

hipError_t launch_tiled(const BeamDesc& d, const Shape& s, int lds_bytes, hipStream_t st)
{
    int idx = -1;
    for (int i = 0; i < kNumShapes; ++i) {
        const Shape& k = kShapes[i].s;
        if (k.kind == 0 && k.nbits == s.nbits && k.waves == s.waves && k.dpw == s.dpw &&
            k.m == s.m && k.cc == s.cc && k.pi == s.pi) {
            idx = i;
            break;
        }
    }
    if (idx < 0) return hipErrorInvalidValue;
    hipError_t e = ensure_lds_attr(idx, kShapes[idx].fn);
    if (e != hipSuccess) return e;
    const long long n = (long long)d.ntiles * d.nblocks;
    if (n <= 0 || n > 0x7fffffffLL) return hipErrorInvalidValue;
    BeamDesc arg = d;
    void* args[] = {&arg};
    return hipLaunchKernel(kShapes[idx].fn, dim3((unsigned)n), dim3(s.waves * 64), args,
                           (size_t)lds_bytes, st);
}

hipError_t launch_untiled(const BeamDesc& d, int nbits, hipStream_t st)
{
    const long long nthreads = (d.nout + 3) / 4;
    const long long gx = (nthreads + 255) / 256;
    if (gx <= 0 || gx > 0x7fffffffLL) return hipErrorInvalidValue;
    const unsigned gy = (unsigned)(d.ndm < 65535 ? d.ndm : 65535);
    BeamDesc arg = d;
    void* args[] = {&arg};
    const void* fn = nbits == 2 ? reinterpret_cast<const void*>(&k_untiled<2>)
                                : reinterpret_cast<const void*>(&k_untiled<8>);
    return hipLaunchKernel(fn, dim3((unsigned)gx, gy), dim3(256), args, 0, st);
}

int persistent_max_grid(int lds_bytes)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_persistent),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_persistent), kPersistentWaves * 64,
            (size_t)lds_bytes) != hipSuccess)
        return 0;
    if (per_cu < 1) per_cu = 1;
    return ncu * per_cu;
}

hipError_t launch_persistent(const BeamDesc* d_descs, int nbeams, long long total_work,
                             unsigned int* d_counters, int lds_bytes, int grid, hipStream_t st)
{
    if (grid <= 0 || nbeams <= 0 || total_work <= 0 || total_work >= 0x7fffffffLL)
        return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_persistent),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kMaxLdsBytes);
    if (e != hipSuccess) return e;
    const BeamDesc* a0 = d_descs;
    int a1 = nbeams;
    long long a2 = total_work;
    unsigned int* a3 = d_counters;
    void* args[] = {&a0, &a1, &a2, &a3};
    return hipLaunchKernel(reinterpret_cast<const void*>(&k_persistent), dim3(grid),
                           dim3(kPersistentWaves * 64), args, (size_t)lds_bytes, st);
}

}  // namespace dedisp
