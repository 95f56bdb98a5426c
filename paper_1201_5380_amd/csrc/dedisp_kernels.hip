// gfx950 kernels for the direct incoherent dedispersion transform
// (Barsdell et al. 2012, Section 2.1, eq. direct):
//
//     out[d][t] = sum_c in[t + delay[d][c]][c]
//
// Two kernels per beam.
//
// 1. Corner turn + unpack (k_unpack, k_unpack_planes, k_unpack_seg).  Reads
//    the packed time-major input with coalesced loads (two row segments, so
//    a stream's history and a new chunk need not be contiguous) and writes
//    it channel-major, one scratch row per live channel: 2-bit codes as
//    nibbles (two samples per byte, eight per 32-bit word) or as two bit
//    planes (32 consecutive samples per word, or 32 time segments per word
//    in the segmented layout), 8-bit codes as bytes.  This is the "corner
//    turn" the paper times separately (Table 2); it costs a few percent of
//    the main kernel's time and turns every later access into aligned
//    contiguous 16-byte loads.
//
// 2. LDS-tiled shifted sum (k_tiled).  A workgroup owns one time tile of
//    64*M scratch words per lane-row (512*M samples of 2-bit or 256*M of
//    8-bit data) and a block of DB = NW*DPW neighbouring trial DMs.  For
//    each chunk of CC channels it stages, per channel, the window of samples
//    the whole DM block needs -- it starts at t0 + base, base being the
//    block's smallest delay in that channel rounded down to 16 bytes of
//    scratch -- into LDS.  Every DM of the block then reads its shifted slice
//    of that window: the temporal reuse discussed in Section 2.2, which pays
//    on gfx950 because LDS is large and the kernel is bound by integer adds
//    and LDS reads.  The loads of chunk k+1 are issued before chunk k is
//    summed and land in registers, so their latency hides behind the
//    arithmetic.
//
//    Each lane owns M consecutive scratch words (8*M or 4*M output samples)
//    of DPW DMs.  For one (DM, channel) pair the delay is wave-uniform: a
//    lane reads M+1 consecutive words at its own word offset plus the
//    delay's whole words and realigns them by the remainder with v_alignbit
//    (nibble granularity, 2-bit data) or spreads them into 16-bit lanes with
//    v_perm (8-bit data).  Lanes are M words apart with M odd, so the 64
//    lanes of a wave hit distinct LDS banks.  The per-(DM, channel) window
//    offsets arrive through vector loads and v_readlane, never through
//    scalar memory, so waits on LDS are never held up by scalar loads.
//
//    The sums use bit-level parallelism (Section 2.3).  2-bit codes held as
//    bit planes are added 32 samples at a time by bit-sliced full adders
//    (plane_body); on the segmented planes a delay is a whole number of
//    words, so a lane reads M words and realigns nothing.  2-bit codes held
//    as nibbles are added eight at a time in the 4-bit lanes of a register
//    (exact for up to (2^4-1)/(2^2-1) = 5 codes, so flushed every 4
//    channels), then in 8-bit lanes (85 codes) and finally in 16-bit lanes
//    (21845 codes).  8-bit codes are added two at a time in 16-bit lanes
//    (257 codes), then in 32-bit accumulators.
//
// Untiled kernel (k_untiled): one thread per 4 outputs of one DM reading the
// packed input directly.  Used when a DM block's delay spread is too large
// for LDS (e.g. a DM list with huge gaps) or the input is misaligned.
//
// Multi-beam kernel (k_multi): one launch over the (beam,
// time tile, DM block) work items of up to 16 beams that may differ in
// channel count, bit depth, length, DM list and tile shape.
#include "dedisp_device.h"

namespace dedisp {

namespace {

// ------------------------------------------------------------ corner turn

constexpr int kUT = 128;   // time rows per unpack tile
constexpr int kUC = 128;   // channels per unpack tile

// Bytes of channel-major scratch per sample: 2-bit codes are stored two per
// byte (sample 2i in the low nibble of byte i, 2i+1 in the high nibble),
// 8-bit codes one per byte.
template <int NBITS>
struct Store {
    static constexpr int kSamplesPerByte = NBITS == 2 ? 2 : 1;
    static constexpr int kRowBytes = kUT / kSamplesPerByte;      // per channel per unpack tile
    static constexpr int kPitch = kRowBytes + 16;                 // LDS row pitch of the unpack tile
};

// xc[row * pitch + byte] for a 128 x 128 (time x channel) tile, where row is
// the channel's scratch row (killed channels have none).  Requires
// row_bytes % 4 == 0 and 4-byte aligned input rows.
template <int NBITS>
__device__ __forceinline__ void unpack_tile(const BeamDesc& b, long long bx, int by, uint8_t* tile)
{
    using S = Store<NBITS>;
    const long long t0 = bx * kUT;
    const int c0 = by * kUC;
    constexpr int WPR = kUC * NBITS / 32;          // 32-bit words per row segment
    constexpr int CPW = 32 / NBITS;                // channels per word
    // item = (row quad, word): four rows of one word -> CPW channels x 4 times
    for (int it = threadIdx.x; it < (kUT / 4) * WPR; it += 256) {
        const int w = it % WPR;
        const int rq = it / WPR;
        const int cw = c0 + w * CPW;               // first channel of the word
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const long long t = t0 + 4 * rq + k;
            v[k] = (t < b.nsamps && cw < b.nchans)
                       ? *reinterpret_cast<const uint32_t*>(row_ptr(b, t) + (long long)cw * NBITS / 8)
                       : 0u;
        }
        if constexpr (NBITS == 2) {
            uint8_t* dst = tile + (size_t)(w * CPW) * S::kPitch + 2 * rq;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // byte q of each row holds 4 channels -> [t0 t1 t2 t3] bytes
                const uint32_t sel = 0x0C0C0000u | ((uint32_t)(q + 4) << 8) | (uint32_t)q;
                const uint32_t lo = __builtin_amdgcn_perm(v[1], v[0], sel);
                const uint32_t hi = __builtin_amdgcn_perm(v[3], v[2], sel);
                const uint32_t w4 = lo | (hi << 16);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // channel 4q+j: code of time k at bits [8k, 8k+1]; pack to nibbles
                    const uint32_t x = (w4 >> (2 * j)) & 0x03030303u;
                    const uint32_t y = x | (x >> 4);          // byte 0: t0|t1<<4, byte 2: t2|t3<<4
                    *reinterpret_cast<uint16_t*>(dst + (size_t)(4 * q + j) * S::kPitch) =
                        (uint16_t)((y & 0xFFu) | ((y >> 8) & 0xFF00u));
                }
            }
        } else {
            uint8_t* dst = tile + (size_t)(w * CPW) * S::kPitch + 4 * rq;
            const uint32_t a01 = __builtin_amdgcn_perm(v[1], v[0], 0x05010400u);
            const uint32_t a23 = __builtin_amdgcn_perm(v[3], v[2], 0x05010400u);
            const uint32_t b01 = __builtin_amdgcn_perm(v[1], v[0], 0x07030602u);
            const uint32_t b23 = __builtin_amdgcn_perm(v[3], v[2], 0x07030602u);
            *reinterpret_cast<uint32_t*>(dst) = __builtin_amdgcn_perm(a23, a01, 0x05040100u);
            *reinterpret_cast<uint32_t*>(dst + S::kPitch) = __builtin_amdgcn_perm(a23, a01, 0x07060302u);
            *reinterpret_cast<uint32_t*>(dst + 2 * S::kPitch) = __builtin_amdgcn_perm(b23, b01, 0x05040100u);
            *reinterpret_cast<uint32_t*>(dst + 3 * S::kPitch) = __builtin_amdgcn_perm(b23, b01, 0x07060302u);
        }
    }
    __syncthreads();
    // write 16-byte pieces to each channel's scratch row (killed channels
    // have none); pieces past the last sample hold zeros
    constexpr int PPR = S::kRowBytes / 16;          // pieces per channel row
    const long long byte0 = t0 / S::kSamplesPerByte;
    // rows and kill flags first (a load inside the store loop would make
    // every store wait for the one before it); without a channel map
    // (sub-band passes keep every channel's row) killed channels are
    // written as zeros
    constexpr int NIT = kUC * PPR / 256;
    static_assert(kUC * PPR % 256 == 0, "whole items per thread");
    int rows[NIT];
    bool killed[NIT];
#pragma unroll
    for (int n = 0; n < NIT; ++n) {
        const int c = c0 + (threadIdx.x + 256 * n) / PPR;
        rows[n] = c < b.nchans ? (b.chanmap ? b.chanmap[c] : c) : -1;
        killed[n] = c < b.nchans && b.mask && b.mask[c] == 0;
    }
#pragma unroll
    for (int n = 0; n < NIT; ++n) {
        const int it = threadIdx.x + 256 * n;
        const int c = it / PPR;
        const int p = it % PPR;
        if (rows[n] < 0 || t0 + 16LL * S::kSamplesPerByte * p >= b.nsamps) continue;
        const u32x4 val = killed[n] ? u32x4{0u, 0u, 0u, 0u}
                                    : *reinterpret_cast<const u32x4*>(tile + (size_t)c * S::kPitch + 16 * p);
        *reinterpret_cast<u32x4*>(b.xc + (long long)rows[n] * b.pitch + byte0 + 16 * p) = val;
    }
    // the padding rows (live channels up to a multiple of 8) read as zeros
    if (b.pad_row >= 0 && by == 0 && threadIdx.x < PPR * (b.nact - b.pad_row)) {
        const int r = b.pad_row + threadIdx.x / PPR;
        const int p = threadIdx.x % PPR;
        if (t0 + 16LL * S::kSamplesPerByte * p < b.nsamps)
            *reinterpret_cast<u32x4*>(b.xc + (long long)r * b.pitch + byte0 + 16 * p) =
                u32x4{0u, 0u, 0u, 0u};
    }
}

// Corner turn into bit planes (2-bit codes, format kFmtPlane).  A workgroup
// covers 128 samples of up to 1024 channels: lane l of wave w takes input
// word column g = 64*by + l (channels 16g .. 16g+15) over the 32 samples
// 128*bx + 32w .. +31.  Its 32 row words form a 32 x 32 bit matrix (row i =
// sample i, bit 2q + p = bit p of channel 16g + q); transposed, word 2q + p
// is plane p of channel 16g + q over the 32 samples.  The words go through
// LDS so that each scratch row receives one 16-byte store of its 128 samples.
constexpr int kPlaneTileT = 128;               // samples per plane corner-turn tile
constexpr int kPlaneTileW = 64;                // input words (16 channels each) per tile
constexpr int kPlaneLdsPitch = kPlaneTileW * 4 + 4;   // LDS words per bit row (+4: fewer conflicts)

// In-place transpose of a 32 x 32 bit matrix (a[r] bit c -> a[c] bit r) by
// block swaps of 16, 8, 4, 2 and 1 bits (two shifts and two bit-field
// selects per row pair and step).
__device__ __forceinline__ void transpose32(uint32_t (&a)[32])
{
#pragma unroll
    for (int st = 0; st < 5; ++st) {
        const int j = 16 >> st;
        const uint32_t m = st == 0 ? 0x0000FFFFu : st == 1 ? 0x00FF00FFu : st == 2 ? 0x0F0F0F0Fu
                           : st == 3 ? 0x33333333u : 0x55555555u;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if (k & j) continue;
            const uint32_t top = a[k], bot = a[k + j];
            a[k] = (top & m) | ((bot << j) & ~m);
            a[k + j] = ((top >> j) & m) | (bot & ~m);
        }
    }
}

//
// The interleaved format (SEG, kFmtSeg) uses the same transpose with other
// rows: workgroup bx covers the four scratch words 4bx .. 4bx+3, wave w word
// j = 4bx + w, whose row i is input sample j + S*i (S = seg_len(nout)); every
// word of the scratch rows is written, zeros past the last sample.
template <bool SEG>
__device__ __forceinline__ void unpack_planes_tile(const BeamDesc& b, long long bx, int by, uint32_t* lds)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ndw = b.nchans >> 4;                  // input words per row
    const int g = by * kPlaneTileW + lane;
    const long long t0 = SEG ? 4 * bx + wave : bx * kPlaneTileT + 32 * wave;
    const long long step = SEG ? seg_len(b.nout) : 1;
    uint32_t a[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const long long t = t0 + step * i;
        a[i] = (t < b.nsamps && g < ndw) ? *reinterpret_cast<const uint32_t*>(row_ptr(b, t) + 4LL * g) : 0u;
    }
    transpose32(a);
#pragma unroll
    for (int k = 0; k < 32; ++k) lds[k * kPlaneLdsPitch + 4 * lane + wave] = a[k];
    __syncthreads();
    // one 16-byte store per (channel, plane) row: item i -> word column
    // i / 32, bit row k = i % 32 (channel 16g + k/2, plane k%2)
    const long long byte0 = SEG ? 16 * bx : bx * (kPlaneTileT / 8);
    if (SEG || bx * kPlaneTileT < b.nsamps) {
        // rows and kill flags of all the thread's items first: a load inside
        // the store loop would make every store wait for the one before it
        // (vector loads and stores share one counter)
        constexpr int NIT = kPlaneTileW * 32 / 256;
        static_assert(kPlaneTileW * 32 % 256 == 0, "whole items per thread");
        int rows[NIT];
        bool killed[NIT];
#pragma unroll
        for (int n = 0; n < NIT; ++n) {
            const int i = threadIdx.x + 256 * n;
            const int c = 16 * (by * kPlaneTileW + (i >> 5)) + ((i & 31) >> 1);
            rows[n] = c < b.nchans ? (b.chanmap ? b.chanmap[c] : c) : -1;
            killed[n] = c < b.nchans && b.mask && b.mask[c] == 0;
        }
#pragma unroll
        for (int n = 0; n < NIT; ++n) {
            if (rows[n] < 0) continue;
            const int i = threadIdx.x + 256 * n;
            const int l = i >> 5, k = i & 31;
            const u32x4 v = killed[n] ? u32x4{0u, 0u, 0u, 0u}
                                      : *reinterpret_cast<const u32x4*>(lds + k * kPlaneLdsPitch + 4 * l);
            *reinterpret_cast<u32x4*>(b.xc + (long long)(2 * rows[n] + (k & 1)) * b.pitch + byte0) = v;
        }
        // the padding rows (live channels up to a multiple of 32) read as zeros
        if (b.pad_row >= 0 && by == 0 && threadIdx.x < 2 * (b.nact - b.pad_row))
            *reinterpret_cast<u32x4*>(b.xc + (long long)(2 * b.pad_row + threadIdx.x) * b.pitch + byte0) =
                u32x4{0u, 0u, 0u, 0u};
    }
}

// Consecutive time tiles write consecutive 16-byte pieces of the same plane
// rows' 128-byte lines, so they go to one XCD (whose L2 merges the pieces)
// rather than round-robin over the eight.
__global__ __launch_bounds__(256) void k_unpack_planes(BeamDesc b)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[32 * kPlaneLdsPitch];
    unpack_planes_tile<false>(b, xcd_remap((int)blockIdx.x, (int)gridDim.x), blockIdx.y, lds);
}

// The single-beam segmented corner turn: kSegTurnWaves waves, words
// W x .. W x + W-1 (W = kSegTurnWaves) of every plane row per workgroup, so
// each row receives 4W bytes of a 128-byte line from one workgroup.
constexpr int kSegTurnWaves = 16;
constexpr int kSegLdsPitch = kPlaneTileW * kSegTurnWaves + 4;   // LDS words per bit row
__global__ __launch_bounds__(64 * kSegTurnWaves) void k_unpack_seg(BeamDesc b)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[32 * kSegLdsPitch];
    const long long bx = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int by = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ndw = b.nchans >> 4;
    const int g = by * kPlaneTileW + lane;
    const long long S = seg_len(b.nout);
    const long long j = kSegTurnWaves * bx + wave;
    uint32_t a[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const long long t = j + S * i;
        a[i] = (t < b.nsamps && g < ndw) ? *reinterpret_cast<const uint32_t*>(row_ptr(b, t) + 4LL * g) : 0u;
    }
    transpose32(a);
#pragma unroll
    for (int k = 0; k < 32; ++k) lds[k * kSegLdsPitch + kSegTurnWaves * lane + wave] = a[k];
    // rows and kill flags first: a load inside the store loop would make
    // every store wait for the one before it
    constexpr int PPR = kSegTurnWaves / 4;           // 16-byte pieces per row and workgroup
    constexpr int NIT = kPlaneTileW * 32 * PPR / (64 * kSegTurnWaves);
    static_assert(NIT * 64 * kSegTurnWaves == kPlaneTileW * 32 * PPR, "whole items per thread");
    int rows[NIT];
    bool killed[NIT];
#pragma unroll
    for (int n = 0; n < NIT; ++n) {
        const int i = threadIdx.x + 64 * kSegTurnWaves * n;
        const int c = 16 * (by * kPlaneTileW + i / (32 * PPR)) + ((i / PPR) % 32 >> 1);
        rows[n] = c < b.nchans ? (b.chanmap ? b.chanmap[c] : c) : -1;
        killed[n] = c < b.nchans && b.mask && b.mask[c] == 0;
    }
    __syncthreads();
    // item i: lane column l = i / (32 PPR), bit row k = (i / PPR) % 32, piece h = i % PPR
    const long long byte0 = 4 * kSegTurnWaves * bx;
#pragma unroll
    for (int n = 0; n < NIT; ++n) {
        if (rows[n] < 0) continue;
        const int i = threadIdx.x + 64 * kSegTurnWaves * n;
        const int l = i / (32 * PPR), k = (i / PPR) % 32, h = i % PPR;
        const u32x4 v = killed[n] ? u32x4{0u, 0u, 0u, 0u}
                                  : *reinterpret_cast<const u32x4*>(lds + k * kSegLdsPitch + kSegTurnWaves * l + 4 * h);
        *reinterpret_cast<u32x4*>(b.xc + (long long)(2 * rows[n] + (k & 1)) * b.pitch + byte0 + 16 * h) = v;
    }
    // the padding rows (live channels up to a multiple of 32) read as zeros
    if (b.pad_row >= 0 && by == 0 && threadIdx.x < 2 * PPR * (b.nact - b.pad_row))
        *reinterpret_cast<u32x4*>(b.xc + (long long)(2 * b.pad_row + threadIdx.x / PPR) * b.pitch + byte0 +
                                  16 * (threadIdx.x % PPR)) = u32x4{0u, 0u, 0u, 0u};
}

template <int NBITS>
__global__ __launch_bounds__(256) void k_unpack(BeamDesc b)
{
    __shared__ __attribute__((aligned(16))) uint8_t tile[kUC * Store<NBITS>::kPitch];
    unpack_tile<NBITS>(b, xcd_remap((int)blockIdx.x, (int)gridDim.x), blockIdx.y, tile);
}

// Corner turns of up to kMaxBatchDescs beams in one launch: workgroup i
// takes unit i of the beams' (time tile, channel tile) units, numbered beam
// by beam; the beam's input bit depth (b.in_nbits) picks the unpack.
__host__ __device__ inline long long unpack_grid_x(const BeamDesc& b)
{
    if (b.xc_fmt == kFmtSeg) return b.pitch / 16;      // four words of every row per workgroup
    const int t = b.xc_fmt == kFmtPlane ? kPlaneTileT : kUT;
    return (b.nsamps + t - 1) / t;
}
__host__ __device__ inline long long unpack_grid_y(const BeamDesc& b)
{
    return fmt_planes(b.xc_fmt) ? ((b.nchans >> 4) + kPlaneTileW - 1) / kPlaneTileW : (b.nchans + kUC - 1) / kUC;
}

__global__ __launch_bounds__(256) void k_unpack_multi(DescBlock blk, int nbeams)
{
    constexpr int kBytes = kUC * Store<8>::kPitch > 128 * kPlaneLdsPitch ? kUC * Store<8>::kPitch
                                                                         : 128 * kPlaneLdsPitch;
    __shared__ __attribute__((aligned(16))) uint8_t tile[kBytes];
    long long id = blockIdx.x;
    for (int i = 0; i < nbeams; ++i) {
        const BeamDesc& b = blk.d[i];
        const long long gx = unpack_grid_x(b);
        const long long units = gx * unpack_grid_y(b);
        if (id < units) {
            const long long bx = id % gx;
            const int by = (int)(id / gx);
            if (b.xc_fmt == kFmtPlane) unpack_planes_tile<false>(b, bx, by, reinterpret_cast<uint32_t*>(tile));
            else if (b.xc_fmt == kFmtSeg) unpack_planes_tile<true>(b, bx, by, reinterpret_cast<uint32_t*>(tile));
            else if (b.in_nbits == 2) unpack_tile<2>(b, bx, by, tile);
            else unpack_tile<8>(b, bx, by, tile);
            return;
        }
        id -= units;
    }
}

// ------------------------------------------------------------ tiled sum

// One (time tile, DM block) work item.
//   xc   channel-major scratch, b.pitch bytes per row, in format FMT: 2-bit
//        codes two per byte (8 samples per 32-bit word), 8-bit codes or
//        small sums one per byte (4 per word), or 16-bit sums (2 per word)
//   base [nblocks][nact]  window start of scratch row k, in samples (a
//        multiple of 16 bytes of scratch)
//   rel  [nblocks*DB][nact/2] window offsets (delay - base, in samples) of a
//        DM row for scratch rows 2p and 2p+1 in the low and high 16 bits
// LDS: CC rows of rw words (rw % 4 == 0).  Channels are summed in pairs so
// the two realigned words of a pair fold into an accumulator with one
// three-operand add, and one v_readlane fetches both offsets.
template <int FMT, int NW, int DPW, int M, int CC, int PM>
__device__ __forceinline__ void tile_body(const BeamDesc& b, int tile, int block, int group,
                                          uint32_t* lds)
{
    static_assert(M % 2 == 1, "lanes must be an odd number of LDS words apart");
    static_assert(CC % NW == 0, "every wave stages the same number of channel rows");
    static_assert(CC <= 84, "2-bit byte lanes hold 85 codes");
    static_assert((64 % (CC / 2)) == 0, "offset pairs of one DM sit in one register");
    constexpr int SPW = fmt_samples_per_word(FMT);   // samples per 32-bit LDS word
    constexpr int BNUM = fmt_bytes_num(FMT);         // scratch bytes per sample =
    constexpr int BDEN = fmt_bytes_den(FMT);         //   BNUM / BDEN
    constexpr int T = 64 * M * SPW;              // tile length in samples
    constexpr int DB = NW * DPW;
    constexpr int CPW = CC / NW;                 // channel rows staged per wave per chunk
    constexpr int CP = CC / 2;                   // channel pairs per chunk
    constexpr int KPR = 64 / CP;                 // DMs per offset register
    constexpr int RV = (DPW + KPR - 1) / KPR;    // registers of offset pairs per wave
    // Packed lanes:
    //  2-bit: a realigned word holds eight 4-bit lanes (samples 0..7), and a
    //         group of 4 channels sums into them exactly (at most 12 < 16).
    //         Every 8 channels the two group sums g, h are folded into
    //           E += (g & 0x0F0F0F0F) + (h & 0x0F0F0F0F)   byte lanes: samples 0, 2, 4, 6
    //           S += (g >> 4) + (h >> 4)
    //         and every FLUSH chunks the odd samples are recovered as
    //           O = S - ((E & 0xFFFFFF00) >> 4)            byte lanes: samples 1, 3, 5, 7
    //         (each group sum's lowest nibble is below 16, so its shift
    //         drops nothing but that nibble; the even nibbles it moves are
    //         exactly E's upper three byte lanes shifted down by 4 bits).
    //         E and O are exact up to 85 codes per lane, and are flushed into
    //         16-bit lanes w16[0..3] = samples {0,4}, {2,6}, {1,5}, {3,7}.
    //  8-bit: sw[0] = 16-bit lanes (samples 0, 1), sw[1] = (2, 3), exact for
    //         257 codes, flushed every FLUSH chunks into 32-bit acc[0..3].
    //  Small byte values (at most V <= 127): sw[0] = byte lanes (samples
    //         0..3) realigned with v_alignbit, flushed every b.flush_every
    //         channels (an even count with flush_every * V <= 255) into
    //         32-bit acc[0..3].
    //  16-bit values (at most V <= 32767): sw[0] = 16-bit lanes (samples 0,
    //         1) realigned with v_alignbit, flushed every b.flush_every
    //         channels (even, flush_every * V <= 65535) into acc[0..1].
    constexpr int NACC = 4;
    constexpr bool kFixedFlush = FMT == kFmtNib || FMT == kFmtByte;
    constexpr int FLUSH = FMT == kFmtNib ? 85 / CC : 257 / CC;
    static_assert(!kFixedFlush || FLUSH >= 1, "chunk too large for the packed lanes");
    static_assert(CC % 8 == 0, "channels are summed in groups of 8");

    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    tile = wave_uniform(tile);
    block = wave_uniform(block);
    group = wave_uniform(group);
    const long long t0 = (long long)tile * T;
    // Every descriptor field is wave-uniform; keep them in scalar registers
    // (the multi-beam kernels read descriptors through a dynamic index).
    const int nchans = wave_uniform(b.nact);   // scratch rows, a multiple of 8
    const int rw = wave_uniform(b.rw);
    const int rq = rw >> 2;                // 16-byte pieces per row
    const long long pitch = wave_uniform64(b.pitch);
    const long long nout = wave_uniform64(b.nout);
    const long long out_stride = wave_uniform64(b.out_stride);
    const int ndm = wave_uniform(b.ndm);
    const uint8_t* xc = wave_uniform_ptr(b.xc) + group * wave_uniform64(b.g_xc);
    uint32_t* out = wave_uniform_ptr(b.out);
    const int32_t* base_row = wave_uniform_ptr(b.base) + group * wave_uniform64(b.g_base) +
                              (size_t)block * nchans;
    const int npairs = nchans >> 1;
    const uint32_t* rel_rows = wave_uniform_ptr(b.rel) + group * wave_uniform64(b.g_rel) +
                               (size_t)(block * DB + wave * DPW) * npairs;

    uint32_t sw[DPW][M][2];
    uint32_t acc[DPW][M][NACC];
#pragma unroll
    for (int k = 0; k < DPW; ++k)
#pragma unroll
        for (int j = 0; j < M; ++j) {
            sw[k][j][0] = sw[k][j][1] = 0u;
#pragma unroll
            for (int e = 0; e < NACC; ++e) acc[k][j][e] = 0u;
        }

    // Chunk prefetch registers.  Every load below is unconditional and in
    // bounds (indices are clamped); results that are not needed are simply
    // not stored, which keeps all of these arrays in registers.
    u32x4 pf[CPW][PM];
    int vbase_nxt = 0;         // lane i < CC: window start of channel c0 + i (next chunk)
    uint32_t vrel_cur[RV], vrel_nxt[RV];
    const int last_c = nchans - 1;
    const int last_p = rq - 1;

#define DEDISP_LOAD_BASE(C0)                                                        \
    vbase_nxt = gload(base_row + min((C0) + (lane < CC ? lane : 0), last_c));
#define DEDISP_LOAD_REL(C0, DST)                                                    \
    _Pragma("unroll") for (int r = 0; r < RV; ++r) {                                \
        const int idx = 64 * r + lane;                                              \
        DST[r] = gload(rel_rows + (size_t)min(idx / CP, DPW - 1) * npairs +         \
                       min(((C0) >> 1) + idx % CP, npairs - 1));                    \
    }
#define DEDISP_LOAD_DATA(C0)                                                        \
    _Pragma("unroll") for (int i = 0; i < CPW; ++i) {                               \
        const int cl = wave + NW * i;                                               \
        const int bs = lane_value(vbase_nxt, cl);                                   \
        const uint8_t* src = xc + (long long)min((C0) + cl, last_c) * pitch + (t0 + bs) * BNUM / BDEN; \
        _Pragma("unroll") for (int q = 0; q < PM; ++q)                              \
            pf[i][q] = gload(reinterpret_cast<const u32x4*>(src + 16 * min(lane + 64 * q, last_p))); \
    }

    DEDISP_LOAD_BASE(0)
    DEDISP_LOAD_DATA(0)
    DEDISP_LOAD_REL(0, vrel_nxt)
    if (CC < nchans) {
        DEDISP_LOAD_BASE(CC)
    }

    int since_flush = 0;                       // chunks (fixed flush) or channels (runtime flush)
    const int flush_chans = wave_uniform(b.flush_every);
    const bool dbuf = wave_uniform(b.dbuf) != 0;
    bool chunk_odd = false;
    for (int c0 = 0; c0 < nchans; c0 += CC) {
        const int ncur = min(CC, nchans - c0);  // a multiple of 8
        // With a double buffer (b.dbuf) the chunk goes to the half the
        // previous chunk did not use, which every wave finished reading before
        // the last barrier; otherwise wait until everyone is done reading.
        uint32_t* lbuf = lds;
        if (dbuf) {
            if (chunk_odd) lbuf += (size_t)CC * rw;
            chunk_odd = !chunk_odd;
        } else {
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            const int cl = wave + NW * i;
            uint32_t* dst = lbuf + (size_t)cl * rw;
#pragma unroll
            for (int q = 0; q < PM; ++q) {
                const int p = lane + 64 * q;
                if (cl < ncur && p < rq) *reinterpret_cast<u32x4*>(dst + 4 * p) = pf[i][q];
            }
        }
#pragma unroll
        for (int r = 0; r < RV; ++r) vrel_cur[r] = vrel_nxt[r];
        __syncthreads();
        if (c0 + CC < nchans) {
            DEDISP_LOAD_DATA(c0 + CC)          // uses the window starts of chunk c0 + CC
            DEDISP_LOAD_REL(c0 + CC, vrel_nxt)
            if (c0 + 2 * CC < nchans) {
                DEDISP_LOAD_BASE(c0 + 2 * CC)
            }
        }
#undef DEDISP_LOAD_BASE
#undef DEDISP_LOAD_REL
#undef DEDISP_LOAD_DATA

        const uint32_t* lrow = lbuf + lane * M;
        if constexpr (FMT == kFmtNib) {
            for (int c = 0; c < ncur; c += 8) {
#pragma unroll
                for (int k = 0; k < DPW; ++k) {
                    // offsets of (DM k, channels c+2q, c+2q+1): register k / KPR,
                    // lane (k % KPR)*CP + c/2 + q
                    uint32_t rr[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        rr[q] = (uint32_t)lane_value((int)vrel_cur[k / KPR], (k % KPR) * CP + (c >> 1) + q);
                    uint32_t w[8][M + 1], sh[8];
#pragma unroll
                    for (int h = 0; h < 8; ++h) {
                        const uint32_t r = (h & 1) ? (rr[h >> 1] >> 16) : (rr[h >> 1] & 0xFFFFu);
                        const uint32_t* src = lrow + (size_t)(c + h) * rw + r / SPW;
#pragma unroll
                        for (int j = 0; j <= M; ++j) w[h][j] = src[j];
                        sh[h] = 4u * (r & 7u);                 // nibble shift
                    }
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        uint32_t a[8];
#pragma unroll
                        for (int h = 0; h < 8; ++h)
                            a[h] = __builtin_amdgcn_alignbit(w[h][j + 1], w[h][j], sh[h]);
                        const uint32_t g = (a[0] + a[1]) + (a[2] + a[3]);
                        const uint32_t g2 = (a[4] + a[5]) + (a[6] + a[7]);
                        sw[k][j][0] += (g & 0x0F0F0F0Fu) + (g2 & 0x0F0F0F0Fu);
                        sw[k][j][1] += (g >> 4) + (g2 >> 4);
                    }
                }
            }
        } else if constexpr (FMT == kFmtByte) {
            for (int c = 0; c < ncur; c += 2) {
                const uint32_t* row0 = lrow + (size_t)c * rw;
                const uint32_t* row1 = row0 + rw;
#pragma unroll
                for (int k = 0; k < DPW; ++k) {
                    const uint32_t rr = (uint32_t)lane_value((int)vrel_cur[k / KPR], (k % KPR) * CP + (c >> 1));
                    const uint32_t r0 = rr & 0xFFFFu, r1 = rr >> 16;
                    const uint32_t* src0 = row0 + r0 / SPW;
                    const uint32_t* src1 = row1 + r1 / SPW;
                    uint32_t w0[M + 1], w1[M + 1];
#pragma unroll
                    for (int j = 0; j <= M; ++j) {
                        w0[j] = src0[j];
                        w1[j] = src1[j];
                    }
                    // bytes s, s+1 -> 16-bit lanes of sw[0]; s+2, s+3 -> sw[1]
                    // (selectors formed in scalar registers: they are
                    // wave-uniform, and vector ALU slots are the bottleneck)
                    uint32_t lo0 = (r0 & 3u) * 0x00010001u + 0x0C010C00u;
                    uint32_t lo1 = (r1 & 3u) * 0x00010001u + 0x0C010C00u;
                    asm volatile("" : "+s"(lo0), "+s"(lo1));
                    const uint32_t hi0 = lo0 + 0x00020002u, hi1 = lo1 + 0x00020002u;
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        sw[k][j][0] += __builtin_amdgcn_perm(w0[j + 1], w0[j], lo0) +
                                       __builtin_amdgcn_perm(w1[j + 1], w1[j], lo1);
                        sw[k][j][1] += __builtin_amdgcn_perm(w0[j + 1], w0[j], hi0) +
                                       __builtin_amdgcn_perm(w1[j + 1], w1[j], hi1);
                    }
                }
            }
        } else {
            // small byte values or 16-bit values, runtime flush interval
            for (int c = 0; c < ncur; c += 2) {
                const uint32_t* row0 = lrow + (size_t)c * rw;
                const uint32_t* row1 = row0 + rw;
#pragma unroll
                for (int k = 0; k < DPW; ++k) {
                    const uint32_t rr = (uint32_t)lane_value((int)vrel_cur[k / KPR], (k % KPR) * CP + (c >> 1));
                    const uint32_t r0 = rr & 0xFFFFu, r1 = rr >> 16;
                    const uint32_t* src0 = row0 + r0 / SPW;
                    const uint32_t* src1 = row1 + r1 / SPW;
                    uint32_t w0[M + 1], w1[M + 1];
#pragma unroll
                    for (int j = 0; j <= M; ++j) {
                        w0[j] = src0[j];
                        w1[j] = src1[j];
                    }
                    // bit shift of the window start within its word
                    const uint32_t s0 = (r0 % SPW) * (32u / SPW), s1 = (r1 % SPW) * (32u / SPW);
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        sw[k][j][0] += __builtin_amdgcn_alignbit(w0[j + 1], w0[j], s0) +
                                       __builtin_amdgcn_alignbit(w1[j + 1], w1[j], s1);
                }
                since_flush += 2;
                if (since_flush + 2 > flush_chans) {
                    since_flush = 0;
#pragma unroll
                    for (int k = 0; k < DPW; ++k)
#pragma unroll
                        for (int j = 0; j < M; ++j) {
                            const uint32_t v = sw[k][j][0];
                            if constexpr (FMT == kFmtByteS) {
                                acc[k][j][0] += v & 0xFFu;
                                acc[k][j][1] += (v >> 8) & 0xFFu;
                                acc[k][j][2] += (v >> 16) & 0xFFu;
                                acc[k][j][3] += v >> 24;
                            } else {
                                acc[k][j][0] += v & 0xFFFFu;
                                acc[k][j][1] += v >> 16;
                            }
                            sw[k][j][0] = 0u;
                        }
                }
            }
        }

        if (kFixedFlush && (++since_flush == FLUSH || c0 + CC >= nchans)) {
            since_flush = 0;
#pragma unroll
            for (int k = 0; k < DPW; ++k)
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    if constexpr (FMT == kFmtNib) {
                        const uint32_t e = sw[k][j][0];
                        const uint32_t o = sw[k][j][1] - ((e & 0xFFFFFF00u) >> 4);
                        acc[k][j][0] += e & 0x00FF00FFu;           // samples 0, 4
                        acc[k][j][1] += (e >> 8) & 0x00FF00FFu;    // samples 2, 6
                        acc[k][j][2] += o & 0x00FF00FFu;           // samples 1, 5
                        acc[k][j][3] += (o >> 8) & 0x00FF00FFu;    // samples 3, 7
                    } else {
                        const uint32_t lo = sw[k][j][0], hi = sw[k][j][1];
                        acc[k][j][0] += lo & 0xFFFFu;
                        acc[k][j][1] += lo >> 16;
                        acc[k][j][2] += hi & 0xFFFFu;
                        acc[k][j][3] += hi >> 16;
                    }
                    sw[k][j][0] = 0u;
                    sw[k][j][1] = 0u;
                }
        }
    }

    if constexpr (!kFixedFlush) {
        if (since_flush > 0) {
#pragma unroll
            for (int k = 0; k < DPW; ++k)
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const uint32_t v = sw[k][j][0];
                    if constexpr (FMT == kFmtByteS) {
                        acc[k][j][0] += v & 0xFFu;
                        acc[k][j][1] += (v >> 8) & 0xFFu;
                        acc[k][j][2] += (v >> 16) & 0xFFu;
                        acc[k][j][3] += v >> 24;
                    } else {
                        acc[k][j][0] += v & 0xFFFFu;
                        acc[k][j][1] += v >> 16;
                    }
                }
        }
    }

    // 16-byte stores need 16-byte aligned rows (SPW >= 4), 8-byte stores
    // 8-byte aligned rows (SPW == 2)
    constexpr int VW = SPW >= 4 ? 4 : 2;
    const bool vec = ((out_stride & (VW - 1)) == 0) &&
                     ((reinterpret_cast<uintptr_t>(out) & (4 * VW - 1)) == 0);
    const int32_t* rowmap = wave_uniform_ptr(b.rowmap);
    const int ndm_here = group == wave_uniform(b.ngroups) - 1 ? wave_uniform(b.ndm_last) : ndm;
    const int out_bytes = wave_uniform(b.out_bytes);
    const int out_shift = wave_uniform(b.out_shift);
    const long long g_out = wave_uniform64(b.g_out);
    // narrow rows take 32-bit stores of 4 bytes or 2 halves when every row
    // starts 4-byte aligned
    const bool nvec = ((reinterpret_cast<uintptr_t>(out) & 3) == 0) && ((out_stride & 3) == 0) &&
                      ((g_out & 3) == 0);
#pragma unroll
    for (int k = 0; k < DPW; ++k) {
        const int d = block * DB + wave * DPW + k;
        if (d >= ndm_here) continue;
        const int orow_idx = rowmap ? wave_uniform(rowmap[d]) : d;
        if (out_bytes != 4) {
            // narrow sums written into a channel-major scratch: row stride
            // and group offset in bytes
            uint8_t* nrow = reinterpret_cast<uint8_t*>(out) + group * g_out +
                            (long long)orow_idx * out_stride;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const long long t = t0 + (long long)SPW * (lane * M + j);
                uint32_t o[SPW];
                if constexpr (FMT == kFmtNib) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        o[4 * h + 0] = (acc[k][j][0] >> (16 * h)) & 0xFFFFu;
                        o[4 * h + 1] = (acc[k][j][2] >> (16 * h)) & 0xFFFFu;
                        o[4 * h + 2] = (acc[k][j][1] >> (16 * h)) & 0xFFFFu;
                        o[4 * h + 3] = (acc[k][j][3] >> (16 * h)) & 0xFFFFu;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < SPW; ++e) o[e] = acc[k][j][e];
                }
#pragma unroll
                for (int e = 0; e < SPW; ++e) o[e] = out_value(o[e], out_shift, out_bytes);
                if (nvec && t + SPW <= nout) {
                    if (out_bytes == 1) {
#pragma unroll
                        for (int g4 = 0; g4 < SPW / 4; ++g4)
                            *reinterpret_cast<uint32_t*>(nrow + t + 4 * g4) =
                                o[4 * g4] | (o[4 * g4 + 1] << 8) | (o[4 * g4 + 2] << 16) | (o[4 * g4 + 3] << 24);
                    } else {
#pragma unroll
                        for (int g2 = 0; g2 < SPW / 2; ++g2)
                            *reinterpret_cast<uint32_t*>(nrow + 2 * (t + 2 * g2)) =
                                o[2 * g2] | (o[2 * g2 + 1] << 16);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < SPW; ++e) {
                        if (t + e < nout) {
                            if (out_bytes == 1) nrow[t + e] = (uint8_t)o[e];
                            else reinterpret_cast<uint16_t*>(nrow)[t + e] = (uint16_t)o[e];
                        }
                    }
                }
            }
            continue;
        }
        uint32_t* orow = out + group * g_out + (size_t)orow_idx * (size_t)out_stride;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const long long t = t0 + (long long)SPW * (lane * M + j);
            uint32_t o[SPW];
            if constexpr (FMT == kFmtNib) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    o[4 * h + 0] = (acc[k][j][0] >> (16 * h)) & 0xFFFFu;
                    o[4 * h + 1] = (acc[k][j][2] >> (16 * h)) & 0xFFFFu;
                    o[4 * h + 2] = (acc[k][j][1] >> (16 * h)) & 0xFFFFu;
                    o[4 * h + 3] = (acc[k][j][3] >> (16 * h)) & 0xFFFFu;
                }
            } else {
#pragma unroll
                for (int e = 0; e < SPW; ++e) o[e] = acc[k][j][e];
            }
            if (out_shift) {
#pragma unroll
                for (int e = 0; e < SPW; ++e) o[e] >>= out_shift;
            }
#pragma unroll
            for (int g = 0; g < SPW / VW; ++g) {
                const long long tg = t + VW * g;
                if (vec && tg + VW - 1 < nout) {
                    if constexpr (VW == 4)
                        *reinterpret_cast<u32x4*>(orow + tg) =
                            u32x4{o[4 * g], o[4 * g + 1], o[4 * g + 2], o[4 * g + 3]};
                    else
                        *reinterpret_cast<u32x2*>(orow + tg) = u32x2{o[2 * g], o[2 * g + 1]};
                } else {
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        if (tg + e < nout) orow[tg + e] = o[VW * g + e];
                }
            }
        }
    }
}

// ------------------------------------------------------------ bit-plane sum
//
// 2-bit codes as two bit planes (format kFmtPlane): a 32-bit word of plane p
// holds bit p of 32 consecutive samples.  For one (DM, channel) a lane
// realigns M words of each plane with v_alignbit (any shift 0..31), giving
// a = bit 0 and b = bit 1 of the channel's 32M shifted samples; the channel
// adds a + 2b to every sample.  The sums are kept bit-sliced: acc[L][j] is
// bit L of the running sum of the 32 samples of word j, and words are added
// by full adders over 32 bit positions at once (Section 2.3's bit-level
// parallelism with one-bit lanes; a full adder is one three-way xor and one
// majority, each a single v_bitop3).  Carries are handed up the levels in a
// fixed schedule over 32 channels (64 full adders, 5 half adders), so no
// lane ever overflows and no flush is needed; at the end a bit transpose
// turns the kPlaneLevels planes of each word into 32 integer sums.

// Full adder over 32 bit positions: s <- s ^ x ^ y; returns the carry
// majority(s, x, y), of twice the weight of s.
__device__ __forceinline__ uint32_t fa(uint32_t& s, uint32_t x, uint32_t y)
{
    const uint32_t c = __builtin_amdgcn_bitop3_b32(s, x, y, 0xE8);
    s = __builtin_amdgcn_bitop3_b32(s, x, y, 0x96);
    return c;
}

__device__ __forceinline__ uint32_t ha(uint32_t& s, uint32_t x)
{
    const uint32_t c = s & x;
    s ^= x;
    return c;
}

// Realigned planes of one channel: bits r .. r + 32M - 1 of the staged rows
// starting `row0` words after the lane's base (plane 1 RWS words after plane
// 0).  The word offset is formed in a scalar register, so one vector add
// gives the address and every read takes an immediate offset.
//
// Interleaved format (SEG): r is the offset in whole words and lane l owns
// words l, l + 64, ..., l + 64(M-1) of the tile, so the words need no
// realignment and the 64 lanes of a read hit 64 consecutive words.
template <int M, int RWS, bool SEG>
__device__ __forceinline__ void plane_words(const uint32_t* lrow, int row0, uint32_t r, uint32_t (&a)[M],
                                            uint32_t (&b)[M])
{
    int off = row0 + (int)(SEG ? r : r >> 5);
    asm volatile("" : "+s"(off));       // keep the constant row part out of the address fold
    const uint32_t* src = lrow + off;
    if constexpr (SEG) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
            a[j] = src[64 * j];
            b[j] = src[RWS + 64 * j];
        }
    } else {
        uint32_t w0[M + 1], w1[M + 1];
#pragma unroll
        for (int j = 0; j <= M; ++j) {
            w0[j] = src[j];
            w1[j] = src[RWS + j];
        }
        const uint32_t sh = r & 31u;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            a[j] = __builtin_amdgcn_alignbit(w0[j + 1], w0[j], sh);
            b[j] = __builtin_amdgcn_alignbit(w1[j + 1], w1[j], sh);
        }
    }
}

// Four channels (LDS rows of channel j at row + 2*j*RWS; offset pairs in
// lanes pair0, pair0 + 1 of voff) into the accumulators; returns their three
// carries of weight 4 in k4.
template <int M, int RWS, bool SEG>
__device__ __forceinline__ void plane_quad(uint32_t (&acc)[kPlaneLevels][M], const uint32_t* lrow, int row,
                                           uint32_t voff, int pair0, uint32_t (&k4)[3][M])
{
    uint32_t a0[M], b0[M], a1[M], b1[M];
    uint32_t k2[2][M];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t rr = (uint32_t)lane_value((int)voff, pair0 + h);
        plane_words<M, RWS, SEG>(lrow, row + (4 * h) * RWS, rr & 0xFFFFu, a0, b0);
        plane_words<M, RWS, SEG>(lrow, row + (4 * h + 2) * RWS, rr >> 16, a1, b1);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            k2[h][j] = fa(acc[0][j], a0[j], a1[j]);
            k4[h][j] = fa(acc[1][j], b0[j], b1[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) k4[2][j] = fa(acc[1][j], k2[0][j], k2[1][j]);
}

// Fold six carries of level L into three of level L + 1.
template <int M>
__device__ __forceinline__ void plane_fold(uint32_t (&accl)[M], const uint32_t (&x)[3][M], const uint32_t (&y)[3][M],
                                           uint32_t (&out)[3][M])
{
#pragma unroll
    for (int j = 0; j < M; ++j) {
        out[0][j] = fa(accl[j], x[0][j], x[1][j]);
        out[1][j] = fa(accl[j], x[2][j], y[0][j]);
        out[2][j] = fa(accl[j], y[1][j], y[2][j]);
    }
}

template <int M, int RWS, bool SEG>
__device__ __forceinline__ void plane_octet(uint32_t (&acc)[kPlaneLevels][M], const uint32_t* lrow, int row,
                                            uint32_t voff, int pair0, uint32_t (&k8)[3][M])
{
    uint32_t p[3][M], q[3][M];
    plane_quad<M, RWS, SEG>(acc, lrow, row, voff, pair0, p);
    plane_quad<M, RWS, SEG>(acc, lrow, row + 8 * RWS, voff, pair0 + 2, q);
    plane_fold<M>(acc[2], p, q, k8);
}

template <int M, int RWS, bool SEG>
__device__ __forceinline__ void plane_sixteen(uint32_t (&acc)[kPlaneLevels][M], const uint32_t* lrow, int row,
                                              uint32_t voff, int pair0, uint32_t (&k16)[3][M])
{
    uint32_t p[3][M], q[3][M];
    plane_octet<M, RWS, SEG>(acc, lrow, row, voff, pair0, p);
    plane_octet<M, RWS, SEG>(acc, lrow, row + 16 * RWS, voff, pair0 + 4, q);
    plane_fold<M>(acc[3], p, q, k16);
}

// 32 channels (LDS rows from word `row` of the lane's base on): the full
// schedule down to the top level (the sum of at most kPlaneMaxChans codes of
// 3 never carries out of it).
template <int M, int RWS, bool SEG>
__device__ __forceinline__ void plane_unit(uint32_t (&acc)[kPlaneLevels][M], const uint32_t* lrow, int row,
                                           uint32_t voff, int pair0)
{
    uint32_t p[3][M], q[3][M], k32[3][M];
    plane_sixteen<M, RWS, SEG>(acc, lrow, row, voff, pair0, p);
    plane_sixteen<M, RWS, SEG>(acc, lrow, row + 32 * RWS, voff, pair0 + 8, q);
    plane_fold<M>(acc[4], p, q, k32);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const uint32_t k64a = fa(acc[5][j], k32[0][j], k32[1][j]);
        const uint32_t k64b = ha(acc[5][j], k32[2][j]);
        uint32_t c = fa(acc[6][j], k64a, k64b);
#pragma unroll
        for (int L = 7; L < kPlaneLevels - 1; ++L) c = ha(acc[L][j], c);
        acc[kPlaneLevels - 1][j] ^= c;
    }
}

// 16 x 16 bit transposes in both 16-bit halves at once: afterwards the low
// half of r[s] holds bits s of the low halves of the input rows, the high
// half bits 16 + s of their high halves.
__device__ __forceinline__ void transpose16x2(uint32_t (&r)[16])
{
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int j = 8 >> st;
        const uint32_t m = st == 0 ? 0x00FF00FFu : st == 1 ? 0x0F0F0F0Fu : st == 2 ? 0x33333333u : 0x55555555u;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k & j) continue;
            const uint32_t top = r[k], bot = r[k + j];
            r[k] = (top & m) | ((bot << j) & ~m);
            r[k + j] = ((top >> j) & m) | (bot & ~m);
        }
    }
}

// One (time tile, DM block) work item of the bit-plane formats: NW waves,
// one DM per wave, M plane words (32M samples) per lane, CC channels per
// staged chunk (a multiple of 32).  LDS: CC channels x 2 planes x RWS words
// (plane p of chunk channel c at row 2c + p); the staged window of a plane is
// b.rw <= RWS words long.  Window tables as for tile_body: offsets in
// samples, window starts multiples of 128 samples (kFmtPlane), or offsets
// and starts in words, the starts multiples of 4 (SEG: kFmtSeg, where a
// tile is the words 64M*tile .. +64M-1 of every row, i.e. 64M outputs of
// each of the 32 segments).
template <int NW, int M, int CC, int PM, bool SEG>
__device__ __forceinline__ void plane_body(const BeamDesc& b, int tile, int block, uint32_t* lds)
{
    constexpr int RWS = SEG ? kSegRowWords : kPlaneRowWords;
    constexpr int T = 64 * M * 32;               // tile length in samples (kFmtPlane)
    constexpr int DB = NW;                       // one DM per wave
    constexpr int RPW = 2 * CC / NW;             // plane rows staged per wave per chunk
    constexpr int CP = CC / 2;                   // channel pairs per chunk
    constexpr int NL = kPlaneLevels;
    static_assert(SEG || M % 2 == 1, "lanes must be an odd number of LDS words apart");
    static_assert(CC % 32 == 0 && (2 * CC) % NW == 0 && CP <= 64, "bad chunk");
    static_assert(SEG || RWS + M < 256, "plane 1 is read at an 8-bit dword offset from plane 0");
    static_assert(RWS % 4 == 0 && RWS >= 64 * M + 8 && RWS <= 256 * PM, "staged rows too short for the tile");

    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    tile = wave_uniform(tile);
    block = wave_uniform(block);
    // first sample (kFmtPlane) or word (SEG) of the tile
    const long long t0 = (long long)tile * (SEG ? 64 * M : T);
    const int nchans = wave_uniform(b.nact);     // a multiple of 32
    const int rw = wave_uniform(b.rw);
    const int rq = rw >> 2;
    const long long pitch = wave_uniform64(b.pitch);
    const long long nout = wave_uniform64(b.nout);
    const long long out_stride = wave_uniform64(b.out_stride);
    const int ndm = wave_uniform(b.ndm);
    const uint8_t* xc = wave_uniform_ptr(b.xc);
    uint32_t* out = wave_uniform_ptr(b.out);
    // SEG: (start, span) pairs, span = the block's largest window offset of the row
    const int32_t* base_row = wave_uniform_ptr(b.base) + (size_t)block * nchans * (SEG ? 2 : 1);
    const int npairs = nchans >> 1;
    const uint32_t* rel_row = wave_uniform_ptr(b.rel) + (size_t)(block * DB + wave) * npairs;
    // Fields the stores need, read now: a scalar load left in flight across
    // the channel loop would make every LDS wait in it a wait for all
    // outstanding reads (scalar and LDS loads share one counter).
    const int32_t* rowmap = wave_uniform_ptr(b.rowmap);
    const int out_bytes = wave_uniform(b.out_bytes);
    const int out_shift = wave_uniform(b.out_shift);
    asm volatile("" ::"s"(rowmap), "s"(out_bytes), "s"(out_shift));

    uint32_t acc[NL][M];
#pragma unroll
    for (int L = 0; L < NL; ++L)
#pragma unroll
        for (int j = 0; j < M; ++j) acc[L][j] = 0u;

    u32x4 pf[RPW][PM] = {};
    int npr[RPW];                 // pieces of each staged row that are loaded (and written to LDS)
    int vbase_nxt = 0;            // lane i < CC: window start of channel c0 + i (next chunk)
    int vspan_nxt = 0;            // SEG, lane i < CC: its span
    uint32_t vrel_cur = 0, vrel_nxt = 0;
    const int last_c = nchans - 1;
    const int last_p = rq - 1;

#define DEDISP_PLOAD_BASE(C0)                                                                         \
    if constexpr (SEG) {                                                                                \
        const int32_t* bp = base_row + 2 * min((C0) + (lane < CC ? lane : 0), last_c);                   \
        vbase_nxt = gload(bp);                                                                          \
        vspan_nxt = gload(bp + 1);                                                                      \
    } else {                                                                                            \
        vbase_nxt = gload(base_row + min((C0) + (lane < CC ? lane : 0), last_c));                        \
    }
#define DEDISP_PLOAD_REL(C0) vrel_nxt = gload(rel_row + min(((C0) >> 1) + (lane < CP ? lane : 0), npairs - 1));
#define DEDISP_PLOAD_DATA(C0)                                                                         \
    _Pragma("unroll") for (int i = 0; i < RPW; ++i) {                                                  \
        const int cl = wave + NW * i;                                                                   \
        const int bs = lane_value(vbase_nxt, cl >> 1);                                                  \
        const uint8_t* src = xc + (long long)(2 * min((C0) + (cl >> 1), last_c) + (cl & 1)) * pitch + \
                             (SEG ? 4 * (t0 + bs) : (t0 + bs) >> 3);                                    \
        /* SEG: only the pieces the row's own span needs (the rest of its LDS row is never read) */     \
        const int np = SEG ? (lane_value(vspan_nxt, cl >> 1) + 64 * M + 3) >> 2 : rq;                  \
        npr[i] = np;                                                                                    \
        _Pragma("unroll") for (int q = 0; q < PM; ++q)                                                  \
            if (!SEG || lane + 64 * q < np)                                                             \
                pf[i][q] = gload(reinterpret_cast<const u32x4*>(src + 16 * min(lane + 64 * q, last_p))); \
    }

    DEDISP_PLOAD_BASE(0)
    DEDISP_PLOAD_DATA(0)
    DEDISP_PLOAD_REL(0)
    if (CC < nchans) {
        DEDISP_PLOAD_BASE(CC)
    }

    const bool dbuf = wave_uniform(b.dbuf) != 0;
    bool chunk_odd = false;
    for (int c0 = 0; c0 < nchans; c0 += CC) {
        const int ncur = min(CC, nchans - c0);   // a multiple of 32
        uint32_t* lbuf = lds;
        if (dbuf) {
            if (chunk_odd) lbuf += (size_t)CC * 2 * RWS;
            chunk_odd = !chunk_odd;
        } else {
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int cl = wave + NW * i;
            uint32_t* dst = lbuf + (size_t)cl * RWS;
#pragma unroll
            for (int q = 0; q < PM; ++q) {
                const int pc = lane + 64 * q;
                if ((cl >> 1) < ncur && pc < npr[i]) *reinterpret_cast<u32x4*>(dst + 4 * pc) = pf[i][q];
            }
        }
        vrel_cur = vrel_nxt;
        __syncthreads();
        if (c0 + CC < nchans) {
            DEDISP_PLOAD_DATA(c0 + CC)
            DEDISP_PLOAD_REL(c0 + CC)
            if (c0 + 2 * CC < nchans) {
                DEDISP_PLOAD_BASE(c0 + 2 * CC)
            }
        }
        const uint32_t* lrow = lbuf + (SEG ? lane : lane * M);
        for (int u = 0; u < ncur; u += 32)
            plane_unit<M, RWS, SEG>(acc, lrow, u * 2 * RWS, vrel_cur, u >> 1);
    }
#undef DEDISP_PLOAD_BASE
#undef DEDISP_PLOAD_REL
#undef DEDISP_PLOAD_DATA

    const int d = block * DB + wave;
    if (d >= ndm) return;
    const int orow_idx = rowmap ? wave_uniform(rowmap[d]) : d;
    if constexpr (SEG) {
        // word w of the tile holds outputs w + S*i of segments i = 0..31;
        // for each (word, segment) the 64 lanes store 64 consecutive outputs
        const long long S = seg_len(nout);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            uint32_t r[16];
#pragma unroll
            for (int L = 0; L < 16; ++L) r[L] = L < NL ? acc[L][j] : 0u;
            transpose16x2(r);
            const long long w = t0 + lane + 64 * j;
            if (w >= S) continue;
            if (out_bytes == 4) {
                uint32_t* orow = out + (size_t)orow_idx * (size_t)out_stride;
#pragma unroll
                for (int i = 0; i < 32; ++i) {
                    const long long t = w + S * i;
                    const uint32_t v = i < 16 ? (r[i] & 0xFFFFu) : (r[i - 16] >> 16);
                    if (t < nout) orow[t] = v >> out_shift;
                }
            } else {
                uint8_t* nrow = reinterpret_cast<uint8_t*>(out) + (long long)orow_idx * out_stride;
#pragma unroll
                for (int i = 0; i < 32; ++i) {
                    const long long t = w + S * i;
                    const uint32_t v = out_value(i < 16 ? (r[i] & 0xFFFFu) : (r[i - 16] >> 16), out_shift,
                                                 out_bytes);
                    if (t < nout) {
                        if (out_bytes == 1) nrow[t] = (uint8_t)v;
                        else reinterpret_cast<uint16_t*>(nrow)[t] = (uint16_t)v;
                    }
                }
            }
        }
        return;
    }
    const bool vec = ((out_stride & 3) == 0) && ((reinterpret_cast<uintptr_t>(out) & 15) == 0);
    const bool nvec = ((reinterpret_cast<uintptr_t>(out) & 3) == 0) && ((out_stride & 3) == 0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        uint32_t r[16];
#pragma unroll
        for (int L = 0; L < 16; ++L) r[L] = L < NL ? acc[L][j] : 0u;
        transpose16x2(r);
        const long long t = t0 + 32LL * (lane * M + j);
        if (out_bytes == 4) {
            uint32_t* orow = out + (size_t)orow_idx * (size_t)out_stride;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const int h = g >> 2;            // 0: samples 0..15 (low halves), 1: 16..31 (high)
                uint32_t o[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t v = r[4 * (g & 3) + e];
                    o[e] = (h ? (v >> 16) : (v & 0xFFFFu)) >> out_shift;
                }
                const long long tg = t + 4 * g;
                if (vec && tg + 3 < nout) {
                    *reinterpret_cast<u32x4*>(orow + tg) = u32x4{o[0], o[1], o[2], o[3]};
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (tg + e < nout) orow[tg + e] = o[e];
                }
            }
        } else {
            uint8_t* nrow = reinterpret_cast<uint8_t*>(out) + (long long)orow_idx * out_stride;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const int h = g >> 2;
                uint32_t o[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t v = r[4 * (g & 3) + e];
                    o[e] = out_value(h ? (v >> 16) : (v & 0xFFFFu), out_shift, out_bytes);
                }
                const long long tg = t + 4 * g;
                if (nvec && tg + 3 < nout) {
                    if (out_bytes == 1) {
                        *reinterpret_cast<uint32_t*>(nrow + tg) = o[0] | (o[1] << 8) | (o[2] << 16) | (o[3] << 24);
                    } else {
                        *reinterpret_cast<uint32_t*>(nrow + 2 * tg) = o[0] | (o[1] << 16);
                        *reinterpret_cast<uint32_t*>(nrow + 2 * tg + 4) = o[2] | (o[3] << 16);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (tg + e < nout) {
                            if (out_bytes == 1) nrow[tg + e] = (uint8_t)o[e];
                            else reinterpret_cast<uint16_t*>(nrow)[tg + e] = (uint16_t)o[e];
                        }
                }
            }
        }
    }
}

template <int FMT, int NW, int DPW, int M, int CC, int PM>
__device__ __forceinline__ void tiled_item(const BeamDesc& b, int tile, int block, int group, uint32_t* lds)
{
    if constexpr (fmt_planes(FMT)) {
        static_assert(DPW == 1, "bit-plane shapes take one DM per wave");
        plane_body<NW, M, CC, PM, FMT == kFmtSeg>(b, tile, block, lds);
    } else {
        tile_body<FMT, NW, DPW, M, CC, PM>(b, tile, block, group, lds);
    }
}

template <int FMT, int NW, int DPW, int M, int CC, int PM>
__global__ __launch_bounds__(NW * 64) void k_tiled(BeamDesc b)
{
    extern __shared__ uint32_t lds_dyn[];
    const int n = b.ntiles * b.nblocks;
    const int logical = xcd_remap((int)blockIdx.x, n);
    int tile, block;
    if constexpr (FMT == kFmtSeg) {
        // DM-block-major: an XCD sweeps the tiles of its blocks in time
        // order, so the workgroups in flight on it read overlapping windows
        // (a block's window spans its delay spread in words, more than a
        // tile), and the eight XCDs sweep the scratch side by side.
        block = logical / b.ntiles;
        tile = logical - block * b.ntiles;
    } else {
        tile = logical / b.nblocks;
        block = logical % b.nblocks;
    }
    tiled_item<FMT, NW, DPW, M, CC, PM>(b, tile, block, (int)blockIdx.y, lds_dyn);
}

// ------------------------------------------------------------ untiled

template <int NBITS>
__device__ __forceinline__ uint32_t sample_at(const BeamDesc& b, long long r, int c)
{
    const uint8_t* row = row_ptr(b, r);
    if constexpr (NBITS == 8) return row[c];
    else return (row[c >> 2] >> (2 * (c & 3))) & 3u;
}

// With b.scrunch = s > 1, output t of a DM row sums, per channel, the s
// input samples that make up scrunched sample t + delay.
template <int NBITS>
__global__ __launch_bounds__(256) void k_untiled(BeamDesc b)
{
    const long long t = ((long long)blockIdx.x * 256 + threadIdx.x) * 4;
    if (t >= b.nout) return;
    const int s = b.scrunch;
    for (int d = blockIdx.y; d < b.ndm; d += gridDim.y) {
        const int32_t* dl = b.table + (size_t)d * b.nchans;
        uint32_t a[4] = {0u, 0u, 0u, 0u};
        for (int c = 0; c < b.nchans; ++c) {
            if (b.mask && b.mask[c] == 0) continue;
            const int off = dl[c];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < b.nout)
                    for (int i = 0; i < s; ++i)
                        a[e] += sample_at<NBITS>(b, (t + e + off) * s + i, c);
        }
        const int orow_idx = b.rowmap ? b.rowmap[d] : d;
        if (b.out_bytes == 4) {
            uint32_t* orow = b.out + (size_t)orow_idx * (size_t)b.out_stride;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < b.nout) orow[t + e] = a[e] >> b.out_shift;
        } else {
            uint8_t* nrow = reinterpret_cast<uint8_t*>(b.out) + (long long)orow_idx * b.out_stride;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < b.nout) {
                    const uint32_t v = out_value(a[e], b.out_shift, b.out_bytes);
                    if (b.out_bytes == 1) nrow[t + e] = (uint8_t)v;
                    else reinterpret_cast<uint16_t*>(nrow)[t + e] = (uint16_t)v;
                }
        }
    }
}

// Untiled pass over a channel-major scratch (grouped passes whose delay
// spread is too large for LDS): one thread per 4 outputs of one DM row of
// group blockIdx.z, reading scratch samples of format FMT straight from
// global memory.  table: [ngroups][ndm][nact] delays of the scratch rows.
template <int FMT>
__device__ __forceinline__ uint32_t xc_sample(const uint8_t* row, long long t)
{
    if constexpr (FMT == kFmtNib) return (row[t >> 1] >> (4 * (t & 1))) & 0xFu;
    else if constexpr (FMT == kFmtHalf) return reinterpret_cast<const uint16_t*>(row)[t];
    else return row[t];
}

template <int FMT>
__global__ __launch_bounds__(256) void k_untiled_xc(BeamDesc b)
{
    // outputs base + threadIdx.x + 256*e, e < 4: consecutive lanes read and
    // write consecutive samples
    const long long base = (long long)blockIdx.x * 1024 + threadIdx.x;
    if (base >= b.nout) return;
    const int g = blockIdx.z;
    const int ndm_here = g == b.ngroups - 1 ? b.ndm_last : b.ndm;
    const uint8_t* xc = b.xc + g * b.g_xc;
    for (int d = blockIdx.y; d < ndm_here; d += gridDim.y) {
        const int32_t* dl = b.table + ((size_t)g * b.ndm + d) * b.nact;
        const int32_t* rs = b.rowsel ? b.rowsel + ((size_t)g * b.ndm + d) * b.nact : nullptr;
        uint32_t a[4] = {0u, 0u, 0u, 0u};
        for (int k = 0; k < b.nact; ++k) {
            const uint8_t* row = xc + (long long)(rs ? rs[k] : k) * b.pitch;
            const long long off = dl[k];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (base + 256 * e < b.nout) a[e] += xc_sample<FMT>(row, base + 256 * e + off);
        }
        if (b.out_bytes == 4) {
            uint32_t* orow = b.out + g * b.g_out + (size_t)d * (size_t)b.out_stride;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (base + 256 * e < b.nout) orow[base + 256 * e] = a[e] >> b.out_shift;
        } else {
            uint8_t* nrow = reinterpret_cast<uint8_t*>(b.out) + g * b.g_out + (long long)d * b.out_stride;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (base + 256 * e < b.nout) {
                    const uint32_t v = out_value(a[e], b.out_shift, b.out_bytes);
                    if (b.out_bytes == 1) nrow[base + 256 * e] = (uint8_t)v;
                    else reinterpret_cast<uint16_t*>(nrow)[base + 256 * e] = (uint16_t)v;
                }
        }
    }
}

// ---------------------------------------------------------------- zero fill

// Zero [base + g*group_stride, + bytes) for g = blockIdx.y with 16-byte
// stores (a fill kernel rather than a memset, so the launch can sit in a
// captured graph).
__global__ __launch_bounds__(256) void k_zero(uint8_t* base, long long group_stride, long long n16)
{
    u32x4* p = reinterpret_cast<u32x4*>(base + (long long)blockIdx.y * group_stride);
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n16; i += (long long)gridDim.x * 256)
        p[i] = u32x4{0u, 0u, 0u, 0u};
}

// ---------------------------------------------------------------- shapes

// (scratch format, waves, DMs per wave, words per lane, channels per chunk,
// pieces, multi): a tile is 64*words scratch words long (2048*words outputs
// of bit planes, 512*words 2-bit nibble, 256*words byte or 128*words 16-bit
// samples); a staged channel row holds at most 64*pieces 16-byte pieces;
// shapes marked multi are also compiled into multi-beam kernel `multi` (which
// allocates registers for the largest of its shapes).  The first shape of
// each format is its default; the segmented bit planes are chosen by tile
// config (sample format 5) or by the tuner.
#define DEDISP_SHAPES(X)                   \
    X(kFmtPlane, 16, 1, 3, 32, 1, 2)       \
    X(kFmtPlane, 8, 1, 3, 32, 1, 1)        \
    X(kFmtPlane, 16, 1, 1, 32, 1, 0)       \
    X(kFmtPlane, 8, 1, 1, 32, 1, 0)        \
    X(kFmtPlane, 16, 1, 3, 64, 1, 0)       \
    X(kFmtSeg, 16, 1, 3, 32, 2, 3)         \
    X(kFmtSeg, 16, 1, 1, 32, 2, 0)         \
    X(kFmtNib, 8, 2, 3, 32, 2, 1)          \
    X(kFmtNib, 8, 2, 3, 16, 4, 1)          \
    X(kFmtNib, 8, 2, 1, 32, 2, 1)          \
    X(kFmtNib, 8, 4, 3, 32, 2, 0)          \
    X(kFmtNib, 8, 2, 5, 32, 2, 0)          \
    X(kFmtNib, 8, 4, 3, 16, 4, 0)          \
    X(kFmtNib, 16, 2, 3, 64, 2, 0)         \
    X(kFmtNib, 16, 1, 5, 64, 2, 2)         \
    X(kFmtNib, 16, 1, 5, 32, 2, 2)         \
    X(kFmtNib, 8, 1, 5, 32, 2, 0)          \
    X(kFmtByte, 8, 2, 5, 32, 2, 1)         \
    X(kFmtByte, 8, 2, 3, 16, 4, 1)         \
    X(kFmtByte, 8, 4, 3, 16, 4, 0)         \
    X(kFmtByte, 8, 4, 3, 32, 2, 0)         \
    X(kFmtByte, 8, 4, 5, 32, 2, 0)         \
    X(kFmtByte, 8, 2, 5, 64, 2, 0)         \
    X(kFmtByte, 16, 2, 5, 64, 2, 2)        \
    X(kFmtByte, 4, 4, 5, 32, 2, 0)         \
    X(kFmtByteS, 8, 2, 3, 32, 2, 0)        \
    X(kFmtByteS, 8, 2, 3, 16, 4, 0)        \
    X(kFmtByteS, 16, 1, 5, 64, 2, 0)       \
    X(kFmtByteS, 8, 2, 5, 32, 2, 0)        \
    X(kFmtHalf, 8, 2, 3, 32, 2, 0)         \
    X(kFmtHalf, 8, 2, 3, 16, 4, 0)         \
    X(kFmtHalf, 16, 1, 5, 64, 2, 0)        \
    X(kFmtHalf, 16, 2, 3, 32, 2, 0)        \
    X(kFmtHalf, 8, 4, 3, 32, 2, 0)         \
    X(kFmtHalf, 8, 2, 5, 32, 2, 0)

struct ShapeEntry {
    Shape s;
    const void* fn;
};

#define DEDISP_ENTRY(FMT, NW, DPW, M, CC, PM, MULTI) \
    {Shape{0, FMT, NW, DPW, M, CC, PM, MULTI}, reinterpret_cast<const void*>(&k_tiled<FMT, NW, DPW, M, CC, PM>)},

const ShapeEntry kShapes[] = {
    DEDISP_SHAPES(DEDISP_ENTRY)
    {Shape{1, 2, 4, 1, 1, 0, 0, 0}, reinterpret_cast<const void*>(&k_untiled<2>)},
    {Shape{1, 8, 4, 1, 1, 0, 0, 0}, reinterpret_cast<const void*>(&k_untiled<8>)},
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// Multi-beam kernels: class c holds the shapes marked multi = c, all with
// multi_waves(c) waves.
template <int CLASS, int FMT, int NW, int DPW, int M, int CC, int PM, int MULTI>
__device__ __forceinline__ bool run_if(int shape_id, int want, const BeamDesc& b, int tile,
                                       int block, uint32_t* lds)
{
    if constexpr (MULTI == CLASS) {
        static_assert(NW == multi_waves(CLASS), "multi-beam shapes of a class share one workgroup size");
        if (shape_id == want) {
            tiled_item<FMT, NW, DPW, M, CC, PM>(b, tile, block, 0, lds);
            return true;
        }
    }
    return false;
}

// Dispatch one work item to its beam's shape.  Beam b owns the items
// [work_begin, work_begin + span) with span = ntiles*nblocks rounded up to a
// multiple of 8 (work_begin is a multiple of 8), so the XCD remap below
// applies within each beam: all eight XCDs sweep one beam at a time, each a
// contiguous range of its (tile, DM block) items, as in a single-beam
// launch.  Items past ntiles*nblocks are padding and return at once.
template <int CLASS>
__device__ __forceinline__ void run_item(const DescBlock& blk, int nbeams, int item, uint32_t* lds)
{
    int bi = 0;
    while (bi + 1 < nbeams && blk.d[bi + 1].work_begin <= item) ++bi;
    bi = wave_uniform(bi);
    const BeamDesc& b = blk.d[bi];
    const int nreal = b.ntiles * b.nblocks;
    const int span = (nreal + 7) & ~7;
    const int local = xcd_remap(item - (int)b.work_begin, span);
    if (local >= nreal) return;
    // the segmented bit planes run DM-block-major, as in k_tiled
    const bool bmajor = wave_uniform(b.xc_fmt) == kFmtSeg;
    const int tile = bmajor ? local % b.ntiles : local / b.nblocks;
    const int block = bmajor ? local / b.ntiles : local - tile * b.nblocks;
    int id = 0;
    bool done = false;
#define DEDISP_RUN(FMT, NW, DPW, M, CC, PM, MULTI) \
    if (!done) done = run_if<CLASS, FMT, NW, DPW, M, CC, PM, MULTI>(b.shape, id, b, tile, block, lds); \
    ++id;
    DEDISP_SHAPES(DEDISP_RUN)
#undef DEDISP_RUN
    (void)done;
}

// Multi-beam launch, one workgroup per work item of every beam (the
// hardware dispatcher balances the uneven items as workgroups finish).
template <int CLASS>
__global__ __launch_bounds__(multi_waves(CLASS) * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_multi(
    DescBlock blk, int nbeams, int total)
{
    extern __shared__ uint32_t lds_dyn[];
    run_item<CLASS>(blk, nbeams, (int)blockIdx.x, lds_dyn);
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

hipError_t launch_unpack(const BeamDesc& d, int nbits, int fmt, hipStream_t st)
{
    if (d.scrunch > 1) return launch_scrunch(d, nbits, fmt, st);
    BeamDesc arg = d;
    arg.xc_fmt = fmt;
    void* args[] = {&arg};
    const long long gx = unpack_grid_x(arg);
    const long long gy = unpack_grid_y(arg);
    if (gx <= 0 || gx > 0x7fffffffLL || gy > 65535) return hipErrorInvalidValue;
    if ((nbits == 2) != (fmt == kFmtNib || fmt_planes(fmt))) return hipErrorInvalidValue;
    if (fmt_planes(fmt) && (d.nchans % 16 || d.row_bytes % 4)) return hipErrorInvalidValue;
    if (fmt == kFmtSeg) {
        if (d.pitch % (4 * kSegTurnWaves) || d.nout <= 0) return hipErrorInvalidValue;
        return hipLaunchKernel(reinterpret_cast<const void*>(&k_unpack_seg),
                               dim3((unsigned)(d.pitch / (4 * kSegTurnWaves)), (unsigned)gy),
                               dim3(64 * kSegTurnWaves), args, 0, st);
    }
    const void* fn = fmt == kFmtPlane ? reinterpret_cast<const void*>(&k_unpack_planes)
                     : nbits == 2     ? reinterpret_cast<const void*>(&k_unpack<2>)
                                      : reinterpret_cast<const void*>(&k_unpack<8>);
    return hipLaunchKernel(fn, dim3((unsigned)gx, (unsigned)gy), dim3(256), args, 0, st);
}

hipError_t launch_unpack_multi(const DescBlock& blk, int nbeams, hipStream_t st)
{
    if (nbeams <= 0 || nbeams > kMaxBatchDescs) return hipErrorInvalidValue;
    long long units = 0;
    for (int i = 0; i < nbeams; ++i) {
        const BeamDesc& b = blk.d[i];
        if (b.scrunch != 1 || (b.in_nbits != 2 && b.in_nbits != 8) || b.nsamps <= 0 || b.nchans <= 0)
            return hipErrorInvalidValue;
        if ((b.in_nbits == 2) != (b.xc_fmt == kFmtNib || fmt_planes(b.xc_fmt))) return hipErrorInvalidValue;
        if (fmt_planes(b.xc_fmt) && (b.nchans % 16 || b.row_bytes % 4)) return hipErrorInvalidValue;
        if (b.xc_fmt == kFmtSeg && (b.pitch % 16 || b.nout <= 0)) return hipErrorInvalidValue;
        units += unpack_grid_x(b) * unpack_grid_y(b);
    }
    if (units > 0x7fffffffLL) return hipErrorInvalidValue;
    DescBlock a0 = blk;
    int a1 = nbeams;
    void* args[] = {&a0, &a1};
    return hipLaunchKernel(reinterpret_cast<const void*>(&k_unpack_multi), dim3((unsigned)units), dim3(256),
                           args, 0, st);
}

hipError_t launch_tiled(const BeamDesc& d, const Shape& s, int lds_bytes, hipStream_t st)
{
    int idx = -1;
    for (int i = 0; i < kNumShapes; ++i) {
        const Shape& k = kShapes[i].s;
        if (k.kind == 0 && k.fmt == s.fmt && k.waves == s.waves && k.dpw == s.dpw &&
            k.m == s.m && k.cc == s.cc && k.pi == s.pi) {
            idx = i;
            break;
        }
    }
    if (idx < 0) return hipErrorInvalidValue;
    hipError_t e = ensure_lds_attr(idx, kShapes[idx].fn);
    if (e != hipSuccess) return e;
    const long long n = (long long)d.ntiles * d.nblocks;
    if (n <= 0 || n > 0x7fffffffLL || d.ngroups < 1 || d.ngroups > 65535) return hipErrorInvalidValue;
    BeamDesc arg = d;
    void* args[] = {&arg};
    return hipLaunchKernel(kShapes[idx].fn, dim3((unsigned)n, (unsigned)d.ngroups), dim3(s.waves * 64),
                           args, (size_t)lds_bytes, st);
}

hipError_t launch_zero(uint8_t* base, long long group_stride, long long bytes, int ngroups,
                       hipStream_t st)
{
    if (bytes <= 0 || ngroups <= 0) return hipSuccess;
    if ((bytes & 15) || (reinterpret_cast<uintptr_t>(base) & 15) || (group_stride & 15) ||
        ngroups > 65535)
        return hipErrorInvalidValue;
    const long long n16 = bytes / 16;
    const long long nb = (n16 + 255) / 256;
    const long long gx = nb < 4096 ? nb : 4096;
    void* args[] = {&base, &group_stride, const_cast<long long*>(&n16)};
    return hipLaunchKernel(reinterpret_cast<const void*>(&k_zero), dim3((unsigned)gx, (unsigned)ngroups),
                           dim3(256), args, 0, st);
}

hipError_t launch_untiled_xc(const BeamDesc& d, int fmt, hipStream_t st)
{
    const long long gx = (d.nout + 1023) / 1024;
    if (gx <= 0 || gx > 0x7fffffffLL || d.ngroups < 1 || d.ngroups > 65535) return hipErrorInvalidValue;
    const unsigned gy = (unsigned)(d.ndm < 65535 ? d.ndm : 65535);
    BeamDesc arg = d;
    void* args[] = {&arg};
    const void* fn = fmt == kFmtNib    ? reinterpret_cast<const void*>(&k_untiled_xc<kFmtNib>)
                     : fmt == kFmtHalf ? reinterpret_cast<const void*>(&k_untiled_xc<kFmtHalf>)
                                       : reinterpret_cast<const void*>(&k_untiled_xc<kFmtByte>);
    return hipLaunchKernel(fn, dim3((unsigned)gx, gy, (unsigned)d.ngroups), dim3(256), args, 0, st);
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

hipError_t launch_multi(const DescBlock& blk, int nbeams, int total_work, int lds_bytes, int cls,
                        hipStream_t st)
{
    if (nbeams <= 0 || nbeams > kMaxBatchDescs || total_work <= 0 || cls < 1 || cls > kMultiClasses)
        return hipErrorInvalidValue;
    const void* fn = cls == 1   ? reinterpret_cast<const void*>(&k_multi<1>)
                     : cls == 2 ? reinterpret_cast<const void*>(&k_multi<2>)
                                : reinterpret_cast<const void*>(&k_multi<3>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess) return e;
    DescBlock a0 = blk;
    int a1 = nbeams;
    int a2 = total_work;
    void* args[] = {&a0, &a1, &a2};
    return hipLaunchKernel(fn, dim3(total_work), dim3(multi_waves(cls) * 64), args, (size_t)lds_bytes, st);
}

}  // namespace dedisp
