// Internal interface between the host library (dedisp_api.cpp) and the
// gfx950 kernels (dedisp_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dedisp {

// Sample format of the channel-major scratch the LDS-tiled kernel sums.
enum Fmt : int {
    kFmtNib = 0,     // 2-bit codes, two per byte (eight per 32-bit word)
    kFmtByte = 1,    // 8-bit codes, one per byte
    kFmtByteS = 2,   // byte values at most 127 (time-scrunched 2-bit codes)
    kFmtHalf = 3,    // 16-bit values at most 32767 (time-scrunched 8-bit, or heavily scrunched 2-bit, codes)
    kFmtPlane = 4,   // 2-bit codes as two bit planes: scratch row 2k + p holds bit p of row k's
                     // codes, 32 samples per 32-bit word (sample 32w + i at bit i of word w)
    kFmtSeg = 5,     // two bit planes of 32 interleaved time segments: the outputs are cut
                     // into 32 segments of S = seg_len(nout) samples and bit i of word j of
                     // row 2k + p holds bit p of sample j + S*i, so a delay of n samples is
                     // a shift of n whole words
};
// bytes per sample of one scratch row = num / den
constexpr int fmt_bytes_num(int fmt) { return fmt == kFmtHalf ? 2 : 1; }
constexpr int fmt_bytes_den(int fmt) { return fmt == kFmtNib ? 2 : fmt == kFmtPlane || fmt == kFmtSeg ? 8 : 1; }
constexpr int fmt_samples_per_word(int fmt) { return 4 * fmt_bytes_den(fmt) / fmt_bytes_num(fmt); }
constexpr bool fmt_planes(int fmt) { return fmt == kFmtPlane || fmt == kFmtSeg; }
// scratch rows per channel row and channel rows per unit of the summation
constexpr int fmt_rows(int fmt) { return fmt_planes(fmt) ? 2 : 1; }
constexpr int fmt_chan_unit(int fmt) { return fmt_planes(fmt) ? 32 : 8; }
// Segment length of the interleaved bit-plane format for nout outputs, and
// the number of words of its scratch rows (every segment's outputs and the
// max_delay samples after the last, plus a staged window of rw words past a
// whole number of 512-word tiles).
__host__ __device__ constexpr long long seg_len(long long nout) { return (nout + 31) / 32; }
constexpr long long seg_row_words(long long nout, long long max_delay, int rw)
{
    return (seg_len(nout) + 511) / 512 * 512 + max_delay + rw + 64;
}

// Bit-plane sums: bit levels kept per sample (sums of up to 3 * 1365 two-bit
// codes) and the LDS row length of one staged plane (32-bit words; plane 1
// of a channel sits this many words after plane 0).
constexpr int kPlaneLevels = 12;
constexpr int kPlaneMaxChans = ((1 << kPlaneLevels) - 1) / 3;
constexpr int kPlaneRowWords = 224;
// LDS row length of one staged plane of the interleaved format: a tile's 64M
// words plus the spread of the DM block's delays, in whole words.
constexpr int kSegRowWords = 512;
// The segmented layout writes seg_len(nout) + max_delay words per plane row
// where the plain planes write (nout + max_delay) / 32, so its corner turn
// costs more than its sum saves unless nout is several times max_delay
// (break-even near 6 on the survey band): below this many max_delays of
// outputs a launch takes the plain bit planes.
constexpr long long kSegMinOutPerDelay = 8;

// One beam (or one stream push) as the kernels see it.  The input is a
// virtual concatenation of two row segments so that a stream's resident
// history and a new chunk can be summed without copying them together:
// rows [0, n0) are at in0, rows [n0, nsamps) at in1.
struct BeamDesc {
    const uint8_t* in0;
    const uint8_t* in1;
    long long n0;
    long long nsamps;
    long long nout;           // outputs per DM row: nsamps / scrunch - max_delay
    uint32_t* out;
    long long out_stride;     // between DM rows: elements (out_bytes 4) or bytes (1, 2)
    uint8_t* xc;              // channel-major scratch written by the unpack or scrunch kernel
    long long pitch;          // bytes between channel rows of xc (multiple of 16)
    const uint32_t* rel;      // [nblocks*DB][nchans/2] window offsets of channel pairs (16+16 bits)
    const int32_t* base;      // [nblocks][nchans] window start (multiple of 16 bytes of scratch);
                              // kFmtSeg: [nblocks][nchans][2] (start, span)
    const int32_t* table;     // [ndm][nchans] full delay table (untiled kernel)
    const int32_t* chanmap;   // [nchans] scratch row of each channel, -1 = killed (NULL = identity)
    const int32_t* mask;      // [nchans] 0/1 kill mask for the untiled kernel (NULL = all on)
    const int32_t* rowmap;    // [ndm] output row of each DM row (NULL = identity)
    const int32_t* rowsel;    // untiled scratch pass: [ngroups][ndm][nact] scratch row of each
                              // term (NULL = term k reads row k)
    int nact;                 // scratch rows the tiled kernel sums (live channels, padded to a multiple of 8)
    int pad_row;              // first of the scratch rows [pad_row, nact) the corner turn zero-fills, or -1
    int nchans;
    int row_bytes;
    int ndm;
    int nblocks;              // ceil(ndm / DB)
    int ntiles;               // ceil(nout / tile length)
    int rw;                   // LDS row length in 32-bit words
    int flush_every;          // channels between packed-lane flushes (small-value formats)
    int shape;                // index into the compiled shape list
    int scrunch;              // samples summed per scratch sample (1 = none)
    // Grouped launches (sub-band dedispersion): gridDim.y = ngroups groups,
    // group g reading its scratch, window tables and writing its outputs at
    // the offsets below times g.  ngroups = 1 and offsets 0 otherwise.
    int ngroups;
    int ndm_last;             // DM rows of the last group (the others have ndm)
    int out_bytes;            // 4: uint32 outputs; 1 or 2: uint8 / uint16 outputs or narrow sums
    int out_shift;            // outputs are min(sum >> out_shift, largest value of out_bytes)
    int dbuf;                 // tiled kernel: two LDS chunk buffers (one barrier per chunk)
    int in_nbits;             // input bit depth (multi-beam corner turn)
    int xc_fmt;               // scratch format the corner turn writes (Fmt)
    long long g_xc;           // bytes
    long long g_rel;          // elements of rel
    long long g_base;         // elements of base
    long long g_out;          // elements (out_bytes 4) or bytes (1, 2)
    long long work_begin;     // first global work item of this beam
};

// A compiled kernel shape.
struct Shape {
    int kind;       // 0 = LDS-tiled, 1 = untiled
    int fmt;        // scratch sample format (tiled) or input bit depth (untiled)
    int waves;
    int dpw;        // DMs per wave
    int m;          // 32-bit scratch words per lane
    int cc;         // channels staged per chunk
    int pi;         // 16-byte pieces per lane per staged row: row <= 64*pi pieces
    int multi;      // multi-beam kernel class it is also compiled into (0 = none)
};

// Shapes compiled into the library (index = shape id).
int shape_count();
const Shape& shape_at(int i);

// Largest dynamic LDS a workgroup may use on this device (bytes).
constexpr int kMaxLdsBytes = 160 * 1024;

// Enqueue the corner turn (time-major packed -> channel-major scratch of
// format fmt in d.xc), summing d.scrunch consecutive samples when above 1.
hipError_t launch_unpack(const BeamDesc& d, int nbits, int fmt, hipStream_t st);
// The scrunching corner turn alone (d.scrunch > 1; fmt = kFmtByteS for 2-bit
// s <= 8, else kFmtHalf).
hipError_t launch_scrunch(const BeamDesc& d, int nbits, int fmt, hipStream_t st);

// Stage 1 of the piecewise linear tree: k = log2(nsub) tree steps (Theta/Phi)
// for each of the npairs (sub-band n, pass p) pairs in pairs[2y], pairs[2y+1]
// (device memory), over the channel-major scratch d.xc (format fmt, every
// channel's row kept) with channel j of the sub-band read p*j samples later;
// pair y's tree DM d' is written as row y*nsub + d' of out (pitch out_pitch
// bytes, 16-byte aligned) for t < len1, one byte (ob = 1: 2-bit input,
// nsub <= 64) or 16 bits (ob = 2) per sample.  The scratch rows must hold
// len1 + tile + nsub + (largest p)(nsub - 1) + 8 samples.
hipError_t launch_tree(const BeamDesc& d, int fmt, int nsub, int ob, const int32_t* pairs, int npairs,
                       uint8_t* out, long long out_pitch, long long len1, hipStream_t st);
// Samples per time tile of the longest stage-1 tile (the scratch rows need this many
// samples of margin past nsamps).
int tree_tile(int nsub);

// Stage 2 of the piecewise linear tree: out[d][t] = sum over the d.nact
// sub-bands n of S[d.rowsel[d*nact + n]][t + d.table[d*nact + n]] for
// t < d.nout, S the stage-1 rows in d.xc (ob bytes per sample, pitch d.pitch
// bytes, rows readable 20 bytes past the last delayed output).  flush =
// terms summed in 16-bit lanes between 32-bit flushes (flush * largest row
// value < 2^16).  d.out / out_bytes / out_shift / out_stride as for the
// other kernels.
// trials (device, ntrials entries) restricts it to those trials (NULL: all).
hipError_t launch_tree_combine(const BeamDesc& d, int ob, int flush, const int32_t* trials, int ntrials,
                               hipStream_t st);

// Stage 2 with LDS staging, byte rows only: for the nblocks trial blocks
// blocks[] (block k = trials k*kTreeBlock .. +kTreeBlock-1), a workgroup
// stages, per sub-band n, rows stage[.][n].lo .. + span, each as wdw (a
// multiple of 4) dwords at LDS dword lds + (row - lo) wdw, segmented within
// the time tile [t0, t0 + kTreeTile): with P = kTreeTile / 4, byte i of
// staged dword k is sample t0 + dmin4 + k + i P (dmin4 a multiple of 4).
// Every trial d of the block then sums, over n, byte i of the LDS dword at
// byte offset off[d][n] + 4 u for its output t0 + u + i P (u < P).  rcp =
// ceil(2^32 / (wdw / 4)).  lds_dwords = LDS per workgroup; at most 128
// sub-bands.  pair: every row value is below 128.  d as for
// launch_tree_combine (32-bit sums: no flush interval).
constexpr int kTreeBlock = 32;
constexpr int kTreeTile = 512;
struct TreeStage {
    int lo, span, dmin4, wdw, lds;
    uint32_t rcp;          // ceil(2^32 / (wdw / 4)): i / (wdw / 4) = umulhi(i, rcp) for i < 2^16
    int pad_[2];
};
hipError_t launch_tree_combine_lds(const BeamDesc& d, const int32_t* blocks, int nblocks, const TreeStage* stage,
                                   const int32_t* off, int lds_dwords, bool pair, hipStream_t st);

// Zero `bytes` (a multiple of 16) at base + g*group_stride for g < ngroups.
hipError_t launch_zero(uint8_t* base, long long group_stride, long long bytes, int ngroups,
                       hipStream_t st);

// Enqueue the transform of one beam with the given shape.
hipError_t launch_tiled(const BeamDesc& d, const Shape& s, int lds_bytes, hipStream_t st);
hipError_t launch_untiled(const BeamDesc& d, int nbits, hipStream_t st);
// Untiled pass over the channel-major scratch of format fmt (grouped passes
// of sub-band dedispersion whose delay spread does not fit in LDS);
// d.table is [ngroups][ndm][nact].
hipError_t launch_untiled_xc(const BeamDesc& d, int fmt, hipStream_t st);

// Multi-beam launches over up to kMaxBatchDescs beams whose descriptors
// travel in the kernel arguments (work_begin = prefix sum of ntiles*nblocks,
// each rounded up to a multiple of 8).  Every beam of a launch must use a
// shape of the launch's multi-beam class (shape.multi): class 1 holds 8-wave
// shapes, class 2 the 16-wave ones, class 3 the 16-wave segmented bit-plane
// shape (in a kernel of its own, so its registers do not add to the others');
// the LDS size is the largest any beam
// needs.
constexpr int kMultiWaves = 8;
constexpr int kMultiClasses = 3;
__host__ __device__ constexpr int multi_waves(int cls) { return cls == 1 ? 8 : 16; }
constexpr int kMaxBatchDescs = 16;
struct DescBlock {
    BeamDesc d[kMaxBatchDescs];
};
static_assert(sizeof(DescBlock) + 16 <= 4096, "multi-beam descriptors must fit the kernel arguments");

// Corner turns (no scrunching) of blk.d[0 .. nbeams) in one launch, each as
// launch_unpack with d.in_nbits as the bit depth.
hipError_t launch_unpack_multi(const DescBlock& blk, int nbeams, hipStream_t st);
// One workgroup per work item of every beam in one launch (cls = the
// beams' multi-beam class).
hipError_t launch_multi(const DescBlock& blk, int nbeams, int total_work, int lds_bytes, int cls,
                        hipStream_t st);

}  // namespace dedisp
