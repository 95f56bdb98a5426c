// Internal interface between the host library (dedisp_api.cpp) and the
// gfx950 kernels (dedisp_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dedisp {

// One beam (or one stream push) as the kernels see it.  The input is a
// virtual concatenation of two row segments so that a stream's resident
// history and a new chunk can be summed without copying them together:
// rows [0, n0) are at in0, rows [n0, nsamps) at in1.
struct BeamDesc {
    const uint8_t* in0;
    const uint8_t* in1;
    long long n0;
    long long nsamps;
    long long nout;           // nsamps - max_delay
    uint32_t* out;
    long long out_stride;     // elements between DM rows
    uint8_t* xc;              // channel-major bytes written by the unpack kernel
    long long pitch;          // bytes between channel rows of xc (multiple of 16)
    const uint32_t* rel;      // [nblocks*DB][nchans/2] window offsets of channel pairs (16+16 bits)
    const int32_t* base;      // [nblocks][nchans] window start (multiple of 16)
    const int32_t* table;     // [ndm][nchans] full delay table (untiled kernel)
    const int32_t* chanmap;   // [nchans] scratch row of each channel, -1 = killed (NULL = identity)
    const int32_t* mask;      // [nchans] 0/1 kill mask for the untiled kernel (NULL = all on)
    int nact;                 // scratch rows the tiled kernel sums (live channels, padded to a multiple of 8)
    int pad_row;              // first of the scratch rows [pad_row, nact) the corner turn zero-fills, or -1
    int nchans;
    int row_bytes;
    int ndm;
    int nblocks;              // ceil(ndm / DB)
    int ntiles;               // ceil(nout / tile length)
    int rw;                   // LDS row length in 32-bit words
    int flush_every;          // chunks between packed-lane flushes
    int shape;                // index into the compiled shape list
    int pad_;
    long long work_begin;     // first global work item of this beam
};

// A compiled kernel shape.
struct Shape {
    int kind;       // 0 = LDS-tiled, 1 = untiled
    int nbits;
    int waves;
    int dpw;        // DMs per wave
    int m;          // 32-bit words per lane (4 samples each)
    int cc;         // channels staged per chunk
    int pi;         // 16-byte pieces per lane per staged row: row <= 64*pi pieces
    int multi;      // also compiled into the multi-beam kernels
};

// Shapes compiled into the library (index = shape id).
int shape_count();
const Shape& shape_at(int i);

// Largest dynamic LDS a workgroup may use on this device (bytes).
constexpr int kMaxLdsBytes = 160 * 1024;

// Enqueue the corner turn (time-major packed -> channel-major bytes in d.xc).
hipError_t launch_unpack(const BeamDesc& d, int nbits, hipStream_t st);

// Enqueue the transform of one beam with the given shape.
hipError_t launch_tiled(const BeamDesc& d, const Shape& s, int lds_bytes, hipStream_t st);
hipError_t launch_untiled(const BeamDesc& d, int nbits, hipStream_t st);

// Multi-beam launches over up to kMaxBatchDescs beams whose descriptors
// travel in the kernel arguments (work_begin = prefix sum of ntiles*nblocks,
// each rounded up to a multiple of 8).  Every
// beam must use a shape marked multi; the LDS size is the largest any
// beam needs.
constexpr int kMultiWaves = 8;
constexpr int kMaxBatchDescs = 16;
struct DescBlock {
    BeamDesc d[kMaxBatchDescs];
};
// One workgroup per work item of every beam in one launch.
hipError_t launch_multi(const DescBlock& blk, int nbeams, int total_work, int lds_bytes,
                        hipStream_t st);
// Grid sized to the machine, workgroups looping over the items.
hipError_t launch_persistent(const DescBlock& blk, int nbeams, int total_work, int lds_bytes,
                             int grid, hipStream_t st);
int persistent_max_grid(int lds_bytes);

}  // namespace dedisp
