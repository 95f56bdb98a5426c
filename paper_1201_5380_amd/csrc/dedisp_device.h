// Device helpers shared by the kernel sources (internal; not installed).
#pragma once

#include "dedisp_internal.h"

namespace dedisp {
namespace {

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Native 4 x 32-bit vector (one 16-byte load or store); unlike HIP's uint4
// struct it stays in registers when held in arrays.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ long long wave_uniform64(long long x)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(x & 0xffffffffLL));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(x >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T* wave_uniform_ptr(T* p)
{
    return reinterpret_cast<T*>(wave_uniform64(reinterpret_cast<long long>(p)));
}

// A load through the global address space (global_load, counted by the
// vector-memory counter only).  Pointers taken from a descriptor are
// generic, and a generic (flat) load also counts against the counter LDS
// reads share, so every LDS wait issued while it is in flight would wait for
// it too -- a prefetch of the next chunk would stall the current one.
template <typename T>
__device__ __forceinline__ T gload(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ int lane_value(int v, int lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

// An output value at the descriptor's width: shifted right, then saturated.
__device__ __forceinline__ uint32_t out_value(uint32_t v, int shift, int bytes)
{
    v >>= shift;
    if (bytes == 1) return v < 0xFFu ? v : 0xFFu;
    if (bytes == 2) return v < 0xFFFFu ? v : 0xFFFFu;
    return v;
}

// Address of input row r in the two-segment virtual input.
__device__ __forceinline__ const uint8_t* row_ptr(const BeamDesc& b, long long r)
{
    return r < b.n0 ? b.in0 + r * (long long)b.row_bytes
                    : b.in1 + (r - b.n0) * (long long)b.row_bytes;
}

// Map the hardware workgroup index to a logical one so that the workgroups
// dispatched to one XCD (round-robin over 8 XCDs) get a contiguous range of
// logical indices, i.e. all DM blocks of the same few time tiles, which read
// overlapping input windows through that XCD's L2.
__device__ __forceinline__ int xcd_remap(int i, int n)
{
    constexpr int kXcds = 8;
    const int per = n / kXcds, rem = n % kXcds;
    const int x = i % kXcds, k = i / kXcds;
    return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

}  // namespace
}  // namespace dedisp
