// Piecewise linear tree dedispersion (Section 3): stage 1 applies the
// tree's steps within every sub-band of the channel-major scratch, stage 2
// combines one tree row per sub-band for every trial.
#include <type_traits>

#include "dedisp_device.h"

namespace dedisp {

namespace {

// ---------------------------------------------------------------- tree

// Stage 1 of the piecewise linear tree (Section 3).  Workgroup (tile,
// (sub-band n, pass p) pair) loads the sub-band's nsub scratch rows -- any
// scratch format: 2-bit nibbles, bytes, scrunched byte or 16-bit sums; row j
// read p*j samples later (the pass's imposed delay), killed channels as
// zeros -- for samples [t0, t0 + T + nsub) into LDS as 16-bit values, two
// per 32-bit word, and
// applies the tree's steps i = 0 .. k-1 out of place (double buffer):
//   B[2v][t]   = A[Phi(r, 2v)][t] + A[Phi(r, 2v+1)][t + Theta(i, 2v)]
//   B[2v+1][t] = A[Phi(r, 2v)][t] + A[Phi(r, 2v+1)][t + Theta(i, 2v+1)]
// with r = 2^i, Theta(i, v) = ((v mod 2^{i+1}) + 1) / 2 and
// Phi(r, v) = (v mod 2) r + v/2 + (v/(2r)) r.  Row d' of the result is the
// sub-band at tree DM d', written as 16-bit values for t < len1 (byte rows
// take k_tree_b below).  Sums stay below 2^16 (nsub codes), so a 32-bit add
// sums two samples without a carry between them.
//
// Theta(i, 2v+1) = Theta(i, 2v) + 1, so both outputs of a pair read the
// same three samples of the second row: one aligned word pair q, q+1 and a
// 16-bit realignment (v_alignbit) give both shifted words.  Every step
// computes all LW words of every row; words past a step's valid length only
// ever feed words past the next step's valid length (each step reads at t
// and above), so the T samples stored at the end are exact.  Rows carry
// RS >= LW + nsub/4 words so the shifted reads stay inside the row.
__host__ __device__ constexpr int tree_tile_len(int nsub) { return 8192 / nsub; }
__host__ __device__ constexpr int tree_row_words(int nsub)
{
    return ((tree_tile_len(nsub) + nsub) / 2 + nsub / 4 + 1 + 3) / 4 * 4;
}

__device__ __forceinline__ int tree_theta(int i, int v) { return ((v & ((2 << i) - 1)) + 1) >> 1; }
// Phi(2^i, v), with v / 2^{i+1} taken as a shift
__device__ __forceinline__ int tree_phi(int i, int v) { return ((v & 1) << i) + (v >> 1) + ((v >> (i + 1)) << i); }

template <int FMT, int NSUB>
__global__ __launch_bounds__(256) void k_tree(BeamDesc b, const int32_t* pairs, uint8_t* out, long long out_pitch,
                                              long long len1)
{
    constexpr int T = tree_tile_len(NSUB);
    constexpr int L = T + NSUB;                    // samples loaded per row (>= T + NSUB - 1)
    constexpr int LW = L / 2;                      // words computed per row
    constexpr int RS = tree_row_words(NSUB);       // LDS row stride in words
    constexpr int K = NSUB == 8 ? 3 : NSUB == 16 ? 4 : NSUB == 32 ? 5 : NSUB == 64 ? 6 : 7;
    static_assert((1 << K) == NSUB, "sub-band width must be a power of two");
    static_assert(RS >= LW + NSUB / 4 && RS % 4 == 0, "row stride covers the shifted reads");
    extern __shared__ __align__(16) uint32_t tw[];             // [2][NSUB][RS]
    uint32_t* A = tw;
    uint32_t* B = tw + NSUB * RS;
    const long long t0 = (long long)blockIdx.x * T;
    const int y = blockIdx.y;
    const int n = pairs[2 * y], pass = pairs[2 * y + 1];
    // load: 32-bit scratch words, spread to two 16-bit samples per LDS word;
    // channel j of the sub-band starts pass*j samples later (the imposed
    // delay), realigned from two consecutive words
    constexpr int SPW = fmt_samples_per_word(FMT);
    constexpr int WPR = L / SPW;                   // scratch words per row
    static_assert(L % SPW == 0, "whole words per row");
    // every load (and kill-mask flag) is issued before the first
    // realignment, so a thread waits for global memory once; a thread's last
    // index may run past the rows (clamped: loaded, not stored)
    constexpr int NLD = (NSUB * WPR + 255) / 256;
    int jj[NLD], ww[NLD], keep[NLD];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int it = threadIdx.x + 256 * k;
        const int ic = it < NSUB * WPR ? it : NSUB * WPR - 1;
        jj[k] = ic / WPR;
        ww[k] = ic % WPR;
    }
    if (b.mask) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) keep[k] = b.mask[n * NSUB + jj[k]];
    } else {
#pragma unroll
        for (int k = 0; k < NLD; ++k) keep[k] = 1;
    }
    u32x2 raw[NLD];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const uint32_t* row = reinterpret_cast<const uint32_t*>(b.xc + (long long)(n * NSUB + jj[k]) * b.pitch);
        __builtin_memcpy(&raw[k], row + t0 / SPW + (pass * jj[k]) / SPW + ww[k], sizeof(u32x2));
    }
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int it = threadIdx.x + 256 * k;
        if (it >= NSUB * WPR) break;
        const int shift = pass * jj[k];
        // killed channels read as zeros (a scrunching corner turn keeps their rows)
        const uint32_t v = __builtin_amdgcn_alignbit(raw[k].y, raw[k].x, (shift % SPW) * (32 / SPW)) &
                           (0u - (uint32_t)(keep[k] != 0));
        uint32_t* dst = A + jj[k] * RS + ww[k] * (SPW / 2);
        if constexpr (FMT == kFmtHalf) {
            dst[0] = v;                            // already two 16-bit samples
        } else if constexpr (FMT == kFmtNib) {
            u32x4 q;
            q.x = (v & 0xFu) | ((v & 0xF0u) << 12);
            q.y = ((v >> 8) & 0xFu) | ((v & 0xF000u) << 4);
            q.z = ((v >> 16) & 0xFu) | ((v >> 4) & 0xF0000u);
            q.w = ((v >> 24) & 0xFu) | ((v >> 12) & 0xF0000u);
            *reinterpret_cast<u32x4*>(dst) = q;
        } else {
            dst[0] = (v & 0xFFu) | ((v & 0xFF00u) << 8);
            dst[1] = ((v >> 16) & 0xFFu) | ((v >> 8) & 0xFF0000u);
        }
    }
    __syncthreads();
    // each pair v of output rows has a team of TPP threads; team lane l takes
    // words l, l + TPP, ... of the row (consecutive lanes on consecutive
    // words), so the pair's rows and shift are computed once per step
    constexpr int TPP = 256 / (NSUB / 2);
    constexpr int WPT = (LW + TPP - 1) / TPP;      // words per thread
    const int v = threadIdx.x / TPP, l = threadIdx.x % TPP;
    // unrolled: each step's Theta/Phi masks and buffer offsets are
    // constants; a step issues all of a thread's LDS reads before its writes
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t* lo = A + tree_phi(i, 2 * v) * RS + l;
        const int th = tree_theta(i, 2 * v);
        const uint32_t* hi = A + tree_phi(i, 2 * v + 1) * RS + (th >> 1) + l;
        uint32_t* o0 = B + (2 * v) * RS + l;
        uint32_t* o1 = B + (2 * v + 1) * RS + l;
        const bool odd = (th & 1) != 0;
        uint32_t ra[WPT], r0[WPT], r1[WPT];
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            if (LW % TPP != 0 && k == WPT - 1 && l + TPP * k >= LW) break;
            ra[k] = lo[TPP * k];
            r0[k] = hi[TPP * k];
            r1[k] = hi[TPP * k + 1];
        }
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            if (LW % TPP != 0 && k == WPT - 1 && l + TPP * k >= LW) break;
            const uint32_t mid = __builtin_amdgcn_alignbit(r1[k], r0[k], 16);
            o0[TPP * k] = ra[k] + (odd ? mid : r0[k]);
            o1[TPP * k] = ra[k] + (odd ? r1[k] : mid);
        }
        __syncthreads();
        uint32_t* tmp = A;
        A = B;
        B = tmp;
    }
    // store rows n*NSUB + d', samples t0 .. t0 + T - 1 below len1, eight
    // 16-bit values per 16-byte store
    for (int it = threadIdx.x; it < NSUB * (T / 8); it += 256) {
        const int dp = it / (T / 8), t = 8 * (it % (T / 8));
        const long long tg = t0 + t;
        if (tg >= len1) continue;
        const u32x4 val = *reinterpret_cast<const u32x4*>(A + dp * RS + t / 2);
        uint16_t* orow = reinterpret_cast<uint16_t*>(out + (long long)(y * NSUB + dp) * out_pitch);
        if (tg + 8 <= len1) {
            *reinterpret_cast<u32x4*>(orow + tg) = val;
        } else {
            const uint32_t wv[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (tg + e < len1) orow[tg + e] = (uint16_t)(wv[e >> 1] >> (16 * (e & 1)));
        }
    }
}

// Stage 1 for byte rows (every sub-band sum below 256: 2-bit codes up to
// nsub = 64, small scrunched sums): the same steps as k_tree on byte lanes,
// four samples per 32-bit LDS word, so a step moves half the LDS bytes per
// sample of the 16-bit form.  512 threads per workgroup in teams of
// TPP >= 32 threads, each team taking one output pair (two for nsub = 64)
// and WPT consecutive-word columns of its rows, so every half-wave reads 32
// consecutive words (no bank conflicts); a step issues all of a thread's
// LDS reads before its first write.
// Theta(i, 2v+1) = Theta(i, 2v) + 1: with s = Theta mod 4, the words of the
// second row shifted by s and s + 1 samples are bytes s .. s+3 and
// s+1 .. s+4 of the aligned pair (h0, h1), one v_perm each.  Byte sums never
// carry into the next lane (values below 256).
constexpr int kTreeBThreads = 512;
// LW words (4 LW samples) computed per row
__host__ __device__ constexpr int tree_b_words(int nsub) { return 4096 / nsub > 128 ? 4096 / nsub : 128; }
// T samples per tile: the 4 LW loaded samples less at least nsub of halo
__host__ __device__ constexpr int tree_tile_len_b(int nsub) { return 4 * tree_b_words(nsub) - (nsub > 16 ? nsub : 16); }
__host__ __device__ constexpr int tree_row_words_b(int nsub) { return (tree_b_words(nsub) + nsub / 8 + 1 + 3) / 4 * 4; }

template <int FMT, int NSUB>
__global__ __launch_bounds__(kTreeBThreads) void k_tree_b(BeamDesc b, const int32_t* pairs, uint8_t* out,
                                                          long long out_pitch, long long len1)
{
    static_assert(FMT == kFmtNib || FMT == kFmtByteS, "byte lanes hold 2-bit codes or small byte sums");
    constexpr int NT = kTreeBThreads;
    constexpr int LW = tree_b_words(NSUB);         // words computed per row
    constexpr int L = 4 * LW;                      // samples loaded per row
    constexpr int T = tree_tile_len_b(NSUB);       // samples stored per row
    constexpr int RS = tree_row_words_b(NSUB);     // LDS row stride in words
    constexpr int K = NSUB == 8 ? 3 : NSUB == 16 ? 4 : NSUB == 32 ? 5 : 6;
    static_assert((1 << K) == NSUB && NSUB <= 64, "sub-band width must be a power of two up to 64");
    static_assert(L >= T + NSUB - 1 && L % 8 == 0 && T % 16 == 0, "halo, whole scratch words, 16-sample stores");
    // Theta <= NSUB / 2 samples: reads reach word LW - 1 + NSUB / 8 + 1
    static_assert(RS >= LW + NSUB / 8 + 1 && RS % 4 == 0, "row stride covers the shifted reads");
    extern __shared__ __align__(16) uint32_t tw[];             // [2][NSUB][RS]
    uint32_t* A = tw;
    uint32_t* B = tw + NSUB * RS;
    const long long t0 = (long long)blockIdx.x * T;
    const int y = blockIdx.y;
    const int n = pairs[2 * y], pass = pairs[2 * y + 1];
    // load: channel j of the sub-band starts pass*j samples later (the
    // imposed delay), realigned from two consecutive scratch words.  Thread
    // x takes word w = x mod WPR of rows j = x / WPR + JS k; every load (and
    // kill-mask flag) is issued before the first realignment, so a thread
    // waits for global memory once
    constexpr int SPW = fmt_samples_per_word(FMT);   // 8 (nibbles) or 4 (bytes)
    constexpr int WPR = L / SPW;
    static_assert(NT % WPR == 0 && (NSUB * WPR) % NT == 0, "whole rows per thread block pass");
    constexpr int JS = NT / WPR;                   // rows per pass over the threads
    constexpr int NLD = NSUB * WPR / NT;           // loads per thread
    const int w = threadIdx.x % WPR, j0 = threadIdx.x / WPR;
    int keep[NLD];
    if (b.mask) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) keep[k] = b.mask[n * NSUB + j0 + JS * k];
    } else {
#pragma unroll
        for (int k = 0; k < NLD; ++k) keep[k] = 1;
    }
    const uint8_t* row0 = b.xc + (long long)(n * NSUB + j0) * b.pitch + (t0 / SPW + w) * 4;
    u32x2 raw[NLD];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int shift = pass * (j0 + JS * k);
        __builtin_memcpy(&raw[k], row0 + (long long)(JS * k) * b.pitch + (shift / SPW) * 4, sizeof(u32x2));
    }
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int shift = pass * (j0 + JS * k);
        // killed channels read as zeros (a scrunching corner turn keeps their rows)
        const uint32_t v = __builtin_amdgcn_alignbit(raw[k].y, raw[k].x, (shift % SPW) * (32 / SPW)) &
                           (0u - (uint32_t)(keep[k] != 0));
        uint32_t* dst = A + (j0 + JS * k) * RS + w * (SPW / 4);
        if constexpr (FMT == kFmtNib) {
            // nibble i (sample i) to byte i of two words: even samples from
            // the low nibbles, odd ones from the high nibbles, interleaved
            const uint32_t ev = v & 0x0F0F0F0Fu, od = (v >> 4) & 0x0F0F0F0Fu;
            u32x2 q;
            q.x = __builtin_amdgcn_perm(od, ev, 0x05010400u);
            q.y = __builtin_amdgcn_perm(od, ev, 0x07030602u);
            *reinterpret_cast<u32x2*>(dst) = q;
        } else {
            dst[0] = v;                            // already four byte samples
        }
    }
    __syncthreads();
    // output pairs v = team + NTEAM q (q < PPT) of a team of TPP threads;
    // team lane l takes words l, l + TPP, ... of the rows
    constexpr int TPP = NT / (NSUB / 2) > 32 ? NT / (NSUB / 2) : 32;
    constexpr int NTEAM = NT / TPP;
    constexpr int PPT = (NSUB / 2) / NTEAM;        // output pairs per team
    constexpr int WPT = LW / TPP;                  // words per thread and row
    static_assert(NTEAM * PPT == NSUB / 2 && TPP * WPT == LW, "whole teams and team passes");
    const int team = threadIdx.x / TPP, l = threadIdx.x % TPP;
    // unrolled: each step's Theta/Phi masks and buffer offsets are constants
#pragma unroll
    for (int i = 0; i < K; ++i) {
        uint32_t a[PPT][WPT], h0[PPT][WPT], h1[PPT][WPT], sel0[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int v = team + NTEAM * q;
            const int th = tree_theta(i, 2 * v);
            const uint32_t* lo = A + tree_phi(i, 2 * v) * RS + l;
            const uint32_t* hi = A + tree_phi(i, 2 * v + 1) * RS + (th >> 2) + l;
            // v_perm selector: bytes s .. s+3 of (h0 = bytes 0-3, h1 = 4-7)
            sel0[q] = 0x03020100u + (uint32_t)(th & 3) * 0x01010101u;
#pragma unroll
            for (int k = 0; k < WPT; ++k) {
                a[q][k] = lo[TPP * k];
                h0[q][k] = hi[TPP * k];
                h1[q][k] = hi[TPP * k + 1];
            }
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            uint32_t* o0 = B + (2 * (team + NTEAM * q)) * RS + l;
            const uint32_t sel1 = sel0[q] + 0x01010101u;   // bytes s+1 .. s+4
#pragma unroll
            for (int k = 0; k < WPT; ++k) {
                o0[TPP * k] = a[q][k] + __builtin_amdgcn_perm(h1[q][k], h0[q][k], sel0[q]);
                o0[RS + TPP * k] = a[q][k] + __builtin_amdgcn_perm(h1[q][k], h0[q][k], sel1);
            }
        }
        __syncthreads();
        uint32_t* tmp = A;
        A = B;
        B = tmp;
    }
    // store rows n*NSUB + d', samples t0 .. t0 + T - 1 below len1, 16 per
    // 16-byte store
    constexpr int PR = T / 16;                     // pieces per row
    uint8_t* obase = out + (long long)y * NSUB * out_pitch + t0;
    const long long rem = len1 - t0;               // samples of this tile below len1
#pragma unroll
    for (int m = 0; m < (NSUB * PR + NT - 1) / NT; ++m) {
        const int it = threadIdx.x + NT * m;
        if ((NSUB * PR) % NT != 0 && it >= NSUB * PR) break;
        const int dp = it / PR, t = 16 * (it - dp * PR);
        if (t >= rem) continue;
        const u32x4 val = *reinterpret_cast<const u32x4*>(A + dp * RS + t / 4);
        uint8_t* o = obase + (long long)dp * out_pitch + t;
        if (t + 16 <= rem) {
            *reinterpret_cast<u32x4*>(o) = val;
        } else {
            const uint32_t wv[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
            for (int e = 0; e < 16; ++e)
                if (t + e < rem) o[e] = (uint8_t)(wv[e >> 2] >> (8 * (e & 3)));
        }
    }
}

// N consecutive outputs t .. t+N-1 of trial d at the descriptor's width.
template <int N>
__device__ __forceinline__ void tree_store(const BeamDesc& b, int d, long long t, const uint32_t (&acc)[N])
{
    if (b.rowmap) d = b.rowmap[d];               // the trial's row of the whole output
    if (b.out_bytes == 4) {
        uint32_t* orow = b.out + (size_t)d * (size_t)b.out_stride;
        if (t + N <= b.nout) {
#pragma unroll
            for (int q = 0; q < N / 4; ++q) {
                const u32x4 v = {acc[4 * q] >> b.out_shift, acc[4 * q + 1] >> b.out_shift,
                                 acc[4 * q + 2] >> b.out_shift, acc[4 * q + 3] >> b.out_shift};
                __builtin_memcpy(orow + t + 4 * q, &v, sizeof(v));
            }
        } else {
#pragma unroll
            for (int e = 0; e < N; ++e)
                if (t + e < b.nout) orow[t + e] = acc[e] >> b.out_shift;
        }
    } else {
        uint8_t* nrow = reinterpret_cast<uint8_t*>(b.out) + (long long)d * b.out_stride;
#pragma unroll
        for (int e = 0; e < N; ++e) {
            if (t + e >= b.nout) continue;
            const uint32_t v = out_value(acc[e], b.out_shift, b.out_bytes);
            if (b.out_bytes == 1) nrow[t + e] = (uint8_t)v;
            else reinterpret_cast<uint16_t*>(nrow)[t + e] = (uint16_t)v;
        }
    }
}

// Stage 2 of the piecewise linear tree (Section 3, the piecewise linear
// combination of sub-bands): out[d][t] = sum over sub-bands n of
// S[rowsel[d][n]][t + table[d][n]], S the stage-1 rows (d.xc, pitch d.pitch
// bytes) of 16-bit values (OB = 2) or bytes (OB = 1).  A lane sums L = 8
// (16-bit) or 16 (byte) consecutive outputs of one trial: per term five
// aligned 32-bit words (a 16-byte load and one more, four terms' loads in
// flight at a time) give the L shifted samples through four realignments
// (v_alignbit by the delay's offset within a word) for 16-bit rows, or
// eight v_perm byte-pair picks for byte rows; they are added in 16-bit
// lanes without a carry between lanes and moved to 32-bit sums every
// `flush` terms (flush * largest row value < 2^16).  The realignment is
// uniform over the wave (t is a multiple of the samples per word).
//
// Work items (time tile of 256 L outputs, trial) are ordered tile-major,
// trial-minor and cut into 8 contiguous ranges, one per XCD (the hardware
// hands workgroup i to XCD i mod 8): the workgroups in flight on an XCD
// cover neighbouring trials of one tile, which share most of their tree
// rows, so the rows stay in that XCD's L2.
template <int OB>
__global__ __launch_bounds__(256) void k_tree_combine(BeamDesc b, int flush, long long per_xcd,
                                                      const int32_t* trials, int ntr)
{
    constexpr int L = OB == 2 ? 8 : 16;           // outputs per lane
    constexpr int SPW = 4 / OB;                   // samples per 32-bit word
    const long long o = (long long)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const long long ndm = trials ? ntr : b.ndm;   // the trials this launch covers
    if (o >= ndm * ((b.nout + 256 * L - 1) / (256 * L))) return;   // no barriers below
    const int d = trials ? trials[o % ndm] : (int)(o % ndm);
    const long long t_out = (o / ndm) * (256 * L) + threadIdx.x * L;
    // every lane stays to the end (the tables below are broadcast from all
    // lanes' registers); lanes past the last output read from sample 0 and
    // store nothing
    const bool live = t_out < b.nout;
    const long long t = live ? t_out : 0;
    const int nsb = b.nact;
    const int32_t* rows = b.rowsel + (size_t)d * nsb;
    const int32_t* dly = b.table + (size_t)d * nsb;
    // up to 128 sub-bands: the trial's rows and delays sit in registers (lane
    // n holds sub-band n's and n + 64's) and are broadcast per term
    const int lane = threadIdx.x & 63;
    const bool in_regs = nsb <= 128;
    const int r_lo = in_regs && lane < nsb ? rows[lane] : 0, r_hi = in_regs && lane + 64 < nsb ? rows[lane + 64] : 0;
    const int d_lo = in_regs && lane < nsb ? dly[lane] : 0, d_hi = in_regs && lane + 64 < nsb ? dly[lane + 64] : 0;
    uint32_t acc[L];
#pragma unroll
    for (int e = 0; e < L; ++e) acc[e] = 0u;
    for (int n0 = 0; n0 < nsb; n0 += flush) {
        const int n1 = min(nsb, n0 + flush);
        // OB = 2: p[k] = samples (2k, 2k+1); OB = 1: p[k] = (4k, 4k+2),
        // q[k] = (4k+1, 4k+3), each pair in the two 16-bit lanes
        uint32_t p[4] = {0u, 0u, 0u, 0u}, q[4] = {0u, 0u, 0u, 0u};
        // U terms at a time: the group's loads are all issued before the
        // first add
        constexpr int U = 4;
        for (int n = n0; n < n1; n += U) {
            uint32_t w[U][5];
            int sh[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int m = n + u < n1 ? n + u : n;   // past the range: repeat n, not added
                const int rn = in_regs ? __builtin_amdgcn_readlane(m < 64 ? r_lo : r_hi, m & 63) : rows[m];
                const int dn = in_regs ? __builtin_amdgcn_readlane(m < 64 ? d_lo : d_hi, m & 63) : dly[m];
                const long long s = t + dn;
                const uint32_t* src = reinterpret_cast<const uint32_t*>(b.xc + (long long)rn * b.pitch) + s / SPW;
                u32x4 v;
                __builtin_memcpy(&v, src, sizeof(v));
                w[u][0] = v.x;
                w[u][1] = v.y;
                w[u][2] = v.z;
                w[u][3] = v.w;
                w[u][4] = src[4];
                sh[u] = (int)(s % SPW);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (n + u >= n1) break;
                if constexpr (OB == 2) {
                    // 16-bit rows: realign by 0 or 16 bits, add both lanes
#pragma unroll
                    for (int k = 0; k < 4; ++k) p[k] += __builtin_amdgcn_alignbit(w[u][k + 1], w[u][k], 16 * sh[u]);
                } else {
                    // byte rows: one v_perm of the aligned pair picks bytes
                    // s, s+2 into p's 16-bit lanes, another s+1, s+3 into q's
                    const uint32_t sa = 0x0C020C00u + (uint32_t)sh[u] * 0x00010001u;
                    const uint32_t sb = sa + 0x00010001u;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        p[k] += __builtin_amdgcn_perm(w[u][k + 1], w[u][k], sa);
                        q[k] += __builtin_amdgcn_perm(w[u][k + 1], w[u][k], sb);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if constexpr (OB == 2) {
                acc[2 * k] += p[k] & 0xFFFFu;
                acc[2 * k + 1] += p[k] >> 16;
            } else {
                acc[4 * k] += p[k] & 0xFFFFu;
                acc[4 * k + 1] += q[k] & 0xFFFFu;
                acc[4 * k + 2] += p[k] >> 16;
                acc[4 * k + 3] += q[k] >> 16;
            }
        }
    }
    if (live) tree_store<L>(b, d, t, acc);
}

// Stage 2 with LDS staging (byte rows).  Consecutive trials of a sorted,
// dense DM list use nearly the same tree rows (d'_n changes slowly with DM)
// at nearly the same delays, so a workgroup stages, for its time tile and
// block of kTreeBlock trials, each sub-band's rows the block uses over the
// block's delay window once, and every trial then reads its terms from LDS.
//
// The staged rows are segmented within the tile: with P = kTreeTile / 4 and
// B = t0 + dmin4 the window's first sample, byte i of staged dword k is
// sample B + k + i P.  A trial whose delay is o samples past dmin4 finds
// the samples of outputs t0 + u + i P (i = 0 .. 3) in dword o + u, so every
// delay is a whole-dword offset: no realignment, one LDS dword per four
// outputs and term.  Lane l takes u = l + 64 j (j < P / 64).  Bytes 0 and 2
// are added in 16-bit lanes (a mask), bytes 1 and 3 through an unmasked
// shift whose byte-2 part is taken out at the end; with PAIR (row values
// below 128) two terms are first added as bytes.
// Staging turns four aligned dwords of the row (samples B + 4c .. + 3 of
// each of the four segments) into four staged dwords with eight v_perm.
__device__ __forceinline__ void tree_store_at(const BeamDesc& b, int drow, long long t, uint32_t v)
{
    if (t >= b.nout) return;
    if (b.out_bytes == 4) {
        b.out[(size_t)drow * (size_t)b.out_stride + t] = v >> b.out_shift;
    } else {
        uint8_t* nrow = reinterpret_cast<uint8_t*>(b.out) + (long long)drow * b.out_stride;
        const uint32_t w = out_value(v, b.out_shift, b.out_bytes);
        if (b.out_bytes == 1) nrow[t] = (uint8_t)w;
        else reinterpret_cast<uint16_t*>(nrow)[t] = (uint16_t)w;
    }
}

// eight waves per workgroup: a workgroup's LDS (the staged rows) then
// carries twice the waves of four, for latency hiding
constexpr int kTreeWaves = 8;
template <bool PAIR>
__global__ __launch_bounds__(64 * kTreeWaves) void k_tree_combine_lds(BeamDesc b, const int32_t* blocks, const TreeStage* stage,
                                                          const int32_t* off, int nblocks)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t sl[];
    constexpr int TT = kTreeTile, TB = kTreeBlock;
    constexpr int P = TT / 4;                      // outputs per segment of the tile
    constexpr int J = P / 64;                      // staged dwords per lane and term
    static_assert(P % 64 == 0, "whole dwords per lane");
    // workgroup i: trial block i mod nblocks of time tile i / nblocks, so the
    // workgroups in flight write long runs of each output row (a tile-fastest
    // order spreads them over every tile of few rows, which writes HBM at
    // about two thirds the rate)
    const int bi = (int)(blockIdx.x % (unsigned)nblocks);
    const long long t0 = (long long)(blockIdx.x / (unsigned)nblocks) * TT;
    const int blk = blocks[bi];
    const int nsb = b.nact;
    const TreeStage* st = stage + (size_t)bi * nsb;
    // staging: item i of sub-band n (i < span * wdw/4: row i / (wdw/4),
    // dword group c = i mod (wdw/4)) fills LDS dwords lds + 4 i .. + 3.
    // Wave w stages sub-bands w, w + kTreeWaves, ...: items lane and lane +
    // 64 of SB sub-bands at a time, all of their loads in flight before the
    // first transpose; items from 128 on in a loop of their own.
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the wave's trials (wave, wave + kTreeWaves, ...) and their rows of the
    // whole output, read before the first store (a vector load issued after
    // the stores would wait for them)
    constexpr int KT = TB / kTreeWaves;
    int drow[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        const int d = blk * TB + wave + kTreeWaves * k;
        const int dd = d < b.ndm ? d : 0;
        drow[k] = b.rowmap ? b.rowmap[dd] : dd;
    }
    // The sub-band's rows lo .. lo + span - 1 are read as one buffer (32-bit
    // offsets: (max(span, 4) + 1) * pitch stays below 2^31, which the host
    // checks): loads past its end read zeros, and loads past the end of an
    // earlier row read the next row's bytes, which only outputs at or past
    // nout see (output t reads sample t + delay < nout + the largest delay
    // <= the row length).
    auto stage_item = [&](const TreeStage& g, int i, uint32_t (&a)[4]) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(b.xc + (long long)g.lo * b.pitch), (short)0, (int)(g.span * b.pitch), 0x00020000);
        // i < 2^14: the rounded-up reciprocal gives the exact quotient
        const int row = (int)__umulhi((uint32_t)i, g.rcp), c = i - row * (g.wdw / 4);
        const int voff = row * (int)b.pitch + (int)(t0 + g.dmin4) + 4 * c;
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff + s * P, 0, 0);
    };
    auto put_item = [&](const TreeStage& g, int i, bool live, const uint32_t (&a)[4]) {
        // 4x4 byte transpose: staged dword e = byte e of a[0 .. 3]
        const uint32_t x01l = __builtin_amdgcn_perm(a[1], a[0], 0x05010400u);
        const uint32_t x01h = __builtin_amdgcn_perm(a[1], a[0], 0x07030602u);
        const uint32_t x23l = __builtin_amdgcn_perm(a[3], a[2], 0x05010400u);
        const uint32_t x23h = __builtin_amdgcn_perm(a[3], a[2], 0x07030602u);
        const u32x4 v = {__builtin_amdgcn_perm(x23l, x01l, 0x05040100u),
                         __builtin_amdgcn_perm(x23l, x01l, 0x07060302u),
                         __builtin_amdgcn_perm(x23h, x01h, 0x05040100u),
                         __builtin_amdgcn_perm(x23h, x01h, 0x07060302u)};
        if (live) *reinterpret_cast<u32x4*>(sl + g.lds + 4 * i) = v;
    };
    // Items past a sub-band's end read zeros (rows past its span lie outside
    // its buffer) and are transposed but not written, so every load's value
    // is consumed on every path and loads of later items never wait for
    // earlier ones.
    // At most 128 sub-bands: four passes of kTreeWaves * SB, unrolled (a
    // loop would make the first loads of a pass wait for the last pass's).
    constexpr int SB = 4, H = 2;
    static_assert(4 * kTreeWaves * SB >= 128, "every sub-band staged");
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int n0 = wave + kTreeWaves * SB * it;
        if (n0 >= nsb) break;                      // uniform
        uint32_t a[SB][H][4];
        int items[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int n = n0 + kTreeWaves * u;
            items[u] = n < nsb ? st[n].span * (st[n].wdw / 4) : 0;
#pragma unroll
            for (int h = 0; h < H; ++h) {
                if (items[u] > 64 * h) stage_item(st[n], lane + 64 * h, a[u][h]);   // uniform
            }
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int n = n0 + kTreeWaves * u;
#pragma unroll
            for (int h = 0; h < H; ++h) {
                if (items[u] > 64 * h) put_item(st[n], lane + 64 * h, lane + 64 * h < items[u], a[u][h]);
            }
        }
    }
    for (int n = wave; n < nsb; n += kTreeWaves) {
        const TreeStage g = st[n];
        for (int i = 64 * H + lane; i < g.span * (g.wdw / 4); i += 64) {
            uint32_t a[4];
            stage_item(g, i, a);
            put_item(g, i, true, a);
        }
    }
    __syncthreads();
    constexpr uint32_t M = 0x00FF00FFu;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
        const int d = blk * TB + wave + kTreeWaves * kt;
        if (d >= b.ndm) break;                     // no barriers below
        // p[j]: outputs u, u + 2P in its 16-bit lanes (bytes 0 and 2 of each
        // term); q[j]: the terms shifted right by 8 bits, unmasked, so that
        // q = S1 + 2^8 S2 + 2^16 S3 (S_i the sum of bytes i, each below 2^15:
        // no wrap), and q - 2^8 S2 holds outputs u + P, u + 3P.
        uint32_t p[J], q[J];
#pragma unroll
        for (int j = 0; j < J; ++j) p[j] = q[j] = 0u;
        // the trial's LDS byte offsets through scalar loads (the table is
        // constant during the launch)
        typedef const __attribute__((address_space(4))) int32_t* coff_t;
        const coff_t od = (coff_t)(off + (size_t)d * nsb);
        // C terms at a time: every LDS read of the group before the first add
        auto terms = [&](auto cnt, const int* o) {
            constexpr int C = decltype(cnt)::value;
            uint32_t w[C][J];
#pragma unroll
            for (int u = 0; u < C; ++u)
#pragma unroll
                for (int j = 0; j < J; ++j)
                    w[u][j] = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(sl) + o[u] + 4 * lane +
                                                                 256 * j);
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if constexpr (PAIR && C % 2 == 0) {
#pragma unroll
                    for (int u = 0; u < C; u += 2) {
                        const uint32_t s = w[u][j] + w[u + 1][j];   // bytes below 128: no carry
                        p[j] += s & M;
                        q[j] += s >> 8;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < C; ++u) {
                        p[j] += w[u][j] & M;
                        q[j] += w[u][j] >> 8;
                    }
                }
            }
        };
        // terms n .. n + C - 1
        auto group = [&](auto cnt, int n) {
            constexpr int C = decltype(cnt)::value;
            int o[C];
#pragma unroll
            for (int u = 0; u < C; ++u) o[u] = od[n + u];
            terms(cnt, o);
        };
        // eight terms at a time, the next eight offsets loaded ahead
        int n = 0;
        int o8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (nsb >= 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) o8[u] = od[u];
        }
        for (; n + 8 <= nsb; n += 8) {
            int o[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) o[u] = o8[u];
            if (n + 16 <= nsb) {
#pragma unroll
                for (int u = 0; u < 8; ++u) o8[u] = od[n + 8 + u];
            }
            terms(std::integral_constant<int, 8>(), o);
        }
        if (n + 4 <= nsb) {
            group(std::integral_constant<int, 4>(), n);
            n += 4;
        }
        if (n + 2 <= nsb) {
            group(std::integral_constant<int, 2>(), n);
            n += 2;
        }
        if (n < nsb) group(std::integral_constant<int, 1>(), n);
#pragma unroll
        for (int j = 0; j < J; ++j) q[j] -= (p[j] >> 16) << 8;
        if (b.out_bytes == 4 && t0 + TT <= b.nout) {
            // a whole tile of 32-bit outputs: one row address, no bounds checks
            uint32_t* orow = b.out + (size_t)drow[kt] * (size_t)b.out_stride + t0 + lane;
            const int sh = b.out_shift;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                orow[64 * j] = (p[j] & 0xFFFFu) >> sh;
                orow[64 * j + P] = (q[j] & 0xFFFFu) >> sh;
                orow[64 * j + 2 * P] = (p[j] >> 16) >> sh;
                orow[64 * j + 3 * P] = (q[j] >> 16) >> sh;
            }
        } else {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const long long t = t0 + 64 * j + lane;
                tree_store_at(b, drow[kt], t, p[j] & 0xFFFFu);
                tree_store_at(b, drow[kt], t + P, q[j] & 0xFFFFu);
                tree_store_at(b, drow[kt], t + 2 * P, p[j] >> 16);
                tree_store_at(b, drow[kt], t + 3 * P, q[j] >> 16);
            }
        }
    }
}

}  // namespace

int tree_tile(int nsub) { return tree_tile_len_b(nsub) > tree_tile_len(nsub) ? tree_tile_len_b(nsub) : tree_tile_len(nsub); }

hipError_t launch_tree_combine_lds(const BeamDesc& d, const int32_t* blocks, int nblocks, const TreeStage* stage,
                                   const int32_t* off, int lds_dwords, bool pair, hipStream_t st)
{
    if (d.nout <= 0 || d.ndm <= 0 || d.nact <= 0 || d.nact > 128 || nblocks <= 0 || nblocks > 65535 ||
        lds_dwords <= 0 || (size_t)lds_dwords * 4 > (size_t)kMaxLdsBytes || (d.pitch & 3) ||
        (reinterpret_cast<uintptr_t>(d.xc) & 3) ||
        (reinterpret_cast<uintptr_t>(d.out) & (d.out_bytes == 4 ? 3 : d.out_bytes - 1)))
        return hipErrorInvalidValue;
    const long long gx = (d.nout + kTreeTile - 1) / kTreeTile * nblocks;
    if (gx > 0x7fffffffLL) return hipErrorInvalidValue;
    const void* fn = pair ? reinterpret_cast<const void*>(&k_tree_combine_lds<true>)
                          : reinterpret_cast<const void*>(&k_tree_combine_lds<false>);
    const size_t lds = (size_t)lds_dwords * 4;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    BeamDesc a0 = d;
    const int32_t* a1 = blocks;
    const TreeStage* a2 = stage;
    const int32_t* a3 = off;
    int a4 = nblocks;
    void* args[] = {&a0, &a1, &a2, &a3, &a4};
    return hipLaunchKernel(fn, dim3((unsigned)gx), dim3(64 * kTreeWaves), args, lds, st);
}

hipError_t launch_tree_combine(const BeamDesc& d, int ob, int flush, const int32_t* trials, int ntrials,
                               hipStream_t st)
{
    if (d.nout <= 0 || d.ndm <= 0 || d.nact <= 0 || flush < 1 || (d.pitch & 3) || (ob != 1 && ob != 2) ||
        (reinterpret_cast<uintptr_t>(d.xc) & 3) ||
        (reinterpret_cast<uintptr_t>(d.out) & (d.out_bytes == 4 ? 3 : d.out_bytes - 1)))
        return hipErrorInvalidValue;
    const long long per_item = ob == 2 ? 2048 : 4096;
    if (trials && ntrials <= 0) return hipErrorInvalidValue;
    const long long items = (long long)(trials ? ntrials : d.ndm) * ((d.nout + per_item - 1) / per_item);
    const long long per_xcd = (items + 7) / 8;
    if (8 * per_xcd > 0x7fffffffLL) return hipErrorInvalidValue;
    BeamDesc a0 = d;
    int a1 = flush;
    long long a2 = per_xcd;
    const int32_t* a3 = trials;
    int a4 = ntrials;
    void* args[] = {&a0, &a1, &a2, &a3, &a4};
    const void* fn = ob == 2 ? reinterpret_cast<const void*>(&k_tree_combine<2>)
                             : reinterpret_cast<const void*>(&k_tree_combine<1>);
    return hipLaunchKernel(fn, dim3((unsigned)(8 * per_xcd)), dim3(256), args, 0, st);
}

hipError_t launch_tree(const BeamDesc& d, int fmt, int nsub, int ob, const int32_t* pairs, int npairs,
                       uint8_t* out, long long out_pitch, long long len1, hipStream_t st)
{
    if (len1 <= 0 || (out_pitch & 15) || (reinterpret_cast<uintptr_t>(out) & 15) || !pairs ||
        (d.pitch & 3))
        return hipErrorInvalidValue;
    const long long T = ob == 1 ? tree_tile_len_b(nsub) : tree_tile_len(nsub);
    const long long gx = (len1 + T - 1) / T;
    const long long gy = npairs;
    if (gx <= 0 || gx > 0x7fffffffLL || gy <= 0 || gy > 65535) return hipErrorInvalidValue;
    const void* fn = nullptr;
    // byte rows (byte lanes in LDS) hold sub-band sums below 256: 2-bit
    // codes up to nsub = 64, small scrunched sums (byte format) for narrow
    // sub-bands; 16-bit rows everything else
#define DEDISP_TREE_B(F, N) \
    if (fmt == F && nsub == N && ob == 1) fn = reinterpret_cast<const void*>(&k_tree_b<F, N>);
#define DEDISP_TREE_CASE(F, N) \
    if (fmt == F && nsub == N && ob == 2) fn = reinterpret_cast<const void*>(&k_tree<F, N>);
    DEDISP_TREE_B(kFmtNib, 8) DEDISP_TREE_B(kFmtNib, 16) DEDISP_TREE_B(kFmtNib, 32) DEDISP_TREE_B(kFmtNib, 64)
    DEDISP_TREE_B(kFmtByteS, 8) DEDISP_TREE_B(kFmtByteS, 16) DEDISP_TREE_B(kFmtByteS, 32)
    DEDISP_TREE_CASE(kFmtNib, 128)
    DEDISP_TREE_CASE(kFmtByte, 8) DEDISP_TREE_CASE(kFmtByte, 16) DEDISP_TREE_CASE(kFmtByte, 32)
    DEDISP_TREE_CASE(kFmtByte, 64) DEDISP_TREE_CASE(kFmtByte, 128)
    DEDISP_TREE_CASE(kFmtByteS, 8) DEDISP_TREE_CASE(kFmtByteS, 16) DEDISP_TREE_CASE(kFmtByteS, 32)
    DEDISP_TREE_CASE(kFmtByteS, 64) DEDISP_TREE_CASE(kFmtByteS, 128)
    DEDISP_TREE_CASE(kFmtHalf, 8) DEDISP_TREE_CASE(kFmtHalf, 16) DEDISP_TREE_CASE(kFmtHalf, 32)
    DEDISP_TREE_CASE(kFmtHalf, 64) DEDISP_TREE_CASE(kFmtHalf, 128)
#undef DEDISP_TREE_B
#undef DEDISP_TREE_CASE
    if (!fn) return hipErrorInvalidValue;
    const size_t lds = 2ull * nsub * (ob == 1 ? tree_row_words_b(nsub) : tree_row_words(nsub)) * sizeof(uint32_t);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    BeamDesc a0 = d;
    const int32_t* a1 = pairs;
    uint8_t* a2 = out;
    long long a3 = out_pitch, a4 = len1;
    void* args[] = {&a0, &a1, &a2, &a3, &a4};
    return hipLaunchKernel(fn, dim3((unsigned)gx, (unsigned)gy), dim3(ob == 1 ? kTreeBThreads : 256), args, lds, st);
}

}  // namespace dedisp
