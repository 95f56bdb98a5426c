// Host side of the dedispersion library: argument validation, the delay
// table, the per-DM-block window tables the LDS-tiled kernel consumes, kernel
// selection and tuning, streams (overlap-save over time) and batches
// (multi-beam, graph-captured launches).  All validation happens before any
// HIP call.
#include "dedisp.h"
#include "dedisp_internal.h"
#include "dedisp_host.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

using dedisp::BeamDesc;
using dedisp::Shape;
using dedisp::kFmtNib;
using dedisp::kFmtByte;
using dedisp::kFmtByteS;
using dedisp::kFmtHalf;

namespace dedisp {
namespace host {

thread_local std::string g_last_error;

dedisp_status fail(dedisp_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

dedisp_status hip_fail(hipError_t e, const char* where)
{
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return DEDISP_ERR_HIP;
}

// Dispersion constant k_DM, MHz^2 pc^-1 cm^3 s (Section 1 of the paper).
constexpr double kDispersionConstant = 4.148808e3;

void destroy_groups(dedisp_plan p);

InFlight::~InFlight()
{
    for (auto& e : ev) (void)hipEventDestroy(e.second);
}

void InFlight::record(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    hipEvent_t e = nullptr;
    for (auto& x : ev)
        if (x.first == s) e = x.second;
    if (!e) {
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            // cannot track this stream: fall back to waiting for the device
            last = s;
            any = true;
            ev.clear();
            return;
        }
        ev.emplace_back(s, e);
    }
    if (hipEventRecord(e, s) != hipSuccess) ev.clear();
    last = s;
    any = true;
}

void InFlight::record_existing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    hipEvent_t e = nullptr;
    for (auto& x : ev)
        if (x.first == s) e = x.second;
    if (!e || hipEventRecord(e, s) != hipSuccess) untracked = true;
    last = s;
    any = true;
}

void InFlight::wait()
{
    if (!any) return;
    bool ok = !ev.empty() && !untracked;
    for (auto& x : ev)
        if (hipEventSynchronize(x.second) != hipSuccess) ok = false;
    if (!ok) (void)hipDeviceSynchronize();
    untracked = false;
}

void free_device(dedisp_plan p)
{
    if (p->d_table || !p->blocks.empty()) p->inflight.wait();
    if (p->d_table) (void)hipFree(p->d_table);
    p->d_table = nullptr;
    for (auto& kv : p->blocks) {
        if (kv.second.d_rel) (void)hipFree(kv.second.d_rel);
        if (kv.second.d_base) (void)hipFree(kv.second.d_base);
    }
    p->blocks.clear();
    free_scratch(p->xc);
    if (p->d_chanmap) (void)hipFree(p->d_chanmap);
    if (p->d_mask) (void)hipFree(p->d_mask);
    p->d_chanmap = nullptr;
    p->d_mask = nullptr;
}

// Drop the cached DM-block tables (their window bases are aligned to the
// scratch format's 16-byte pieces) before a plan's format changes.
void drop_block_tables(dedisp_plan p)
{
    if (p->blocks.empty()) return;
    p->inflight.wait();
    for (auto& kv : p->blocks) {
        if (kv.second.d_rel) (void)hipFree(kv.second.d_rel);
        if (kv.second.d_base) (void)hipFree(kv.second.d_base);
    }
    p->blocks.clear();
}

bool is_finite(double x) { return std::isfinite(x); }

// Section 2.1: DeltaT(nu) = (k_DM/dtau) (1/(nu0 + nu dnu)^2 - 1/nu0^2) and
// delay = round(DM * DeltaT), half away from zero, evaluated in binary64 in
// this order (the host is compiled with -ffp-contract=off).
bool build_delay_table(const dedisp_plan_s& p, const double* dms, int ndm,
                       std::vector<int32_t>& table, int& max_delay)
{
    std::vector<double> dT(p.nchans);
    const double inv_f0_sq = 1.0 / (p.f_top * p.f_top);
    const double samples_per_unit = kDispersionConstant / p.dt;
    for (int c = 0; c < p.nchans; ++c) {
        const double f = p.f_top + static_cast<double>(c) * p.df;
        dT[c] = samples_per_unit * (1.0 / (f * f) - inv_f0_sq);
    }
    table.assign(static_cast<size_t>(ndm) * p.nchans, 0);
    max_delay = 0;
    for (int d = 0; d < ndm; ++d) {
        for (int c = 0; c < p.nchans; ++c) {
            const double x = dms[d] * dT[c];
            if (!(x < 2147483647.0)) return false;
            const long long v = std::llround(x);
            table[static_cast<size_t>(d) * p.nchans + c] = static_cast<int32_t>(v);
            max_delay = std::max(max_delay, static_cast<int>(v));
        }
    }
    return true;
}

// Window tables for blocks of `db` consecutive DM rows, over the scratch
// rows (the live channels in order, then zero rows up to a multiple of 8):
// base[b][k] is the smallest delay of row k's channel over the block,
// rounded down to 16 bytes of scratch (32 two-bit or 16 eight-bit samples,
// 128 samples of a bit plane, 4 words of the interleaved bit planes, whose
// words advance one sample each, so staged windows start on 16-byte
// boundaries); the window offset of DM row d, scratch row k is
// delay[d][c(k)] - base[b][k] (0 for padding DM rows past ndm and for the
// zero rows), stored for row pairs: rel[d][p] = off(2p) | off(2p+1) << 16.
// relmax is the largest offset (always < 2^16 for a shape that fits).  For
// the interleaved bit planes base holds (start, span) pairs, span = the
// largest offset of the row over the block, so a row's window is staged only
// as far as its own DMs read.
void build_block_tables(const dedisp_plan_s& p, int db, int fmt, BlockTables& bt)
{
    const int bstride = fmt == dedisp::kFmtSeg ? 2 : 1;
    const int align = fmt == dedisp::kFmtSeg ? 4 : 16 * dedisp::fmt_bytes_den(fmt) / dedisp::fmt_bytes_num(fmt);
    const int ndm = static_cast<int>(p.dms.size());
    const int nch = p.nchans;
    const int nrow = p.nact_padded();     // scratch rows: live channels, then zero rows
    const int nlive = p.nact();
    const int np = nrow / 2;
    bt.db = db;
    bt.nblocks = (ndm + db - 1) / db;
    const size_t rel_per_group = static_cast<size_t>(bt.nblocks) * db * np;
    const size_t base_per_group = static_cast<size_t>(bt.nblocks) * nrow * bstride;
    bt.rel.assign(rel_per_group * p.ngroups, 0u);
    bt.base.assign(base_per_group * p.ngroups, 0);
    bt.relmax = 0;
    for (int g = 0; g < p.ngroups; ++g) {
        const int32_t* table = p.table.data() + static_cast<size_t>(g) * ndm * nch;
        uint32_t* rel = bt.rel.data() + g * rel_per_group;
        int32_t* base = bt.base.data() + g * base_per_group;
        for (int b = 0; b < bt.nblocks; ++b) {
        const int d0 = b * db, d1 = std::min(ndm, d0 + db);
        for (int k = 0; k < nlive; ++k) {
            const int c = p.source_channel(k);
            int mn = 0x7fffffff;
            for (int d = d0; d < d1; ++d)
                mn = std::min(mn, table[static_cast<size_t>(d) * nch + c]);
            mn &= ~(align - 1);
            int span = 0;
            for (int d = d0; d < d1; ++d) {
                const int r = table[static_cast<size_t>(d) * nch + c] - mn;
                bt.relmax = std::max(bt.relmax, r);
                span = std::max(span, r);
                const uint32_t v = static_cast<uint32_t>(std::min(r, 0xFFFF));
                rel[static_cast<size_t>(d) * np + k / 2] |= (k & 1) ? (v << 16) : v;
            }
            const size_t at = (static_cast<size_t>(b) * nrow + k) * bstride;
            base[at] = mn;
            if (bstride == 2) base[at + 1] = span;
        }
        }
    }
}

// A bit-plane plan also runs the interleaved bit-plane shapes.
bool shape_matches(const Shape& s, const dedisp_plan_s& p)
{
    if (s.kind != 0) return s.fmt == p.nbits;
    return s.fmt == p.fmt || (s.fmt == dedisp::kFmtSeg && p.fmt == dedisp::kFmtPlane);
}

// The shape of config c: for a bit-plane plan, sample_format kFmtSeg picks
// the interleaved layout and any other value the plain one.
const Shape* find_shape(const dedisp_tile_config& c, const dedisp_plan_s& p, int* index)
{
    for (int i = 0; i < dedisp::shape_count(); ++i) {
        const Shape& s = dedisp::shape_at(i);
        if (!shape_matches(s, p) || s.kind != c.kind) continue;
        if (s.kind == 0 && (s.fmt == dedisp::kFmtSeg) != (c.sample_format == dedisp::kFmtSeg)) continue;
        if (s.kind == 1 || (s.waves == c.waves && s.dpw == c.dms_per_wave &&
                            s.m == c.words_per_lane && s.cc == c.chunk_chans)) {
            if (index) *index = i;
            return &s;
        }
    }
    return nullptr;
}

// Default shape: the first compiled tiled shape of this scratch format.
dedisp_tile_config default_config(int fmt)
{
    dedisp_tile_config c{};
    for (int i = 0; i < dedisp::shape_count(); ++i) {
        const Shape& s = dedisp::shape_at(i);
        if (s.kind == 0 && s.fmt == fmt) {
            c.kind = 0;
            c.waves = s.waves;
            c.dms_per_wave = s.dpw;
            c.words_per_lane = s.m;
            c.chunk_chans = s.cc;
            return c;
        }
    }
    c.kind = 1;
    return c;
}

dedisp_status ensure_device_table(dedisp_plan p)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (p->device >= 0 && p->device != dev)
        return fail(DEDISP_ERR_UNSUPPORTED, "plan used on a second device");
    p->device = dev;
    if (!p->d_table) {
        const size_t bytes = p->table.size() * sizeof(int32_t);
        hipError_t e = hipMalloc(&p->d_table, bytes);
        if (e != hipSuccess) {
            p->d_table = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc delay table");
        }
        HIP_TRY(hipMemcpy(p->d_table, p->table.data(), bytes, hipMemcpyHostToDevice));
    }
    if (!p->killmask.empty() && !p->d_chanmap) {
        std::vector<int32_t> map(p->nchans, -1);
        for (size_t k = 0; k < p->active.size(); ++k) map[p->active[k]] = static_cast<int32_t>(k);
        const size_t bytes = map.size() * sizeof(int32_t);
        if (hipMalloc(&p->d_chanmap, bytes) != hipSuccess) {
            p->d_chanmap = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc channel map");
        }
        if (hipMalloc(&p->d_mask, bytes) != hipSuccess) {
            p->d_mask = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc kill mask");
        }
        HIP_TRY(hipMemcpy(p->d_chanmap, map.data(), bytes, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_mask, p->killmask.data(), bytes, hipMemcpyHostToDevice));
    }
    return DEDISP_OK;
}

dedisp_status ensure_block_tables(dedisp_plan p, int db, int fmt, BlockTables** out)
{
    auto it = p->blocks.find(block_key(db, fmt));
    if (it == p->blocks.end()) {
        BlockTables bt;
        build_block_tables(*p, db, fmt, bt);
        it = p->blocks.emplace(block_key(db, fmt), std::move(bt)).first;
    }
    BlockTables& bt = it->second;
    if (!bt.d_rel) {
        dedisp_status st = ensure_device_table(p);
        if (st != DEDISP_OK) return st;
        const size_t rb = bt.rel.size() * sizeof(uint32_t), bb = bt.base.size() * sizeof(int32_t);
        if (hipMalloc(&bt.d_rel, rb) != hipSuccess) {
            bt.d_rel = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc window table");
        }
        if (hipMalloc(&bt.d_base, bb) != hipSuccess) {
            (void)hipFree(bt.d_rel);
            bt.d_rel = nullptr;
            bt.d_base = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc window table");
        }
        HIP_TRY(hipMemcpy(bt.d_rel, bt.rel.data(), rb, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(bt.d_base, bt.base.data(), bb, hipMemcpyHostToDevice));
    }
    *out = &bt;
    return DEDISP_OK;
}

// Window length (32-bit words per channel row in LDS, a multiple of 4) of
// shape s: a lane reads words up to rel / (samples per word) + 64*m.
// (Interleaved bit planes: offsets are in words, and a lane reads no word
// past its last.)
int window_words(const BlockTables& bt, const Shape& s)
{
    if (s.fmt == dedisp::kFmtSeg) return (bt.relmax + 64 * s.m + 3) & ~3;
    return ((bt.relmax / dedisp::fmt_samples_per_word(s.fmt) + 64 * s.m + 1) + 3) & ~3;
}

// LDS bytes of one staged chunk: bit-plane shapes stage both planes of
// every channel in rows of a fixed length.
int chunk_lds_bytes(const Shape& s, int rw)
{
    if (s.fmt == dedisp::kFmtPlane) return s.cc * 2 * dedisp::kPlaneRowWords * 4;
    if (s.fmt == dedisp::kFmtSeg) return s.cc * 2 * dedisp::kSegRowWords * 4;
    return s.cc * rw * 4;
}

bool shape_fits(const BlockTables& bt, const Shape& s)
{
    const int rw = window_words(bt, s);
    if (s.fmt == dedisp::kFmtPlane && rw > dedisp::kPlaneRowWords) return false;
    if (s.fmt == dedisp::kFmtSeg && rw > dedisp::kSegRowWords) return false;
    return bt.relmax < 0x10000 && (rw >> 2) <= 64 * s.pi &&
           static_cast<long long>(chunk_lds_bytes(s, rw)) <= dedisp::kMaxLdsBytes;
}

// The tiled path reads input rows as 32-bit words and keeps unscrunched
// 2-bit sums in 16-bit lanes.
bool tiled_supported(const dedisp_plan_s& p)
{
    return (p.internal || p.row_bytes % 4 == 0) && p.nact() >= 1 &&
           (p.fmt != kFmtNib || p.nact_padded() <= 21845) &&
           (p.fmt != dedisp::kFmtPlane || (p.nact_padded() <= dedisp::kPlaneMaxChans && p.ngroups == 1));
}

// Channels summed into the packed lanes of the small-value formats between
// flushes: an even count whose sum cannot carry out of a lane.
int flush_channels(const dedisp_plan_s& p)
{
    const int v = p.value_bound();
    const int lane_max = p.fmt == kFmtByteS ? 255 : 65535;
    return std::max(2, std::min(1 << 20, lane_max / v) & ~1);
}

// Resolve the shape used for this plan: the requested one if its LDS window
// fits, else the first compiled tiled shape of the same bit depth that fits,
// else the untiled kernel.  Host-only (no HIP call) when `upload` is false.
dedisp_status resolve_launch(dedisp_plan p, const dedisp_tile_config& want, bool upload,
                             LaunchPlan& lp, bool multi_only, long long nout)
{
    const bool seg_ok = nout < 0 || nout >= dedisp::kSegMinOutPerDelay * p->max_delay;
    int idx = -1;
    if (!find_shape(want, *p, &idx)) return fail(DEDISP_ERR_INVALID_ARG, "unknown tile shape");
    std::vector<int> order{idx};
    for (int i = 0; i < dedisp::shape_count(); ++i)
        if (i != idx) order.push_back(i);
    if (multi_only) {
        std::vector<int> keep;
        for (int i : order)
            if (dedisp::shape_at(i).multi) keep.push_back(i);
        order.swap(keep);
    }
    std::map<int, BlockTables> host_tables;
    if (want.kind == 1 && !multi_only) order.clear();
    for (int i : order) {
        const Shape& s = dedisp::shape_at(i);
        if (s.kind != 0 || !shape_matches(s, *p) || !tiled_supported(*p)) continue;
        if (s.fmt == dedisp::kFmtSeg && !seg_ok) continue;
        const int db = s.waves * s.dpw;
        const int key = block_key(db, s.fmt);
        const BlockTables* bt = nullptr;
        auto it = p->blocks.find(key);
        if (it != p->blocks.end()) {
            bt = &it->second;
        } else {
            auto h = host_tables.find(key);
            if (h == host_tables.end()) {
                h = host_tables.emplace(key, BlockTables{}).first;
                build_block_tables(*p, db, s.fmt, h->second);
            }
            bt = &h->second;
        }
        if (!shape_fits(*bt, s)) continue;
        lp.shape_index = i;
        lp.shape = s;
        lp.cc = s.cc;
        lp.rw = window_words(*bt, s);
        lp.lds = chunk_lds_bytes(s, lp.rw);
        // Double-buffer the staged chunk (one barrier per chunk instead of
        // two) when that keeps as many workgroups resident per CU: at most
        // 16 waves per CU run at the tiled kernels' register counts, so a
        // CU holds min(16 / waves, LDS / bytes per workgroup) workgroups.
        {
            const int by_waves = std::max(1, 16 / s.waves);
            const int single = std::min(by_waves, dedisp::kMaxLdsBytes / lp.lds);
            const int twice = std::min(by_waves, dedisp::kMaxLdsBytes / (2 * lp.lds));
            lp.dbuf = (twice >= 1 && twice >= single) ? 1 : 0;
        }
        if (lp.dbuf) lp.lds *= 2;
        lp.nbits = p->nbits;
        lp.flush_every = flush_channels(*p);
        lp.bt = nullptr;
        if (upload) {
            BlockTables* dbt = nullptr;
            dedisp_status st = ensure_block_tables(p, db, s.fmt, &dbt);
            if (st != DEDISP_OK) return st;
            lp.bt = dbt;
        }
        return DEDISP_OK;
    }
    if (p->internal) {
        // a grouped pass: read the scratch straight from global memory
        lp.shape_index = -1;
        lp.shape = Shape{2, p->fmt, 4, 1, 1, 0, 0, 0};
        lp.nbits = p->nbits;
        lp.cc = lp.rw = lp.lds = 0;
        lp.flush_every = 1;
        lp.bt = nullptr;
        if (upload) return ensure_device_table(p);
        return DEDISP_OK;
    }
    dedisp_tile_config u{};
    u.kind = 1;
    if (!find_shape(u, *p, &idx)) return fail(DEDISP_ERR_UNSUPPORTED, "no untiled kernel");
    lp.shape_index = idx;
    lp.nbits = p->nbits;
    lp.shape = dedisp::shape_at(idx);
    lp.cc = lp.rw = lp.lds = 0;
    lp.bt = nullptr;
    if (upload) return ensure_device_table(p);
    return DEDISP_OK;
}

long long tile_len(const Shape& s) { return 64LL * dedisp::fmt_samples_per_word(s.fmt) * s.m; }

// Row pitch in bytes of the channel-major scratch holding nsamps samples of
// format fmt: a staged window starts before the last sample and spans 4*rw
// bytes.  The interleaved bit planes hold seg_row_words words (a window
// starts before word seg_len + max_delay).
long long xc_pitch(long long nsamps, int fmt, int rw, long long max_delay)
{
    if (fmt == dedisp::kFmtSeg)
        return ((4 * dedisp::seg_row_words(nsamps - max_delay, max_delay, rw) + 63) / 64) * 64;
    const long long num = dedisp::fmt_bytes_num(fmt), den = dedisp::fmt_bytes_den(fmt);
    const long long bytes = (nsamps * num + den - 1) / den;
    return ((bytes + 4LL * rw + 63) / 64) * 64;
}

void free_scratch(Scratch& x)
{
    if (x.ptr) {
        if (x.owner) x.owner->wait();
        else (void)hipDeviceSynchronize();
        (void)hipFree(x.ptr);
    }
    x.ptr = nullptr;
    x.bytes = 0;
}

dedisp_status ensure_scratch(Scratch& x, size_t need)
{
    if (x.ptr && x.bytes >= need) return DEDISP_OK;
    free_scratch(x);
    if (hipMalloc(&x.ptr, need) != hipSuccess) {
        x.ptr = nullptr;
        return fail(DEDISP_ERR_OOM, "hipMalloc channel-major scratch");
    }
    x.bytes = need;
    return DEDISP_OK;
}

dedisp_status ensure_xc(const dedisp_plan_s& p, Scratch& x, long long nsamps, const LaunchPlan& lp)
{
    if (lp.shape.kind != 0) return DEDISP_OK;
    const long long ns = nsamps / p.scrunch;
    return ensure_scratch(x, static_cast<size_t>(xc_pitch(ns, lp.shape.fmt, lp.rw, p.max_delay)) * p.nact_padded() *
                                 dedisp::fmt_rows(lp.shape.fmt));
}

void fill_desc(dedisp_plan p, const LaunchPlan& lp, const void* in0, long long n0,
               const void* in1, long long nsamps, uint32_t* out, long long stride,
               uint8_t* xc, BeamDesc& d)
{
    std::memset(&d, 0, sizeof(d));
    d.in0 = static_cast<const uint8_t*>(in0);
    d.in1 = static_cast<const uint8_t*>(in1);
    d.n0 = n0;
    d.nsamps = nsamps;
    d.nout = nsamps / p->scrunch - p->max_delay;
    d.scrunch = p->scrunch;
    d.rowmap = nullptr;
    d.ngroups = 1;
    d.ndm_last = static_cast<int>(p->dms.size());
    d.out = out;
    d.out_bytes = p->out_nbits / 8;
    d.out_shift = p->out_shift;
    // narrow outputs: row stride in bytes
    d.out_stride = d.out_bytes == 4 ? stride : stride * d.out_bytes;
    d.table = p->d_table;
    d.chanmap = p->d_chanmap;
    d.mask = p->d_mask;
    d.nact = p->nact_padded();
    d.pad_row = p->nact() < p->nact_padded() ? p->nact() : -1;
    d.nchans = p->nchans;
    d.row_bytes = p->row_bytes;
    d.ndm = static_cast<int>(p->dms.size());
    d.shape = lp.shape_index;
    if (lp.shape.kind == 0) {
        d.xc = xc;
        d.xc_fmt = lp.shape.fmt;
        d.pitch = xc_pitch(nsamps / p->scrunch, lp.shape.fmt, lp.rw, p->max_delay);
        d.rel = lp.bt->d_rel;
        d.base = lp.bt->d_base;
        d.nblocks = lp.bt->nblocks;
        d.ntiles = static_cast<int>((d.nout + tile_len(lp.shape) - 1) / tile_len(lp.shape));
        d.rw = lp.rw;
        d.flush_every = lp.flush_every;
        d.dbuf = lp.dbuf;
    }
}

hipError_t launch_desc(const BeamDesc& d, const LaunchPlan& lp, hipStream_t st)
{
    if (lp.shape.kind == 0) {
        hipError_t e = dedisp::launch_unpack(d, lp.nbits, lp.shape.fmt, st);
        if (e != hipSuccess) return e;
        return dedisp::launch_tiled(d, lp.shape, lp.lds, st);
    }
    return dedisp::launch_untiled(d, lp.nbits, st);
}


// --------------------------------------------------------------- tune cache

std::string cache_key(dedisp_plan p, size_t nsamps)
{
    size_t bucket = 1;
    while (bucket < nsamps) bucket <<= 1;
    std::ostringstream os;
    os << "nbits=" << p->nbits << ",fmt=" << p->fmt << ",scrunch=" << p->scrunch
       << ",nchans=" << p->nchans << ",ndm=" << p->dms.size()
       << ",max_delay=" << p->max_delay << ",nsamps<=" << bucket;
    return os.str();
}

// The cache file is a JSON object {"key": [kind, waves, dpw, m, cc, ms], ...}.
std::map<std::string, std::vector<double>> read_cache(const char* path)
{
    std::map<std::string, std::vector<double>> m;
    if (!path) return m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while (true) {
        size_t k0 = s.find('"', i);
        if (k0 == std::string::npos) break;
        size_t k1 = s.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        size_t a0 = s.find('[', k1);
        size_t a1 = s.find(']', a0 == std::string::npos ? k1 : a0);
        if (a0 == std::string::npos || a1 == std::string::npos) break;
        std::vector<double> v;
        std::stringstream vs(s.substr(a0 + 1, a1 - a0 - 1));
        std::string tok;
        while (std::getline(vs, tok, ',')) v.push_back(std::atof(tok.c_str()));
        m[s.substr(k0 + 1, k1 - k0 - 1)] = v;
        i = a1 + 1;
    }
    return m;
}

void write_cache(const char* path, const std::map<std::string, std::vector<double>>& m)
{
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\n";
        size_t n = 0;
        for (const auto& kv : m) {
            f << "  \"" << kv.first << "\": [";
            for (size_t j = 0; j < kv.second.size(); ++j) f << (j ? ", " : "") << kv.second[j];
            f << "]" << (++n < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

void destroy_tree(dedisp_plan p)
{
    if (p->d_tree_rows || p->d_tree_delay || p->d_tree_pairs || p->d_tree_stage || p->d_tree_sblocks ||
        p->d_tree_off || p->d_tree_gtrials)
        p->inflight.wait();
    if (p->d_tree_rows) (void)hipFree(p->d_tree_rows);
    if (p->d_tree_delay) (void)hipFree(p->d_tree_delay);
    if (p->d_tree_pairs) (void)hipFree(p->d_tree_pairs);
    if (p->d_tree_stage) (void)hipFree(p->d_tree_stage);
    if (p->d_tree_sblocks) (void)hipFree(p->d_tree_sblocks);
    if (p->d_tree_off) (void)hipFree(p->d_tree_off);
    if (p->d_tree_gtrials) (void)hipFree(p->d_tree_gtrials);
    p->d_tree_rows = p->d_tree_delay = p->d_tree_pairs = nullptr;
    p->d_tree_stage = nullptr;
    p->d_tree_sblocks = p->d_tree_off = p->d_tree_gtrials = nullptr;
    p->tree_stage.clear();
    p->tree_sblocks.clear();
    p->tree_off.clear();
    p->tree_gtrials.clear();
    p->tree_lds = 0;
    p->tree_span = 0;
    p->tree_rows.clear();
    p->tree_delay.clear();
    p->tree_pairs.clear();
    p->tree_nsub = 0;
    p->tree_maxdelay = 0;
    p->tree_npass = 0;
    for (auto& g : p->groups)
        if (g.sub && g.sub->tree_nsub) destroy_tree(g.sub);
}

void destroy_subband(dedisp_plan p)
{
    if (p->sb_step1 || p->sb_step2) p->inflight.wait();   // the passes' tables serve p's executes
    dedisp_plan_destroy(p->sb_step1);
    dedisp_plan_destroy(p->sb_step2);
    p->sb_step1 = p->sb_step2 = nullptr;
    free_scratch(p->sb_xc2);
    p->sb_nsub = p->sb_ngroup = 0;
}

// An internal plan for one pass of a grouped (sub-band) transform.
dedisp_plan new_internal(const dedisp_plan_s& p)
{
    dedisp_plan q = new (std::nothrow) dedisp_plan_s;
    if (!q) return nullptr;
    q->nbits = p.nbits;
    q->dt = p.dt;
    q->f_top = p.f_top;
    q->df = p.df;
    q->row_bytes = 4;
    q->internal = true;
    q->has_dms = true;
    return q;
}

void destroy_groups(dedisp_plan p)
{
    if (!p->groups.empty()) p->inflight.wait();   // the groups' tables serve p's executes
    for (auto& g : p->groups) {
        if (g.d_rows) (void)hipFree(g.d_rows);
        dedisp_plan_destroy(g.sub);
    }
    p->groups.clear();
    p->scrunch_factors.clear();
}

// Time-scrunching: the diagonal DM of the band (Section 2.1), where the delay
// between the last two channels -- the steepest part of the trail -- is one
// sample.
double diagonal_dm(const dedisp_plan_s& p)
{
    if (p.nchans < 2) return HUGE_VAL;
    const double inv_f0_sq = 1.0 / (p.f_top * p.f_top);
    const double samples_per_unit = kDispersionConstant / p.dt;
    const double fa = p.f_top + static_cast<double>(p.nchans - 2) * p.df;
    const double fb = p.f_top + static_cast<double>(p.nchans - 1) * p.df;
    const double dTa = samples_per_unit * (1.0 / (fa * fa) - inv_f0_sq);
    const double dTb = samples_per_unit * (1.0 / (fb * fb) - inv_f0_sq);
    return 1.0 / (dTb - dTa);
}

// Scratch format of the direct transform at full resolution: 2-bit codes as
// bit planes while every sum fits the planes' levels, else as nibbles; 8-bit
// codes as bytes.
int direct_format(int nbits, int nchans)
{
    if (nbits != 2) return kFmtByte;
    const int u = dedisp::fmt_chan_unit(dedisp::kFmtPlane);
    return (nchans + u - 1) / u * u <= dedisp::kPlaneMaxChans ? dedisp::kFmtPlane : kFmtNib;
}

// Scratch format of a scrunch group: sums of up to 8 two-bit codes stay in
// byte lanes (four samples per add, flushed at least every 10 channels);
// larger two-bit sums (at most 3*64 = 192) are bytes read through the 8-bit
// code path (one v_perm spreads two bytes into 16-bit lanes), the same VALU
// per sample as 16-bit scratch with half the bytes; 8-bit sums take 16 bits.
int scrunch_format(int nbits, int nchans, int s)
{
    if (s == 1) return direct_format(nbits, nchans);
    if (nbits == 2) return s <= 8 ? kFmtByteS : kFmtByte;
    return kFmtHalf;
}

constexpr int kMaxScrunch = 64;

// Valid outputs per row of a scrunch group for nsamps input rows (<= 0: too few).
long long group_nout(const ScrunchGroup& g, size_t nsamps)
{
    return static_cast<long long>(nsamps / g.s) - g.sub->max_delay;
}

}  // namespace host
}  // namespace dedisp

using namespace dedisp::host;

// =================================================================== C ABI

extern "C" {

const char* dedisp_status_string(dedisp_status s)
{
    switch (s) {
        case DEDISP_OK: return "DEDISP_OK";
        case DEDISP_ERR_INVALID_ARG: return "DEDISP_ERR_INVALID_ARG";
        case DEDISP_ERR_NO_DM_LIST: return "DEDISP_ERR_NO_DM_LIST";
        case DEDISP_ERR_TOO_FEW_SAMPLES: return "DEDISP_ERR_TOO_FEW_SAMPLES";
        case DEDISP_ERR_OOM: return "DEDISP_ERR_OOM";
        case DEDISP_ERR_HIP: return "DEDISP_ERR_HIP";
        case DEDISP_ERR_UNSUPPORTED: return "DEDISP_ERR_UNSUPPORTED";
        default: return "DEDISP_ERR_UNKNOWN";
    }
}

const char* dedisp_last_error(void) { return g_last_error.c_str(); }

dedisp_status dedisp_plan_create(dedisp_plan* out, int nchans, double dt_s, double f_top_mhz,
                                 double df_mhz, int nbits)
{
    if (!out) return fail(DEDISP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nchans <= 0) return fail(DEDISP_ERR_INVALID_ARG, "nchans must be positive");
    if (nbits != 2 && nbits != 8) return fail(DEDISP_ERR_INVALID_ARG, "nbits must be 2 or 8");
    if ((static_cast<long long>(nchans) * nbits) % 8)
        return fail(DEDISP_ERR_INVALID_ARG, "nchans*nbits must be a multiple of 8");
    if (!is_finite(dt_s) || !(dt_s > 0)) return fail(DEDISP_ERR_INVALID_ARG, "dt must be > 0");
    if (!is_finite(f_top_mhz) || !(f_top_mhz > 0))
        return fail(DEDISP_ERR_INVALID_ARG, "f_top must be > 0");
    if (!is_finite(df_mhz) || !(df_mhz < 0)) return fail(DEDISP_ERR_INVALID_ARG, "df must be < 0");
    if (!(f_top_mhz + static_cast<double>(nchans - 1) * df_mhz > 0))
        return fail(DEDISP_ERR_INVALID_ARG, "band reaches zero frequency");
    dedisp_plan p = new (std::nothrow) dedisp_plan_s;
    if (!p) return fail(DEDISP_ERR_OOM, "plan allocation");
    p->nchans = nchans;
    p->nbits = nbits;
    p->dt = dt_s;
    p->f_top = f_top_mhz;
    p->df = df_mhz;
    p->row_bytes = nchans * nbits / 8;
    p->fmt = direct_format(nbits, nchans);
    p->cfg = default_config(p->fmt);
    *out = p;
    return DEDISP_OK;
}

void dedisp_plan_destroy(dedisp_plan p)
{
    if (!p) return;
    destroy_tree(p);
    destroy_subband(p);
    destroy_groups(p);
    free_device(p);
    delete p;
}

dedisp_status dedisp_set_dm_list(dedisp_plan p, const double* dms, int ndm)
{
    if (!p || !dms) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (ndm <= 0) return fail(DEDISP_ERR_INVALID_ARG, "ndm must be positive");
    for (int d = 0; d < ndm; ++d)
        if (!is_finite(dms[d]) || dms[d] < 0)
            return fail(DEDISP_ERR_INVALID_ARG, "DMs must be finite and >= 0");
    std::vector<int32_t> table;
    int mx = 0;
    if (!build_delay_table(*p, dms, ndm, table, mx))
        return fail(DEDISP_ERR_INVALID_ARG, "a delay does not fit in int32");
    destroy_tree(p);
    destroy_subband(p);
    destroy_groups(p);
    free_device(p);
    p->dms.assign(dms, dms + ndm);
    p->table.swap(table);
    p->max_delay = mx;
    p->has_dms = true;
    return DEDISP_OK;
}

dedisp_status dedisp_set_killmask(dedisp_plan p, const int32_t* mask)
{
    if (!p) return fail(DEDISP_ERR_INVALID_ARG, "NULL plan");
    std::vector<int32_t> km, act;
    if (mask) {
        bool all_on = true;
        for (int c = 0; c < p->nchans; ++c) {
            if (mask[c] != 0 && mask[c] != 1)
                return fail(DEDISP_ERR_INVALID_ARG, "kill mask entries must be 0 or 1");
            if (mask[c]) act.push_back(c);
            else all_on = false;
        }
        if (!all_on) km.assign(mask, mask + p->nchans);
        else act.clear();
    }
    for (auto& g : p->groups) {
        dedisp_status st = dedisp_set_killmask(g.sub, mask);
        if (st != DEDISP_OK) return st;
    }
    free_device(p);
    p->killmask.swap(km);
    p->active.swap(act);
    return DEDISP_OK;
}

dedisp_status dedisp_get_nchans(dedisp_plan p, int* v)
{
    if (!p || !v) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    *v = p->nchans;
    return DEDISP_OK;
}

dedisp_status dedisp_get_nbits(dedisp_plan p, int* v)
{
    if (!p || !v) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    *v = p->nbits;
    return DEDISP_OK;
}

dedisp_status dedisp_get_dm_count(dedisp_plan p, int* v)
{
    if (!p || !v) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    *v = static_cast<int>(p->dms.size());
    return DEDISP_OK;
}

dedisp_status dedisp_get_max_delay(dedisp_plan p, int* v)
{
    if (!p || !v) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    *v = p->max_delay;
    return DEDISP_OK;
}

dedisp_status dedisp_get_delay_table(dedisp_plan p, int32_t* host_out)
{
    if (!p || !host_out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    std::memcpy(host_out, p->table.data(), p->table.size() * sizeof(int32_t));
    return DEDISP_OK;
}

int dedisp_tile_config_count(void) { return dedisp::shape_count(); }

dedisp_status dedisp_tile_config_get(int i, dedisp_tile_config* c)
{
    if (!c || i < 0 || i >= dedisp::shape_count())
        return fail(DEDISP_ERR_INVALID_ARG, "bad index");
    const Shape& s = dedisp::shape_at(i);
    c->kind = s.kind;
    c->waves = s.kind == 0 ? s.waves : 4;
    c->dms_per_wave = s.dpw;
    c->words_per_lane = s.m;
    c->chunk_chans = s.cc;
    c->sample_format = s.kind == 0 ? s.fmt : -1;
    return DEDISP_OK;
}

dedisp_status dedisp_set_tile_config(dedisp_plan p, const dedisp_tile_config* c)
{
    if (!p || !c) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!find_shape(*c, *p)) return fail(DEDISP_ERR_INVALID_ARG, "unknown tile shape");
    p->cfg = *c;
    for (auto& g : p->groups)
        if (find_shape(*c, *g.sub)) g.sub->cfg = *c;
    for (dedisp_plan q : {p->sb_step1, p->sb_step2})
        if (q && c->kind == 0 && find_shape(*c, *q)) q->cfg = *c;
    return DEDISP_OK;
}

dedisp_status dedisp_get_tile_config(dedisp_plan p, dedisp_tile_config* c)
{
    if (!p || !c) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    LaunchPlan lp;
    dedisp_status st = resolve_launch(p, p->cfg, false, lp);
    if (st != DEDISP_OK) return st;
    c->kind = lp.shape.kind;
    c->waves = lp.shape.kind == 0 ? lp.shape.waves : 4;
    c->dms_per_wave = lp.shape.dpw;
    c->words_per_lane = lp.shape.m;
    c->chunk_chans = lp.cc;
    c->sample_format = lp.shape.kind == 0 ? lp.shape.fmt : -1;
    return DEDISP_OK;
}

static dedisp_status execute_groups(dedisp_plan p, const void* d_in, size_t nsamps,
                                    uint32_t* d_out, size_t stride, void* stream)
{
    if (nsamps > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "nsamps too large");
    long long width = 0;
    for (const auto& g : p->groups) {
        const long long n = group_nout(g, nsamps);
        if (n <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps / s <= max delay of a scrunch group");
        width = std::max(width, n);
    }
    if (stride == 0) stride = static_cast<size_t>(width);
    if (stride < static_cast<size_t>(width))
        return fail(DEDISP_ERR_INVALID_ARG, "out_row_stride < longest output row");
    // resolve every group first (all validation before any launch)
    std::vector<LaunchPlan> lps(p->groups.size());
    size_t need = 0;
    for (size_t i = 0; i < p->groups.size(); ++i) {
        dedisp_plan sub = p->groups[i].sub;
        const long long gout = static_cast<long long>(nsamps) / sub->scrunch - sub->max_delay;
        dedisp_status st = resolve_launch(sub, sub->cfg, true, lps[i], false, gout);
        if (st != DEDISP_OK) return st;
        if (lps[i].shape.kind == 0 && (reinterpret_cast<uintptr_t>(d_in) & 3)) {
            dedisp_tile_config u{};
            u.kind = 1;
            st = resolve_launch(sub, u, true, lps[i]);
            if (st != DEDISP_OK) return st;
        }
        if (lps[i].shape.kind == 0) {
            const long long ns = static_cast<long long>(nsamps) / sub->scrunch;
            need = std::max(need, static_cast<size_t>(xc_pitch(ns, lps[i].shape.fmt, lps[i].rw, sub->max_delay)) *
                                      sub->nact_padded() * dedisp::fmt_rows(lps[i].shape.fmt));
        }
        ScrunchGroup& g = p->groups[i];
        if (!g.d_rows) {
            const size_t bytes = g.rows.size() * sizeof(int32_t);
            if (hipMalloc(&g.d_rows, bytes) != hipSuccess) {
                g.d_rows = nullptr;
                return fail(DEDISP_ERR_OOM, "hipMalloc scrunch row map");
            }
            HIP_TRY(hipMemcpy(g.d_rows, g.rows.data(), bytes, hipMemcpyHostToDevice));
        }
    }
    // the groups run one after another on one stream and share one scratch
    dedisp_status st = ensure_scratch(p->xc, std::max<size_t>(need, 1));
    if (st != DEDISP_OK) return st;
    for (size_t i = 0; i < p->groups.size(); ++i) {
        BeamDesc d;
        fill_desc(p->groups[i].sub, lps[i], d_in, static_cast<long long>(nsamps), nullptr,
                  static_cast<long long>(nsamps), d_out, static_cast<long long>(stride),
                  p->xc.ptr, d);
        d.rowmap = p->groups[i].d_rows;
        hipError_t e = launch_desc(d, lps[i], static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    return DEDISP_OK;
}

// Sub-band dedispersion: sub-band sums of step 1 (lengths len1) and the
// outputs of step 2 (nout) for nsamps input rows.
static void subband_lengths(const dedisp_plan_s& p, size_t nsamps, long long& len1, long long& nout)
{
    len1 = static_cast<long long>(nsamps) - p.sb_step1->max_delay;
    nout = len1 - p.sb_step2->max_delay;
}

static dedisp_status tree_upload(dedisp_plan p);
static dedisp_status combine_rows(dedisp_plan q, const dedisp_plan_s& outp, uint8_t* xc, long long pitch, int ob,
                                  int nsb, int row_max, int ndm, long long nout, uint32_t* d_out, size_t stride,
                                  const int32_t* rowmap, hipStream_t hs);

static dedisp_status execute_subband(dedisp_plan p, const void* d_in, size_t nsamps,
                                     uint32_t* d_out, size_t stride, void* stream)
{
    if (nsamps > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "nsamps too large");
    dedisp_plan s1 = p->sb_step1, s2 = p->sb_step2;
    long long len1 = 0, nout = 0;
    subband_lengths(*p, nsamps, len1, nout);
    if (len1 <= 0 || nout <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps too short for the sub-band passes");
    if (stride == 0) stride = static_cast<size_t>(nout);
    if (stride < static_cast<size_t>(nout)) return fail(DEDISP_ERR_INVALID_ARG, "out_row_stride < nout");
    if (reinterpret_cast<uintptr_t>(d_in) & 3)
        return fail(DEDISP_ERR_INVALID_ARG, "sub-band passes need 4-byte aligned input");
    LaunchPlan lp1, lp2;
    dedisp_status st = resolve_launch(s1, s1->cfg, true, lp1);
    if (st != DEDISP_OK) return st;
    st = resolve_launch(s2, s2->cfg, true, lp2);
    if (st != DEDISP_OK) return st;
    st = ensure_device_table(p);
    if (st != DEDISP_OK) return st;
    const int nsub = p->sb_nsub, ngroup = p->sb_ngroup;
    const int nsb = p->nchans / nsub, nsb_p = s2->nchans, nnom = s1->ndm_last;
    const long long pitch1 = xc_pitch(static_cast<long long>(nsamps), s1->fmt, lp1.rw, 0);
    const long long pitch2 = xc_pitch(len1, s2->fmt, lp2.rw, 0);
    st = ensure_scratch(p->xc, static_cast<size_t>(pitch1) * p->nchans);
    if (st != DEDISP_OK) return st;
    st = ensure_scratch(p->sb_xc2, static_cast<size_t>(pitch2) * nsb_p * nnom);
    if (st != DEDISP_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);

    // corner turn: every channel keeps its row (killed channels are zeros)
    BeamDesc d0;
    std::memset(&d0, 0, sizeof(d0));
    d0.in0 = static_cast<const uint8_t*>(d_in);
    d0.n0 = d0.nsamps = static_cast<long long>(nsamps);
    d0.xc = p->xc.ptr;
    d0.pitch = pitch1;
    d0.mask = p->d_mask;
    d0.nact = p->nchans;
    d0.pad_row = -1;
    d0.nchans = p->nchans;
    d0.row_bytes = p->row_bytes;
    d0.scrunch = 1;
    d0.ngroups = 1;
    d0.out_bytes = 4;
    hipError_t e = dedisp::launch_unpack(d0, p->nbits, s1->fmt, hs);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (nsb_p > nsb) {
        e = dedisp::launch_zero(p->sb_xc2.ptr + static_cast<long long>(nsb) * pitch2,
                                static_cast<long long>(nsb_p) * pitch2,
                                static_cast<long long>(nsb_p - nsb) * pitch2, nnom, hs);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    // step 1: every sub-band at every nominal DM, written as narrow sums into
    // row m*nsb_p + n of the intermediate scratch
    BeamDesc d1;
    std::memset(&d1, 0, sizeof(d1));
    d1.xc = p->xc.ptr;
    d1.pitch = pitch1;
    d1.nact = nsub;
    d1.pad_row = -1;
    d1.nchans = nsub;
    d1.ndm = d1.ndm_last = nnom;
    d1.nout = len1;
    if (lp1.shape.kind == 0) {
        d1.rel = lp1.bt->d_rel;
        d1.base = lp1.bt->d_base;
        d1.nblocks = lp1.bt->nblocks;
        d1.ntiles = static_cast<int>((len1 + tile_len(lp1.shape) - 1) / tile_len(lp1.shape));
        d1.g_rel = static_cast<long long>(lp1.bt->nblocks) * lp1.bt->db * (nsub / 2);
        d1.g_base = static_cast<long long>(lp1.bt->nblocks) * nsub;
    }
    d1.table = s1->d_table;
    d1.rw = lp1.rw;
    d1.flush_every = lp1.flush_every;
    d1.dbuf = lp1.dbuf;
    d1.shape = lp1.shape_index;
    d1.scrunch = 1;
    d1.ngroups = nsb;
    d1.g_xc = static_cast<long long>(nsub) * pitch1;
    d1.out = reinterpret_cast<uint32_t*>(p->sb_xc2.ptr);
    d1.out_bytes = dedisp::fmt_bytes_num(s2->fmt);
    d1.out_stride = static_cast<long long>(nsb_p) * pitch2;
    d1.g_out = pitch2;
    e = lp1.shape.kind == 0 ? dedisp::launch_tiled(d1, lp1.shape, lp1.lds, hs)
                            : dedisp::launch_untiled_xc(d1, s1->fmt, hs);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (!s2->tree_rows.empty() && s2->fmt != kFmtHalf) {
        // step 2 as the combination of per-sub-band rows (byte sums)
        st = tree_upload(s2);
        if (st != DEDISP_OK) return st;
        return combine_rows(s2, *p, p->sb_xc2.ptr, pitch2, 1, nsb, s2->vbound, static_cast<int>(p->dms.size()), nout,
                            d_out, stride, nullptr, hs);
    }
    // step 2: for every nominal DM, its trials over the miniature filterbank
    BeamDesc d2;
    std::memset(&d2, 0, sizeof(d2));
    d2.xc = p->sb_xc2.ptr;
    d2.pitch = pitch2;
    d2.nact = nsb_p;
    d2.pad_row = -1;
    d2.nchans = nsb_p;
    d2.ndm = ngroup;
    d2.ndm_last = s2->ndm_last;
    d2.nout = nout;
    if (lp2.shape.kind == 0) {
        d2.rel = lp2.bt->d_rel;
        d2.base = lp2.bt->d_base;
        d2.nblocks = lp2.bt->nblocks;
        d2.ntiles = static_cast<int>((nout + tile_len(lp2.shape) - 1) / tile_len(lp2.shape));
        d2.g_rel = static_cast<long long>(lp2.bt->nblocks) * lp2.bt->db * (nsb_p / 2);
        d2.g_base = static_cast<long long>(lp2.bt->nblocks) * nsb_p;
    }
    d2.table = s2->d_table;
    d2.rw = lp2.rw;
    d2.flush_every = lp2.flush_every;
    d2.dbuf = lp2.dbuf;
    d2.shape = lp2.shape_index;
    d2.scrunch = 1;
    d2.ngroups = nnom;
    d2.g_xc = static_cast<long long>(nsb_p) * pitch2;
    d2.out = d_out;
    d2.out_bytes = p->out_nbits / 8;
    d2.out_shift = p->out_shift;
    {
        const long long unit = d2.out_bytes == 4 ? 1 : d2.out_bytes;   // narrow: bytes
        d2.out_stride = static_cast<long long>(stride) * unit;
        d2.g_out = static_cast<long long>(ngroup) * static_cast<long long>(stride) * unit;
    }
    e = lp2.shape.kind == 0 ? dedisp::launch_tiled(d2, lp2.shape, lp2.lds, hs)
                            : dedisp::launch_untiled_xc(d2, s2->fmt, hs);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return DEDISP_OK;
}

// Piecewise linear tree: stage-1 length and outputs for nsamps input rows.
static void tree_lengths(const dedisp_plan_s& p, size_t nsamps, long long& len1, long long& nout)
{
    // on the plan's (scrunched) samples: pass p reads p (nsub - 1) samples
    // further, and its tree another nsub - 1
    len1 = static_cast<long long>(nsamps) / p.scrunch - static_cast<long long>(p.tree_npass) * (p.tree_nsub - 1);
    nout = len1 - p.tree_maxdelay;
}

// The plan whose rows a tree run covers: the plan itself, or each scrunch
// group's plan (rows placed through the group's row map).
static dedisp_status tree_upload(dedisp_plan p)
{
    dedisp_status st = ensure_device_table(p);
    if (st != DEDISP_OK) return st;
    if (!p->d_tree_rows) {
        const size_t bytes = p->tree_rows.size() * sizeof(int32_t);
        if (hipMalloc(&p->d_tree_rows, bytes) != hipSuccess) {
            p->d_tree_rows = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc tree tables");
        }
        if (hipMalloc(&p->d_tree_delay, bytes) != hipSuccess) {
            p->d_tree_delay = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc tree tables");
        }
        HIP_TRY(hipMemcpy(p->d_tree_rows, p->tree_rows.data(), bytes, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_tree_delay, p->tree_delay.data(), bytes, hipMemcpyHostToDevice));
    }
    if (!p->d_tree_pairs && !p->tree_pairs.empty()) {
        const size_t bytes = p->tree_pairs.size() * sizeof(int32_t);
        if (hipMalloc(&p->d_tree_pairs, bytes) != hipSuccess) {
            p->d_tree_pairs = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc tree tables");
        }
        HIP_TRY(hipMemcpy(p->d_tree_pairs, p->tree_pairs.data(), bytes, hipMemcpyHostToDevice));
    }
    auto upload = [](void** dst, const void* src, size_t bytes) -> dedisp_status {
        if (*dst || bytes == 0) return DEDISP_OK;
        if (hipMalloc(dst, bytes) != hipSuccess) {
            *dst = nullptr;
            return fail(DEDISP_ERR_OOM, "hipMalloc tree tables");
        }
        HIP_TRY(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return DEDISP_OK;
    };
    dedisp_status s2 = upload(reinterpret_cast<void**>(&p->d_tree_stage), p->tree_stage.data(),
                              p->tree_stage.size() * sizeof(dedisp::TreeStage));
    if (s2 == DEDISP_OK)
        s2 = upload(reinterpret_cast<void**>(&p->d_tree_sblocks), p->tree_sblocks.data(),
                    p->tree_sblocks.size() * sizeof(int32_t));
    if (s2 == DEDISP_OK)
        s2 = upload(reinterpret_cast<void**>(&p->d_tree_off), p->tree_off.data(), p->tree_off.size() * sizeof(int32_t));
    if (s2 == DEDISP_OK)
        s2 = upload(reinterpret_cast<void**>(&p->d_tree_gtrials), p->tree_gtrials.data(),
                    p->tree_gtrials.size() * sizeof(int32_t));
    return s2;
}

// Tree rows are bytes while the largest sub-band sum fits (3 nsub for 2-bit
// codes up to nsub = 64, small scrunched sums), else 16 bits.
static int tree_row_bytes(const dedisp_plan_s& p)
{
    return static_cast<long long>(p.value_bound()) * p.tree_nsub <= 255 ? 1 : 2;
}

// The combination of per-sub-band rows (tree stage 2; sub-band step 2 with
// byte sums): out[d][t] = sum over the nsb sub-bands n of row q->tree_rows[d][n]
// of xc (pitch bytes, ob bytes per sample, values at most row_max) at sample
// t + q->tree_delay[d][n], for the ndm trials and t < nout, in outp's output
// format.  Dense trial blocks whose rows fit go through LDS (q->tree_sblocks),
// the rest are gathered.  Tables must be on the device (tree_upload).
static dedisp_status combine_rows(dedisp_plan q, const dedisp_plan_s& outp, uint8_t* xc, long long pitch, int ob,
                                  int nsb, int row_max, int ndm, long long nout, uint32_t* d_out, size_t stride,
                                  const int32_t* rowmap, hipStream_t hs)
{
    BeamDesc dg;
    std::memset(&dg, 0, sizeof(dg));
    dg.xc = xc;
    dg.pitch = pitch;
    dg.table = q->d_tree_delay;
    dg.rowsel = q->d_tree_rows;
    dg.rowmap = rowmap;
    dg.nact = nsb;
    dg.nchans = nsb;
    dg.ndm = dg.ndm_last = ndm;
    dg.ngroups = 1;
    dg.nout = nout;
    dg.scrunch = 1;
    dg.out = d_out;
    dg.out_bytes = outp.out_nbits / 8;
    dg.out_shift = outp.out_shift;
    dg.out_stride = static_cast<long long>(stride) * (dg.out_bytes == 4 ? 1 : dg.out_bytes);
    // 16-bit partial sums of at most 65535 / (largest row value) terms
    const int flush = 65535 / row_max;
    hipError_t e;
    // the staged kernel addresses a sub-band's rows with 32-bit offsets
    if (!q->tree_sblocks.empty() &&
        (std::max<long long>(q->tree_span, 4) + 1) * dg.pitch + 4LL * dedisp::kTreeTile < (1LL << 31)) {
        // the staged trial blocks through LDS, the rest gathered
        // rows below 128 let two terms be added as bytes first
        e = dedisp::launch_tree_combine_lds(dg, q->d_tree_sblocks, static_cast<int>(q->tree_sblocks.size()),
                                            q->d_tree_stage, q->d_tree_off, q->tree_lds, 2 * row_max <= 255, hs);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        if (!q->tree_gtrials.empty())
            e = dedisp::launch_tree_combine(dg, ob, flush, q->d_tree_gtrials,
                                            static_cast<int>(q->tree_gtrials.size()), hs);
    } else {
        e = dedisp::launch_tree_combine(dg, ob, flush, nullptr, 0, hs);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return DEDISP_OK;
}

// Enqueue one plan's tree: corner turn (scrunching for a group's plan),
// stage 1 per (sub-band, pass) pair, stage 2 into d_out rows (through rowmap
// when set).  Lengths, strides and tables are checked by the caller.
static dedisp_status run_tree(dedisp_plan p, const void* d_in, size_t nsamps, uint32_t* d_out,
                              size_t stride, const int32_t* rowmap, hipStream_t hs)
{
    long long len1 = 0, nout = 0;
    tree_lengths(*p, nsamps, len1, nout);
    const int nsub = p->tree_nsub, nsb = p->nchans / nsub;
    const int npairs = static_cast<int>(p->tree_pairs.size() / 2);
    const long long ns = static_cast<long long>(nsamps) / p->scrunch;
    // the tree kernel reads whole tiles (and one more word) past the last
    // sample, up to (npass - 1)(nsub - 1) samples further under an imposed
    // delay
    // stage 1 reads one row per channel: 2-bit codes as nibbles
    const int tfmt = p->fmt == dedisp::kFmtPlane ? kFmtNib : p->fmt;
    const long long pitch1 = xc_pitch(ns + dedisp::tree_tile(nsub) + nsub +
                                          static_cast<long long>(p->tree_npass - 1) * (nsub - 1) + 8,
                                      tfmt, 0, 0);
    const int ob = tree_row_bytes(*p);
    const long long pitch2 = ((ob * len1 + 64) + 63) / 64 * 64;
    dedisp_status st = ensure_scratch(p->xc, static_cast<size_t>(pitch1) * p->nchans);
    if (st != DEDISP_OK) return st;
    st = ensure_scratch(p->sb_xc2, static_cast<size_t>(pitch2) * npairs * nsub);
    if (st != DEDISP_OK) return st;
    // corner turn: every channel keeps its row (stage 1 reads killed ones as zeros)
    BeamDesc d0;
    std::memset(&d0, 0, sizeof(d0));
    d0.in0 = static_cast<const uint8_t*>(d_in);
    d0.n0 = d0.nsamps = static_cast<long long>(nsamps);
    d0.xc = p->xc.ptr;
    d0.pitch = pitch1;
    d0.mask = p->d_mask;
    d0.nact = p->nchans;
    d0.pad_row = -1;
    d0.nchans = p->nchans;
    d0.row_bytes = p->row_bytes;
    d0.scrunch = p->scrunch;
    d0.ngroups = 1;
    d0.out_bytes = 4;
    hipError_t e = dedisp::launch_unpack(d0, p->nbits, tfmt, hs);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    e = dedisp::launch_tree(d0, tfmt, nsub, ob, p->d_tree_pairs, npairs, p->sb_xc2.ptr, pitch2, len1, hs);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    // stage 2: every trial sums, over the sub-bands, its tree row at its delay
    return combine_rows(p, *p, p->sb_xc2.ptr, pitch2, ob, nsb, p->value_bound() * nsub,
                        static_cast<int>(p->dms.size()), nout, d_out, stride, rowmap, hs);
}

static dedisp_status execute_tree(dedisp_plan p, const void* d_in, size_t nsamps, uint32_t* d_out,
                                  size_t stride, void* stream)
{
    if (nsamps > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "nsamps too large");
    if (reinterpret_cast<uintptr_t>(d_in) & 3)
        return fail(DEDISP_ERR_INVALID_ARG, "tree passes need 4-byte aligned input");
    // the plans that run: this one, or every scrunch group's (Section 3's
    // tree on time-scrunched data); validate them all before any launch
    std::vector<std::pair<dedisp_plan, const int32_t*>> runs;
    if (p->groups.empty()) {
        runs.emplace_back(p, nullptr);
    } else {
        for (auto& g : p->groups) {
            if (!g.d_rows) {
                const size_t bytes = g.rows.size() * sizeof(int32_t);
                if (hipMalloc(&g.d_rows, bytes) != hipSuccess) {
                    g.d_rows = nullptr;
                    return fail(DEDISP_ERR_OOM, "hipMalloc scrunch row map");
                }
                HIP_TRY(hipMemcpy(g.d_rows, g.rows.data(), bytes, hipMemcpyHostToDevice));
            }
            runs.emplace_back(g.sub, g.d_rows);
        }
    }
    long long width = 0;
    for (auto& r : runs) {
        long long len1 = 0, nout = 0;
        tree_lengths(*r.first, nsamps, len1, nout);
        if (len1 <= 0 || nout <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps too short for the tree passes");
        width = std::max(width, nout);
    }
    if (stride == 0) stride = static_cast<size_t>(width);
    if (stride < static_cast<size_t>(width)) return fail(DEDISP_ERR_INVALID_ARG, "out_row_stride < nout");
    for (auto& r : runs) {
        dedisp_status st = tree_upload(r.first);
        if (st != DEDISP_OK) return st;
    }
    for (auto& r : runs) {
        dedisp_status st = run_tree(r.first, d_in, nsamps, d_out, stride, r.second,
                                    static_cast<hipStream_t>(stream));
        if (st != DEDISP_OK) return st;
    }
    return DEDISP_OK;
}

dedisp_status dedisp_execute(dedisp_plan p, const void* d_in, size_t nsamps, uint32_t* d_out,
                             size_t stride, void* stream)
{
    if (!p || !d_in || !d_out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (p->tree_nsub || p->sb_step1 || !p->groups.empty()) {
        const dedisp_status st = p->tree_nsub  ? execute_tree(p, d_in, nsamps, d_out, stride, stream)
                                 : p->sb_step1 ? execute_subband(p, d_in, nsamps, d_out, stride, stream)
                                               : execute_groups(p, d_in, nsamps, d_out, stride, stream);
        if (st == DEDISP_OK) p->inflight.record(static_cast<hipStream_t>(stream));
        return st;
    }
    // (an internal scrunch-group plan, run on its own while tuning, sums
    // p->scrunch input rows per sample)
    if (nsamps / p->scrunch <= static_cast<size_t>(p->max_delay))
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps <= max_delay");
    if (nsamps > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "nsamps too large");
    const size_t nout = nsamps / p->scrunch - p->max_delay;
    if (stride == 0) stride = nout;
    if (stride < nout) return fail(DEDISP_ERR_INVALID_ARG, "out_row_stride < nsamps - max_delay");
    LaunchPlan lp;
    dedisp_status st = resolve_launch(p, p->cfg, true, lp, false, static_cast<long long>(nout));
    if (st != DEDISP_OK) return st;
    if (lp.shape.kind == 0 && (reinterpret_cast<uintptr_t>(d_in) & 3)) {
        // the corner turn reads 32-bit words
        dedisp_tile_config u{};
        u.kind = 1;
        st = resolve_launch(p, u, true, lp);
        if (st != DEDISP_OK) return st;
    }
    st = ensure_xc(*p, p->xc, static_cast<long long>(nsamps), lp);
    if (st != DEDISP_OK) return st;
    BeamDesc d;
    fill_desc(p, lp, d_in, static_cast<long long>(nsamps), nullptr,
              static_cast<long long>(nsamps), d_out, static_cast<long long>(stride), p->xc.ptr, d);
    hipError_t e = launch_desc(d, lp, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    p->inflight.record(static_cast<hipStream_t>(stream));
    return DEDISP_OK;
}

dedisp_status dedisp_tune(dedisp_plan p, const void* d_in, size_t nsamps, uint32_t* d_out,
                          size_t stride, void* stream, const char* cache_path, float* best_ms)
{
    if (!p || !d_in || !d_out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (p->tree_nsub) {
        // the tree's passes have one shape each: time the transform
        hipStream_t hs = static_cast<hipStream_t>(stream);
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        dedisp_status rc = dedisp_execute(p, d_in, nsamps, d_out, stride, stream);
        float ms = 0.f;
        if (rc == DEDISP_OK) {
            HIP_TRY(hipEventRecord(e0, hs));
            rc = dedisp_execute(p, d_in, nsamps, d_out, stride, stream);
            HIP_TRY(hipEventRecord(e1, hs));
            HIP_TRY(hipEventSynchronize(e1));
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (best_ms) *best_ms = ms;
        return rc;
    }
    if (p->sb_step1) {
        // each pass in turn: time whole transforms over the pass's shapes;
        // where the sub-band sums fit a byte, for both intermediate widths
        // (bytes read as 8-bit codes, 16-bit values), keeping the faster
        long long len1 = 0, nout = 0;
        subband_lengths(*p, nsamps, len1, nout);
        if (len1 <= 0 || nout <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps too short for the sub-band passes");
        hipStream_t hs = static_cast<hipStream_t>(stream);
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        dedisp_plan s1 = p->sb_step1, s2 = p->sb_step2;
        auto tune_passes = [&](float& total) -> dedisp_status {
            total = 0.f;
            for (dedisp_plan q : {s1, s2}) {
                float best = 1e30f;
                dedisp_tile_config best_cfg = q->cfg;
                for (int i = 0; i < dedisp::shape_count(); ++i) {
                    const Shape& s = dedisp::shape_at(i);
                    if (s.kind != 0 || !shape_matches(s, *q)) continue;
                    dedisp_tile_config c{};
                    c.kind = 0;
                    c.waves = s.waves;
                    c.dms_per_wave = s.dpw;
                    c.words_per_lane = s.m;
                    c.chunk_chans = s.cc;
                    LaunchPlan probe;
                    if (resolve_launch(q, c, false, probe) != DEDISP_OK || probe.shape_index != i) continue;
                    const dedisp_tile_config saved = q->cfg;
                    q->cfg = c;
                    dedisp_status rc = dedisp_execute(p, d_in, nsamps, d_out, stride, stream);
                    float ms = 0.f;
                    if (rc == DEDISP_OK) {
                        HIP_TRY(hipEventRecord(e0, hs));
                        for (int r = 0; r < 3 && rc == DEDISP_OK; ++r)
                            rc = dedisp_execute(p, d_in, nsamps, d_out, stride, stream);
                        HIP_TRY(hipEventRecord(e1, hs));
                        HIP_TRY(hipEventSynchronize(e1));
                        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                        ms /= 3;
                    }
                    q->cfg = saved;
                    if (rc != DEDISP_OK) return rc;
                    if (ms < best) {
                        best = ms;
                        best_cfg = c;
                    }
                }
                q->cfg = best_cfg;
                // each timing is a whole transform: the last pass's best is
                // the tuned transform's time
                if (best < 1e29f) total = best;
            }
            return DEDISP_OK;
        };
        std::vector<int> fmts{s2->fmt};
        if (s2->fmt == dedisp::kFmtByte) fmts.push_back(kFmtHalf);
        else if (s2->fmt == kFmtHalf && s2->vbound <= 255) fmts.push_back(dedisp::kFmtByte);
        float best_total = 0.f;
        int best_fmt = s2->fmt;
        dedisp_tile_config best1 = s1->cfg, best2 = s2->cfg;
        dedisp_status rc = DEDISP_OK;
        for (size_t k = 0; k < fmts.size() && rc == DEDISP_OK; ++k) {
            if (k > 0) {
                drop_block_tables(s2);
                s2->fmt = fmts[k];
                s1->cfg = default_config(s1->fmt);
                s2->cfg = default_config(s2->fmt);
            }
            float total = 0.f;
            rc = tune_passes(total);
            if (rc == DEDISP_OK && (k == 0 || total < best_total)) {
                best_total = total;
                best_fmt = s2->fmt;
                best1 = s1->cfg;
                best2 = s2->cfg;
            }
        }
        if (s2->fmt != best_fmt) {
            drop_block_tables(s2);
            s2->fmt = best_fmt;
        }
        s1->cfg = best1;
        s2->cfg = best2;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != DEDISP_OK) return rc;
        if (best_ms) *best_ms = best_total;
        return DEDISP_OK;
    }
    if (!p->groups.empty()) {
        // each scrunch group on its own (its rows land at the top of d_out,
        // which the next execute overwrites)
        size_t width = 0;
        for (const auto& g : p->groups) {
            const long long n = group_nout(g, nsamps);
            if (n <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps / s <= max delay of a scrunch group");
            width = std::max(width, static_cast<size_t>(n));
        }
        if (stride == 0) stride = width;
        if (stride < width) return fail(DEDISP_ERR_INVALID_ARG, "out_row_stride < longest output row");
        float total = 0.f;
        for (auto& g : p->groups) {
            float ms = 0.f;
            dedisp_status st = dedisp_tune(g.sub, d_in, nsamps, d_out, stride, stream, cache_path, &ms);
            if (st != DEDISP_OK) return st;
            total += ms;
        }
        if (best_ms) *best_ms = total;
        return DEDISP_OK;
    }
    if (nsamps / p->scrunch <= static_cast<size_t>(p->max_delay))
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps <= max_delay");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const std::string key = cache_key(p, nsamps);
    auto cache = read_cache(cache_path);
    auto hit = cache.find(key);
    if (hit != cache.end() && hit->second.size() >= 5) {
        dedisp_tile_config c{};
        c.kind = static_cast<int>(hit->second[0]);
        c.waves = static_cast<int>(hit->second[1]);
        c.dms_per_wave = static_cast<int>(hit->second[2]);
        c.words_per_lane = static_cast<int>(hit->second[3]);
        c.chunk_chans = static_cast<int>(hit->second[4]);
        c.sample_format = hit->second.size() > 6 ? static_cast<int>(hit->second[6]) : -1;
        if (find_shape(c, *p)) {
            p->cfg = c;
            if (best_ms) *best_ms = hit->second.size() > 5 ? static_cast<float>(hit->second[5]) : 0.f;
            return DEDISP_OK;
        }
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const dedisp_tile_config saved = p->cfg;
    float best = 1e30f;
    dedisp_tile_config best_cfg = saved;
    for (int i = 0; i < dedisp::shape_count(); ++i) {
        const Shape& s = dedisp::shape_at(i);
        if (!shape_matches(s, *p)) continue;
        {
            dedisp_tile_config c{};
            c.kind = s.kind;
            c.waves = s.waves;
            c.dms_per_wave = s.dpw;
            c.words_per_lane = s.m;
            c.chunk_chans = s.cc;
            c.sample_format = s.kind == 0 ? s.fmt : -1;
            // a shape whose window does not fit would silently time another one
            LaunchPlan probe;
            const long long tout = static_cast<long long>(nsamps) / p->scrunch - p->max_delay;
            if (resolve_launch(p, c, false, probe, false, tout) != DEDISP_OK || probe.shape_index != i) continue;
            p->cfg = c;
            // the untiled kernel is timed only on small problems or when no
            // tiled shape fits: elsewhere it is never the fastest, and one
            // launch over a survey-sized input takes hundreds of milliseconds
            if (s.kind == 1 && best < 1e29f && static_cast<double>(nsamps) * p->nchans * p->dms.size() > 1e9)
                continue;
            dedisp_status rc = dedisp_execute(p, d_in, nsamps, d_out, stride, stream);
            if (rc != DEDISP_OK) {
                p->cfg = saved;
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc;
            }
            const int reps = 3;
            HIP_TRY(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) {
                rc = dedisp_execute(p, d_in, nsamps, d_out, stride, stream);
                if (rc != DEDISP_OK) break;
            }
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            if (rc != DEDISP_OK) {
                p->cfg = saved;
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc;
            }
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            ms /= reps;
            if (ms < best) {
                best = ms;
                best_cfg = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->cfg = best_cfg;
    if (best_ms) *best_ms = best;
    if (cache_path) {
        cache[key] = {static_cast<double>(best_cfg.kind), static_cast<double>(best_cfg.waves),
                      static_cast<double>(best_cfg.dms_per_wave),
                      static_cast<double>(best_cfg.words_per_lane),
                      static_cast<double>(best_cfg.chunk_chans), static_cast<double>(best),
                      static_cast<double>(best_cfg.sample_format)};
        write_cache(cache_path, cache);
    }
    return DEDISP_OK;
}

dedisp_status dedisp_get_diagonal_dm(dedisp_plan p, double* dm)
{
    if (!p || !dm) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    *dm = diagonal_dm(*p);
    return DEDISP_OK;
}

dedisp_status dedisp_default_scrunch_factors(dedisp_plan p, int max_factor, int32_t* factors)
{
    if (!p || !factors) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (max_factor < 1 || max_factor > kMaxScrunch || (max_factor & (max_factor - 1)))
        return fail(DEDISP_ERR_INVALID_ARG, "max_factor must be a power of two in [1, 64]");
    const double diag = diagonal_dm(*p);
    for (size_t d = 0; d < p->dms.size(); ++d) {
        int s = 1;
        double threshold = diag;
        while (s < max_factor && p->dms[d] > threshold) {
            s *= 2;
            threshold *= 2.0;
        }
        factors[d] = s;
    }
    return DEDISP_OK;
}

dedisp_status dedisp_set_scrunching(dedisp_plan p, const int32_t* factors)
{
    if (!p) return fail(DEDISP_ERR_INVALID_ARG, "NULL plan");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (p->scrunch != 1 || p->internal) return fail(DEDISP_ERR_INVALID_ARG, "not a user plan");
    if (p->sb_step1 && factors) return fail(DEDISP_ERR_UNSUPPORTED, "time-scrunching excludes sub-band mode");
    // the tree is built on the scrunch groups: switch it off before changing them
    if (p->tree_nsub) return fail(DEDISP_ERR_UNSUPPORTED, "set time-scrunching before the tree");
    const int ndm = static_cast<int>(p->dms.size());
    bool any = false;
    if (factors) {
        for (int d = 0; d < ndm; ++d) {
            const int s = factors[d];
            if (s < 1 || s > kMaxScrunch || (s & (s - 1)))
                return fail(DEDISP_ERR_INVALID_ARG, "scrunch factors must be powers of two in [1, 64]");
            any |= s > 1;
        }
    }
    destroy_groups(p);
    if (!any) return DEDISP_OK;
    p->scrunch_factors.assign(factors, factors + ndm);
    for (int s = 1; s <= kMaxScrunch; s *= 2) {
        ScrunchGroup g;
        g.s = s;
        std::vector<double> dms;
        for (int d = 0; d < ndm; ++d)
            if (factors[d] == s) {
                g.rows.push_back(d);
                dms.push_back(p->dms[d]);
            }
        if (g.rows.empty()) continue;
        dedisp_plan sub = new (std::nothrow) dedisp_plan_s;
        if (!sub) {
            destroy_groups(p);
            return fail(DEDISP_ERR_OOM, "plan allocation");
        }
        sub->nchans = p->nchans;
        sub->nbits = p->nbits;
        sub->dt = p->dt * s;
        sub->f_top = p->f_top;
        sub->df = p->df;
        sub->row_bytes = p->row_bytes;
        sub->scrunch = s;
        sub->fmt = scrunch_format(p->nbits, p->nchans, s);
        sub->cfg = default_config(sub->fmt);
        sub->killmask = p->killmask;
        sub->active = p->active;
        sub->out_nbits = p->out_nbits;
        sub->out_shift = p->out_shift;
        g.sub = sub;
        p->groups.push_back(g);
        std::vector<int32_t> table;
        int mx = 0;
        if (!build_delay_table(*sub, dms.data(), static_cast<int>(dms.size()), table, mx)) {
            destroy_groups(p);
            return fail(DEDISP_ERR_INVALID_ARG, "a delay does not fit in int32");
        }
        sub->dms = dms;
        sub->table.swap(table);
        sub->max_delay = mx;
        sub->has_dms = true;
    }
    return DEDISP_OK;
}

// Staging tables of the combination of per-sub-band rows (byte rows, at
// most 128 sub-bands): per block of kTreeBlock consecutive trials and
// sub-band, the rows the block uses and its delay window; a block whose rows
// exceed the LDS budget is gathered instead.  rows and delay are
// [ndm][nsb].
struct Stage2Tables {
    std::vector<dedisp::TreeStage> stage;
    std::vector<int32_t> sblocks, off, gtrials;
    int lds_max = 0, span_max = 0;
    void assign_to(dedisp_plan q)
    {
        if (sblocks.empty()) return;
        q->tree_stage.swap(stage);
        q->tree_sblocks.swap(sblocks);
        q->tree_off.swap(off);
        q->tree_gtrials.swap(gtrials);
        q->tree_lds = lds_max;
        q->tree_span = span_max;
    }
};

static Stage2Tables stage2_tables(int ndm, int nsb, const std::vector<int32_t>& rows,
                                  const std::vector<int32_t>& delay)
{
    constexpr int TB = dedisp::kTreeBlock, TT = dedisp::kTreeTile;
    constexpr long long kTreeLdsDwords = 16 * 1024;          // 64 KB: two workgroups per CU
    Stage2Tables r;
    r.off.assign(static_cast<size_t>(ndm) * nsb, 0);
    std::vector<dedisp::TreeStage> st(nsb);
    for (int b = 0; b * TB < ndm; ++b) {
        const int d0 = b * TB, d1 = std::min(ndm, d0 + TB);
        long long lds = 0;
        for (int n = 0; n < nsb; ++n) {
            int lo = 0x7fffffff, hi = -1, dmin = 0x7fffffff, dmax = -1;
            for (int d = d0; d < d1; ++d) {
                const size_t i = static_cast<size_t>(d) * nsb + n;
                lo = std::min(lo, rows[i]);
                hi = std::max(hi, rows[i]);
                dmin = std::min(dmin, delay[i]);
                dmax = std::max(dmax, delay[i]);
            }
            dedisp::TreeStage& g = st[n];
            g = dedisp::TreeStage{};
            g.lo = lo;
            g.span = hi - lo + 1;
            g.dmin4 = dmin & ~3;
            // staged rows are segmented within the tile (four segments of
            // TT/4 outputs, one byte of each per dword): the window covers
            // a segment and the block's delay spread, in whole groups of
            // four dwords
            g.wdw = ((dmax - g.dmin4) + TT / 4 + 3) / 4 * 4;
            g.rcp = static_cast<uint32_t>(((1ull << 32) + g.wdw / 4 - 1) / (g.wdw / 4));
            g.lds = static_cast<int>(std::min<long long>(lds, 0x7fffffff));
            lds += static_cast<long long>(g.span) * g.wdw;
        }
        if (lds > kTreeLdsDwords) {
            for (int d = d0; d < d1; ++d) r.gtrials.push_back(d);
            continue;
        }
        for (int n = 0; n < nsb; ++n)
            for (int d = d0; d < d1; ++d) {
                const size_t i = static_cast<size_t>(d) * nsb + n;
                const dedisp::TreeStage& g = st[n];
                r.off[i] = 4 * (g.lds + (rows[i] - g.lo) * g.wdw + (delay[i] - g.dmin4));
            }
        r.sblocks.push_back(b);
        r.stage.insert(r.stage.end(), st.begin(), st.end());
        r.lds_max = std::max(r.lds_max, static_cast<int>(lds));
        for (const auto& g : st) r.span_max = std::max(r.span_max, g.span);
    }
    return r;
}

dedisp_status dedisp_set_subband(dedisp_plan p, int nsub, int ngroup)
{
    if (!p) return fail(DEDISP_ERR_INVALID_ARG, "NULL plan");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (p->internal || p->scrunch != 1) return fail(DEDISP_ERR_INVALID_ARG, "not a user plan");
    if (nsub == 0 && ngroup == 0) {
        destroy_subband(p);
        return DEDISP_OK;
    }
    if (nsub < 8 || nsub % 8 || p->nchans % nsub)
        return fail(DEDISP_ERR_INVALID_ARG, "nsub must be a multiple of 8 that divides nchans");
    if (ngroup < 1) return fail(DEDISP_ERR_INVALID_ARG, "ngroup must be positive");
    if (!p->groups.empty() || p->tree_nsub)
        return fail(DEDISP_ERR_UNSUPPORTED, "sub-band mode excludes time-scrunching and the tree");
    if (p->row_bytes % 4) return fail(DEDISP_ERR_UNSUPPORTED, "sub-band passes need whole 32-bit words per row");
    const int vsum = (p->nbits == 2 ? 3 : 255) * nsub;      // largest sub-band sum
    if (vsum > 32767) return fail(DEDISP_ERR_UNSUPPORTED, "sub-band sums do not fit 16 bits");
    const int ndm = static_cast<int>(p->dms.size());
    const int nnom = (ndm + ngroup - 1) / ngroup;
    const int nsb = p->nchans / nsub;
    const int nsb_p = (nsb + 7) & ~7;
    if (nnom > 65535 || nsb > 65535) return fail(DEDISP_ERR_UNSUPPORTED, "too many sub-bands or nominal DMs");
    std::vector<double> nom(nnom);
    for (int m = 0; m < nnom; ++m) nom[m] = p->dms[static_cast<size_t>(m) * ngroup];
    std::vector<int32_t> tab_nom;
    int mx = 0;
    if (!build_delay_table(*p, nom.data(), nnom, tab_nom, mx))
        return fail(DEDISP_ERR_INVALID_ARG, "a delay does not fit in int32");
    dedisp_plan s1 = new_internal(*p), s2 = new_internal(*p);
    if (!s1 || !s2) {
        dedisp_plan_destroy(s1);
        dedisp_plan_destroy(s2);
        return fail(DEDISP_ERR_OOM, "plan allocation");
    }
    // step 1: group n = sub-band n, rows = nominal DMs, delays relative to
    // the sub-band's first channel
    s1->nchans = nsub;
    s1->fmt = p->nbits == 2 ? kFmtNib : dedisp::kFmtByte;   // grouped passes: one row per channel
    s1->ngroups = nsb;
    s1->dms = nom;
    s1->ndm_last = nnom;
    s1->table.assign(static_cast<size_t>(nsb) * nnom * nsub, 0);
    s1->max_delay = 0;
    for (int n = 0; n < nsb; ++n)
        for (int m = 0; m < nnom; ++m)
            for (int j = 0; j < nsub; ++j) {
                const int32_t* row = tab_nom.data() + static_cast<size_t>(m) * p->nchans + n * nsub;
                const int32_t v = row[j] - row[0];
                s1->table[(static_cast<size_t>(n) * nnom + m) * nsub + j] = v;
                s1->max_delay = std::max(s1->max_delay, static_cast<int>(v));
            }
    s1->cfg = default_config(s1->fmt);
    // step 2: group m = nominal DM m, rows = its trials, channels = sub-bands
    // (padded with zero rows to a multiple of 8), delays of each sub-band's
    // first channel
    s2->nchans = nsb_p;
    // intermediate sums: byte lanes with periodic flushes while a flush
    // comes at most every 6 channels (1.5 + 8/6 VALU per channel and 4
    // samples); else bytes spread to 16-bit lanes (the 8-bit code path: 3
    // VALU, exact up to 255) or 16-bit values (also 3 VALU, twice the bytes
    // through HBM and LDS).  The 8-bit shapes fill with 32 or more sub-bands
    // and trials per nominal DM, so bytes are the default there; the tuner
    // times both widths wherever sums fit a byte
    s2->fmt = vsum <= 42                               ? kFmtByteS
              : vsum <= 255 && nsb >= 32 && ngroup >= 32 ? dedisp::kFmtByte
                                                         : kFmtHalf;
    s2->vbound = vsum;
    s2->ngroups = nnom;
    s2->dms.assign(ngroup, 0.0);
    s2->ndm_last = ndm - (nnom - 1) * ngroup;
    s2->table.assign(static_cast<size_t>(nnom) * ngroup * nsb_p, 0);
    s2->max_delay = 0;
    for (int m = 0; m < nnom; ++m)
        for (int k = 0; k < ngroup; ++k) {
            const int d = std::min(m * ngroup + k, ndm - 1);
            for (int n = 0; n < nsb; ++n) {
                const int32_t v = p->table[static_cast<size_t>(d) * p->nchans + n * nsub];
                s2->table[(static_cast<size_t>(m) * ngroup + k) * nsb_p + n] = v;
                s2->max_delay = std::max(s2->max_delay, static_cast<int>(v));
            }
        }
    s2->cfg = default_config(s2->fmt);
    // byte sums: step 2 is the combination of per-sub-band rows, trial d
    // summing row (d / ngroup) * nsb_p + n at the delay of sub-band n's first
    // channel -- the tree's stage-2 kernels, used while the sums are bytes
    // and every block of trials stages in LDS (ngroup a multiple of the
    // block size); else the grouped tiled launch
    if (vsum <= 255 && nsb <= 128) {
        std::vector<int32_t> rows(static_cast<size_t>(ndm) * nsb), delay(rows.size());
        for (int d = 0; d < ndm; ++d)
            for (int n = 0; n < nsb; ++n) {
                rows[static_cast<size_t>(d) * nsb + n] = (d / ngroup) * nsb_p + n;
                delay[static_cast<size_t>(d) * nsb + n] = p->table[static_cast<size_t>(d) * p->nchans + n * nsub];
            }
        Stage2Tables t = stage2_tables(ndm, nsb, rows, delay);
        if (!t.sblocks.empty() && t.gtrials.empty()) {
            s2->tree_rows.swap(rows);
            s2->tree_delay.swap(delay);
            t.assign_to(s2);
        }
    }
    destroy_subband(p);
    p->sb_nsub = nsub;
    p->sb_ngroup = ngroup;
    p->sb_step1 = s1;
    p->sb_step2 = s2;
    return DEDISP_OK;
}


// Tables of the piecewise tree with sub-bands of nsub channels for plan q's
// trials, at q's resolution (dt, or s*dt for a scrunch group's plan).
static dedisp_status build_tree(dedisp_plan q, int nsub)
{
    const int nsb = q->nchans / nsub;
    const int ndm = static_cast<int>(q->dms.size());
    // Section 3, eq. combining_subbands, in binary64 in this order:
    // d'_n = round(DM [DeltaT(v_{n+1}) - DeltaT(v_n)]),
    // dt''_n = round(DM * (sum of those brackets over the sub-bands before n))
    const double inv_f0_sq = 1.0 / (q->f_top * q->f_top);
    const double samples_per_unit = kDispersionConstant / q->dt;
    std::vector<double> step(nsb);
    for (int n = 0; n < nsb; ++n) {
        const double fa = q->f_top + static_cast<double>(n * nsub) * q->df;
        const double fb = q->f_top + static_cast<double>((n + 1) * nsub) * q->df;
        step[n] = samples_per_unit * (1.0 / (fb * fb) - inv_f0_sq) - samples_per_unit * (1.0 / (fa * fa) - inv_f0_sq);
    }
    // past the diagonal (Section 3, computing larger DMs): sub-band n of
    // trial d reads stage-1 pass p = d' / nsub (a delay of p samples per
    // channel imposed within the sub-band) at tree DM d' mod nsub
    std::vector<int32_t> dprime(static_cast<size_t>(ndm) * nsb), delay(dprime.size());
    int mx = 0, maxpass = 0;
    for (int d = 0; d < ndm; ++d) {
        double acc = 0.0;
        for (int n = 0; n < nsb; ++n) {
            const double dp = std::round(q->dms[d] * step[n]);
            const double dd = std::round(q->dms[d] * acc);
            if (!(dd < 2.0e9) || !(dp < 2.0e9)) return fail(DEDISP_ERR_INVALID_ARG, "a delay does not fit in int32");
            dprime[static_cast<size_t>(d) * nsb + n] = static_cast<int32_t>(dp);
            delay[static_cast<size_t>(d) * nsb + n] = static_cast<int32_t>(dd);
            mx = std::max(mx, static_cast<int>(dd));
            maxpass = std::max(maxpass, static_cast<int>(dp) / nsub);
            acc += step[n];
        }
    }
    if (maxpass >= 65535)
        return fail(DEDISP_ERR_UNSUPPORTED, "more than 65535 (sub-band, pass) pairs for the tree's stage 1");
    // the (sub-band, pass) pairs in use, sub-band major
    std::vector<int32_t> pair_of(static_cast<size_t>(nsb) * (maxpass + 1), -1);
    for (size_t i = 0; i < dprime.size(); ++i)
        pair_of[(i % nsb) * (maxpass + 1) + dprime[i] / nsub] = 0;
    std::vector<int32_t> pairs;
    for (int n = 0; n < nsb; ++n)
        for (int ps = 0; ps <= maxpass; ++ps) {
            int32_t& y = pair_of[static_cast<size_t>(n) * (maxpass + 1) + ps];
            if (y < 0) continue;
            y = static_cast<int32_t>(pairs.size() / 2);
            pairs.push_back(n);
            pairs.push_back(ps);
        }
    if (pairs.size() / 2 > 65535)
        return fail(DEDISP_ERR_UNSUPPORTED, "more than 65535 (sub-band, pass) pairs for the tree's stage 1");
    std::vector<int32_t> rows(dprime.size());
    for (size_t i = 0; i < dprime.size(); ++i) {
        const int n = static_cast<int>(i % nsb), ps = dprime[i] / nsub;
        rows[i] = pair_of[static_cast<size_t>(n) * (maxpass + 1) + ps] * nsub + dprime[i] % nsub;
    }
    // LDS staging of stage 2 (byte rows only; the kernel keeps a trial's
    // offsets in two registers: up to 128 sub-bands)
    Stage2Tables s2t;
    if (static_cast<long long>(q->value_bound()) * nsub <= 255 && nsb <= 128) s2t = stage2_tables(ndm, nsb, rows, delay);
    destroy_tree(q);
    q->tree_nsub = nsub;
    q->tree_maxdelay = mx;
    q->tree_npass = maxpass + 1;
    q->tree_pairs.swap(pairs);
    q->tree_rows.swap(rows);
    q->tree_delay.swap(delay);
    s2t.assign_to(q);
    return DEDISP_OK;
}

dedisp_status dedisp_set_tree(dedisp_plan p, int nsub)
{
    if (!p) return fail(DEDISP_ERR_INVALID_ARG, "NULL plan");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (p->internal || p->scrunch != 1) return fail(DEDISP_ERR_INVALID_ARG, "not a user plan");
    if (nsub == 0) {
        destroy_tree(p);
        return DEDISP_OK;
    }
    if (nsub < 8 || nsub > 128 || (nsub & (nsub - 1)) || p->nchans % nsub)
        return fail(DEDISP_ERR_INVALID_ARG, "nsub must be a power of two in [8, 128] dividing nchans");
    if (p->sb_step1) return fail(DEDISP_ERR_UNSUPPORTED, "the tree excludes sub-band mode");
    if (p->row_bytes % 4) return fail(DEDISP_ERR_UNSUPPORTED, "tree passes need whole 32-bit words per row");
    if (!(p->f_top + static_cast<double>(p->nchans) * p->df > 0))
        return fail(DEDISP_ERR_UNSUPPORTED, "the band edge past the last channel reaches zero frequency");
    if (p->groups.empty()) return build_tree(p, nsub);
    // time-scrunched trials: one tree per scrunch group over its s-sample
    // sums, whose sub-band sums must stay below 2^16
    for (const auto& g : p->groups)
        if (static_cast<long long>(g.sub->value_bound()) * nsub > 65535)
            return fail(DEDISP_ERR_UNSUPPORTED, "a scrunch group's sub-band sums exceed 16 bits");
    destroy_tree(p);
    for (auto& g : p->groups) {
        dedisp_status st = build_tree(g.sub, nsub);
        if (st != DEDISP_OK) {
            destroy_tree(p);
            return st;
        }
    }
    p->tree_nsub = nsub;
    return DEDISP_OK;
}

dedisp_status dedisp_set_output_format(dedisp_plan p, int nbits, int shift)
{
    if (!p) return fail(DEDISP_ERR_INVALID_ARG, "NULL plan");
    if (p->internal) return fail(DEDISP_ERR_INVALID_ARG, "not a user plan");
    if (nbits != 8 && nbits != 16 && nbits != 32)
        return fail(DEDISP_ERR_INVALID_ARG, "output bits must be 8, 16 or 32");
    if (shift < 0 || shift > 31) return fail(DEDISP_ERR_INVALID_ARG, "shift must be in [0, 31]");
    p->out_nbits = nbits;
    p->out_shift = shift;
    for (auto& g : p->groups) {
        g.sub->out_nbits = nbits;
        g.sub->out_shift = shift;
    }
    return DEDISP_OK;
}

dedisp_status dedisp_get_output_format(dedisp_plan p, int* nbits, int* shift)
{
    if (!p || !nbits || !shift) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    *nbits = p->out_nbits;
    *shift = p->out_shift;
    return DEDISP_OK;
}

dedisp_status dedisp_get_output_lengths(dedisp_plan p, size_t nsamps, size_t* nout)
{
    if (!p || !nout) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (p->tree_nsub && p->groups.empty()) {
        long long len1 = 0, n = 0;
        tree_lengths(*p, nsamps, len1, n);
        if (len1 <= 0 || n <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps too short for the tree passes");
        for (size_t d = 0; d < p->dms.size(); ++d) nout[d] = static_cast<size_t>(n);
        return DEDISP_OK;
    }
    if (p->tree_nsub) {
        for (const auto& g : p->groups) {
            long long len1 = 0, n = 0;
            tree_lengths(*g.sub, nsamps, len1, n);
            if (len1 <= 0 || n <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps too short for the tree passes");
            for (int32_t r : g.rows) nout[r] = static_cast<size_t>(n);
        }
        return DEDISP_OK;
    }
    if (p->sb_step1) {
        long long len1 = 0, n = 0;
        subband_lengths(*p, nsamps, len1, n);
        if (len1 <= 0 || n <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps too short for the sub-band passes");
        for (size_t d = 0; d < p->dms.size(); ++d) nout[d] = static_cast<size_t>(n);
        return DEDISP_OK;
    }
    if (p->groups.empty()) {
        if (nsamps <= static_cast<size_t>(p->max_delay))
            return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps <= max_delay");
        for (size_t d = 0; d < p->dms.size(); ++d) nout[d] = nsamps - p->max_delay;
        return DEDISP_OK;
    }
    for (const auto& g : p->groups) {
        const long long n = group_nout(g, nsamps);
        if (n <= 0) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps / s <= max delay of a scrunch group");
        for (int32_t r : g.rows) nout[r] = static_cast<size_t>(n);
    }
    return DEDISP_OK;
}

}  // extern "C"
