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

// Largest number of codes that can be summed in one packed lane without a
// carry into the next: 255/3 for 2-bit codes in 8-bit lanes (Section 2.3),
// 65535/255 for 8-bit codes in 16-bit lanes.
constexpr int kLaneSum2Bit = 85;
constexpr int kLaneSum8Bit = 257;

void free_device(dedisp_plan p)
{
    if (p->d_table || !p->blocks.empty()) (void)hipDeviceSynchronize();
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
// so staged windows start on 16-byte boundaries); the window offset of DM row d, scratch row k is
// delay[d][c(k)] - base[b][k] (0 for padding DM rows past ndm and for the
// zero rows), stored for row pairs: rel[d][p] = off(2p) | off(2p+1) << 16.
// relmax is the largest offset (always < 2^16 for a shape that fits).
void build_block_tables(const dedisp_plan_s& p, int db, BlockTables& bt)
{
    const int ndm = static_cast<int>(p.dms.size());
    const int nch = p.nchans;
    const int nrow = p.nact_padded();     // scratch rows: live channels, then zero rows
    const int nlive = p.nact();
    const int np = nrow / 2;
    bt.db = db;
    bt.nblocks = (ndm + db - 1) / db;
    bt.rel.assign(static_cast<size_t>(bt.nblocks) * db * np, 0u);
    bt.base.assign(static_cast<size_t>(bt.nblocks) * nrow, 0);
    bt.relmax = 0;
    for (int b = 0; b < bt.nblocks; ++b) {
        const int d0 = b * db, d1 = std::min(ndm, d0 + db);
        for (int k = 0; k < nlive; ++k) {
            const int c = p.source_channel(k);
            int mn = 0x7fffffff;
            for (int d = d0; d < d1; ++d)
                mn = std::min(mn, p.table[static_cast<size_t>(d) * nch + c]);
            mn &= p.nbits == 2 ? ~31 : ~15;
            bt.base[static_cast<size_t>(b) * nrow + k] = mn;
            for (int d = d0; d < d1; ++d) {
                const int r = p.table[static_cast<size_t>(d) * nch + c] - mn;
                bt.relmax = std::max(bt.relmax, r);
                const uint32_t v = static_cast<uint32_t>(std::min(r, 0xFFFF));
                bt.rel[static_cast<size_t>(d) * np + k / 2] |= (k & 1) ? (v << 16) : v;
            }
        }
    }
}

const Shape* find_shape(const dedisp_tile_config& c, int nbits, int* index)
{
    for (int i = 0; i < dedisp::shape_count(); ++i) {
        const Shape& s = dedisp::shape_at(i);
        if (s.nbits != nbits || s.kind != c.kind) continue;
        if (s.kind == 1 || (s.waves == c.waves && s.dpw == c.dms_per_wave &&
                            s.m == c.words_per_lane && s.cc == c.chunk_chans)) {
            if (index) *index = i;
            return &s;
        }
    }
    return nullptr;
}

// Default shape: the first compiled tiled shape of this bit depth (the
// shape list is ordered by measured speed on the survey-beam workload).
dedisp_tile_config default_config(int nbits)
{
    dedisp_tile_config c{};
    for (int i = 0; i < dedisp::shape_count(); ++i) {
        const Shape& s = dedisp::shape_at(i);
        if (s.kind == 0 && s.nbits == nbits) {
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

dedisp_status ensure_block_tables(dedisp_plan p, int db, BlockTables** out)
{
    auto it = p->blocks.find(db);
    if (it == p->blocks.end()) {
        BlockTables bt;
        build_block_tables(*p, db, bt);
        it = p->blocks.emplace(db, std::move(bt)).first;
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

// Samples per 32-bit word of the channel-major scratch: 2-bit codes are
// stored as nibbles (8 per word), 8-bit codes as bytes (4 per word).
int samples_per_word(int nbits) { return nbits == 2 ? 8 : 4; }

// Window length (32-bit words per channel row in LDS, a multiple of 4) of
// shape s: a lane reads words up to rel / samples_per_word + 64*m.
int window_words(const BlockTables& bt, const Shape& s)
{
    return ((bt.relmax / samples_per_word(s.nbits) + 64 * s.m + 1) + 3) & ~3;
}

bool shape_fits(const BlockTables& bt, const Shape& s)
{
    const int rw = window_words(bt, s);
    return bt.relmax < 0x10000 && (rw >> 2) <= 64 * s.pi &&
           static_cast<long long>(s.cc) * rw * 4 <= dedisp::kMaxLdsBytes;
}

// The tiled path reads input rows as 32-bit words and keeps 2-bit sums in
// 16-bit lanes.
bool tiled_supported(const dedisp_plan_s& p)
{
    return p.row_bytes % 4 == 0 && p.nact() >= 1 && (p.nbits == 8 || p.nchans <= 21845);
}

// Resolve the shape used for this plan: the requested one if its LDS window
// fits, else the first compiled tiled shape of the same bit depth that fits,
// else the untiled kernel.  Host-only (no HIP call) when `upload` is false.
dedisp_status resolve_launch(dedisp_plan p, const dedisp_tile_config& want, bool upload,
                             LaunchPlan& lp, bool multi_only)
{
    int idx = -1;
    if (!find_shape(want, p->nbits, &idx)) return fail(DEDISP_ERR_INVALID_ARG, "unknown tile shape");
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
        if (s.nbits != p->nbits || s.kind != 0 || !tiled_supported(*p)) continue;
        const int db = s.waves * s.dpw;
        const BlockTables* bt = nullptr;
        auto it = p->blocks.find(db);
        if (it != p->blocks.end()) {
            bt = &it->second;
        } else {
            auto h = host_tables.find(db);
            if (h == host_tables.end()) {
                h = host_tables.emplace(db, BlockTables{}).first;
                build_block_tables(*p, db, h->second);
            }
            bt = &h->second;
        }
        if (!shape_fits(*bt, s)) continue;
        lp.shape_index = i;
        lp.shape = s;
        lp.cc = s.cc;
        lp.rw = window_words(*bt, s);
        lp.lds = s.cc * lp.rw * 4;
        const int lane_sum = p->nbits == 2 ? kLaneSum2Bit : kLaneSum8Bit;
        lp.flush_every = std::max(1, lane_sum / s.cc);
        lp.bt = nullptr;
        if (upload) {
            BlockTables* dbt = nullptr;
            dedisp_status st = ensure_block_tables(p, db, &dbt);
            if (st != DEDISP_OK) return st;
            lp.bt = dbt;
        }
        return DEDISP_OK;
    }
    dedisp_tile_config u{};
    u.kind = 1;
    if (!find_shape(u, p->nbits, &idx)) return fail(DEDISP_ERR_UNSUPPORTED, "no untiled kernel");
    lp.shape_index = idx;
    lp.shape = dedisp::shape_at(idx);
    lp.cc = lp.rw = lp.lds = 0;
    lp.bt = nullptr;
    if (upload) return ensure_device_table(p);
    return DEDISP_OK;
}

long long tile_len(const Shape& s) { return 64LL * samples_per_word(s.nbits) * s.m; }

// Row pitch in bytes of the channel-major scratch: a staged window starts
// before the last sample and spans 4*rw bytes.
long long xc_pitch(long long nsamps, int nbits, int rw)
{
    const long long bytes = nbits == 2 ? (nsamps + 1) / 2 : nsamps;
    return ((bytes + 4LL * rw + 63) / 64) * 64;
}

void free_scratch(Scratch& x)
{
    if (x.ptr) {
        (void)hipDeviceSynchronize();
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
    return ensure_scratch(x, static_cast<size_t>(xc_pitch(nsamps, lp.shape.nbits, lp.rw)) * p.nact_padded());
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
    d.nout = nsamps - p->max_delay;
    d.out = out;
    d.out_stride = stride;
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
        d.pitch = xc_pitch(nsamps, lp.shape.nbits, lp.rw);
        d.rel = lp.bt->d_rel;
        d.base = lp.bt->d_base;
        d.nblocks = lp.bt->nblocks;
        d.ntiles = static_cast<int>((d.nout + tile_len(lp.shape) - 1) / tile_len(lp.shape));
        d.rw = lp.rw;
        d.flush_every = lp.flush_every;
    }
}

hipError_t launch_desc(const BeamDesc& d, const LaunchPlan& lp, hipStream_t st)
{
    if (lp.shape.kind == 0) {
        hipError_t e = dedisp::launch_unpack(d, lp.shape.nbits, st);
        if (e != hipSuccess) return e;
        return dedisp::launch_tiled(d, lp.shape, lp.lds, st);
    }
    return dedisp::launch_untiled(d, lp.shape.nbits, st);
}


// --------------------------------------------------------------- tune cache

std::string cache_key(dedisp_plan p, size_t nsamps)
{
    size_t bucket = 1;
    while (bucket < nsamps) bucket <<= 1;
    std::ostringstream os;
    os << "nbits=" << p->nbits << ",nchans=" << p->nchans << ",ndm=" << p->dms.size()
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
    p->cfg = default_config(nbits);
    *out = p;
    return DEDISP_OK;
}

void dedisp_plan_destroy(dedisp_plan p)
{
    if (!p) return;
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
    return DEDISP_OK;
}

dedisp_status dedisp_set_tile_config(dedisp_plan p, const dedisp_tile_config* c)
{
    if (!p || !c) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!find_shape(*c, p->nbits)) return fail(DEDISP_ERR_INVALID_ARG, "unknown tile shape");
    p->cfg = *c;
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
    return DEDISP_OK;
}

dedisp_status dedisp_execute(dedisp_plan p, const void* d_in, size_t nsamps, uint32_t* d_out,
                             size_t stride, void* stream)
{
    if (!p || !d_in || !d_out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (nsamps <= static_cast<size_t>(p->max_delay))
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps <= max_delay");
    if (nsamps > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "nsamps too large");
    const size_t nout = nsamps - p->max_delay;
    if (stride == 0) stride = nout;
    if (stride < nout) return fail(DEDISP_ERR_INVALID_ARG, "out_row_stride < nsamps - max_delay");
    LaunchPlan lp;
    dedisp_status st = resolve_launch(p, p->cfg, true, lp);
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
    return DEDISP_OK;
}

dedisp_status dedisp_tune(dedisp_plan p, const void* d_in, size_t nsamps, uint32_t* d_out,
                          size_t stride, void* stream, const char* cache_path, float* best_ms)
{
    if (!p || !d_in || !d_out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (nsamps <= static_cast<size_t>(p->max_delay))
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
        if (find_shape(c, p->nbits)) {
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
        if (s.nbits != p->nbits) continue;
        {
            dedisp_tile_config c{};
            c.kind = s.kind;
            c.waves = s.waves;
            c.dms_per_wave = s.dpw;
            c.words_per_lane = s.m;
            c.chunk_chans = s.cc;
            // a shape whose window does not fit would silently time another one
            LaunchPlan probe;
            if (resolve_launch(p, c, false, probe) != DEDISP_OK || probe.shape_index != i) continue;
            p->cfg = c;
            // skip the untiled kernel on big problems: it is never the fastest
            if (s.kind == 1 && static_cast<double>(nsamps) * p->nchans * p->dms.size() > 1e11)
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
                      static_cast<double>(best_cfg.chunk_chans), static_cast<double>(best)};
        write_cache(cache_path, cache);
    }
    return DEDISP_OK;
}

}  // extern "C"
