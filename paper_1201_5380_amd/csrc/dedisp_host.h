// Host-side internals shared by the library's translation units: the plan
// object behind the opaque dedisp_plan handle and the helpers that turn a
// plan plus buffers into kernel launches.  Not part of the ABI.
#pragma once

#include "dedisp.h"
#include "dedisp_internal.h"

#include <map>
#include <string>
#include <vector>

#define HIP_TRY(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) return ::dedisp::host::hip_fail(e_, #call);      \
    } while (0)

namespace dedisp {
namespace host {

// Record an error message for dedisp_last_error and return the status.
dedisp_status fail(dedisp_status st, const std::string& msg);
dedisp_status hip_fail(hipError_t e, const char* where);

// Window tables of one DM-block size (see build_block_tables).
struct BlockTables {
    int db = 0;
    int nblocks = 0;
    int relmax = 0;
    std::vector<uint32_t> rel;   // [nblocks*db][nchans/2], channel pairs packed 16+16 bits
    std::vector<int32_t> base;   // [nblocks][nchans] ([nblocks][nchans][2] start, span: kFmtSeg)
    uint32_t* d_rel = nullptr;
    int32_t* d_base = nullptr;
};

// Work enqueued on behalf of one object (a plan, stream or batch): one event
// per HIP stream the object was used on, recorded after each enqueue (not
// while that stream is capturing a graph).  wait() blocks the calling host
// thread until that work is done -- other work on the device goes on -- so
// the object's device memory can be freed or rewritten.
struct InFlight {
    std::vector<std::pair<hipStream_t, hipEvent_t>> ev;
    hipStream_t last = nullptr;    // most recent stream recorded on
    bool any = false;
    bool untracked = false;        // work on a stream without an event: wait() waits for the device
    InFlight() = default;
    InFlight(const InFlight&) = delete;
    InFlight& operator=(const InFlight&) = delete;
    ~InFlight();
    void record(hipStream_t s);
    // record() without creating an event: a stream seen before reuses its
    // event, work on a new one is marked untracked.
    void record_existing(hipStream_t s);
    void wait();
};

// A device buffer that only grows; freeing it waits for its owner's work.
struct Scratch {
    uint8_t* ptr = nullptr;
    size_t bytes = 0;
    InFlight* owner = nullptr;     // NULL: freeing waits for the whole device
};

// A resolved launch for one beam: shape, LDS size and window length.
struct LaunchPlan {
    int shape_index = -1;
    Shape shape{};
    int nbits = 0;       // input bit depth (selects the corner-turn kernel)
    int cc = 0, rw = 0, lds = 0, flush_every = 1;
    int dbuf = 0;        // two LDS chunk buffers (lds counts both)
    BlockTables* bt = nullptr;
};

// Shapes usable by plan p: tiled shapes of its scratch format, the untiled
// kernel of its input bit depth.
bool shape_matches(const Shape& s, const struct ::dedisp_plan_s& p);
const Shape* find_shape(const dedisp_tile_config& c, const struct ::dedisp_plan_s& p,
                        int* index = nullptr);
dedisp_tile_config default_config(int fmt);
bool tiled_supported(const struct ::dedisp_plan_s& p);

// Resolve the shape used for plan p (requested one if it fits, else another
// tiled shape, else the untiled kernel).  `upload` makes the device tables.
// With multi_only, only shapes compiled into the multi-beam kernels are
// considered before the untiled fallback.  nout (outputs per DM row of the
// launch, -1 if not known) excludes the segmented bit planes from launches
// shorter than kSegMinOutPerDelay * max_delay.
dedisp_status resolve_launch(::dedisp_plan p, const dedisp_tile_config& want, bool upload,
                             LaunchPlan& lp, bool multi_only = false, long long nout = -1);

long long tile_len(const Shape& s);
// Row pitch (bytes) of the channel-major scratch for nsamps input samples
// (max_delay: the plan's, which fixes the interleaved format's segments).
long long xc_pitch(long long nsamps, int fmt, int rw, long long max_delay);
// Key of a plan's window tables: DM-block size and window granularity (the
// interleaved bit-plane format aligns windows to 4 words, the others to 16
// bytes of scratch).
inline int block_key(int db, int fmt) { return 2 * db + (fmt == dedisp::kFmtSeg ? 1 : 0); }
void free_scratch(Scratch& x);
dedisp_status ensure_scratch(Scratch& x, size_t need);
dedisp_status ensure_xc(const struct ::dedisp_plan_s& p, Scratch& x, long long nsamps,
                        const LaunchPlan& lp);
dedisp_status ensure_device_table(::dedisp_plan p);

// Descriptor of one transform over the virtual input [in0 (n0 rows) | in1].
void fill_desc(::dedisp_plan p, const LaunchPlan& lp, const void* in0, long long n0,
               const void* in1, long long nsamps, uint32_t* out, long long stride,
               uint8_t* xc, BeamDesc& d);
// Corner turn (tiled shapes) + transform, on one stream.
hipError_t launch_desc(const BeamDesc& d, const LaunchPlan& lp, hipStream_t st);

// One transform ready to enqueue.
struct Item {
    BeamDesc d{};
    LaunchPlan lp;
};
// Enqueue every item on one stream: the corner turns, then the tiled items as
// multi-beam launches of up to kMaxBatchDescs beams each (every tiled item
// must use a multi-beam shape), then the untiled items one launch each.
hipError_t enqueue_items(std::vector<Item>& items, hipStream_t st);

std::string cache_key(::dedisp_plan p, size_t nsamps);
std::map<std::string, std::vector<double>> read_cache(const char* path);
void write_cache(const char* path, const std::map<std::string, std::vector<double>>& m);

}  // namespace host
}  // namespace dedisp

// A group of trials that share one time-scrunching factor: an internal plan
// over those DMs at s times the sampling time, and the output row of each.
struct ScrunchGroup {
    int s = 1;
    std::vector<int32_t> rows;
    struct dedisp_plan_s* sub = nullptr;
    int32_t* d_rows = nullptr;
};

// The object behind dedisp_plan.
struct dedisp_plan_s {
    dedisp_plan_s()
    {
        xc.owner = &inflight;
        sb_xc2.owner = &inflight;
    }
    dedisp_plan_s(const dedisp_plan_s&) = delete;
    dedisp_plan_s& operator=(const dedisp_plan_s&) = delete;
    // work enqueued with this plan's tables and scratch (its own executes,
    // and the pushes and batch launches that read its tables)
    dedisp::host::InFlight inflight;
    int nchans = 0;
    int nbits = 0;
    int fmt = 0;                    // scratch sample format (dedisp::Fmt)
    int scrunch = 1;                // input samples summed per scratch sample
    int out_nbits = 32;             // output width: 8, 16 or 32 bits
    int out_shift = 0;              // outputs are min(sum >> out_shift, 2^out_nbits - 1)
    double dt = 0, f_top = 0, df = 0;
    int row_bytes = 0;
    std::vector<double> dms;
    std::vector<int32_t> table;     // [ndm][nchans]
    int max_delay = 0;
    bool has_dms = false;
    dedisp_tile_config cfg{};
    int device = -1;
    int32_t* d_table = nullptr;
    std::map<int, dedisp::host::BlockTables> blocks;  // keyed by block_key(DM-block size, format)
    dedisp::host::Scratch xc;                          // channel-major scratch for execute
    // Channel kill mask (empty = every channel on): live channels in order,
    // and the device copies the kernels read.
    std::vector<int32_t> killmask;
    std::vector<int32_t> active;
    int32_t* d_chanmap = nullptr;
    int32_t* d_mask = nullptr;
    // Time-scrunching (empty = off): factor per trial and the groups.
    std::vector<int32_t> scrunch_factors;
    std::vector<ScrunchGroup> groups;
    // Sub-band dedispersion (0 = off): channels per sub-band, trials per
    // nominal DM, the two grouped passes and the intermediate scratch.
    int sb_nsub = 0, sb_ngroup = 0;
    struct dedisp_plan_s* sb_step1 = nullptr;
    struct dedisp_plan_s* sb_step2 = nullptr;
    dedisp::host::Scratch sb_xc2;
    // Internal plans of grouped passes: the table holds ngroups blocks of
    // [ndm][nchans]; the last group has ndm_last valid rows; vbound (when
    // set) bounds one scratch sample.
    // Piecewise linear tree (0 = off): sub-band width; the (sub-band, pass)
    // pairs stage 1 computes, pair y's rows at y*nsub .. y*nsub + nsub - 1;
    // per (trial, sub-band) the stage-1 row of d'_n(d) and the delay
    // dt''_n(d); passes in use = largest pass + 1.
    int tree_nsub = 0;
    int tree_maxdelay = 0;
    int tree_npass = 0;
    std::vector<int32_t> tree_pairs;        // [npairs][2] = (sub-band, pass)
    std::vector<int32_t> tree_rows, tree_delay;
    int32_t* d_tree_rows = nullptr;
    int32_t* d_tree_delay = nullptr;
    int32_t* d_tree_pairs = nullptr;
    // LDS-staged stage 2 (byte rows): staged trial blocks with their tables,
    // per (trial, sub-band) LDS byte offsets, and the trials of the blocks
    // whose rows do not fit (gathered from global memory instead)
    std::vector<dedisp::TreeStage> tree_stage;
    std::vector<int32_t> tree_sblocks, tree_off, tree_gtrials;
    int tree_lds = 0;                       // dwords per workgroup
    int tree_span = 0;                      // most rows a staged block reads of one sub-band
    dedisp::TreeStage* d_tree_stage = nullptr;
    int32_t* d_tree_sblocks = nullptr;
    int32_t* d_tree_off = nullptr;
    int32_t* d_tree_gtrials = nullptr;
    bool internal = false;
    int ngroups = 1;
    int ndm_last = 0;
    int vbound = 0;

    // largest value of one scratch sample
    int value_bound() const { return vbound ? vbound : (nbits == 2 ? 3 : 255) * scrunch; }

    int nact() const { return killmask.empty() ? nchans : static_cast<int>(active.size()); }
    // channel rows the tiled kernel sums: live channels padded with zero rows
    // to a whole number of its channel units (8, or 32 for bit planes)
    int nact_padded() const
    {
        const int u = dedisp::fmt_chan_unit(fmt);
        return (nact() + u - 1) / u * u;
    }
    int source_channel(int row) const { return killmask.empty() ? row : active[row]; }
};
