// Streams: overlap-save dedispersion of an unbounded input.
//
// A stream keeps the last max_delay input rows of everything pushed so far
// on the device (its history).  A push of L rows dedisperses the virtual
// input [history | chunk] -- the kernels read the two segments in place, so
// the chunk is never copied next to the history -- which yields exactly the
// outputs the data seen so far fully covers, and then replaces the history
// with the last max_delay rows of that virtual input.  Concatenating the
// outputs of all pushes gives the one-shot transform of the concatenated
// input (the time-division processing of Section 6 of the paper, without
// dropping the samples at chunk boundaries).
//
// dedisp_stream_push_many runs several streams' pushes as one multi-beam
// launch: the continuous-batching step of a serving loop.
#include "dedisp_host.h"

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

using dedisp::BeamDesc;
using namespace dedisp::host;

struct dedisp_stream_s {
    dedisp_stream_s() { xc.owner = &inflight; }
    InFlight inflight;                        // this stream's pushes
    dedisp_plan plan = nullptr;
    int row_bytes = 0;
    int max_delay = 0;
    uint8_t* hist[2] = {nullptr, nullptr};   // ping-pong history buffers, max_delay rows each
    int cur = 0;
    size_t hist_rows = 0;
    uint64_t total = 0;
    Scratch xc;                               // channel-major scratch of this stream
};

namespace {

// What one push needs enqueued.
struct PushPlan {
    size_t L = 0;
    bool has_output = false;
    size_t nout = 0;
    Item item;
};

dedisp_status check_stream(dedisp_stream s)
{
    if (!s || !s->plan) return fail(DEDISP_ERR_INVALID_ARG, "NULL stream");
    if (!s->plan->has_dms || s->plan->max_delay != s->max_delay)
        return fail(DEDISP_ERR_INVALID_ARG, "the plan's DM list changed after the stream was created");
    if (!s->plan->groups.empty() || s->plan->sb_step1 || s->plan->tree_nsub)
        return fail(DEDISP_ERR_UNSUPPORTED, "streams support the direct transform only");
    return DEDISP_OK;
}

// Validate a push and build its launch (no device work yet).
dedisp_status prepare_push(dedisp_stream s, const void* chunk, size_t L, uint32_t* out,
                           size_t stride, bool multi, PushPlan& pp)
{
    dedisp_status st = check_stream(s);
    if (st != DEDISP_OK) return st;
    if (L > 0 && !chunk) return fail(DEDISP_ERR_INVALID_ARG, "NULL chunk");
    if (L > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "chunk too large");
    pp.L = L;
    const size_t N = s->hist_rows + L;
    pp.has_output = N > static_cast<size_t>(s->max_delay);
    if (!pp.has_output) return DEDISP_OK;
    pp.nout = N - s->max_delay;
    if (!out) return fail(DEDISP_ERR_INVALID_ARG, "NULL output for a push that produces output");
    if (stride == 0) stride = pp.nout;
    if (stride < pp.nout) return fail(DEDISP_ERR_INVALID_ARG, "out_row_stride < new outputs");
    dedisp_plan p = s->plan;
    LaunchPlan lp;
    st = resolve_launch(p, p->cfg, true, lp, multi, static_cast<long long>(pp.nout));
    if (st != DEDISP_OK) return st;
    if (lp.shape.kind == 0 && (reinterpret_cast<uintptr_t>(chunk) & 3)) {
        dedisp_tile_config u{};
        u.kind = 1;
        st = resolve_launch(p, u, true, lp);
        if (st != DEDISP_OK) return st;
    }
    st = ensure_xc(*p, s->xc, static_cast<long long>(N), lp);
    if (st != DEDISP_OK) return st;
    pp.item.lp = lp;
    fill_desc(p, lp, s->hist[s->cur], static_cast<long long>(s->hist_rows), chunk,
              static_cast<long long>(N), out, static_cast<long long>(stride), s->xc.ptr,
              pp.item.d);
    return DEDISP_OK;
}

// Enqueue the history update after the push's kernels (same stream).
dedisp_status update_history(dedisp_stream s, const void* chunk, const PushPlan& pp,
                             hipStream_t st)
{
    const size_t rb = static_cast<size_t>(s->row_bytes);
    const size_t md = static_cast<size_t>(s->max_delay);
    const size_t L = pp.L;
    if (L == 0) return DEDISP_OK;
    if (!pp.has_output) {
        // still priming: append the chunk
        HIP_TRY(hipMemcpyAsync(s->hist[s->cur] + s->hist_rows * rb, chunk, L * rb,
                               hipMemcpyDeviceToDevice, st));
        s->hist_rows += L;
        s->total += L;
        return DEDISP_OK;
    }
    const int other = 1 - s->cur;
    if (md > 0) {
        if (L >= md) {
            HIP_TRY(hipMemcpyAsync(s->hist[other], static_cast<const uint8_t*>(chunk) + (L - md) * rb,
                                   md * rb, hipMemcpyDeviceToDevice, st));
        } else {
            const size_t keep = md - L;
            HIP_TRY(hipMemcpyAsync(s->hist[other], s->hist[s->cur] + (s->hist_rows - keep) * rb,
                                   keep * rb, hipMemcpyDeviceToDevice, st));
            HIP_TRY(hipMemcpyAsync(s->hist[other] + keep * rb, chunk, L * rb,
                                   hipMemcpyDeviceToDevice, st));
        }
    }
    s->cur = other;
    s->hist_rows = md;
    s->total += L;
    return DEDISP_OK;
}

}  // namespace

extern "C" {

dedisp_status dedisp_stream_create(dedisp_plan plan, dedisp_stream* out)
{
    if (!out) return fail(DEDISP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!plan) return fail(DEDISP_ERR_INVALID_ARG, "plan is NULL");
    if (!plan->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (!plan->groups.empty() || plan->sb_step1 || plan->tree_nsub)
        return fail(DEDISP_ERR_UNSUPPORTED, "streams support the direct transform only");
    dedisp_stream s = new (std::nothrow) dedisp_stream_s;
    if (!s) return fail(DEDISP_ERR_OOM, "stream allocation");
    s->plan = plan;
    s->row_bytes = plan->row_bytes;
    s->max_delay = plan->max_delay;
    const size_t bytes = std::max<size_t>(1, static_cast<size_t>(s->max_delay)) * s->row_bytes;
    for (int i = 0; i < 2; ++i) {
        if (hipMalloc(&s->hist[i], bytes) != hipSuccess) {
            s->hist[i] = nullptr;
            dedisp_stream_destroy(s);
            return fail(DEDISP_ERR_OOM, "hipMalloc history");
        }
    }
    *out = s;
    return DEDISP_OK;
}

void dedisp_stream_destroy(dedisp_stream s)
{
    if (!s) return;
    s->inflight.wait();
    for (int i = 0; i < 2; ++i)
        if (s->hist[i]) (void)hipFree(s->hist[i]);
    free_scratch(s->xc);
    delete s;
}

dedisp_status dedisp_stream_reserve(dedisp_stream s, size_t max_chunk)
{
    dedisp_status st = check_stream(s);
    if (st != DEDISP_OK) return st;
    if (max_chunk == 0 || max_chunk > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "bad max_chunk");
    // the longest push scans max_delay history rows plus the chunk, with the
    // shape a batched push (multi-beam shapes) or a single push resolves to
    const long long n = static_cast<long long>(s->max_delay + max_chunk);
    for (bool multi : {true, false}) {
        LaunchPlan lp;
        st = resolve_launch(s->plan, s->plan->cfg, false, lp, multi, static_cast<long long>(max_chunk));
        if (st != DEDISP_OK) return st;
        st = ensure_xc(*s->plan, s->xc, n, lp);
        if (st != DEDISP_OK) return st;
    }
    return DEDISP_OK;
}

dedisp_status dedisp_stream_push(dedisp_stream s, const void* chunk, size_t nsamps,
                                 uint32_t* out, size_t stride, size_t* n_out, void* stream)
{
    if (!n_out) return fail(DEDISP_ERR_INVALID_ARG, "n_out is NULL");
    *n_out = 0;
    PushPlan pp;
    dedisp_status st = prepare_push(s, chunk, nsamps, out, stride, false, pp);
    if (st != DEDISP_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (pp.has_output) {
        hipError_t e = launch_desc(pp.item.d, pp.item.lp, hs);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    st = update_history(s, chunk, pp, hs);
    if (st != DEDISP_OK) return st;
    s->inflight.record(hs);
    s->plan->inflight.record(hs);
    *n_out = pp.nout;
    return DEDISP_OK;
}

dedisp_status dedisp_stream_push_many(dedisp_stream* streams, const void* const* chunks,
                                      const size_t* nsamps, uint32_t* const* outs,
                                      const size_t* strides, size_t* n_outs, int n, void* stream)
{
    if (!streams || !chunks || !nsamps || !outs || !n_outs || n < 0)
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    for (int i = 0; i < n; ++i) {
        n_outs[i] = 0;
        for (int j = 0; j < i; ++j)
            if (streams[i] == streams[j]) return fail(DEDISP_ERR_INVALID_ARG, "a stream appears twice");
    }
    std::vector<PushPlan> pps(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        dedisp_status st = prepare_push(streams[i], chunks[i], nsamps[i], outs[i],
                                        strides ? strides[i] : 0, true, pps[i]);
        if (st != DEDISP_OK) return st;
    }
    std::vector<Item> items;
    for (auto& pp : pps)
        if (pp.has_output) items.push_back(pp.item);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (!items.empty()) {
        hipError_t e = enqueue_items(items, hs);
        if (e != hipSuccess) return hip_fail(e, "batched launch");
    }
    for (int i = 0; i < n; ++i) {
        dedisp_status st = update_history(streams[i], chunks[i], pps[i], hs);
        if (st != DEDISP_OK) return st;
        streams[i]->inflight.record(hs);
        streams[i]->plan->inflight.record(hs);
        n_outs[i] = pps[i].nout;
    }
    return DEDISP_OK;
}

dedisp_status dedisp_stream_get_device_bytes(dedisp_stream s, size_t* bytes)
{
    if (!s || !bytes) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    const size_t hist = std::max<size_t>(1, static_cast<size_t>(s->max_delay)) * s->row_bytes;
    *bytes = 2 * hist + s->xc.bytes;
    return DEDISP_OK;
}

dedisp_status dedisp_stream_get_state(dedisp_stream s, size_t* history_rows, uint64_t* total_rows)
{
    if (!s || !history_rows || !total_rows) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    *history_rows = s->hist_rows;
    *total_rows = s->total;
    return DEDISP_OK;
}

dedisp_status dedisp_stream_get_history(dedisp_stream s, void* host_buf, size_t* nsamps)
{
    if (!s || !nsamps) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    *nsamps = s->hist_rows;
    if (s->hist_rows == 0) return DEDISP_OK;
    if (!host_buf) return fail(DEDISP_ERR_INVALID_ARG, "host_buf is NULL");
    // after this stream's pushes only, on the stream they last ran on
    s->inflight.wait();
    HIP_TRY(hipMemcpyAsync(host_buf, s->hist[s->cur], s->hist_rows * s->row_bytes, hipMemcpyDeviceToHost,
                           s->inflight.last));
    HIP_TRY(hipStreamSynchronize(s->inflight.last));
    return DEDISP_OK;
}

dedisp_status dedisp_stream_set_history(dedisp_stream s, const void* host_buf, size_t nsamps,
                                        uint64_t total_rows)
{
    dedisp_status st = check_stream(s);
    if (st != DEDISP_OK) return st;
    const size_t md = static_cast<size_t>(s->max_delay);
    if (nsamps > md || total_rows < nsamps) return fail(DEDISP_ERR_INVALID_ARG, "bad history size");
    if (total_rows > md ? nsamps != md : nsamps != total_rows)
        return fail(DEDISP_ERR_INVALID_ARG, "history rows inconsistent with total_rows");
    if (nsamps > 0 && !host_buf) return fail(DEDISP_ERR_INVALID_ARG, "host_buf is NULL");
    s->inflight.wait();
    if (nsamps > 0) {
        HIP_TRY(hipMemcpyAsync(s->hist[s->cur], host_buf, nsamps * s->row_bytes, hipMemcpyHostToDevice,
                               s->inflight.last));
        HIP_TRY(hipStreamSynchronize(s->inflight.last));
    }
    s->hist_rows = nsamps;
    s->total = total_rows;
    return DEDISP_OK;
}

dedisp_status dedisp_stream_reset(dedisp_stream s)
{
    if (!s) return fail(DEDISP_ERR_INVALID_ARG, "NULL stream");
    s->hist_rows = 0;
    s->total = 0;
    return DEDISP_OK;
}

}  // extern "C"
