// Batches: several beams -- differing in channel count, bit depth, length,
// DM list and tile shape -- dedispersed by one multi-beam launch (after one
// multi-beam corner-turn launch), captured once into a HIP graph.  Tile shapes
// are chosen per beam by timing the candidates on the beam's own buffers,
// with results kept in a JSON cache keyed by the beam's shape.
#include "dedisp_host.h"

#include <algorithm>
#include <new>
#include <vector>

using dedisp::BeamDesc;
using dedisp::DescBlock;
using dedisp::Shape;
using namespace dedisp::host;

namespace dedisp {
namespace host {

hipError_t enqueue_items(std::vector<Item>& items, hipStream_t st)
{
    // corner turns of the tiled beams, up to kMaxBatchDescs per launch
    {
        DescBlock ub{};
        int n = 0;
        for (const Item& it : items) {
            if (it.lp.shape.kind != 0) continue;
            ub.d[n] = it.d;
            ub.d[n].in_nbits = it.lp.nbits;
            if (++n == kMaxBatchDescs) {
                hipError_t e = launch_unpack_multi(ub, n, st);
                if (e != hipSuccess) return e;
                n = 0;
            }
        }
        if (n > 0) {
            hipError_t e = launch_unpack_multi(ub, n, st);
            if (e != hipSuccess) return e;
        }
    }
    // multi-beam launches per class, up to kMaxBatchDescs beams each
    for (int cls = 1; cls <= dedisp::kMultiClasses; ++cls) {
        std::vector<Item*> tiled;
        for (Item& it : items) {
            if (it.lp.shape.kind != 0) continue;
            if (it.lp.shape.multi < 1 || it.lp.shape.multi > dedisp::kMultiClasses) return hipErrorInvalidValue;
            if (it.lp.shape.multi == cls) tiled.push_back(&it);
        }
        for (size_t g0 = 0; g0 < tiled.size(); g0 += kMaxBatchDescs) {
            const size_t g1 = std::min(tiled.size(), g0 + kMaxBatchDescs);
            DescBlock blk{};
            long long total = 0;
            int lds = 0;
            for (size_t i = g0; i < g1; ++i) {
                BeamDesc& d = tiled[i]->d;
                d.work_begin = total;   // a multiple of 8: see the multi-beam kernel
                total += (static_cast<long long>(d.ntiles) * d.nblocks + 7) / 8 * 8;
                lds = std::max(lds, tiled[i]->lp.lds);
                blk.d[i - g0] = d;
            }
            if (total > 0x7fffffffLL) return hipErrorInvalidValue;
            hipError_t e = launch_multi(blk, static_cast<int>(g1 - g0), static_cast<int>(total), lds, cls, st);
            if (e != hipSuccess) return e;
        }
    }
    for (const Item& it : items)
        if (it.lp.shape.kind != 0) {
            hipError_t e = launch_untiled(it.d, it.lp.nbits, st);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace host
}  // namespace dedisp

struct dedisp_batch_s {
    InFlight inflight;                // this batch's launches
    std::vector<dedisp_beam> beams;
    std::vector<Item> items;
    std::vector<Scratch> xcs;         // channel-major scratch per beam
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

dedisp_tile_config config_of(const Shape& s)
{
    dedisp_tile_config c{};
    c.kind = s.kind;
    c.waves = s.waves;
    c.dms_per_wave = s.dpw;
    c.words_per_lane = s.m;
    c.chunk_chans = s.cc;
    c.sample_format = s.kind == 0 ? s.fmt : -1;
    return c;
}

// Pick the fastest multi-beam shape for one beam: from the cache when it has
// the beam's key, else by timing each candidate (plain single-beam launches
// on the beam's own buffers).
dedisp_status tune_beam(const dedisp_beam& bm, std::map<std::string, std::vector<double>>& cache,
                        bool& cache_dirty, hipStream_t st, dedisp_tile_config& best)
{
    dedisp_plan p = bm.plan;
    const std::string key = "multi:" + cache_key(p, bm.nsamps);
    auto hit = cache.find(key);
    if (hit != cache.end() && hit->second.size() >= 5) {
        dedisp_tile_config c{};
        c.kind = static_cast<int>(hit->second[0]);
        c.waves = static_cast<int>(hit->second[1]);
        c.dms_per_wave = static_cast<int>(hit->second[2]);
        c.words_per_lane = static_cast<int>(hit->second[3]);
        c.chunk_chans = static_cast<int>(hit->second[4]);
        c.sample_format = hit->second.size() > 6 ? static_cast<int>(hit->second[6]) : -1;
        int idx = -1;
        if (find_shape(c, *p, &idx) && dedisp::shape_at(idx).multi) {
            best = c;
            return DEDISP_OK;
        }
    }
    std::vector<int> cands;
    for (int i = 0; i < dedisp::shape_count(); ++i) {
        const Shape& s = dedisp::shape_at(i);
        if (!shape_matches(s, *p) || s.kind != 0 || !s.multi) continue;
        LaunchPlan probe;
        if (resolve_launch(p, config_of(s), false, probe, true,
                           static_cast<long long>(bm.nsamps) - p->max_delay) != DEDISP_OK ||
            probe.shape_index != i)
            continue;
        cands.push_back(i);
    }
    if (cands.empty()) {
        best = dedisp_tile_config{};
        best.kind = 1;
        return DEDISP_OK;
    }
    if (cands.size() == 1) {
        best = config_of(dedisp::shape_at(cands[0]));
        return DEDISP_OK;
    }
    const dedisp_tile_config saved = p->cfg;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 1e30f;
    dedisp_status rc = DEDISP_OK;
    for (int i : cands) {
        p->cfg = config_of(dedisp::shape_at(i));
        rc = dedisp_execute(p, bm.d_in, bm.nsamps, bm.d_out, bm.out_row_stride, st);
        if (rc != DEDISP_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = DEDISP_ERR_HIP; break; }
        for (int r = 0; r < 3 && rc == DEDISP_OK; ++r)
            rc = dedisp_execute(p, bm.d_in, bm.nsamps, bm.d_out, bm.out_row_stride, st);
        if (rc != DEDISP_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = DEDISP_ERR_HIP;
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            best = p->cfg;
        }
    }
    p->cfg = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DEDISP_OK) return rc;
    cache[key] = {static_cast<double>(best.kind), static_cast<double>(best.waves),
                  static_cast<double>(best.dms_per_wave), static_cast<double>(best.words_per_lane),
                  static_cast<double>(best.chunk_chans), static_cast<double>(best_ms / 3),
                  static_cast<double>(best.sample_format)};
    cache_dirty = true;
    return DEDISP_OK;
}

// A batch launch reads every beam's plan tables: track it on the batch and
// on those plans.
void record_batch(dedisp_batch b, hipStream_t st)
{
    b->inflight.record(st);
    for (const auto& bm : b->beams) bm.plan->inflight.record(st);
}

}  // namespace

extern "C" {

dedisp_status dedisp_batch_create(const dedisp_beam* beams, int nbeams, const char* cache_path,
                                  void* stream, dedisp_batch* out)
{
    if (!out) return fail(DEDISP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!beams || nbeams <= 0) return fail(DEDISP_ERR_INVALID_ARG, "no beams");
    for (int i = 0; i < nbeams; ++i) {
        const dedisp_beam& b = beams[i];
        if (!b.plan || !b.d_in || !b.d_out) return fail(DEDISP_ERR_INVALID_ARG, "NULL beam field");
        if (!b.plan->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "beam without DM list");
        if (!b.plan->groups.empty() || b.plan->sb_step1 || b.plan->tree_nsub)
            return fail(DEDISP_ERR_UNSUPPORTED, "batches support the direct transform only");
        if (b.nsamps <= static_cast<size_t>(b.plan->max_delay))
            return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "beam nsamps <= max_delay");
        if (b.nsamps > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "beam too long");
        const size_t nout = b.nsamps - b.plan->max_delay;
        if (b.out_row_stride != 0 && b.out_row_stride < nout)
            return fail(DEDISP_ERR_INVALID_ARG, "beam out_row_stride too small");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    dedisp_batch bt = new (std::nothrow) dedisp_batch_s;
    if (!bt) return fail(DEDISP_ERR_OOM, "batch allocation");
    bt->beams.assign(beams, beams + nbeams);
    bt->items.resize(static_cast<size_t>(nbeams));
    bt->xcs.resize(static_cast<size_t>(nbeams));
    for (auto& x : bt->xcs) x.owner = &bt->inflight;
    auto cache = read_cache(cache_path);
    bool dirty = false;
    dedisp_status rc = DEDISP_OK;
    for (int i = 0; i < nbeams && rc == DEDISP_OK; ++i) {
        const dedisp_beam& b = beams[i];
        dedisp_tile_config cfg{};
        rc = tune_beam(b, cache, dirty, st, cfg);
        if (rc != DEDISP_OK) break;
        LaunchPlan lp;
        rc = resolve_launch(b.plan, cfg, true, lp, cfg.kind == 0,
                            static_cast<long long>(b.nsamps) - b.plan->max_delay);
        if (rc != DEDISP_OK) break;
        if (lp.shape.kind == 0 && (reinterpret_cast<uintptr_t>(b.d_in) & 3)) {
            dedisp_tile_config u{};
            u.kind = 1;
            rc = resolve_launch(b.plan, u, true, lp);
            if (rc != DEDISP_OK) break;
        }
        rc = ensure_xc(*b.plan, bt->xcs[i], static_cast<long long>(b.nsamps), lp);
        if (rc != DEDISP_OK) break;
        const size_t nout = b.nsamps - b.plan->max_delay;
        bt->items[i].lp = lp;
        fill_desc(b.plan, lp, b.d_in, static_cast<long long>(b.nsamps), nullptr,
                  static_cast<long long>(b.nsamps), b.d_out,
                  static_cast<long long>(b.out_row_stride ? b.out_row_stride : nout),
                  bt->xcs[i].ptr, bt->items[i].d);
    }
    if (rc == DEDISP_OK && dirty) write_cache(cache_path, cache);
    if (rc == DEDISP_OK && hipStreamSynchronize(st) != hipSuccess) rc = hip_fail(hipErrorUnknown, "sync");
    // Capture the launch sequence once on a private stream.
    if (rc == DEDISP_OK && hipStreamCreateWithFlags(&bt->capture, hipStreamNonBlocking) != hipSuccess)
        rc = hip_fail(hipErrorUnknown, "hipStreamCreate");
    if (rc == DEDISP_OK) {
        hipError_t e = hipStreamBeginCapture(bt->capture, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = enqueue_items(bt->items, bt->capture);
            e = hipStreamEndCapture(bt->capture, &bt->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "graph capture");
    }
    if (rc != DEDISP_OK) {
        dedisp_batch_destroy(bt);
        return rc;
    }
    *out = bt;
    return DEDISP_OK;
}

dedisp_status dedisp_batch_execute(dedisp_batch b, void* stream)
{
    if (!b || !b->exec) return fail(DEDISP_ERR_INVALID_ARG, "NULL batch");
    HIP_TRY(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
    record_batch(b, static_cast<hipStream_t>(stream));
    return DEDISP_OK;
}

dedisp_status dedisp_batch_execute_direct(dedisp_batch b, void* stream)
{
    if (!b) return fail(DEDISP_ERR_INVALID_ARG, "NULL batch");
    hipError_t e = enqueue_items(b->items, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    record_batch(b, static_cast<hipStream_t>(stream));
    return DEDISP_OK;
}

void dedisp_batch_destroy(dedisp_batch b)
{
    if (!b) return;
    b->inflight.wait();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (auto& x : b->xcs) free_scratch(x);
    delete b;
}

}  // extern "C"
