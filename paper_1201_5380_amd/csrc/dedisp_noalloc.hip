// Allocation-free direct transform (dedisp_execute_noalloc): the corner turn
// and the tiled kernel of dedisp_execute, with the channel-major scratch
// taken from a fixed device array of this file instead of a plan-owned
// buffer, so the call itself never allocates or frees device memory.
//
// The array is a file-scope device variable.  In host code its name is only a
// host-side stand-in; the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device (with that device current) on
// the first call there, and only that address is handed to kernels.
#include "dedisp_host.h"

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>

namespace {

static __device__ __align__(256) uint8_t scratch[DEDISP_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::unordered_map<int, uint8_t*> g_scratch_ptr;   // device ordinal -> that device's copy

// Device address of the current device's copy of the array.
dedisp_status device_scratch(int dev, uint8_t** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        uint8_t* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch));
        if (e != hipSuccess) return dedisp::host::hip_fail(e, "hipGetSymbolAddress(no-alloc scratch)");
        if (!ptr) return dedisp::host::fail(DEDISP_ERR_HIP, "hipGetSymbolAddress(no-alloc scratch): null address");
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return DEDISP_OK;
}

}  // namespace

extern "C" dedisp_status dedisp_execute_noalloc(dedisp_plan p, const void* d_in, size_t nsamps,
                                                uint32_t* d_out, size_t stride, void* stream)
{
    using namespace dedisp::host;
    if (!p || !d_in || !d_out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_dms) return fail(DEDISP_ERR_NO_DM_LIST, "no DM list");
    if (p->tree_nsub || p->sb_step1 || !p->groups.empty())
        return fail(DEDISP_ERR_UNSUPPORTED,
                    "the no-alloc call runs the plain direct transform only (tree, sub-band and "
                    "time-scrunching modes are not served)");
    if (nsamps <= static_cast<size_t>(p->max_delay))
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps <= max_delay");
    if (nsamps > (1ULL << 40)) return fail(DEDISP_ERR_INVALID_ARG, "nsamps too large");
    const long long nout = static_cast<long long>(nsamps) - p->max_delay;
    if (stride == 0) stride = static_cast<size_t>(nout);
    if (stride < static_cast<size_t>(nout))
        return fail(DEDISP_ERR_INVALID_ARG, "out_row_stride < nsamps - max_delay");

    // the shape dedisp_execute would use, resolved without touching the device
    LaunchPlan lp;
    dedisp_status st = resolve_launch(p, p->cfg, false, lp, false, nout);
    if (st != DEDISP_OK) return st;
    if (lp.shape.kind == 0 && (reinterpret_cast<uintptr_t>(d_in) & 3)) {
        dedisp_tile_config u{};
        u.kind = 1;
        st = resolve_launch(p, u, false, lp);
        if (st != DEDISP_OK) return st;
    }
    // every device table must already be resident: building one allocates
    const char* not_built =
        "the plan's device tables for its current DM list, kill mask and tile shape are not built "
        "on this device (run dedisp_execute or dedisp_tune on the plan once first)";
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (p->device != dev || !p->d_table) return fail(DEDISP_ERR_UNSUPPORTED, not_built);
    if (!p->killmask.empty() && (!p->d_chanmap || !p->d_mask)) return fail(DEDISP_ERR_UNSUPPORTED, not_built);
    if (lp.shape.kind == 0) {
        auto it = p->blocks.find(block_key(lp.shape.waves * lp.shape.dpw, lp.shape.fmt));
        if (it == p->blocks.end() || !it->second.d_rel || !it->second.d_base)
            return fail(DEDISP_ERR_UNSUPPORTED, not_built);
        lp.bt = &it->second;
    }
    const hipStream_t hs = static_cast<hipStream_t>(stream);

    if (lp.shape.kind != 0) {
        // the untiled kernel reads the input directly: no scratch at all
        dedisp::BeamDesc d;
        fill_desc(p, lp, d_in, static_cast<long long>(nsamps), nullptr, static_cast<long long>(nsamps),
                  d_out, static_cast<long long>(stride), nullptr, d);
        const hipError_t e = launch_desc(d, lp, hs);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        p->inflight.record_existing(hs);
        return DEDISP_OK;
    }

    // Time slices whose channel-major scratch fits the array: slice k covers
    // outputs [k*T, k*T + T) and reads input rows [k*T, k*T + T + max_delay)
    // (overlap-save), T a whole number of time tiles.
    const long long rows = static_cast<long long>(p->nact_padded()) * dedisp::fmt_rows(lp.shape.fmt);
    const long long cap = static_cast<long long>(DEDISP_NOALLOC_SCRATCH_BYTES);
    auto need = [&](long long ns) { return xc_pitch(ns, lp.shape.fmt, lp.rw, p->max_delay) * rows; };
    const long long tl = tile_len(lp.shape);
    long long T = nout;
    if (need(static_cast<long long>(nsamps)) > cap) {
        // the most whole tiles per slice whose scratch fits (need grows with ns)
        long long lo = 0, hi = (nout + tl - 1) / tl;
        while (lo < hi) {
            const long long mid = (lo + hi + 1) / 2;
            if (need(mid * tl + p->max_delay) <= cap) lo = mid;
            else hi = mid - 1;
        }
        T = lo * tl;
        if (T <= 0)
            return fail(DEDISP_ERR_UNSUPPORTED,
                        "one time tile plus max_delay rows of this plan's channel-major scratch (" +
                            std::to_string(need(tl + p->max_delay)) + " bytes) exceeds the no-alloc scratch (" +
                            std::to_string(cap) + " bytes)");
    }
    uint8_t* xc = nullptr;
    st = device_scratch(dev, &xc);
    if (st != DEDISP_OK) return st;
    const long long ob = p->out_nbits / 8;
    for (long long t0 = 0; t0 < nout; t0 += T) {
        const long long n = std::min(T, nout - t0);
        const long long ns = n + p->max_delay;
        const uint8_t* in = static_cast<const uint8_t*>(d_in) + t0 * p->row_bytes;
        uint32_t* out = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(d_out) + t0 * ob);
        dedisp::BeamDesc d;
        fill_desc(p, lp, in, ns, nullptr, ns, out, static_cast<long long>(stride), xc, d);
        const hipError_t e = launch_desc(d, lp, hs);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    p->inflight.record_existing(hs);
    return DEDISP_OK;
}
