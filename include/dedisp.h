/*
 * dedisp.h -- C ABI of the MI355X (gfx950) direct incoherent dedispersion
 * library.
 *
 * The transform (Barsdell, Bailes, Barnes & Fluke 2012, "Accelerating
 * incoherent dedispersion", Section 2.1, eq. direct):
 *
 *     out[d][t] = sum_{c=0}^{nchans-1} in[t + delay[d][c]][c]
 *
 * with the per-channel delay of the Section 2.1 delay equations,
 *
 *     DeltaT[c]   = (k_DM / dt) * (1/(f_top + c*df)^2 - 1/f_top^2)
 *     delay[d][c] = round(DM[d] * DeltaT[c])        (half away from zero)
 *
 * k_DM = 4.148808e3 MHz^2 pc^-1 cm^3 s (Section 1), dt in seconds,
 * frequencies in MHz, DM in pc cm^-3.  Delays are computed once on the host
 * in IEEE binary64 in exactly that order and uploaded as an int32 table; the
 * GPU never recomputes them.  Sums are exact 32-bit unsigned integers.
 *
 * Conventions shared by every entry point:
 *   - Input ("filterbank"): nsamps rows, one per time sample, each
 *     nchans*nbits/8 bytes, channel fastest (time-major).  nbits is 2 or 8.
 *     2-bit: channel c is bits [2*(c%4), 2*(c%4)+1] of byte c/4 of its row.
 *     Samples are raw unsigned codes (0..3 or 0..255), summed as they are.
 *   - Channel 0 is the top of the band (frequency f_top, zero delay);
 *     df < 0 so delays grow with channel index.
 *   - Output: ndm rows of uint32, row d at out + d*out_row_stride elements
 *     (out_row_stride = 0 means nsamps - max_delay).  Only fully covered
 *     outputs exist: t in [0, nsamps - max_delay).
 *   - Device pointers are HIP device addresses owned by the caller; they must
 *     stay valid until the work enqueued on `stream` has finished.  Host
 *     pointers are only read during the call.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Every compute call is asynchronous on that stream and returns as soon
 *     as the work is enqueued.
 *   - Every argument is validated on the host before any HIP call; an
 *     invalid call changes nothing and returns an error code.  No C++
 *     exception crosses this interface.
 *   - A plan, stream or batch is used by one host thread at a time.
 */
#ifndef DEDISP_H
#define DEDISP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dedisp_plan_s*   dedisp_plan;    /* observing set-up + DM list + device tables */
typedef struct dedisp_stream_s* dedisp_stream;  /* one unbounded input stream (owns its history) */
typedef struct dedisp_batch_s*  dedisp_batch;   /* a fixed set of beams run as one launch */
typedef int dedisp_status;

enum {
    DEDISP_OK                  = 0,
    DEDISP_ERR_INVALID_ARG     = -1,  /* a null pointer, size or parameter out of range */
    DEDISP_ERR_NO_DM_LIST      = -2,  /* compute requested before dedisp_set_dm_list */
    DEDISP_ERR_TOO_FEW_SAMPLES = -3,  /* nsamps <= max_delay: no output is fully covered */
    DEDISP_ERR_OOM             = -4,  /* a device or host allocation failed */
    DEDISP_ERR_HIP             = -5,  /* a HIP runtime call failed; see dedisp_last_error */
    DEDISP_ERR_UNSUPPORTED     = -6   /* valid request this build cannot serve */
};

/* Human-readable name of a status code (static storage). */
const char* dedisp_status_string(dedisp_status status);

/* Text of the most recent error on the calling host thread (static,
 * thread-local storage; "" if none).  Holds the HIP error string after
 * DEDISP_ERR_HIP. */
const char* dedisp_last_error(void);

/* ---------------------------------------------------------------- plans */

/* Create a plan for `nchans` channels of `nbits`-bit samples taken every
 * `dt_s` seconds, channel 0 at `f_top_mhz`, channel spacing `df_mhz`
 * (Section 2.1: the band start nu_0 and channel spacing Delta nu).
 * Host-only: no HIP call is made.
 * Errors: INVALID_ARG if out == NULL, nchans <= 0, nbits not in {2, 8},
 * nchans*nbits not a multiple of 8, dt_s <= 0, f_top_mhz <= 0, df_mhz >= 0,
 * f_top_mhz + (nchans-1)*df_mhz <= 0, or any value not finite.
 * The caller owns *out and releases it with dedisp_plan_destroy. */
dedisp_status dedisp_plan_create(dedisp_plan* out, int nchans, double dt_s,
                                 double f_top_mhz, double df_mhz, int nbits);

/* Release a plan and its device tables (NULL is ignored).  Waits, on the
 * host, for the work enqueued with the plan (its executes and the stream
 * pushes and batch launches that read its tables) before freeing; other work
 * on the device is not waited for by the library (the HIP runtime's free may
 * still synchronise the device).  Streams and batches using the plan must
 * be destroyed first. */
void dedisp_plan_destroy(dedisp_plan plan);

/* Set the trial DMs (the DM(d) array of Section 2.1), `ndm` values in
 * pc cm^-3, any order, copied from host memory.  Computes the delay table on
 * the host; the device copy is made by the next compute call.
 * Errors: INVALID_ARG if dms == NULL, ndm <= 0, a DM is negative or not
 * finite, or a delay does not fit in int32. */
dedisp_status dedisp_set_dm_list(dedisp_plan plan, const double* dms, int ndm);

/* Channel kill mask (Section 2.3): mask[c] = 1 sums channel c, 0 skips it;
 * NULL (or all ones) restores every channel.  Host array of nchans int32,
 * copied; entries other than 0/1 are INVALID_ARG.  The delay table, max_delay
 * and the output range do not change.  Killed channels cost nothing in the
 * tiled kernel: the corner turn leaves them out of the channel-major
 * scratch.  Waits for the plan's own enqueued work before it drops the
 * device tables. */
dedisp_status dedisp_set_killmask(dedisp_plan plan, const int32_t* mask);

/* Plan queries (host-only).  NO_DM_LIST before dedisp_set_dm_list for the
 * DM-dependent ones. */
dedisp_status dedisp_get_nchans(dedisp_plan plan, int* nchans);
dedisp_status dedisp_get_nbits(dedisp_plan plan, int* nbits);
dedisp_status dedisp_get_dm_count(dedisp_plan plan, int* ndm);
dedisp_status dedisp_get_max_delay(dedisp_plan plan, int* max_delay);

/* Copy the delay table, row-major int32 [ndm][nchans] (row = DM), to host
 * memory `host_out` of at least ndm*nchans elements. */
dedisp_status dedisp_get_delay_table(dedisp_plan plan, int32_t* host_out);

/* The transform over one resident block of input.
 * d_in: device, nsamps rows of the input layout above.
 * d_out: device, ndm rows of out_row_stride (0 = nsamps - max_delay, or
 * the longest row under time-scrunching) elements of the plan's output
 * format (uint32 unless dedisp_set_output_format chose 8 or 16 bits); only
 * t < nsamps - max_delay is written (under time-scrunching, the row lengths
 * dedisp_get_output_lengths gives).
 * Errors: INVALID_ARG (null pointer, stride too small), NO_DM_LIST,
 * TOO_FEW_SAMPLES (nsamps <= max_delay, or nsamps/s <= the largest delay of
 * a scrunch group), OOM, HIP. */
dedisp_status dedisp_execute(dedisp_plan plan, const void* d_in, size_t nsamps,
                             uint32_t* d_out, size_t out_row_stride, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the plain
 * direct transform of dedisp_execute, same arguments and results, with its
 * channel-major scratch taken from one fixed device array of
 * DEDISP_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call makes no hipMalloc, hipFree or other
 * allocating call.  When one transform's scratch would not fit the array the
 * input is processed in consecutive time slices (each a whole number of time
 * tiles of outputs plus max_delay rows of input), which gives the same
 * outputs.
 * Preconditions: the plan's device tables for its current DM list, kill mask
 * and tile shape are already built on the current device, i.e. dedisp_execute
 * or dedisp_tune ran on the plan after the last change to any of them;
 * time-scrunching, sub-band and tree modes are off.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (no output depends on what an earlier call left there): calls
 * that overlap on one GPU (on different HIP streams, or from several host
 * threads) race and must be serialised by the caller, e.g. by issuing them
 * on one HIP stream.
 * Errors: INVALID_ARG (null pointer, stride too small), NO_DM_LIST,
 * TOO_FEW_SAMPLES, UNSUPPORTED (a mode other than the direct transform,
 * device tables not built, or one time tile plus max_delay rows of scratch
 * larger than the array), HIP. */
#define DEDISP_NOALLOC_SCRATCH_BYTES (128u << 20)
dedisp_status dedisp_execute_noalloc(dedisp_plan plan, const void* d_in, size_t nsamps,
                                     uint32_t* d_out, size_t out_row_stride, void* stream);

/* ----------------------------------------------------- time-scrunching */

/* Section 2.1: once a trial's dispersion trail crosses more than one sample
 * per channel (beyond the "diagonal" DM) the time resolution can be reduced
 * by adding adjacent samples, halving the work of those trials.
 *
 * The diagonal DM of the band: the DM at which the delay between the last
 * two channels -- the steepest part of the trail -- is one sample,
 * 1 / (DeltaT(nchans-1) - DeltaT(nchans-2)) with DeltaT of the partial_delay
 * equation.  +inf for a single channel.  Host-only. */
dedisp_status dedisp_get_diagonal_dm(dedisp_plan plan, double* dm);

/* The default factor of every trial of the DM list, written to host array
 * `factors` (ndm int32): 1 up to the diagonal DM, 2 once the DM exceeds it,
 * 4 once it exceeds twice the diagonal, and so on, capped at `max_factor`
 * (a power of two in [1, 64]).  Host-only.
 * Errors: INVALID_ARG, NO_DM_LIST. */
dedisp_status dedisp_default_scrunch_factors(dedisp_plan plan, int max_factor, int32_t* factors);

/* Switch time-scrunching on with one factor per trial (host array of ndm
 * int32 powers of two in [1, 64], copied) or off (NULL, or all factors 1).
 * A trial with factor s is dedispersed from s-sample sums, sample t' of a
 * channel being the sum of input samples s*t' .. s*t'+s-1 (a trailing
 * partial group is dropped), with the delay equation evaluated at the
 * sampling time s*dt.  Row d then holds nsamps/s - (largest delay of the
 * trials sharing its factor) outputs at resolution s*dt.  Setting a new DM
 * list switches scrunching off; the delay table and max_delay queries keep
 * describing the full-resolution list.  Streams and batches reject a plan
 * with scrunching on (UNSUPPORTED).  Set it before dedisp_set_tree (each
 * factor group then runs the tree); while the tree is on any call, and with
 * sub-band mode on a call with factors, is UNSUPPORTED.  Waits for the plan's own enqueued work
 * before it replaces device tables.
 * Errors: INVALID_ARG, NO_DM_LIST, OOM, UNSUPPORTED. */
dedisp_status dedisp_set_scrunching(dedisp_plan plan, const int32_t* factors);

/* Valid outputs of every row for an input of nsamps rows, written to host
 * array `nout` (ndm entries): nsamps - max_delay without scrunching.
 * Host-only.  Errors: INVALID_ARG, NO_DM_LIST, TOO_FEW_SAMPLES. */
dedisp_status dedisp_get_output_lengths(dedisp_plan plan, size_t nsamps, size_t* nout);

/* ------------------------------------------- piecewise linear tree */

/* Section 3: tree dedispersion over sub-bands of nsub channels (a power of
 * two in [8, 128] dividing nchans), combined into the plan's DM trials.
 * Stage 1 applies the tree algorithm's first log2(nsub) steps -- the
 * out-of-place updates with the delay function Theta and the shuffle Phi --
 * to every sub-band, giving its series at the nsub tree DMs
 * (linear trails from 0 to d' samples across the sub-band).  Stage 2 sums,
 * for each trial d, sub-band n's series at tree DM
 * d'_n(d) = round(DM(d) [DeltaT(v_{n+1}) - DeltaT(v_n)]) delayed by
 * dt''_n(d) = round(DM(d) * sum over m < n of [DeltaT(v_{m+1}) - DeltaT(v_m)])
 * (v_n = n*nsub; v_{nchans/nsub} = nchans is the channel just past the band),
 * evaluated in binary64 in that order.  An approximation of the direct
 * transform whose error Appendix A bounds.  Outputs exist for
 * t < nsamps - (nsub - 1) - (largest dt''); dedisp_get_output_lengths gives
 * it.  Trials past the piecewise diagonal (d'_n(d) >= nsub) use further
 * passes of stage 1 over the data with a delay of p samples per channel
 * imposed within each sub-band (Section 3, computing larger DMs): sub-band n
 * of trial d reads pass p = d'_n(d) / nsub at tree DM d'_n(d) mod nsub, and
 * outputs then exist for t < nsamps - (P + 1)(nsub - 1) - (largest dt''),
 * P the largest pass.  Stage 1 runs once per (sub-band, pass) pair in use
 * (at most 65535 pairs, else UNSUPPORTED).  With time-scrunching set first
 * (dedisp_set_scrunching; setting it afterwards is UNSUPPORTED), every scrunch
 * group runs its own tree over its s-sample sums at resolution s*dt, as the
 * paper combines the two for large DMs; its rows' lengths then follow from
 * nsamps / s, and a group whose sub-band sums can exceed 16 bits (largest
 * s-sample sum times nsub above 65535) makes the call UNSUPPORTED.
 * nsub = 0 switches the mode off; a new DM list does too.  Excludes sub-band
 * mode; streams and batches reject such a plan.  Needs 4-byte aligned input rows and a band
 * whose edge past the last channel is above zero frequency.
 * Errors: INVALID_ARG, NO_DM_LIST, UNSUPPORTED. */
dedisp_status dedisp_set_tree(dedisp_plan plan, int nsub);

/* ------------------------------------------------------ output format */

/* Output width (Section 4: the final output is written with a chosen number
 * of bits per sample): nbits = 32 (default), 16 or 8, and every output is
 * min(sum >> shift, 2^nbits - 1) -- exact whenever the shifted sum fits
 * (with 2-bit data a 16-bit output is exact up to 21845 channels).  d_out of
 * every compute call then holds uint8 / uint16 / uint32 elements, and row
 * strides count those elements.  Applies to execute, streams, batches,
 * time-scrunching and sub-band mode alike.  Host-only.
 * Errors: INVALID_ARG (nbits not 8/16/32, shift outside [0, 31]). */
dedisp_status dedisp_set_output_format(dedisp_plan plan, int nbits, int shift);
dedisp_status dedisp_get_output_format(dedisp_plan plan, int* nbits, int* shift);

/* ----------------------------------------------- sub-band dedispersion */

/* Section 4: the channels form nchans/nsub sub-bands of nsub channels and
 * the trials groups of ngroup consecutive list entries, each group's first
 * trial being its nominal DM.  Step 1 dedisperses every sub-band at every
 * nominal DM, with delays relative to the sub-band's first channel; step 2
 * dedisperses, for each trial, the nominal DM's sub-band series with the
 * trial's delay at each sub-band's first channel (the early-edge alignment
 * of Appendix B).  Sample c of trial d is thus taken at delay
 * dt(d, n*nsub) + dt(m, c) - dt(m, n*nsub) (n = c/nsub, m = d/ngroup): an
 * approximation of the direct transform whose error Appendix B bounds, and
 * the direct transform itself when ngroup = 1.  Outputs exist for
 * t < len1 - (largest step-2 delay), len1 = nsamps - (largest step-1
 * delay); dedisp_get_output_lengths gives it.  The sub-band sums are kept
 * on the device in 8 or 16 bits (at most 3*nsub or 255*nsub).
 * nsub: a multiple of 8 dividing nchans (255*nsub <= 32767 for 8-bit
 * data); ngroup >= 1; (0, 0) switches sub-band mode off.  Setting a new DM
 * list switches it off; it excludes time-scrunching (UNSUPPORTED) and
 * streams and batches reject such a plan.  Needs 4-byte aligned input rows.
 * Waits for the plan's own enqueued work before it replaces device tables.
 * Errors: INVALID_ARG, NO_DM_LIST, UNSUPPORTED, OOM. */
dedisp_status dedisp_set_subband(dedisp_plan plan, int nsub, int ngroup);

/* ----------------------------------------------------- kernel selection */

/* Shape of the LDS-tiled kernel: `waves` wavefronts per workgroup share one
 * staged time tile; each wave sums `dms_per_wave` neighbouring trial DMs;
 * each lane owns `words_per_lane` consecutive 32-bit words of the
 * channel-major scratch, i.e. words_per_lane times the samples a word holds
 * (`sample_format`: 0 = 2-bit codes as nibbles, 8 per word; 1 = bytes, 4;
 * 2 = small byte sums, 4; 3 = 16-bit sums, 2; 4 = 2-bit codes as two bit
 * planes, 32 per word of each plane; 5 = the same bit planes with the output
 * cut into 32 time segments, bit i of a word holding segment i, so that a
 * delay moves whole words), so a tile is 64 lanes times that;
 * `chunk_chans` channels are staged in LDS at a time.  kind = 0 is the
 * LDS-tiled kernel, kind = 1 the untiled fallback (no LDS; used
 * automatically when a tile would not fit).  The plan's bit depth and
 * channel count fix the scratch format (2-bit codes are bit planes up to
 * 1365 channels, nibbles beyond); `sample_format` is reported by the getters;
 * dedisp_set_tile_config reads it only on a bit-plane plan, where 5 selects
 * the segmented planes and any other value the plain ones. */
typedef struct {
    int kind;
    int waves;
    int dms_per_wave;
    int words_per_lane;
    int chunk_chans;
    int sample_format;
} dedisp_tile_config;

/* Number of tile shapes compiled into this library, and the i-th one. */
int dedisp_tile_config_count(void);
dedisp_status dedisp_tile_config_get(int index, dedisp_tile_config* cfg);

/* Choose the tile shape used by later compute calls on this plan
 * (must be one of the compiled shapes; chunk_chans a multiple of 4 in
 * [4, 256]).  Host-only.  INVALID_ARG for an unknown shape. */
dedisp_status dedisp_set_tile_config(dedisp_plan plan, const dedisp_tile_config* cfg);
/* (Under time-scrunching the shape also applies to every scrunch group
 * whose scratch format has it; dedisp_tune picks one per group.) */

/* The tile shape the next compute call will use (after falling back if the
 * chosen one does not fit in LDS).  A segmented bit-plane shape (sample
 * format 5) is reported as chosen; a call producing fewer than 8 max_delays
 * of outputs per DM runs the plain bit planes instead (for short inputs the
 * segmented layout's corner turn costs more than its sum saves). */
dedisp_status dedisp_get_tile_config(dedisp_plan plan, dedisp_tile_config* cfg);

/* Autotune: time every compiled shape on the given input/output buffers
 * (the output is overwritten with a valid result), keep the fastest on the
 * plan, and if `cache_path` is not NULL read/update a JSON cache keyed by
 * (nbits, nchans, ndm, max_delay, nsamps bucket).  Synchronises `stream`.
 * In sub-band mode each pass is tuned in turn, and where the sub-band sums
 * fit a byte both widths of the intermediate sums (bytes, 16-bit values)
 * are timed and the faster kept.
 * `best_ms` (nullable) receives the best time of one call. */
dedisp_status dedisp_tune(dedisp_plan plan, const void* d_in, size_t nsamps,
                          uint32_t* d_out, size_t out_row_stride, void* stream,
                          const char* cache_path, float* best_ms);

/* ------------------------------------------------------------- streams */

/* An unbounded input stream: each push appends a chunk of input rows and
 * produces every output that the data seen so far fully covers, so that the
 * concatenated outputs of all pushes equal dedisp_execute on the
 * concatenated input (overlap-save over the time axis).  The stream keeps the
 * last max_delay input rows on the device as its history.
 * The plan must have a DM list and must outlive the stream.
 * Allocates device memory for the history.  Errors: INVALID_ARG,
 * NO_DM_LIST, OOM, HIP. */
dedisp_status dedisp_stream_create(dedisp_plan plan, dedisp_stream* out);
void dedisp_stream_destroy(dedisp_stream s);

/* Push `nsamps` rows at device address d_chunk.  *n_out receives the number
 * of new output samples per DM written to d_out (rows of out_row_stride
 * elements; 0 = n_out): while the stream has seen at most max_delay rows it
 * is 0 and the rows are only kept; after that it is nsamps (the first push
 * past max_delay yields total - max_delay).  d_out may be NULL only when
 * *n_out will be 0.  The caller must not reuse d_chunk before the stream's
 * work on `stream` has finished.  Errors: INVALID_ARG, OOM, HIP. */
dedisp_status dedisp_stream_push(dedisp_stream s, const void* d_chunk, size_t nsamps,
                                 uint32_t* d_out, size_t out_row_stride, size_t* n_out,
                                 void* stream);

/* Several streams' pushes as one launch (the continuous-batching step of a
 * serving loop).  Arrays of length n; streams must be distinct and share
 * nothing but, possibly, their plans.  Same per-stream semantics as
 * dedisp_stream_push. */
dedisp_status dedisp_stream_push_many(dedisp_stream* streams, const void* const* d_chunks,
                                      const size_t* nsamps, uint32_t* const* d_outs,
                                      const size_t* out_row_strides, size_t* n_outs, int n,
                                      void* stream);

/* Size the stream's channel-major scratch for pushes of up to max_chunk rows
 * with the plan's current tile shape (call after tuning the plan).  A push
 * longer than any seen before otherwise grows the scratch, and freeing the
 * old one waits for this stream's queued pushes (and the HIP runtime's free
 * may synchronise the device): in a serving loop that stalls the tick.
 * Synchronous.  Errors: INVALID_ARG, OOM. */
dedisp_status dedisp_stream_reserve(dedisp_stream s, size_t max_chunk);

/* Device memory the stream holds between pushes (the benchmark spec serving form:
 * admission by HBM budget): its two history buffers of max(1, max_delay)
 * packed rows each plus its channel-major scratch as currently sized
 * (dedisp_stream_reserve sizes it for the longest chunk).  The chunk and the
 * outputs of a push are the caller's and are not counted.  Host-only; errors:
 * INVALID_ARG (NULL argument). */
dedisp_status dedisp_stream_get_device_bytes(dedisp_stream s, size_t* bytes);

/* Rows currently held as history, and total rows pushed since creation or
 * the last reset / set_history. */
dedisp_status dedisp_stream_get_state(dedisp_stream s, size_t* history_rows,
                                      uint64_t* total_rows);

/* Checkpoint / restore of the history (synchronous host copies, after this
 * stream's own pushes, on the stream they last ran on; other streams keep
 * running).
 * get: host_buf of at least history_rows * row_bytes bytes; *nsamps receives
 * history_rows.  set: replaces the history with nsamps <= max_delay rows
 * (the stream then behaves as if exactly those rows had been pushed, with
 * total = nsamps ... unless nsamps == max_delay, which marks it as primed). */
dedisp_status dedisp_stream_get_history(dedisp_stream s, void* host_buf, size_t* nsamps);
dedisp_status dedisp_stream_set_history(dedisp_stream s, const void* host_buf, size_t nsamps,
                                        uint64_t total_rows);
dedisp_status dedisp_stream_reset(dedisp_stream s);

/* ------------------------------------------------------------- batches */

/* One beam of a batch: its plan (observing set-up and DM list), resident
 * input and output.  Beams borrow plans and buffers, which must outlive the
 * batch; different beams may differ in nchans, nbits, nsamps and DM list. */
typedef struct {
    dedisp_plan plan;
    const void* d_in;
    size_t      nsamps;
    uint32_t*   d_out;
    size_t      out_row_stride;   /* elements; 0 = nsamps - max_delay */
} dedisp_beam;

/* Build a batch: pick a tile shape per beam (from `tune_cache_path` when it
 * holds the beam's key, else by timing the candidates on the beam's own
 * buffers and recording the result there), upload a device descriptor table
 * and a flat work list, and capture one multi-beam launch (one workgroup per
 * work item of every beam) into a HIP graph.
 * Uses `stream` for tuning and capture and synchronises it.
 * Errors: INVALID_ARG, NO_DM_LIST, TOO_FEW_SAMPLES, OOM, HIP. */
dedisp_status dedisp_batch_create(const dedisp_beam* beams, int nbeams,
                                  const char* tune_cache_path, void* stream,
                                  dedisp_batch* out);

/* Run every beam of the batch: one graph launch on `stream`. */
dedisp_status dedisp_batch_execute(dedisp_batch b, void* stream);

/* Run every beam with the same multi-beam launch but without the graph (for
 * comparison and for callers that re-point buffers between runs). */
dedisp_status dedisp_batch_execute_direct(dedisp_batch b, void* stream);

void dedisp_batch_destroy(dedisp_batch b);

#ifdef __cplusplus
}
#endif

#endif /* DEDISP_H */
