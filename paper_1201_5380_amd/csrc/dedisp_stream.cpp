// Streams and batches: filled in below.
#include "dedisp.h"
extern "C" {
dedisp_status dedisp_stream_create(dedisp_plan, dedisp_stream* out) { if (out) *out = nullptr; return DEDISP_ERR_UNSUPPORTED; }
void dedisp_stream_destroy(dedisp_stream) {}
dedisp_status dedisp_stream_push(dedisp_stream, const void*, size_t, uint32_t*, size_t, size_t*, void*) { return DEDISP_ERR_UNSUPPORTED; }
dedisp_status dedisp_stream_push_many(dedisp_stream*, const void* const*, const size_t*, uint32_t* const*, const size_t*, size_t*, int, void*) { return DEDISP_ERR_UNSUPPORTED; }
dedisp_status dedisp_stream_get_state(dedisp_stream, size_t*, uint64_t*) { return DEDISP_ERR_UNSUPPORTED; }
dedisp_status dedisp_stream_get_history(dedisp_stream, void*, size_t*) { return DEDISP_ERR_UNSUPPORTED; }
dedisp_status dedisp_stream_set_history(dedisp_stream, const void*, size_t, uint64_t) { return DEDISP_ERR_UNSUPPORTED; }
dedisp_status dedisp_stream_reset(dedisp_stream) { return DEDISP_ERR_UNSUPPORTED; }
dedisp_status dedisp_batch_create(const dedisp_beam*, int, const char*, void*, dedisp_batch* out) { if (out) *out = nullptr; return DEDISP_ERR_UNSUPPORTED; }
dedisp_status dedisp_batch_execute(dedisp_batch, void*) { return DEDISP_ERR_UNSUPPORTED; }
dedisp_status dedisp_batch_execute_direct(dedisp_batch, void*) { return DEDISP_ERR_UNSUPPORTED; }
void dedisp_batch_destroy(dedisp_batch) {}
}
