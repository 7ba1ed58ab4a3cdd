// Serving loop (continuous batching) -- placeholder entry points until the
// scheduler lands; every call reports CSPD_E_UNSUPPORTED.
#include "cspd_internal.h"

using namespace cspd;

extern "C" {

cspd_status cspd_serve_create(int32_t, int64_t, int32_t, cspd_server_t *out)
{
    if (out) *out = nullptr;
    return set_error(CSPD_E_UNSUPPORTED, "serving is not built yet");
}

cspd_status cspd_serve_submit(cspd_server_t, const cspd_job *, uint64_t *)
{
    return set_error(CSPD_E_UNSUPPORTED, "serving is not built yet");
}

cspd_status cspd_serve_poll(cspd_server_t, uint64_t, int64_t, cspd_job_stats *)
{
    return set_error(CSPD_E_UNSUPPORTED, "serving is not built yet");
}

void cspd_serve_destroy(cspd_server_t) {}

}  // extern "C"
