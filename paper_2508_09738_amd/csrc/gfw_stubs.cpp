// Temporary entry points for the batched solver and the server (replaced by their
// implementations in gfw_batch.hip / gfw_server.cpp).
#include "../../include/gfw.h"

namespace gfw {
void set_error(const char *fmt, ...);
}

extern "C" {
gfw_status_t gfw_server_create(gfw_context_t, size_t, int32_t, gfw_server_t *)
{
    gfw::set_error("server not available in this build");
    return GFW_E_UNSUPPORTED;
}
gfw_status_t gfw_server_submit(gfw_server_t, const gfw_problem_t *, const gfw_params_t *, uint64_t *)
{
    return GFW_E_UNSUPPORTED;
}
gfw_status_t gfw_server_poll(gfw_server_t, uint64_t, int, void *, int32_t *, gfw_stats_t *)
{
    return GFW_E_UNSUPPORTED;
}
gfw_status_t gfw_server_destroy(gfw_server_t) { return GFW_E_UNSUPPORTED; }
}
