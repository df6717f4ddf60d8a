// Request server with continuous batching (filled in below the ABI stubs).
#include "api_internal.h"

using namespace citron;

struct citron_server {
    int dummy;
};

extern "C" {

citron_server* citron_server_create(int64_t, int32_t, const citron_tuning*)
{
    fail(CITRON_EINVAL, "server not available yet");
    return nullptr;
}
citron_status citron_server_add_graph(citron_server*, citron_graph*, int32_t*)
{
    return fail(CITRON_EINVAL, "server not available yet");
}
citron_status citron_server_submit(citron_server*, int32_t, int32_t, uint64_t)
{
    return fail(CITRON_EINVAL, "server not available yet");
}
int32_t citron_server_poll(citron_server*, citron_result*, int32_t) { return 0; }
int32_t citron_server_pending(citron_server*) { return 0; }
void citron_server_destroy(citron_server*) {}

}  // extern "C"
