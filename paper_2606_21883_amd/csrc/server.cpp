// Continuous-batching server: placeholder until the scheduler lands.
#include "host_internal.h"
#include "mpwos.h"

using namespace mpwos;

extern "C" {
mpwos_status mpwos_server_create(size_t, int64_t, mpwos_server**) { return fail(MPWOS_EINVAL, "server not built"); }
mpwos_status mpwos_submit(mpwos_server*, const mpwos_request*, uint64_t*) { return fail(MPWOS_EINVAL, "server not built"); }
mpwos_status mpwos_poll(mpwos_server*, uint64_t, int32_t*, int32_t*) { return fail(MPWOS_EINVAL, "server not built"); }
mpwos_status mpwos_wait(mpwos_server*, uint64_t, int64_t, int32_t*) { return fail(MPWOS_EINVAL, "server not built"); }
mpwos_status mpwos_server_stats_get(mpwos_server*, mpwos_server_stats*) { return fail(MPWOS_EINVAL, "server not built"); }
mpwos_status mpwos_server_destroy(mpwos_server*) { return fail(MPWOS_EINVAL, "server not built"); }
}
