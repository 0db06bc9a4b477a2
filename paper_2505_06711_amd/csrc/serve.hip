// Serving engine: placeholder entry points until the continuous-batching engine lands.
#include "runtime.hpp"

extern "C" {
reann_status reann_server_create(const reann_model *, const reann_server_opts *, reann_server **) { return REANN_E_UNSUPPORTED; }
reann_status reann_server_set_masses(reann_server *, const double *) { return REANN_E_UNSUPPORTED; }
reann_status reann_system_add(reann_server *, const int32_t *, int64_t, const double *, const int32_t *, const double *,
                              const double *, uint64_t *) { return REANN_E_UNSUPPORTED; }
reann_status reann_submit(reann_server *, const reann_request *, uint64_t *) { return REANN_E_UNSUPPORTED; }
reann_status reann_poll(reann_server *, uint64_t, reann_result *) { return REANN_E_UNSUPPORTED; }
reann_status reann_server_stats(reann_server *, int64_t *) { return REANN_E_UNSUPPORTED; }
void reann_server_destroy(reann_server *) {}
}
