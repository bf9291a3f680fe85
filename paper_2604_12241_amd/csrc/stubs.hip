// Entry points whose subsystems are not built yet: they fail cleanly.
#include "api_internal.h"

static amlm_status not_built(const char *what) {
  set_error(std::string(what) + " is not available in this build");
  return AMLM_E_INVALID;
}

extern "C" amlm_status amlm_server_create(amlm_graph *, const amlm_params *, uint64_t, uint32_t, amlm_server **) {
  return not_built("amlm_server_create");
}
extern "C" amlm_status amlm_server_submit(amlm_server *, const uint32_t *, const uint32_t *, const int64_t *,
                                          uint64_t, int, uint64_t *) {
  return not_built("amlm_server_submit");
}
extern "C" amlm_status amlm_server_wait(amlm_server *, uint64_t, uint32_t *, uint64_t *, uint64_t *, uint32_t *,
                                        uint32_t *, uint64_t) {
  return not_built("amlm_server_wait");
}
extern "C" amlm_status amlm_server_ticket_times(amlm_server *, uint64_t, double *, double *, double *) {
  return not_built("amlm_server_ticket_times");
}
extern "C" void amlm_server_destroy(amlm_server *) {}
