// Continuous-batching server (placeholder until the serving loop lands).
#include "nuri_internal.h"

extern "C" {
int nuri_server_create(nuri_graph *, uint64_t, uint32_t, nuri_server **) {
  nuri::set_error("the server is not available in this build");
  return NURI_EINVAL;
}
int nuri_server_submit(nuri_server *, const nuri_query *, uint64_t *) {
  nuri::set_error("the server is not available in this build");
  return NURI_EINVAL;
}
int nuri_server_poll(nuri_server *, uint64_t, nuri_result **) {
  nuri::set_error("the server is not available in this build");
  return NURI_EINVAL;
}
void nuri_server_destroy(nuri_server *) {}
}
