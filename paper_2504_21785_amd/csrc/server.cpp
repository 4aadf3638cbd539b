// Serving entry points (scheduler not built yet).
#include "common.h"

extern "C" {
int fggc_server_create(fggc_ctx *, int, fggc_server **out) {
  if (out) *out = nullptr;
  fggc::set_last_error("fggc_server_create: not available");
  return FGGC_EUNSUPPORTED;
}
int fggc_server_submit(fggc_server *, const fggc_packets *, double, const fggc_grid *,
                       const fggc_strategy *, double, int, void *, fggc_ticket *) {
  return FGGC_EUNSUPPORTED;
}
int fggc_server_wait(fggc_server *, fggc_ticket, double) { return FGGC_EUNSUPPORTED; }
int fggc_server_stats(fggc_server *, double *, double *, double *, int64_t *) {
  return FGGC_EUNSUPPORTED;
}
void fggc_server_destroy(fggc_server *) {}
}
