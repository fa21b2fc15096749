// Continuous-batching server (see include/cbic.h).
#include "runtime.hpp"

using namespace cbic;

extern "C" {

cbic_status cbic_server_opts_default(cbic_server_opts* o) {
  if (!o) { set_error("opts is NULL"); return CBIC_E_INVALID; }
  o->struct_size = sizeof(cbic_server_opts);
  o->mem_cap_bytes = size_t(32) << 30;
  o->slots_per_class = 4096;
  o->t_max = 200;
  o->iters_per_launch = 4;
  return CBIC_OK;
}

cbic_status cbic_server_create(cbic_context*, const cbic_server_opts*, cbic_server** out) {
  if (out) *out = nullptr;
  set_error("server not available");
  return CBIC_E_UNSUPPORTED;
}
cbic_status cbic_server_submit(cbic_server*, const cbic_system*, int32_t, const double*, const double*,
                               const cbic_solve_opts*, uint64_t*) {
  set_error("server not available");
  return CBIC_E_UNSUPPORTED;
}
cbic_status cbic_server_poll(cbic_server*, uint64_t, cbic_result*) {
  set_error("server not available");
  return CBIC_E_UNSUPPORTED;
}
double cbic_server_clock(const cbic_server*) { return 0.0; }
cbic_status cbic_server_drain(cbic_server*) {
  set_error("server not available");
  return CBIC_E_UNSUPPORTED;
}
cbic_status cbic_server_destroy(cbic_server*) {
  set_error("server not available");
  return CBIC_E_UNSUPPORTED;
}

}  // extern "C"
