// Serving loop (continuous batching): placeholder entry points until the
// scheduler lands; every call reports RGF_EINVAL.
#include "engine.h"

extern "C" {
int transport_open(const rgf_server_opts*, void** server) {
  if (server) *server = nullptr;
  rgf::set_error("serving is not available in this build");
  return RGF_EINVAL;
}
int transport_submit(void*, const rgf_device*, uint64_t, uint64_t, const double*, int64_t, double, int,
                     uint64_t*) {
  rgf::set_error("serving is not available in this build");
  return RGF_EINVAL;
}
int transport_poll(void*, uint64_t, double*, int32_t*, double*) {
  rgf::set_error("serving is not available in this build");
  return RGF_EINVAL;
}
int transport_close(void*) { return RGF_OK; }
int transport_stats(void*, rgf_server_stats*) {
  rgf::set_error("serving is not available in this build");
  return RGF_EINVAL;
}
}
