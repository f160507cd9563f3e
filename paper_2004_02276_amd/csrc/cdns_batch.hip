// cdns_batch.hip -- batched runner over many resident instances.
#include <hip/hip_runtime.h>

#include "../../include/cdns.h"
#include "cdns_internal.h"

extern "C" {

size_t cdns_batch_workspace_bytes(int32_t max_slots) {
  return max_slots > 0 ? (size_t)max_slots * 4096 : 0;
}

cdns_status cdns_batch_create(int32_t, void*, size_t, void*, cdns_batch** out) {
  if (out) *out = nullptr;
  return CDNS_EUNSUP;
}
cdns_status cdns_batch_attach(cdns_batch*, cdns_ctx*, int32_t*) { return CDNS_EUNSUP; }
cdns_status cdns_batch_detach(cdns_batch*, int32_t) { return CDNS_EUNSUP; }
cdns_status cdns_batch_set_step(cdns_batch*, int32_t, double, double) { return CDNS_EUNSUP; }
cdns_status cdns_batch_step(cdns_batch*, int32_t) { return CDNS_EUNSUP; }
cdns_status cdns_batch_destroy(cdns_batch*) { return CDNS_EUNSUP; }

}  // extern "C"
