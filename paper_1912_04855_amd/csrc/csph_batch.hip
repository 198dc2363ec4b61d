// csph_batch.hip -- batches of simulations (to be filled in).
#include <hip/hip_runtime.h>

#include "../../include/csph.h"

extern "C" {

csph_status csph_batch_create(csph_dtype, void*, size_t, csph_batch** out) {
  if (out) *out = nullptr;
  return CSPH_ERR_ARG;
}
csph_status csph_batch_add(csph_batch*, csph_sim*, int64_t, double, int32_t*) { return CSPH_ERR_ARG; }
csph_status csph_batch_advance(csph_batch*, int32_t, int32_t*) { return CSPH_ERR_ARG; }
csph_status csph_batch_poll(csph_batch*, int32_t*, int32_t, int32_t*) { return CSPH_ERR_ARG; }
csph_status csph_batch_remove(csph_batch*, int32_t) { return CSPH_ERR_ARG; }
csph_status csph_batch_destroy(csph_batch*) { return CSPH_OK; }

}
