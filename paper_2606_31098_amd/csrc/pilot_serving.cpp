// pilot_serving.cpp -- continuous-batching entry points (placeholder until
// the slot runtime lands).
#include <hip/hip_runtime.h>

#include "../../include/pilot.h"

extern "C" {

int pilot_admit_cost(pilot_ctx *, const pilot_frame *, size_t *) { return PILOT_EUNSUPPORTED; }
int pilot_admit(pilot_ctx *, const pilot_frame *, const pilot_result *, int *) { return PILOT_EUNSUPPORTED; }
int pilot_step(pilot_ctx *) { return PILOT_EUNSUPPORTED; }
int pilot_poll(pilot_ctx *, int) { return PILOT_EUNSUPPORTED; }
int pilot_serving_state(pilot_ctx *, int *, size_t *) { return PILOT_EUNSUPPORTED; }

}  // extern "C"
