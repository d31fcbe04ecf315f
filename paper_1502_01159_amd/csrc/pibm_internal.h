// pibm_internal.h -- calls between the library's translation units (not part
// of the C ABI).
#ifndef PIBM_INTERNAL_H
#define PIBM_INTERNAL_H

#include <hip/hip_runtime.h>

#include "../../include/pibm.h"

// The network's forward pass on a given stream (the simulation's), for the
// one-point closure step.
int pibm_mlp_forward_on(pibm_mlp *m, const void *dev_x, float *dev_y, int n, hipStream_t stream);

#endif
