// Even-odd Schur complement kernels of the FP64 GCR comparator (see eo.hip).
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

// out = MOUT(alpha * MAUX(aux) + beta * H in) on the sites of parity p, half
// fields; maux: 0 = identity, 1 = A; mout: 0 = identity, 1 = A^{-1}.
int launch_eo(Ctx *c, int p, int maux, int mout, const void *in, const void *aux, double alpha, double beta, void *out);
int launch_eo_split(Ctx *c, const void *full, void *even, void *odd);
int launch_eo_merge(Ctx *c, const void *even, const void *odd, void *full);

}  // namespace mgdd
