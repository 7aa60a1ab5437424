// Third level of the hierarchy (see level2.hip and sap2.hip).
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

// tables and buffers for level-2 aggregates agg2 (in coarse sites) and N2 test vectors
int level2_setup(Ctx *c, const int *agg2, int N2);
void level2_free(Ctx *c);
// P2 from N2 coarse FP64 vectors (copied; FP32 copy made), MGDD_ERANK if rank deficient
int launch_build_P2(Ctx *c, const void *tv2);
// D_cc = P2^H D_c P2 (FP64, then the FP32 copy); marks the level ready
int launch_dcc_build(Ctx *c);
int launch_restrict2(Ctx *c, int prec, int nrhs, const void *in, void *out);
int launch_prolong2(Ctx *c, int prec, int nrhs, const void *in, void *out);

}  // namespace mgdd
