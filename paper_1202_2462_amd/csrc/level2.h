// Third level of the hierarchy: the two-level construction of Section 3
// applied to the coarse operator D_c.
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

// tables and buffers for level-2 aggregates agg2 (in coarse sites) and N2 test vectors
int level2_setup(Ctx *c, const int *agg2, int N2);
// releases the third level; keep_blocks keeps the level-2 Schwarz block tables
void level2_free(Ctx *c, bool keep_blocks = false);
// P2 from N2 coarse FP64 vectors (copied; FP32 copy made), MGDD_ERANK if rank deficient
int launch_build_P2(Ctx *c, const void *tv2);
// D_cc = P2^H D_c P2 (FP64, then the FP32 copy); marks the level ready
int launch_dcc_build(Ctx *c);
// blocks of the level-2 Schwarz smoother (block2 in coarse sites)
int level2_sap_setup(Ctx *c, const int *block2);
// nsweeps red-black Schwarz sweeps on D_c z = b (z in/out), MR(mr) block solves
int launch_sap2(Ctx *c, int prec, int nrhs, int nsweeps, int mr, const void *b, void *z);
int launch_restrict2(Ctx *c, int prec, int nrhs, const void *in, void *out);
int launch_prolong2(Ctx *c, int prec, int nrhs, const void *in, void *out);

}  // namespace mgdd
