// Aggregation interpolation, restriction, prolongation and the coarse
// operator (see transfer.hip).
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

struct AggGeom {
    int a[4];
};

// tables and buffers of the coarse level for aggregates agg and N test vectors
int transfer_setup(Ctx *c, const int *agg, int N);
// P from N FP64 fine fields (device layout); FP32 copy made too. MGDD_ERANK if rank deficient.
int launch_build_P(Ctx *c, const void *tv64);
int launch_restrict(Ctx *c, int prec, int nrhs, const void *fine, void *coarse);
int launch_restrict_ex(Ctx *c, int prec, int nrhs, const void *P, const void *fine, void *out, size_t ostride,
                       size_t rstride);
int launch_prolong(Ctx *c, int prec, int nrhs, const void *coarse, void *fine);
int launch_coarse_build(Ctx *c);
int launch_coarse_apply(Ctx *c, int prec, int nrhs, const void *in, void *out);

// Fused Arnoldi process on D_c for the coarse GMRES (arnoldi.hip); m <= 15.
constexpr int ARNOLDI_FUSED_MAX_STEPS = 15;
size_t coarse_arnoldi_scratch(const Ctx *c, int m, int nb);
// w <- w - V V^H w twice (nb segments of n), three passes; k <= 16 vectors.
constexpr int FUSED_CGS2_MAX = 16;
int fused_cgs2(Ctx *c, int p, size_t n, int nb, void *const *V, int k, void *w, double2 *h1, double2 *h2,
               double2 *nrm);
int launch_coarse_arnoldi(Ctx *c, int p, int m, int nb, const void *b, void *const *V, void *work0, void *work1,
                          void *scratch, double2 *H1, double2 *H2, double2 *NR);

}  // namespace mgdd
