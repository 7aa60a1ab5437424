// Aggregation interpolation, restriction, prolongation and the coarse
// operator (see transfer.hip).
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

struct AggGeom {
    int a[4];
};

// A 9-point stencil operator with 2N x 2N complex blocks per site (D_c on the
// coarse lattice, D_cc on the level-3 lattice): sites, N, neighbour table
// [V][9] (self first), blocks [V][9][col][row] in FP64 and FP32.
struct StencilOp {
    int V = 0, N = 0;
    const int *nbr = nullptr;
    const void *D64 = nullptr, *D32 = nullptr;
    const void *H32 = nullptr;   // [V][5][col][row] FP32 self and forward blocks, or null
    const int *order = nullptr;  // [V] visiting order of the sites (null: index order)
};
inline StencilOp level1_op(const Ctx *c) {
    StencilOp o;
    o.V = c->c.Vc;
    o.N = c->c.N;
    o.nbr = c->c.cnbr;
    o.D64 = c->c.Dc64;
    o.D32 = c->c.Dc32;
    o.H32 = c->c.Dh32;
    o.order = c->c.corder;
    return o;
}
inline StencilOp level2_op(const Ctx *c) {
    StencilOp o;
    o.V = c->c2.Vcc;
    o.N = c->c2.N2;
    o.nbr = c->c2.cnbr2;
    o.D64 = c->c2.Dcc64;
    o.D32 = c->c2.Dcc32;
    return o;
}
int launch_stencil_apply(Ctx *c, const StencilOp &op, int prec, int nrhs, const void *in, void *out);

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
size_t coarse_arnoldi_scratch(const StencilOp &op, int m, int nb);
// w <- w - V V^H w twice (nb segments of n), three passes; k <= 64 vectors.
constexpr int FUSED_CGS2_MAX = 64;
int fused_cgs2(Ctx *c, int p, size_t n, int nb, void *const *V, int k, void *w, double2 *h1, double2 *h2,
               double2 *nrm);
int launch_coarse_arnoldi(Ctx *c, const StencilOp &op, int p, int m, int nb, const void *b, void *const *V,
                          void *work0, void *work1, void *scratch, double2 *H1, double2 *H2, double2 *NR);
// Least squares of a GMRES cycle on the device (arnoldi.hip): coef[i][s] = y_i
// of min ||beta e_1 - H y|| from the Gram-Schmidt outputs h1, h2, nr of m
// steps (the layout of launch_coarse_arnoldi); *status (may be null) set to
// 1 on a non-finite result. m <= LSQ_MAX_STEPS.
constexpr int LSQ_MAX_STEPS = 32;
int launch_hessenberg_lsq(Ctx *c, int m, int nb, const double2 *h1, const double2 *h2, const double2 *nr, double2 *coef,
                          int *status);

}  // namespace mgdd
