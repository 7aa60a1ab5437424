// Host-driven solvers and setup (see solver.hip).
#pragma once

#include <complex>

#include "mgdd_internal.h"
#include "schwarz.h"
#include "transfer.h"

namespace mgdd {

// Bump allocator over the context workspace. take() returns nullptr (and
// records the size needed) when the workspace is too small.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, off = 0, need = 0;
    void *take(size_t bytes);
};
int arena_open(Ctx *c, size_t bytes, Arena &a);
std::complex<double> *host_buf(Ctx *c, size_t n);

// Parameters of the multilevel preconditioner. Two levels: nu Schwarz
// sweeps (mr MR steps per block) after a coarse correction by cit GMRES steps
// on D_c. Three levels: the coarse equation is solved instead by k2 steps of
// flexible GMRES on D_c, preconditioned by nu2 level-2 Schwarz sweeps (mr2
// MR steps per block) after a correction by cit GMRES steps on D_cc.
struct MgOpts {
    int nu = 1, mr = 4, cit = 12;
    int levels = 2;
    int k2 = 0, nu2 = 0, mr2 = 0;
    int gmres_blocks = 0;   // smoother block solves: 0 MR(mr), 1 GMRES(mr)
    int additive = 0;       // smoother: 0 red-black multiplicative, 1 additive
};
MgOpts mg_opts(const mgdd_solve_params *sp);

// nb: number of right-hand sides handled together (stacked fields)
size_t coarse_gmres_bytes(const Ctx *c, int p, int m, int nb);
size_t precond_bytes(const Ctx *c, int p, const MgOpts &o, int nb);
size_t solve_bytes(const Ctx *c, const mgdd_solve_params *sp, int nb);
int coarse_gmres(Ctx *c, int p, int m, int nb, const void *b, void *x, Arena &A, int *status = nullptr);
size_t stencil_gmres_bytes(const StencilOp &op, int p, int m, int nb);
int stencil_gmres(Ctx *c, const StencilOp &op, int p, int m, int nb, const void *b, void *x, Arena &A,
                  int *status = nullptr);
int mg_precond(Ctx *c, int p, int nb, const void *r64, void *z, const MgOpts &o, Arena &A);
int solve_prec(const mgdd_solve_params *sp);
int solve_batch(Ctx *c, const mgdd_solve_params *sp, int nb, const void *b, void *z, mgdd_solve_stats *st);
int bootstrap(Ctx *c, const mgdd_setup_params *sp, const void *rv64, const void *start64);
int level2_bootstrap(Ctx *c, const mgdd_level2_params *lp, const void *random2);
struct NetShape;
int setup_learned(Ctx *c, const NetShape &sh, const double2 *W64, const mgdd_setup_params *sp, const void *rv64,
                  const void *start64);

}  // namespace mgdd
