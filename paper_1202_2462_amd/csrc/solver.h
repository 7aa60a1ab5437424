// Host-driven solvers and setup (see solver.hip).
#pragma once

#include <complex>

#include "mgdd_internal.h"
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

// nb: number of right-hand sides handled together (stacked fields)
size_t coarse_gmres_bytes(const Ctx *c, int p, int m, int nb);
size_t precond_bytes(const Ctx *c, int p, int cit, int nb);
size_t solve_bytes(const Ctx *c, const mgdd_solve_params *sp, int nb);
int coarse_gmres(Ctx *c, int p, int m, int nb, const void *b, void *x, Arena &A);
size_t stencil_gmres_bytes(const StencilOp &op, int p, int m, int nb);
int stencil_gmres(Ctx *c, const StencilOp &op, int p, int m, int nb, const void *b, void *x, Arena &A);
int mg_precond(Ctx *c, int p, int nb, const void *r64, void *z, int nu, int mr, int cit, Arena &A);
int solve_batch(Ctx *c, const mgdd_solve_params *sp, int nb, const void *b, void *z, mgdd_solve_stats *st);
int bootstrap(Ctx *c, const mgdd_setup_params *sp, const void *rv64, const void *start64);

}  // namespace mgdd
