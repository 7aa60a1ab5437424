// Level-1 device kernels on flat complex arrays (see blas.hip).
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

constexpr int MAXV = 16;  // vectors per kernel pass
struct PtrList {
    const void *p[MAXV];
};

// out[i] = <x_i, w> = sum conj(x_i) w for i < nvec (device double2 array).
int blas_multidot(Ctx *c, int px, int pw, size_t n, const void *const *xs, int nvec, const void *w, double2 *out);
// y = beta y + alpha sum_i coef[i] x_i   (coef: device double2 array)
int blas_lincomb(Ctx *c, int px, int py, size_t n, const void *const *xs, int nvec, const double2 *coef, double alpha,
                 double beta, void *y);
// y = (coef ? coef[0] * alpha : alpha) x   (x and y may alias)
int blas_scale(Ctx *c, int px, int py, size_t n, const void *x, const double2 *coef, double2 alpha, void *y);
// y = x / sqrt(re nrm2[0]) (y = 0 when that is 0); x and y may alias
int blas_normalize(Ctx *c, int px, int py, size_t n, const void *x, const double2 *nrm2, void *y);
// coef[0] = 1/sqrt(re v[0])
int blas_rsqrt(Ctx *c, const double2 *v, double2 *coef);

}  // namespace mgdd
