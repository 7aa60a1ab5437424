// Level-1 device kernels on flat complex arrays (see blas.hip).
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

constexpr int MAXV = 16;  // vectors per kernel pass
constexpr int WIDE = 2 * MAXV;  // vectors per launch of the outer Gram-Schmidt kernels
struct PtrList {
    const void *p[MAXV];
};

// Every array holds nseg segments of n complex numbers (segment s at offset
// s * n); the operation is applied to each segment independently.
//
// out[i * nseg + s] = <x_i, w>_s = sum conj(x_i) w over segment s, i < nvec
int blas_multidot(Ctx *c, int px, int pw, size_t n, const void *const *xs, int nvec, const void *w, double2 *out,
                  int nseg = 1);
// y_s = beta y_s + alpha sum_i coef[i * nseg + s] x_i,s   (coef on the device)
int blas_lincomb(Ctx *c, int px, int py, size_t n, const void *const *xs, int nvec, const double2 *coef, double alpha,
                 double beta, void *y, int nseg = 1);
// y_s <- y_s - sum_i coef[i * nseg + s] x_i,s (same precision p for all), then
// out[i * nseg + s] = <x_i, y>_s, or out[s] = ||y_s||^2 when norm_only;
// nvec <= MAXV. The sums are deterministic.
int blas_update_dot(Ctx *c, int p, size_t n, const void *const *xs, int nvec, const double2 *coef, void *y,
                    double2 *out, int norm_only, int nseg = 1);
// Outer Gram-Schmidt step with a lagged second pass (FP64), in two passes over
// the basis instead of three:
// pass A, in one pass over x_0 ... x_{nvec-1}:
//   out_w[i * nseg + s] = <x_i, w>_s and out_v[i * nseg + s] = <x_i, v>_s;
int blas_dots2(Ctx *c, size_t n, const void *const *xs, int nvec, const void *w, const void *v, double2 *out_w,
               double2 *out_v, int nseg = 1);
// pass B, in one pass over x_0 ... x_{nvec-1} (nvec >= 0; v and w are not
// among them), coefficients of segment s at coef[q * nseg + s] (q = 0: a,
// 1: c, 2 + i: -s_i, 2 + nvec + i: -t_i):
//   v <- a (v - sum_i s_i x_i),   w <- w - sum_i t_i x_i + c v   (new v),
// nrm[s] = ||w_s||^2 after.
int blas_dcgs_update(Ctx *c, size_t n, const void *const *xs, int nvec, const double2 *coef, void *v, void *w,
                     double2 *nrm, int nseg = 1);
// y_s = (coef ? coef[s] * alpha : alpha) x_s   (x and y may alias)
int blas_scale(Ctx *c, int px, int py, size_t n, const void *x, const double2 *coef, double2 alpha, void *y,
               int nseg = 1);
// y_s = x_s / sqrt(re nrm2[s]) (y_s = 0 when that is 0); x and y may alias
int blas_normalize(Ctx *c, int px, int py, size_t n, const void *x, const double2 *nrm2, void *y, int nseg = 1);
// FP64 vector sets (at most 64 each, length n): out[i * ny + j] = <x_i, y_j>
int blas_gram(Ctx *c, size_t n, const void *const *xs, int nx, const void *const *ys, int ny, double2 *out);
// FP64: y_k = sum_i M[i * ny + k] x_i for k < ny (M on the device); any y_k may be one of the x_i
// upper: M is upper triangular (M[i * ny + k] = 0 for i > k), which lets some
// of the kernels skip those terms
int blas_transform(Ctx *c, size_t n, const void *const *xs, int nx, const double2 *M, int ny, void *const *ys,
                   int upper = 0);
// y = gamma_5 x for nrhs fine fields of V sites (x and y may alias)
int blas_gamma5(Ctx *c, int p, size_t V, int nrhs, const void *x, void *y);
// coef[0] = 1/sqrt(re v[0])
int blas_rsqrt(Ctx *c, const double2 *v, double2 *coef);

}  // namespace mgdd
