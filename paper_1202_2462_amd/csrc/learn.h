// Gauge-covariant network of the learned setup (learn.hip).
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

constexpr int NET_MAX_LAYERS = 8;
constexpr int NET_MAX_WIDTH = 16;

struct NetShape {
    int nlayers = 0;
    int widths[NET_MAX_LAYERS + 1] = {};
    size_t nweights() const {   // complex weights of all layers
        size_t n = 0;
        for (int l = 0; l < nlayers; l++) n += (size_t)widths[l + 1] * widths[l] * 9;
        return n;
    }
    size_t offset(int l) const {
        size_t n = 0;
        for (int k = 0; k < l; k++) n += (size_t)widths[k + 1] * widths[k] * 9;
        return n;
    }
};

// y = layer(W) x for ns samples: x [ns][cin][12][V], y [ns][cout][12][V]
// (FP32), W FP32 complex [cout][cin][9]
int launch_net_layer(Ctx *c, int cin, int cout, const float2 *W, int ns, const void *x, void *y);
// Wa[c'][c][h] = conj(W[c][c'][hbar]) (the adjoint layer's weights), FP32 from FP64
int launch_net_adjoint_weights(Ctx *c, int cin, int cout, const double2 *W, float2 *Wa);
// FP32 copy of FP64 weights
int launch_net_weights32(Ctx *c, size_t n, const double2 *W, float2 *W32);
// out (FP64) = T_h in (FP32) for nf fields
int launch_net_hop(Ctx *c, int h, int nf, const void *in32, void *out64);
// grad[(c * cin + c') * 9 + h] += G[c' * cout + c] (a Gram block <T_h x_c', g_c>)
int launch_net_grad_add(Ctx *c, int cin, int cout, int h, const double2 *G, double2 *grad);
// Adam step on n complex weights (re and im parts separately)
int launch_net_adam(Ctx *c, size_t n, double2 *W, const double2 *grad, double2 *m, double2 *v, int step, double lr,
                    double beta1, double beta2, double eps);

struct Arena;
// bytes of workspace of net_forward / net_grad for ns samples
size_t net_forward_bytes(const Ctx *c, const NetShape &sh, int ns);
size_t net_grad_bytes(const Ctx *c, const NetShape &sh, int ns);
// out = net(in) for ns samples of one channel (FP32 fields); W64: FP64 weights
int net_forward(Ctx *c, const NetShape &sh, const double2 *W64, int ns, const void *in32, void *out32, Arena &A);
// mean over the ns samples of L = ||(1 - P P^H) f||^2 / ||f||^2 (f = net(in),
// P the context's interpolation) and its gradient dL/dconj(W) (FP64, written)
int net_grad(Ctx *c, const NetShape &sh, const double2 *W64, int ns, const void *in32, double *loss, double2 *grad,
             Arena &A);
bool net_shape_valid(const NetShape &sh);
int check_net_shape(Ctx *c, const NetShape &sh);

}  // namespace mgdd
