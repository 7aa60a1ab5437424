// Gauge-covariant network of the learned setup: kernels for inference and
// training. A layer maps cin spinor channels to cout channels,
//     y[c] = sum_{c', h} W[c, c', h] T_h x[c'],
// with T_0 = 1 and T_h the colour hops of the Wilson stencil (forward:
// U_mu(x) x(x + mu); backward: U_mu(x - mu)^H x(x - mu); the antiperiodic
// sign is folded into the links), applied to every spin. One thread per
// (site, spin): for each input channel and hop it forms the three colour
// components once and adds them, weighted, to all output channels held in
// registers; the weights are the same for the whole grid (scalar loads).
#include <cmath>
#include <vector>

#include "blas.h"
#include "learn.h"
#include "solver.h"
#include "stencil.h"
#include "transfer.h"

namespace mgdd {

namespace {

constexpr int TPB = 256;   // 64 sites x 4 spins

// S samples per thread (blockIdx.y covers samples S at a time): each link
// leaves memory once for the S samples of a site
template <int CIN, int COUT, int S>
__global__ __launch_bounds__(TPB) void net_layer_kernel(Geom g, const float2 *__restrict__ Up,
                                                        const float2 *__restrict__ W, const float2 *__restrict__ x,
                                                        float2 *__restrict__ y, int ns) {
    const int t = blockIdx.x * TPB + threadIdx.x;
    const int i = t >> 2, s = t & 3;
    if (i >= g.V) return;
    const int d = site_in_lex_block_order(g, i);
    int nbr[8];
    site_neighbours(g, d, nbr);
    const size_t V = g.V;
    const int smp0 = blockIdx.y * S;
    LinkViews<float> U(Up, V);
    float2 acc[S][COUT][3];
#pragma unroll
    for (int q = 0; q < S; q++)
#pragma unroll
        for (int c = 0; c < COUT; c++)
#pragma unroll
            for (int a = 0; a < 3; a++) acc[q][c][a] = make_float2(0.f, 0.f);
    // hop outermost: the link of a hop is loaded once and applied to every
    // input channel of every sample
#pragma unroll
    for (int h = 0; h < 9; h++) {
        const int mu = h > 0 ? (h - 1) >> 1 : 0;
        const bool back = h > 0 && ((h - 1) & 1);
        const int dn = h > 0 ? nbr[h - 1] : d;
        float2 u[9];
        if (h > 0) {
            const FieldView<float> &uf = mu == 0 ? U.u0 : mu == 1 ? U.u1 : mu == 2 ? U.u2 : U.u3;
#pragma unroll
            for (int k = 0; k < 9; k++) u[k] = uf.ld(k, back ? dn : d);
        }
#pragma unroll 1
        for (int cp = 0; cp < CIN; cp++) {
#pragma unroll
            for (int q = 0; q < S; q++) {
                if (S > 1 && smp0 + q >= ns) break;   // the same for the whole workgroup
                const FieldView<float> xf(x + ((size_t)(smp0 + q) * CIN + cp) * 12 * V, V, 12);
                float2 v[3], w[3];
#pragma unroll
                for (int a = 0; a < 3; a++) v[a] = xf.ld_lane(a, dn, 3u * s * xf.cs);
                if (h == 0) {
#pragma unroll
                    for (int a = 0; a < 3; a++) w[a] = v[a];
                } else if (back) {
                    su3_mv<float, true>(u, v, w);
                } else {
                    su3_mv<float, false>(u, v, w);
                }
#pragma unroll
                for (int c = 0; c < COUT; c++) {
                    const float2 wt = W[((size_t)c * CIN + cp) * 9 + h];
#pragma unroll
                    for (int a = 0; a < 3; a++) cfma(acc[q][c][a], wt, w[a]);
                }
            }
        }
        // one hop's link in registers at a time
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int q = 0; q < S; q++) {
        if (S > 1 && smp0 + q >= ns) break;
#pragma unroll
        for (int c = 0; c < COUT; c++) {
            const FieldView<float> yf(y + ((size_t)(smp0 + q) * COUT + c) * 12 * V, V, 12);
#pragma unroll
            for (int a = 0; a < 3; a++) yf.st_lane(a, d, 3u * s * yf.cs, acc[q][c][a]);
        }
    }
}

// out (FP64) = T_h in (FP32), one thread per (site, spin), blockIdx.y the field
__global__ __launch_bounds__(TPB) void net_hop_kernel(Geom g, const float2 *__restrict__ Up, int h,
                                                      const float2 *__restrict__ in, double2 *__restrict__ out) {
    const int t = blockIdx.x * TPB + threadIdx.x;
    const int i = t >> 2, s = t & 3;
    if (i >= g.V) return;
    const int d = site_in_lex_block_order(g, i);
    const size_t V = g.V, foff = (size_t)blockIdx.y * 12 * V;
    const FieldView<float> xf(in + foff, V, 12);
    float2 w[3];
    if (h == 0) {
#pragma unroll
        for (int a = 0; a < 3; a++) w[a] = xf.ld_lane(a, d, 3u * s * xf.cs);
    } else {
        int nbr[8];
        site_neighbours(g, d, nbr);
        LinkViews<float> U(Up, V);
        const int mu = (h - 1) >> 1;
        const bool back = (h - 1) & 1;
        const int dn = nbr[h - 1];
        float2 v[3], u[9];
#pragma unroll
        for (int a = 0; a < 3; a++) v[a] = xf.ld_lane(a, dn, 3u * s * xf.cs);
        const FieldView<float> &uf = mu == 0 ? U.u0 : mu == 1 ? U.u1 : mu == 2 ? U.u2 : U.u3;
#pragma unroll
        for (int k = 0; k < 9; k++) u[k] = uf.ld(k, back ? dn : d);
        if (back) su3_mv<float, true>(u, v, w);
        else su3_mv<float, false>(u, v, w);
    }
#pragma unroll
    for (int a = 0; a < 3; a++) out[foff + (size_t)(3 * s + a) * V + d] = make_double2(w[a].x, w[a].y);
}

__global__ void adjoint_weights_kernel(int cin, int cout, const double2 *__restrict__ W, float2 *__restrict__ Wa) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;   // index of Wa: (cp * cout + c) * 9 + h
    if (q >= cin * cout * 9) return;
    const int h = q % 9, c = (q / 9) % cout, cp = q / (9 * cout);
    const int hb = h == 0 ? 0 : ((h - 1) & 1 ? h - 1 : h + 1);
    const double2 w = W[((size_t)c * cin + cp) * 9 + hb];
    Wa[q] = make_float2((float)w.x, (float)-w.y);
}

__global__ void weights32_kernel(size_t n, const double2 *__restrict__ W, float2 *__restrict__ W32) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) W32[q] = make_float2((float)W[q].x, (float)W[q].y);
}

__global__ void grad_add_kernel(int cin, int cout, int h, const double2 *__restrict__ G, double2 *__restrict__ grad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;   // (c', c)
    if (q >= cin * cout) return;
    const int cp = q / cout, c = q % cout;
    double2 &o = grad[((size_t)c * cin + cp) * 9 + h];
    o.x += G[q].x;
    o.y += G[q].y;
}

__device__ inline double adam1(double &w, double g, double &m, double &v, double b1, double b2, double c1, double c2,
                               double lr, double eps) {
    m = b1 * m + (1 - b1) * g;
    v = b2 * v + (1 - b2) * g * g;
    w -= lr * (m / c1) / (sqrt(v / c2) + eps);
    return w;
}

__global__ void adam_kernel(size_t n, double2 *__restrict__ W, const double2 *__restrict__ grad, double2 *__restrict__ m,
                            double2 *__restrict__ v, double b1, double b2, double c1, double c2, double lr, double eps) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double2 w = W[q], mm = m[q], vv = v[q];
    adam1(w.x, grad[q].x, mm.x, vv.x, b1, b2, c1, c2, lr, eps);
    adam1(w.y, grad[q].y, mm.y, vv.y, b1, b2, c1, c2, lr, eps);
    W[q] = w;
    m[q] = mm;
    v[q] = vv;
}

template <int CIN, int COUT>
void layer_launch(Ctx *c, const float2 *W, int ns, const void *x, void *y) {
    // samples per thread: as many as keep the accumulators near 48 complex numbers
    constexpr int S = COUT <= 4 ? 4 : COUT <= 8 ? 2 : 1;
    const unsigned nwg = (unsigned)((4 * (size_t)c->g.V + TPB - 1) / TPB);
    net_layer_kernel<CIN, COUT, S><<<dim3(nwg, (ns + S - 1) / S), TPB, 0, c->stream>>>(
        c->g, (const float2 *)c->U32, W, (const float2 *)x, (float2 *)y, ns);
}

}  // namespace

int launch_net_layer(Ctx *c, int cin, int cout, const float2 *W, int ns, const void *x, void *y) {
#define L(A, B) \
    if (cin == A && cout == B) { layer_launch<A, B>(c, W, ns, x, y); return hip_check(c, hipGetLastError(), "network layer"); }
    L(1, 16) L(16, 16) L(16, 1) L(1, 8) L(8, 8) L(8, 1) L(1, 4) L(4, 4) L(4, 1) L(1, 2) L(2, 2) L(2, 1) L(1, 1)
    L(16, 8) L(8, 16) L(8, 4) L(4, 8) L(4, 2) L(2, 4)
#undef L
    return fail(c, MGDD_EINVAL, "network widths must be 1, 2, 4, 8 or 16, with neighbouring widths at most 2x apart or 1");
}

int launch_net_adjoint_weights(Ctx *c, int cin, int cout, const double2 *W, float2 *Wa) {
    const int n = cin * cout * 9;
    adjoint_weights_kernel<<<(n + 255) / 256, 256, 0, c->stream>>>(cin, cout, W, Wa);
    return hip_check(c, hipGetLastError(), "adjoint weights");
}

int launch_net_weights32(Ctx *c, size_t n, const double2 *W, float2 *W32) {
    weights32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(n, W, W32);
    return hip_check(c, hipGetLastError(), "weights");
}

int launch_net_hop(Ctx *c, int h, int nf, const void *in32, void *out64) {
    const unsigned nwg = (unsigned)((4 * (size_t)c->g.V + TPB - 1) / TPB);
    net_hop_kernel<<<dim3(nwg, nf), TPB, 0, c->stream>>>(c->g, (const float2 *)c->U32, h, (const float2 *)in32,
                                                         (double2 *)out64);
    return hip_check(c, hipGetLastError(), "network hop");
}

int launch_net_grad_add(Ctx *c, int cin, int cout, int h, const double2 *G, double2 *grad) {
    const int n = cin * cout;
    grad_add_kernel<<<(n + 255) / 256, 256, 0, c->stream>>>(cin, cout, h, G, grad);
    return hip_check(c, hipGetLastError(), "gradient");
}

int launch_net_adam(Ctx *c, size_t n, double2 *W, const double2 *grad, double2 *m, double2 *v, int step, double lr,
                    double beta1, double beta2, double eps) {
    const double c1 = 1 - std::pow(beta1, step), c2 = 1 - std::pow(beta2, step);
    adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(n, W, grad, m, v, beta1, beta2, c1, c2, lr, eps);
    return hip_check(c, hipGetLastError(), "adam");
}

// ---------------------------------------------------------------- host side

static bool width_ok(int w) { return w == 1 || w == 2 || w == 4 || w == 8 || w == 16; }

bool net_shape_valid(const NetShape &sh) {
    if (sh.nlayers < 1 || sh.nlayers > NET_MAX_LAYERS) return false;
    if (sh.widths[0] != 1 || sh.widths[sh.nlayers] != 1) return false;
    for (int l = 0; l <= sh.nlayers; l++)
        if (!width_ok(sh.widths[l])) return false;
    for (int l = 0; l < sh.nlayers; l++) {
        const int a = sh.widths[l], b = sh.widths[l + 1];
        if (!(a == 1 || b == 1 || a == b || a == 2 * b || b == 2 * a)) return false;
    }
    return true;
}

int check_net_shape(Ctx *c, const NetShape &sh) {
    if (!net_shape_valid(sh))
        return fail(c, MGDD_EINVAL,
                    "network: 1 to 8 layers, one input and one output channel, widths 1, 2, 4, 8 or 16 with "
                    "neighbouring widths equal, 2x apart, or one of them 1");
    return MGDD_OK;
}

static size_t field32(const Ctx *c) { return (size_t)12 * c->g.V * 8; }

static int max_width(const NetShape &sh) {
    int w = 1;
    for (int l = 0; l <= sh.nlayers; l++) w = sh.widths[l] > w ? sh.widths[l] : w;
    return w;
}

// inference: two activation buffers of the widest layer, used in turn
size_t net_forward_bytes(const Ctx *c, const NetShape &sh, int ns) {
    return sh.nweights() * 8 + 2 * ((size_t)ns * max_width(sh) * field32(c) + 256) + 4096;
}

// training: every layer's activations are kept for the backward pass
static size_t net_acts_bytes(const Ctx *c, const NetShape &sh, int ns) {
    size_t b = sh.nweights() * 8 + 4096;
    for (int l = 1; l <= sh.nlayers; l++) b += (size_t)ns * sh.widths[l] * field32(c) + 256;
    return b;
}

size_t net_grad_bytes(const Ctx *c, const NetShape &sh, int ns) {
    int wmax = 1;
    for (int l = 0; l <= sh.nlayers; l++) wmax = sh.widths[l] > wmax ? sh.widths[l] : wmax;
    const size_t nc = (size_t)c->c.Vc * 2 * c->c.N;
    return net_acts_bytes(c, sh, ns) + sh.nweights() * 8 + (size_t)NET_MAX_WIDTH * NET_MAX_WIDTH * 9 * 8 +
           2 * (size_t)ns * wmax * field32(c) +                      // gradients of two neighbouring layers (FP32)
           2 * (size_t)ns * wmax * field32(c) * 2 +                  // FP64 gradient and hopped activations
           2 * (size_t)ns * field32(c) + (size_t)ns * nc * 8 +      // P P^H f, (1 - P P^H) f, P^H f
           (size_t)NET_MAX_WIDTH * NET_MAX_WIDTH * 16 + 64 * (size_t)ns * 16 + 65536;
}

// activations x_1 .. x_L in the arena (x_0 = the input); W32 the FP32 weights
static int forward_acts(Ctx *c, const NetShape &sh, const double2 *W64, int ns, const void *in32, Arena &A,
                        std::vector<const void *> &xs, float2 *&W32) {
    W32 = (float2 *)A.take(sh.nweights() * 8);
    if (!W32) return fail(c, MGDD_ENOMEM, "network workspace");
    int rc = launch_net_weights32(c, sh.nweights(), W64, W32);
    xs.assign(sh.nlayers + 1, nullptr);
    xs[0] = in32;
    for (int l = 0; l < sh.nlayers && !rc; l++) {
        void *y = A.take((size_t)ns * sh.widths[l + 1] * field32(c));
        if (!y) return fail(c, MGDD_ENOMEM, "network workspace");
        rc = launch_net_layer(c, sh.widths[l], sh.widths[l + 1], W32 + sh.offset(l), ns, xs[l], y);
        xs[l + 1] = y;
    }
    return rc;
}

int net_forward(Ctx *c, const NetShape &sh, const double2 *W64, int ns, const void *in32, void *out32, Arena &A) {
    const size_t mark = A.off;
    float2 *W32 = (float2 *)A.take(sh.nweights() * 8);
    void *buf[2] = {A.take((size_t)ns * max_width(sh) * field32(c)), A.take((size_t)ns * max_width(sh) * field32(c))};
    if (!buf[1]) return fail(c, MGDD_ENOMEM, "network workspace");
    int rc = launch_net_weights32(c, sh.nweights(), W64, W32);
    const void *x = in32;
    for (int l = 0; l < sh.nlayers && !rc; l++) {
        void *y = l + 1 == sh.nlayers ? out32 : buf[l & 1];
        rc = launch_net_layer(c, sh.widths[l], sh.widths[l + 1], W32 + sh.offset(l), ns, x, y);
        x = y;
    }
    A.off = mark;
    return rc;
}

int net_grad(Ctx *c, const NetShape &sh, const double2 *W64, int ns, const void *in32, double *loss, double2 *grad,
             Arena &A) {
    const size_t mark = A.off, n = (size_t)12 * c->g.V, nc = (size_t)c->c.Vc * 2 * c->c.N;
    std::vector<const void *> xs;
    float2 *W32 = nullptr;
    int rc = forward_acts(c, sh, W64, ns, in32, A, xs, W32);
    if (rc) return rc;
    int wmax = 1;
    for (int l = 0; l <= sh.nlayers; l++) wmax = sh.widths[l] > wmax ? sh.widths[l] : wmax;
    float2 *Wa = (float2 *)A.take((size_t)NET_MAX_WIDTH * NET_MAX_WIDTH * 9 * 8);
    void *ga = A.take((size_t)ns * wmax * field32(c)), *gb = A.take((size_t)ns * wmax * field32(c));
    void *g64 = A.take((size_t)ns * wmax * field32(c) * 2), *xh64 = A.take((size_t)ns * wmax * field32(c) * 2);
    void *pf = A.take((size_t)ns * field32(c)), *qf = A.take((size_t)ns * field32(c)), *cf = A.take((size_t)ns * nc * 8);
    double2 *G = (double2 *)A.take((size_t)NET_MAX_WIDTH * NET_MAX_WIDTH * 16);
    double2 *sc = (double2 *)A.take(64 * (size_t)ns * 16);
    if (!sc) return fail(c, MGDD_ENOMEM, "network workspace");
    const void *f = xs[sh.nlayers];
    // (1 - P P^H) f and the norms
    rc = launch_restrict(c, MGDD_F32, ns, f, cf);
    if (!rc) rc = launch_prolong(c, MGDD_F32, ns, cf, pf);
    double2 *one = sc, *coef = sc + ns, *nrm = sc + 3 * ns;
    std::vector<double2> h((size_t)4 * ns);
    for (int s = 0; s < ns; s++) h[s] = make_double2(1.0, 0.0);
    if (!rc) rc = hip_check(c, hipMemcpyAsync(one, h.data(), (size_t)ns * 16, hipMemcpyHostToDevice, c->stream), "write");
    if (!rc) rc = hip_check(c, hipMemcpyAsync(qf, pf, (size_t)ns * field32(c), hipMemcpyDeviceToDevice, c->stream), "copy");
    if (!rc) rc = blas_lincomb(c, MGDD_F32, MGDD_F32, n, &f, 1, one, 1.0, -1.0, qf, ns);   // qf = f - P P^H f
    const void *qp = qf;
    if (!rc) rc = blas_multidot(c, MGDD_F32, MGDD_F32, n, &f, 1, f, nrm, ns);
    if (!rc) rc = blas_multidot(c, MGDD_F32, MGDD_F32, n, &qp, 1, qf, nrm + ns, ns);
    if (!rc) rc = hip_check(c, hipMemcpyAsync(h.data(), nrm, (size_t)2 * ns * 16, hipMemcpyDeviceToHost, c->stream), "read");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (rc) return rc;
    double Lsum = 0;
    std::vector<double2> cw((size_t)2 * ns);
    for (int s = 0; s < ns; s++) {
        const double ff = h[s].x, qq = h[ns + s].x;
        if (!(ff > 0) || !std::isfinite(ff) || !std::isfinite(qq)) return fail(c, MGDD_ENAN, "network output is zero or not finite");
        const double L = qq / ff;
        Lsum += L;
        // g = (qf - L f) / (ff ns): the gradient of the mean
        cw[s] = make_double2(1.0 / (ff * ns), 0.0);
        cw[ns + s] = make_double2(-L / (ff * ns), 0.0);
    }
    *loss = Lsum / ns;
    const void *qfl[2] = {qf, f};
    rc = hip_check(c, hipMemcpyAsync(coef, cw.data(), (size_t)2 * ns * 16, hipMemcpyHostToDevice, c->stream), "write");
    if (!rc) rc = blas_lincomb(c, MGDD_F32, MGDD_F32, n, qfl, 2, coef, 1.0, 0.0, ga, ns);
    if (!rc) rc = hip_check(c, hipMemsetAsync(grad, 0, sh.nweights() * 16, c->stream), "memset");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");   // cw and h are reused below
    // backward through the layers; ga holds dL/dconj(x_{l+1})
    for (int l = sh.nlayers - 1; l >= 0 && !rc; l--) {
        const int cin = sh.widths[l], cout = sh.widths[l + 1];
        rc = launch_convert(c, MGDD_F32, MGDD_F64, (size_t)ns * cout * n, ga, g64);
        for (int hh = 0; hh < 9 && !rc; hh++) {
            rc = launch_net_hop(c, hh, ns * cin, xs[l], xh64);
            for (int s = 0; s < ns && !rc; s++) {
                const void *xp[NET_MAX_WIDTH], *yp[NET_MAX_WIDTH];
                for (int i = 0; i < cin; i++) xp[i] = (const char *)xh64 + ((size_t)s * cin + i) * n * 16;
                for (int j = 0; j < cout; j++) yp[j] = (const char *)g64 + ((size_t)s * cout + j) * n * 16;
                rc = blas_gram(c, n, xp, cin, yp, cout, G);
                if (!rc) rc = launch_net_grad_add(c, cin, cout, hh, G, grad + sh.offset(l));
            }
        }
        if (l > 0 && !rc) {
            rc = launch_net_adjoint_weights(c, cin, cout, W64 + sh.offset(l), Wa);
            if (!rc) rc = launch_net_layer(c, cout, cin, Wa, ns, ga, gb);
            std::swap(ga, gb);
        }
    }
    A.off = mark;
    if (!rc && A.need) rc = fail(c, MGDD_ENOMEM, "network workspace estimate too small");
    return rc;
}

}  // namespace mgdd
