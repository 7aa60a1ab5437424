// Even-odd (Schur complement) pieces of the plain FP64 GCR comparator.
// With D = A - 1/2 H split by site parity, the odd-site system is
//   D_hat = A_oo - 1/4 H_oe A_ee^{-1} H_eo,
//   b_hat = b_o + 1/2 H_oe A_ee^{-1} b_e,   z_e = A_ee^{-1} (b_e + 1/2 H_eo z_o).
// Half fields hold the sites of one parity only, compactly: half index
// h = pos * Vb/2 + (local index within that parity's half of the block), and
// are stored [12][V/2] like full fields.
#include "eo.h"
#include "stencil.h"

namespace mgdd {

namespace {

constexpr int TPB = 256;

__device__ inline int dev_of_half(const Geom &g, int h, int p) {
    const int hb = g.Vb >> 1;
    return ((h / hb) << g.lgVb) + p * hb + (h % hb);
}
__device__ inline int half_of_dev(const Geom &g, int d) {
    const int hb = g.Vb >> 1;
    return (d >> g.lgVb) * hb + (d & (hb - 1));
}

template <typename T> __device__ inline void load_half(const FieldView<T> &f, int h, C<T> *s) { load_spinor<T>(f, h, s); }

// out = MOUT( alpha * MAUX(aux) + beta * H in ), on the sites of parity p.
// MAUX: 0 identity, 1 A. MOUT: 0 identity, 1 A^{-1}. beta == 0 skips the hop
// (and `in` is not read); alpha == 0 skips aux.
template <int MAUX, int MOUT>
__global__ __launch_bounds__(TPB) void eo_kernel(Geom g, int p, const double2 *__restrict__ Up,
                                                 const double2 *__restrict__ Ap, const double2 *__restrict__ Aip,
                                                 const double2 *__restrict__ in, const double2 *__restrict__ aux,
                                                 double alpha, double beta, double2 *__restrict__ out) {
    const int h = blockIdx.x * TPB + threadIdx.x;
    const int Vh = g.V >> 1;
    if (h >= Vh) return;
    const int d = dev_of_half(g, h, p);
    const size_t V = g.V;
    double2 acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = make_double2(0, 0);
    if (beta != 0.0) {
        int nbr[8];
        site_neighbours(g, d, nbr);
        LinkViews<double> U(Up, V);
        FieldView<double> fin(in, (size_t)Vh, 12);
        double2 psi[12], u[9];
        // the neighbours have the other parity: read them from the half field
#define EO_HOP(MU, FWD, K)                                            \
    load_spinor<double>(fin, half_of_dev(g, nbr[K]), psi);           \
    load_link<double, MU>(U, FWD ? d : nbr[K], u);                   \
    hop<double, MU, FWD>(acc, u, psi);
        EO_HOP(0, true, 0) EO_HOP(0, false, 1) EO_HOP(1, true, 2) EO_HOP(1, false, 3)
        EO_HOP(2, true, 4) EO_HOP(2, false, 5) EO_HOP(3, true, 6) EO_HOP(3, false, 7)
#undef EO_HOP
#pragma unroll
        for (int c = 0; c < 12; c++) acc[c] = cscale(acc[c], beta);
    }
    if (alpha != 0.0) {
        FieldView<double> fa(aux, (size_t)Vh, 12);
        double2 x[12], y[12];
        load_spinor<double>(fa, h, x);
        if (MAUX == 1) {
            CloverViews<double> A(Ap, V);
            clover_mv<double>(A, d, x, y);
        } else {
#pragma unroll
            for (int c = 0; c < 12; c++) y[c] = x[c];
        }
#pragma unroll
        for (int c = 0; c < 12; c++) acc[c] = cadd(acc[c], cscale(y[c], alpha));
    }
    FieldView<double> fo(out, (size_t)Vh, 12);
    if (MOUT == 1) {
        CloverViews<double> Ai(Aip, V);
        double2 y[12];
        clover_mv<double>(Ai, d, acc, y);
        store_spinor<double>(fo, h, y);
    } else {
        store_spinor<double>(fo, h, acc);
    }
}

// full field <-> two half fields
__global__ void eo_split_kernel(Geom g, const double2 *__restrict__ full, double2 *__restrict__ even,
                                double2 *__restrict__ odd) {
    const int d = blockIdx.x * TPB + threadIdx.x;
    if (d >= g.V) return;
    const int Vh = g.V >> 1;
    const int p = (d & (g.Vb - 1)) >= (g.Vb >> 1);
    const int h = half_of_dev(g, d);
    double2 *dst = p ? odd : even;
    for (int c = 0; c < 12; c++) dst[(size_t)c * Vh + h] = full[(size_t)c * g.V + d];
}

__global__ void eo_merge_kernel(Geom g, const double2 *__restrict__ even, const double2 *__restrict__ odd,
                                double2 *__restrict__ full) {
    const int d = blockIdx.x * TPB + threadIdx.x;
    if (d >= g.V) return;
    const int Vh = g.V >> 1;
    const int p = (d & (g.Vb - 1)) >= (g.Vb >> 1);
    const int h = half_of_dev(g, d);
    const double2 *src = p ? odd : even;
    for (int c = 0; c < 12; c++) full[(size_t)c * g.V + d] = src[(size_t)c * Vh + h];
}

}  // namespace

int launch_eo(Ctx *c, int p, int maux, int mout, const void *in, const void *aux, double alpha, double beta, void *out) {
    const Geom &g = c->g;
    unsigned nwg = (unsigned)((g.V / 2 + TPB - 1) / TPB);
    auto U = (const double2 *)c->U64;
    auto A = (const double2 *)c->A64;
    auto Ai = (const double2 *)c->Ainv64;
    auto I = (const double2 *)in;
    auto X = (const double2 *)aux;
    auto O = (double2 *)out;
    if (maux == 0 && mout == 0) eo_kernel<0, 0><<<nwg, TPB, 0, c->stream>>>(g, p, U, A, Ai, I, X, alpha, beta, O);
    else if (maux == 1 && mout == 0) eo_kernel<1, 0><<<nwg, TPB, 0, c->stream>>>(g, p, U, A, Ai, I, X, alpha, beta, O);
    else if (maux == 0 && mout == 1) eo_kernel<0, 1><<<nwg, TPB, 0, c->stream>>>(g, p, U, A, Ai, I, X, alpha, beta, O);
    else eo_kernel<1, 1><<<nwg, TPB, 0, c->stream>>>(g, p, U, A, Ai, I, X, alpha, beta, O);
    return hip_check(c, hipGetLastError(), "even-odd kernel");
}

int launch_eo_split(Ctx *c, const void *full, void *even, void *odd) {
    unsigned nwg = (unsigned)((c->g.V + TPB - 1) / TPB);
    eo_split_kernel<<<nwg, TPB, 0, c->stream>>>(c->g, (const double2 *)full, (double2 *)even, (double2 *)odd);
    return hip_check(c, hipGetLastError(), "even-odd split");
}

int launch_eo_merge(Ctx *c, const void *even, const void *odd, void *full) {
    unsigned nwg = (unsigned)((c->g.V + TPB - 1) / TPB);
    eo_merge_kernel<<<nwg, TPB, 0, c->stream>>>(c->g, (const double2 *)even, (const double2 *)odd, (double2 *)full);
    return hip_check(c, hipGetLastError(), "even-odd merge");
}

}  // namespace mgdd
