// Wilson-clover operator D = A - 1/2 H (Section 1): one thread per site,
// site-major loads of the 8 neighbour spinors and links, spin projection to
// half spinors before the SU(3) products.
#include "dirac.h"
#include "stencil.h"

namespace mgdd {

namespace {

constexpr int TPB = 256;

// One thread per (site, right-hand side). Workgroup w covers TPB sites of one
// right-hand side; the right-hand sides of one range of sites are consecutive
// workgroups on one XCD, so the links and the clover term of those sites come
// from HBM once and from L2 for the other right-hand sides.
// S: storage type of the spinors (T, or _Float16 with T = float: half
// storage, FP32 arithmetic, links and clover term in FP32)
template <typename T, typename S = T> struct SpinorView { using type = FieldView<T>; };
template <> struct SpinorView<float, _Float16> { using type = HalfFieldView; };

template <typename T, typename S = T>
__global__ __launch_bounds__(TPB) void dirac_kernel(Geom g, const C<T> *__restrict__ Up, const C<T> *__restrict__ Ap,
                                                    const C<S> *__restrict__ in, C<S> *__restrict__ out, int nrhs,
                                                    int nwg) {
    const int w = xcd_block(nwg);
    const int r = w % nrhs;
    const int i = (w / nrhs) * TPB + threadIdx.x;
    if (i >= g.V) return;
    const int d = site_in_lex_block_order(g, i);
    int nbr[8];
    site_neighbours(g, d, nbr);
    const size_t V = g.V;
    LinkViews<T> U(Up, V);
    CloverViews<T> A(Ap, V);
    using FV = typename SpinorView<T, S>::type;
    FV f(in + (size_t)r * 12 * V, V, 12), o(out + (size_t)r * 12 * V, V, 12);
    C<T> acc[12], psi[12], res[12];
    hop_sum<T>(U, f, d, nbr, acc);
    load_spinor<T>(f, d, psi);
    clover_mv<T>(A, d, psi, res);
#pragma unroll
    for (int k = 0; k < 12; k++) res[k] = csub(res[k], cscale(acc[k], (T)0.5));
    store_spinor<T>(o, d, res);
}

// FP32 spinors read as FP64 (the widening is exact)
struct WidenView {
    FieldView<float> f;
    __device__ WidenView(const float2 *base, size_t V, int ncomp) : f(base, V, ncomp) {}
    __device__ double2 ld(int comp, int site, unsigned salt = 0) const {
        const float2 v = f.ld(comp, site, salt);
        return make_double2((double)v.x, (double)v.y);
    }
};

// dirac_kernel<double> with FP32 input: the FP64 apply of an FP32 field
// without a converted copy
__global__ __launch_bounds__(TPB) void dirac_widen_kernel(Geom g, const double2 *__restrict__ Up,
                                                          const double2 *__restrict__ Ap, const float2 *__restrict__ in,
                                                          double2 *__restrict__ out, int nrhs, int nwg) {
    const int w = xcd_block(nwg);
    const int r = w % nrhs;
    const int i = (w / nrhs) * TPB + threadIdx.x;
    if (i >= g.V) return;
    const int d = site_in_lex_block_order(g, i);
    int nbr[8];
    site_neighbours(g, d, nbr);
    const size_t V = g.V;
    LinkViews<double> U(Up, V);
    CloverViews<double> A(Ap, V);
    WidenView f(in + (size_t)r * 12 * V, V, 12);
    FieldView<double> o(out + (size_t)r * 12 * V, V, 12);
    double2 acc[12], psi[12], res[12];
    hop_sum<double>(U, f, d, nbr, acc);
    load_spinor<double>(f, d, psi);
    clover_mv<double>(A, d, psi, res);
#pragma unroll
    for (int k = 0; k < 12; k++) res[k] = csub(res[k], cscale(acc[k], 0.5));
    store_spinor<double>(o, d, res);
}

}  // namespace

int launch_dirac_widen(Ctx *c, int nrhs, const void *in32, void *out64) {
    int nwg = ((c->g.V + TPB - 1) / TPB) * nrhs;
    const int slot = kt_begin(c);
    dirac_widen_kernel<<<nwg, TPB, 0, c->stream>>>(c->g, (const double2 *)c->U64, (const double2 *)c->A64,
                                                   (const float2 *)in32, (double2 *)out64, nrhs, nwg);
    // links and clover term once per launch, FP32 in and FP64 out per field
    kt_end(c, slot, KF_DIRAC, MGDD_F64, (double)c->g.V * nrhs, (double)c->g.V * (1152.0 + 288.0 * nrhs));
    return hip_check(c, hipGetLastError(), "dirac kernel");
}

int launch_dirac(Ctx *c, int prec, int nrhs, const void *in, void *out) {
    int nwg = ((c->g.V + TPB - 1) / TPB) * nrhs;
    const int slot = kt_begin(c);
    if (prec == MGDD_F64)
        dirac_kernel<double><<<nwg, TPB, 0, c->stream>>>(c->g, (const double2 *)c->U64, (const double2 *)c->A64,
                                                         (const double2 *)in, (double2 *)out, nrhs, nwg);
    else if (prec == MGDD_F32)
        dirac_kernel<float><<<nwg, TPB, 0, c->stream>>>(c->g, (const float2 *)c->U32, (const float2 *)c->A32,
                                                        (const float2 *)in, (float2 *)out, nrhs, nwg);
    else
        dirac_kernel<float, _Float16><<<nwg, TPB, 0, c->stream>>>(c->g, (const float2 *)c->U32,
                                                                  (const float2 *)c->A32, (const half_cx *)in,
                                                                  (half_cx *)out, nrhs, nwg);
    // links and clover term once per launch (FP64, or FP32 for FP32 and half
    // spinors), spinor in and out per field
    const double lc = prec == MGDD_F64 ? 1152.0 : 576.0, sp = 2.0 * 12 * csize(prec);
    kt_end(c, slot, KF_DIRAC, prec, (double)c->g.V * nrhs, (double)c->g.V * (lc + sp * nrhs));
    return hip_check(c, hipGetLastError(), "dirac kernel");
}

}  // namespace mgdd
