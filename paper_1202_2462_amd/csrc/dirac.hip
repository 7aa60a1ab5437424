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

// STAGE (lattice blocks of TPB sites, so that a workgroup is one block): the
// workgroup first puts its own spinors in LDS, and the neighbours inside the
// block (three quarters of them for 4^4 blocks) are read from there; only the
// neighbours outside the block are read from memory, where the cache need not
// have kept them since another workgroup read them.
// RECON: the links are special unitary, rows 0 and 1 are read and row 2 is
// rebuilt (a third fewer link bytes); antiperiodic: the sign of the time
// links at the boundary, which the rebuilt row must carry
template <typename T, typename S = T, bool RECON = false, bool STAGE = false>
__global__ __launch_bounds__(TPB) void dirac_kernel(Geom g, const C<T> *__restrict__ Up, const C<T> *__restrict__ Ap,
                                                    const C<S> *__restrict__ in, C<S> *__restrict__ out, int nrhs,
                                                    int nwg, int antiperiodic) {
    const int w = xcd_block(nwg);
    const int r = w % nrhs;
    const int i = (w / nrhs) * TPB + threadIdx.x;
    if (!STAGE && i >= g.V) return;  // staged: V is a multiple of TPB
    const int d = site_in_lex_block_order(g, i);
    int nbr[8];
    site_neighbours(g, d, nbr);
    T sf = 1, sb = 1;
    if (RECON) time_link_signs<T>(g, d, antiperiodic, sf, sb);
    const size_t V = g.V;
    LinkViews<T> U(Up, V);
    CloverViews<T> A(Ap, V);
    using FV = typename SpinorView<T, S>::type;
    FV f(in + (size_t)r * 12 * V, V, 12), o(out + (size_t)r * 12 * V, V, 12);
    C<T> acc[12], psi[12], res[12];
    load_spinor<T>(f, d, psi);
    if (STAGE) {
        __shared__ C<T> sp[12 * TPB];
#pragma unroll
        for (int k = 0; k < 12; k++) sp[k * TPB + (d & (TPB - 1))] = psi[k];
        __syncthreads();
        hop_sum_staged<T, T, RECON, TPB>(U, (const C<T> *)in + (size_t)r * 12 * V, V, sp, d >> g.lgVb, g.lgVb, d,
                                         nbr, acc, sf, sb);
    } else {
        hop_sum<T, RECON>(U, f, d, nbr, acc, sf, sb);
    }
    clover_mv<T, true>(A, d, psi, res);
#pragma unroll
    for (int k = 0; k < 12; k++) res[k] = csub(res[k], cscale(acc[k], (T)0.5));
    store_spinor<T, true>(o, d, res);
}

// FP32 or half-precision spinors (S) read as FP64 (the widening is exact)
template <typename S> struct WidenView {
    typename F32Store<S>::view f;
    __device__ WidenView(const C<S> *base, size_t V, int ncomp) : f((const float2 *)base, V, ncomp) {}
    __device__ double2 ld(int comp, int site, unsigned salt = 0) const {
        const float2 v = f.ld(comp, site, salt);
        return make_double2((double)v.x, (double)v.y);
    }
};

// dirac_kernel<double> with FP32 or half-precision input (S): the FP64 apply
// of such a field without a converted copy
template <bool RECON, bool STAGE, typename S = float>
__global__ __launch_bounds__(TPB) void dirac_widen_kernel(Geom g, const double2 *__restrict__ Up,
                                                          const double2 *__restrict__ Ap, const C<S> *__restrict__ in,
                                                          double2 *__restrict__ out, int nrhs, int nwg,
                                                          int antiperiodic) {
    const int w = xcd_block(nwg);
    const int r = w % nrhs;
    const int i = (w / nrhs) * TPB + threadIdx.x;
    if (!STAGE && i >= g.V) return;
    const int d = site_in_lex_block_order(g, i);
    int nbr[8];
    site_neighbours(g, d, nbr);
    double sf = 1, sb = 1;
    if (RECON) time_link_signs<double>(g, d, antiperiodic, sf, sb);
    const size_t V = g.V;
    LinkViews<double> U(Up, V);
    CloverViews<double> A(Ap, V);
    WidenView<S> f(in + (size_t)r * 12 * V, V, 12);
    FieldView<double> o(out + (size_t)r * 12 * V, V, 12);
    double2 acc[12], psi[12], res[12];
    if (STAGE) {
        __shared__ C<S> sp[12 * TPB];
        const C<S> *fin = in + (size_t)r * 12 * V;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const float2 v = f.f.ld(k, d);   // exact: back to S unchanged below
            sp[k * TPB + (d & (TPB - 1))] = mk<S>((S)v.x, (S)v.y);
            psi[k] = make_double2((double)v.x, (double)v.y);
        }
        __syncthreads();
        hop_sum_staged<double, S, RECON, TPB>(U, fin, V, sp, d >> g.lgVb, g.lgVb, d, nbr, acc, sf, sb);
    } else {
        hop_sum<double, RECON>(U, f, d, nbr, acc, sf, sb);
        load_spinor<double>(f, d, psi);
    }
    clover_mv<double, true>(A, d, psi, res);
#pragma unroll
    for (int k = 0; k < 12; k++) res[k] = csub(res[k], cscale(acc[k], 0.5));
    store_spinor<double, true>(o, d, res);
}

}  // namespace

// algorithmic bytes of one apply per site: links (two rows of each when they
// are rebuilt) and clover term once per launch, spinors in and out per field
static double dirac_launch_bytes(const Ctx *c, int prec, size_t in_bytes, size_t out_bytes, int nrhs) {
    const double real = prec == MGDD_F64 ? 8.0 : 4.0;
    const double links = 4 * (c->links_su3 ? 6 : 9) * 2 * real, clover = 72 * real;
    return (double)c->g.V * (links + clover + (double)(in_bytes + out_bytes) * nrhs);
}

// The staged kernels take one workgroup per lattice block: blocks of TPB
// sites. -1: an option the context cannot run.
static int dirac_staged(Ctx *c) {
    if (c->dirac_stage == 1 && c->g.Vb != TPB) {
        fail(c, MGDD_ESHAPE, "the staged Wilson-clover apply needs blocks of 256 sites");
        return -1;
    }
    return c->dirac_stage >= 0 && c->g.Vb == TPB ? 1 : 0;
}

int launch_dirac_widen(Ctx *c, int nrhs, const void *in32, void *out64, int in_prec) {
    int nwg = ((c->g.V + TPB - 1) / TPB) * nrhs;
    const int anti = c->t_antiperiodic ? 1 : 0;
    const int st = dirac_staged(c);
    if (st < 0) return MGDD_ESHAPE;
    const bool stage = st == 1;
    const int slot = kt_begin(c);
#define WIDEN(R, G, S)                                                                                                \
    dirac_widen_kernel<R, G, S><<<nwg, TPB, 0, c->stream>>>(c->g, (const double2 *)c->U64, (const double2 *)c->A64,  \
                                                            (const C<S> *)in32, (double2 *)out64, nrhs, nwg, anti)
#define WIDEN_S(S)                                                                                                    \
    do {                                                                                                              \
        if (c->links_su3) {                                                                                           \
            if (stage) WIDEN(true, true, S); else WIDEN(true, false, S);                                              \
        } else {                                                                                                      \
            if (stage) WIDEN(false, true, S); else WIDEN(false, false, S);                                            \
        }                                                                                                             \
    } while (0)
    if (in_prec == MGDD_F16) WIDEN_S(_Float16); else WIDEN_S(float);
#undef WIDEN_S
#undef WIDEN
    kt_end(c, slot, KF_DIRAC, MGDD_F64, (double)c->g.V * nrhs,
           dirac_launch_bytes(c, MGDD_F64, 12 * csize(in_prec), 192, nrhs));
    return hip_check(c, hipGetLastError(), "dirac kernel");
}

int launch_dirac(Ctx *c, int prec, int nrhs, const void *in, void *out) {
    int nwg = ((c->g.V + TPB - 1) / TPB) * nrhs;
    const int anti = c->t_antiperiodic ? 1 : 0;
    const int st = dirac_staged(c);
    if (st < 0) return MGDD_ESHAPE;
    const bool stage = st == 1;
    const int slot = kt_begin(c);
#define DIRAC(T, S, R, G)                                                                                             \
    dirac_kernel<T, S, R, G><<<nwg, TPB, 0, c->stream>>>(c->g, (const C<T> *)(prec == MGDD_F64 ? c->U64 : c->U32),    \
                                                         (const C<T> *)(prec == MGDD_F64 ? c->A64 : c->A32),          \
                                                         (const C<S> *)in, (C<S> *)out, nrhs, nwg, anti)
#define DIRAC_STAGED(T)                                                                                               \
    do {                                                                                                              \
        if (c->links_su3) {                                                                                           \
            if (stage) DIRAC(T, T, true, true); else DIRAC(T, T, true, false);                                        \
        } else {                                                                                                      \
            if (stage) DIRAC(T, T, false, true); else DIRAC(T, T, false, false);                                      \
        }                                                                                                             \
    } while (0)
    if (prec == MGDD_F64) {
        DIRAC_STAGED(double);
    } else if (prec == MGDD_F32) {
        DIRAC_STAGED(float);
    } else {
        if (c->links_su3) DIRAC(float, _Float16, true, false); else DIRAC(float, _Float16, false, false);
    }
#undef DIRAC_STAGED
#undef DIRAC
    const size_t sp = 12 * csize(prec);
    kt_end(c, slot, KF_DIRAC, prec, (double)c->g.V * nrhs, dirac_launch_bytes(c, prec, sp, sp, nrhs));
    return hip_check(c, hipGetLastError(), "dirac kernel");
}

}  // namespace mgdd
