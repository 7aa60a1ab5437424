// Schwarz variants (Section 2): the block systems I^T (D - shift) I e = I^T r
// solved by k steps of GMRES from e = 0 (the block solver of the paper's
// experiments, Section 4), and additive Schwarz (the first error propagator
// of eq. (2.1): every block solved for one residual per sweep). Red-black
// sweeps with MR block solves are the Schwarz kernels of sap.hip.
//
// GMRES kernel: one workgroup per block of the current colour, one thread
// per site. The thread keeps its site's 12 components of every basis vector
// v_0..v_k in registers; the vector being applied is also in LDS, where the
// in-block neighbours read it (hops leaving the block dropped). Arnoldi with
// classical Gram-Schmidt and one re-orthogonalisation (two block-wide sums of
// all coefficients at once, then one for the norm); every thread then solves
// the same (k+1) x k least-squares problem by Givens rotations and forms
// e = sum_i y_i v_i.
#include "schwarz.h"
#include "stencil.h"

namespace mgdd {

namespace {

// deterministic block-wide sums of NV values: an XOR butterfly inside each
// wave, then the per-wave sums added in wave order by every thread
template <typename T, int NV> __device__ inline void block_sum_n(T (&v)[NV], T *red) {
#pragma unroll
    for (int i = 0; i < NV; i++)
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v[i] += __shfl_xor(v[i], m, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++) red[NV * w + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; i++) {
        T s = 0;
        for (int q = 0; q < nw; q++) s += red[NV * q + i];
        v[i] = s;
    }
    __syncthreads();
}

// acc += hop along MU from the in-block neighbour ln (dropped when ln < 0),
// the vector read from LDS ([12][Vb])
template <typename T, int MU, bool FWD>
__device__ inline void lds_hop(C<T> *acc, const LinkViews<T> &U, int d, int dn, int ln, const C<T> *v, int Vb,
                               unsigned salt) {
    if (ln < 0) return;
    C<T> psi[12], u[9];
#pragma unroll
    for (int k = 0; k < 12; k++) psi[k] = v[k * Vb + ln];
    load_link<T, MU>(U, FWD ? d : dn, u, salt);
    hop<T, MU, FWD>(acc, u, psi);
}

template <typename V> __device__ inline V cdiv(V a, V b) {
    const auto n = b.x * b.x + b.y * b.y;
    V q;
    q.x = (a.x * b.x + a.y * b.y) / n;
    q.y = (a.y * b.x - a.x * b.y) / n;
    return q;
}

template <typename V> __device__ inline V cconj(V a) {
    a.y = -a.y;
    return a;
}

template <typename T, int K>
__global__ __launch_bounds__(256) void sap_gmres_kernel(Geom g, const C<T> *__restrict__ Up, const C<T> *__restrict__ Ap,
                                                        const C<T> *__restrict__ b, C<T> *__restrict__ z, int colour,
                                                        T sre, T sim) {
    extern __shared__ unsigned char smem[];
    const int Vb = g.Vb;
    C<T> *v_lds = (C<T> *)smem;                           // [12][Vb]
    T *red = (T *)(smem + sizeof(C<T>) * 12 * Vb);        // [2K][waves]
    const size_t V = g.V;
    const int pos = (colour ? g.ncol0 : 0) + xcd_block(gridDim.x);
    const int l = threadIdx.x;
    const int d = (pos << g.lgVb) + l;
    const size_t roff = (size_t)blockIdx.y * 12 * V;
    LinkViews<T> U(Up, V);
    CloverViews<T> A(Ap, V);
    FieldView<T> bf(b + roff, V, 12), zf(z + roff, V, 12);
    const C<T> shift = mk<T>(sre, sim);

    int x[4], nbr[8], ln[8];
    local_coords(g, l, x);
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        const int bm = 1 << g.lb[mu];
        nbr[2 * mu] = neighbour(g, pos, x, mu, +1);
        nbr[2 * mu + 1] = neighbour(g, pos, x, mu, -1);
        int y[4] = {x[0], x[1], x[2], x[3]};
        const bool wrap = g.nb[mu] == 1;   // a block spanning the lattice keeps its wrap-around hops
        y[mu] = x[mu] + 1;
        if (wrap) y[mu] &= bm - 1;
        ln[2 * mu] = (y[mu] < bm) ? local_index(g, y) : -1;
        y[mu] = x[mu] - 1;
        if (wrap) y[mu] = (y[mu] + bm) & (bm - 1);
        ln[2 * mu + 1] = (y[mu] >= 0) ? local_index(g, y) : -1;
    }

    // r = b - (D - shift) z on this site
    C<T> r[12], tmp[12], zs[12];
    {
        C<T> q[12];
        hop_sum<T>(U, zf, d, nbr, tmp);
        load_spinor<T>(zf, d, zs);
        clover_mv<T>(A, d, zs, q);
        load_spinor<T>(bf, d, r);
#pragma unroll
        for (int k = 0; k < 12; k++) r[k] = csub(r[k], csub(csub(q[k], cscale(tmp[k], (T)0.5)), cmul(shift, zs[k])));
    }
    T nv[2 * K];
#pragma unroll
    for (int i = 0; i < 2 * K; i++) nv[i] = 0;
#pragma unroll
    for (int k = 0; k < 12; k++) nv[0] += r[k].x * r[k].x + r[k].y * r[k].y;
    block_sum_n<T, 2 * K>(nv, red);
    const T beta = sqrt(nv[0]);
    if (beta > (T)0) {   // the same in every thread of the block
        C<T> v[K + 1][12], H[K + 1][K];
#pragma unroll
        for (int i = 0; i <= K; i++)
#pragma unroll
            for (int j = 0; j < K; j++) H[i][j] = mk<T>(0, 0);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            v[0][k] = mk<T>(r[k].x / beta, r[k].y / beta);
            v_lds[k * Vb + l] = v[0][k];
        }
        __syncthreads();
        int kk = K;
#pragma unroll
        for (int j = 0; j < K; j++) {
            if (j < kk) {
                const unsigned salt = opaque_zero();
                C<T> w[12];
#pragma unroll
                for (int k = 0; k < 12; k++) tmp[k] = mk<T>(0, 0);
                lds_hop<T, 0, true>(tmp, U, d, nbr[0], ln[0], v_lds, Vb, salt);
                lds_hop<T, 0, false>(tmp, U, d, nbr[1], ln[1], v_lds, Vb, salt);
                lds_hop<T, 1, true>(tmp, U, d, nbr[2], ln[2], v_lds, Vb, salt);
                lds_hop<T, 1, false>(tmp, U, d, nbr[3], ln[3], v_lds, Vb, salt);
                lds_hop<T, 2, true>(tmp, U, d, nbr[4], ln[4], v_lds, Vb, salt);
                lds_hop<T, 2, false>(tmp, U, d, nbr[5], ln[5], v_lds, Vb, salt);
                lds_hop<T, 3, true>(tmp, U, d, nbr[6], ln[6], v_lds, Vb, salt);
                lds_hop<T, 3, false>(tmp, U, d, nbr[7], ln[7], v_lds, Vb, salt);
                clover_mv<T>(A, d, v[j], w, salt);
#pragma unroll
                for (int k = 0; k < 12; k++) w[k] = csub(csub(w[k], cscale(tmp[k], (T)0.5)), cmul(shift, v[j][k]));
                // two Gram-Schmidt passes against v_0..v_j
#pragma unroll
                for (int pass = 0; pass < 2; pass++) {
                    T part[2 * K];
#pragma unroll
                    for (int i = 0; i < 2 * K; i++) part[i] = 0;
#pragma unroll
                    for (int i = 0; i <= j; i++)
#pragma unroll
                        for (int k = 0; k < 12; k++) {   // conj(v_i) w
                            part[2 * i] += v[i][k].x * w[k].x + v[i][k].y * w[k].y;
                            part[2 * i + 1] += v[i][k].x * w[k].y - v[i][k].y * w[k].x;
                        }
                    block_sum_n<T, 2 * K>(part, red);
#pragma unroll
                    for (int i = 0; i <= j; i++) {
                        const C<T> h = mk<T>(part[2 * i], part[2 * i + 1]);
                        H[i][j] = cadd(H[i][j], h);
#pragma unroll
                        for (int k = 0; k < 12; k++) w[k] = csub(w[k], cmul(h, v[i][k]));
                    }
                }
                T nn[2 * K];
#pragma unroll
                for (int i = 0; i < 2 * K; i++) nn[i] = 0;
#pragma unroll
                for (int k = 0; k < 12; k++) nn[0] += w[k].x * w[k].x + w[k].y * w[k].y;
                block_sum_n<T, 2 * K>(nn, red);
                const T hn = sqrt(nn[0]);
                H[j + 1][j] = mk<T>(hn, 0);
                if (hn == (T)0) {
                    kk = j + 1;   // exact breakdown: the Krylov space is invariant
                } else {
#pragma unroll
                    for (int k = 0; k < 12; k++) v[j + 1][k] = mk<T>(w[k].x / hn, w[k].y / hn);
                    if (j + 1 < K) {
                        // every read of v_lds in this step lies before the barriers of the sums
#pragma unroll
                        for (int k = 0; k < 12; k++) v_lds[k * Vb + l] = v[j + 1][k];
                        __syncthreads();
                    }
                }
            }
        }
        // min || beta e_1 - H y || over the first kk columns: Givens rotations
        // applied to each column as it is reached, then back substitution
        T cs[K];
        C<T> sn[K], gv[K + 1], y[K];
#pragma unroll
        for (int i = 0; i <= K; i++) gv[i] = mk<T>(i == 0 ? beta : (T)0, 0);
#pragma unroll
        for (int j = 0; j < K; j++) {
            if (j < kk) {
#pragma unroll
                for (int i = 0; i < j; i++) {
                    const C<T> a = H[i][j], bb = H[i + 1][j];
                    H[i][j] = cadd(cscale(a, cs[i]), cmul(sn[i], bb));
                    H[i + 1][j] = csub(cscale(bb, cs[i]), cmul(cconj(sn[i]), a));
                }
                const C<T> a = H[j][j], bb = H[j + 1][j];
                const T aa = sqrt(a.x * a.x + a.y * a.y), ab = sqrt(bb.x * bb.x + bb.y * bb.y);
                if (ab == (T)0) {
                    cs[j] = 1;
                    sn[j] = mk<T>(0, 0);
                } else if (aa == (T)0) {
                    cs[j] = 0;
                    sn[j] = mk<T>(1, 0);
                    H[j][j] = bb;
                } else {
                    const T rr = sqrt(aa * aa + ab * ab);
                    const C<T> ph = mk<T>(a.x / aa, a.y / aa);
                    cs[j] = aa / rr;
                    sn[j] = cscale(cmul(ph, cconj(bb)), (T)1 / rr);
                    H[j][j] = cscale(ph, rr);
                }
                H[j + 1][j] = mk<T>(0, 0);
                const C<T> gj = gv[j];
                gv[j] = cscale(gj, cs[j]);
                gv[j + 1] = mk<T>(0, 0);
                gv[j + 1] = csub(gv[j + 1], cmul(cconj(sn[j]), gj));
            }
        }
#pragma unroll
        for (int i = K - 1; i >= 0; i--) {
            y[i] = mk<T>(0, 0);
            if (i < kk) {
                C<T> t = gv[i];
#pragma unroll
                for (int q = i + 1; q < K; q++)
                    if (q < kk) t = csub(t, cmul(H[i][q], y[q]));
                y[i] = cdiv(t, H[i][i]);
            }
        }
#pragma unroll
        for (int k = 0; k < 12; k++) {
            C<T> e = mk<T>(0, 0);
#pragma unroll
            for (int i = 0; i < K; i++)
                if (i < kk) cfma(e, y[i], v[i][k]);
            zs[k] = cadd(zs[k], e);
        }
        store_spinor<T>(zf, d, zs);
    }
}

template <typename T> __global__ void sub_kernel(size_t n, const C<T> *__restrict__ b, C<T> *__restrict__ r) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = csub(b[i], r[i]);
}

template <typename T>
__global__ void add2_kernel(size_t n, const C<T> *__restrict__ e0, const C<T> *__restrict__ e1, C<T> *__restrict__ z) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = cadd(z[i], cadd(e0[i], e1[i]));
}

template <typename T, int K>
void gmres_launch(Ctx *c, int nrhs, int col, const void *U, const void *A, const void *b, void *z, T sre, T sim) {
    const Geom &g = c->g;
    const int nblocks = col ? g.nblocks - g.ncol0 : g.ncol0;
    if (nblocks == 0) return;
    const size_t lds = sizeof(C<T>) * 12 * (size_t)g.Vb + sizeof(T) * 2 * K * (g.Vb / 64);
    sap_gmres_kernel<T, K><<<dim3(nblocks, nrhs), g.Vb, lds, c->stream>>>(
        g, (const C<T> *)U, (const C<T> *)A, (const C<T> *)b, (C<T> *)z, col, sre, sim);
}

// one colour step with GMRES(k) block solves
int gmres_colour(Ctx *c, int prec, int nrhs, int col, int k, double sre, double sim, const void *b, void *z) {
    const bool dp = prec == MGDD_F64;
    const void *U = dp ? c->U64 : c->U32, *A = dp ? c->A64 : c->A32;
#define GL(KK)                                                                                   \
    case KK:                                                                                     \
        if (dp) gmres_launch<double, KK>(c, nrhs, col, U, A, b, z, sre, sim);                    \
        else gmres_launch<float, KK>(c, nrhs, col, U, A, b, z, (float)sre, (float)sim);         \
        break;
    switch (k) {
        GL(1)
        GL(2)
        GL(3)
        default: return fail(c, MGDD_EINVAL, "GMRES block solves take 1 to 3 steps");
    }
#undef GL
    return hip_check(c, hipGetLastError(), "GMRES Schwarz kernel");
}

int colour_step(Ctx *c, int prec, int nrhs, const SchwarzOpts &o, int col, double sre, double sim, const void *b,
                void *z) {
    if (o.gmres) return gmres_colour(c, prec, nrhs, col, o.k, sre, sim, b, z);
    return launch_sap_colour(c, prec, nrhs, col, o.k, sre, sim, b, z);
}

}  // namespace

size_t schwarz_work_bytes(const Ctx *c, int prec, int nrhs, const SchwarzOpts &o) {
    if (!o.additive) return 0;
    return 3 * ((size_t)12 * c->g.V * nrhs * csize(prec) + 256);
}

int launch_schwarz(Ctx *c, int prec, int nrhs, const SchwarzOpts &o, double sre, double sim, const void *b, void *z,
                   void *work) {
    const Geom &g = c->g;
    if (g.Vb < 64 || g.Vb > 256) return fail(c, MGDD_ESHAPE, "the Schwarz kernels need 64 <= block volume <= 256");
    if (o.gmres && (o.k < 1 || o.k > SCHWARZ_GMRES_MAX))
        return fail(c, MGDD_EINVAL, "GMRES block solves take 1 to 3 steps");
    if (!o.additive) {
        if (!o.gmres) return launch_sap(c, prec, nrhs, o.nsweeps, o.k, sre, sim, b, z);
        for (int s = 0; s < o.nsweeps; s++)
            for (int col = 0; col < 2; col++) {
                int rc = colour_step(c, prec, nrhs, o, col, sre, sim, b, z);
                if (rc) return rc;
            }
        return MGDD_OK;
    }
    if (sre != 0.0 || sim != 0.0) return fail(c, MGDD_EINVAL, "additive Schwarz is implemented without a shift");
    if (!work) return fail(c, MGDD_EINVAL, "additive Schwarz needs workspace");
    // r = b - D z once per sweep; each colour's blocks solve for r from a zero
    // start in a field of their own (the kernels form r - D 0 = r on their
    // blocks and never read the other colour's corrections); z += e0 + e1
    const size_t n = (size_t)12 * g.V * nrhs, fb = n * csize(prec);
    char *r = (char *)work, *e0 = r + ((fb + 255) & ~(size_t)255), *e1 = e0 + ((fb + 255) & ~(size_t)255);
    const unsigned nwg = (unsigned)((n + 255) / 256);
    for (int s = 0; s < o.nsweeps; s++) {
        int rc = launch_dirac(c, prec, nrhs, z, r);
        if (rc) return rc;
        if (prec == MGDD_F64) sub_kernel<double><<<nwg, 256, 0, c->stream>>>(n, (const double2 *)b, (double2 *)r);
        else sub_kernel<float><<<nwg, 256, 0, c->stream>>>(n, (const float2 *)b, (float2 *)r);
        rc = hip_check(c, hipMemsetAsync(e0, 0, fb, c->stream), "memset");
        if (!rc) rc = hip_check(c, hipMemsetAsync(e1, 0, fb, c->stream), "memset");
        if (!rc) rc = colour_step(c, prec, nrhs, o, 0, 0.0, 0.0, r, e0);
        if (!rc) rc = colour_step(c, prec, nrhs, o, 1, 0.0, 0.0, r, e1);
        if (rc) return rc;
        if (prec == MGDD_F64)
            add2_kernel<double><<<nwg, 256, 0, c->stream>>>(n, (const double2 *)e0, (const double2 *)e1, (double2 *)z);
        else
            add2_kernel<float><<<nwg, 256, 0, c->stream>>>(n, (const float2 *)e0, (const float2 *)e1, (float2 *)z);
        rc = hip_check(c, hipGetLastError(), "additive Schwarz");
        if (rc) return rc;
    }
    return MGDD_OK;
}

}  // namespace mgdd
