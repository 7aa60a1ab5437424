// Red-Black Schwarz (Section 2, Algorithm 2.1) with minimal-residual block
// solves. One workgroup per lattice block of the current colour, one thread
// per site: the residual r = b - (D - shift) z is formed on the block from
// global memory, then mr steps of MR on I^T (D - shift) I run with the block's
// iterate rho resident in LDS (in-block neighbours read from LDS, hops leaving
// the block dropped), block-wide dot products by wavefront butterflies plus
// one LDS exchange, and finally z += e. Blocks of one colour never touch each
// other, so all of them run at once.
#include "stencil.h"

namespace mgdd {

namespace {

template <typename T> struct Red3 { T a, b, c; };

// deterministic block-wide sum of three values: an XOR butterfly inside each
// 64-lane wave (every lane ends with the same bits), then the per-wave sums
// added in wave order by every thread.
template <typename T> __device__ inline Red3<T> block_sum3(Red3<T> v, T *red) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        v.a += __shfl_xor(v.a, m, 64);
        v.b += __shfl_xor(v.b, m, 64);
        v.c += __shfl_xor(v.c, m, 64);
    }
    int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[3 * w] = v.a;
        red[3 * w + 1] = v.b;
        red[3 * w + 2] = v.c;
    }
    __syncthreads();
    Red3<T> s{0, 0, 0};
    for (int i = 0; i < nw; i++) {
        s.a += red[3 * i];
        s.b += red[3 * i + 1];
        s.c += red[3 * i + 2];
    }
    __syncthreads();
    return s;
}

template <typename T, int MU, bool FWD>
__device__ inline void block_hop(C<T> *acc, const LinkViews<T> &U, int d, int dn, int ln, const C<T> *rho_lds, int Vb,
                                 unsigned salt) {
    if (ln < 0) return;  // neighbour outside the block: dropped in I^T D I
    C<T> psi[12], u[9];
#pragma unroll
    for (int k = 0; k < 12; k++) psi[k] = rho_lds[k * Vb + ln];
    load_link<T, MU>(U, FWD ? d : dn, u, salt);
    hop<T, MU, FWD>(acc, u, psi);
}

template <typename T>
__global__ __launch_bounds__(256) void sap_colour_kernel(Geom g, const C<T> *__restrict__ Up,
                                                         const C<T> *__restrict__ Ap, const C<T> *__restrict__ b,
                                                         C<T> *__restrict__ z, int colour, int mr, T sre, T sim) {
    extern __shared__ unsigned char smem[];
    const int Vb = g.Vb;
    C<T> *rho_lds = (C<T> *)smem;                        // [12][Vb]
    T *red = (T *)(smem + sizeof(C<T>) * 12 * Vb);      // [3 * waves]
    const size_t V = g.V;
    const int pos = (colour ? g.ncol0 : 0) + blockIdx.x;
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
        int bm = 1 << g.lb[mu];
        nbr[2 * mu] = neighbour(g, pos, x, mu, +1);
        nbr[2 * mu + 1] = neighbour(g, pos, x, mu, -1);
        int y[4] = {x[0], x[1], x[2], x[3]};
        // a block that spans the whole lattice in mu keeps its wrap-around hops
        bool wrap = g.nb[mu] == 1;
        y[mu] = x[mu] + 1;
        if (wrap) y[mu] &= bm - 1;
        ln[2 * mu] = (y[mu] < bm) ? local_index(g, y) : -1;
        y[mu] = x[mu] - 1;
        if (wrap) y[mu] = (y[mu] + bm) & (bm - 1);
        ln[2 * mu + 1] = (y[mu] >= 0) ? local_index(g, y) : -1;
    }

    // r = b - (D - shift) z on this site
    C<T> rho[12], e[12], q[12], tmp[12];
    {
        C<T> zs[12];
        hop_sum<T>(U, zf, d, nbr, tmp);
        load_spinor<T>(zf, d, zs);
        clover_mv<T>(A, d, zs, q);
        load_spinor<T>(bf, d, rho);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            C<T> dz = csub(csub(q[k], cscale(tmp[k], (T)0.5)), cmul(shift, zs[k]));
            rho[k] = csub(rho[k], dz);
            e[k] = mk<T>(0, 0);
        }
    }
#pragma unroll
    for (int k = 0; k < 12; k++) rho_lds[k * Vb + l] = rho[k];
    __syncthreads();

    for (int it = 0; it < mr; it++) {
        const unsigned salt = opaque_zero();
        // q = I^T (D - shift) I rho
#pragma unroll
        for (int k = 0; k < 12; k++) tmp[k] = mk<T>(0, 0);
        block_hop<T, 0, true>(tmp, U, d, nbr[0], ln[0], rho_lds, Vb, salt);
        block_hop<T, 0, false>(tmp, U, d, nbr[1], ln[1], rho_lds, Vb, salt);
        block_hop<T, 1, true>(tmp, U, d, nbr[2], ln[2], rho_lds, Vb, salt);
        block_hop<T, 1, false>(tmp, U, d, nbr[3], ln[3], rho_lds, Vb, salt);
        block_hop<T, 2, true>(tmp, U, d, nbr[4], ln[4], rho_lds, Vb, salt);
        block_hop<T, 2, false>(tmp, U, d, nbr[5], ln[5], rho_lds, Vb, salt);
        block_hop<T, 3, true>(tmp, U, d, nbr[6], ln[6], rho_lds, Vb, salt);
        block_hop<T, 3, false>(tmp, U, d, nbr[7], ln[7], rho_lds, Vb, salt);
        clover_mv<T>(A, d, rho, q, salt);
        Red3<T> part{0, 0, 0};
#pragma unroll
        for (int k = 0; k < 12; k++) {
            q[k] = csub(csub(q[k], cscale(tmp[k], (T)0.5)), cmul(shift, rho[k]));
            part.a += q[k].x * q[k].x + q[k].y * q[k].y;
            part.b += q[k].x * rho[k].x + q[k].y * rho[k].y;   // conj(q) rho
            part.c += q[k].x * rho[k].y - q[k].y * rho[k].x;
        }
        Red3<T> s = block_sum3<T>(part, red);
        if (s.a == (T)0) break;
        C<T> alpha = mk<T>(s.b / s.a, s.c / s.a);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cfma(e[k], alpha, rho[k]);
            rho[k] = csub(rho[k], cmul(alpha, q[k]));
        }
        if (it + 1 < mr) {
#pragma unroll
            for (int k = 0; k < 12; k++) rho_lds[k * Vb + l] = rho[k];
            __syncthreads();
        }
    }
    C<T> zs[12];
    load_spinor<T>(zf, d, zs);
#pragma unroll
    for (int k = 0; k < 12; k++) zs[k] = cadd(zs[k], e[k]);
    store_spinor<T>(zf, d, zs);
}

}  // namespace

int launch_sap(Ctx *c, int prec, int nrhs, int nsweeps, int mr, double sre, double sim, const void *b, void *z) {
    const Geom &g = c->g;
    if (g.Vb < 64 || g.Vb > 256)
        return fail(c, MGDD_ESHAPE, "the Schwarz kernel needs 64 <= block volume <= 256");
    size_t lds = (prec == MGDD_F64 ? 16 : 8) * 12 * (size_t)g.Vb + (prec == MGDD_F64 ? 8 : 4) * 3 * (g.Vb / 64);
    for (int s = 0; s < nsweeps; s++)
        for (int col = 0; col < 2; col++) {
            int nblocks = col ? g.nblocks - g.ncol0 : g.ncol0;
            if (nblocks == 0) continue;
            dim3 grid(nblocks, nrhs);
            if (prec == MGDD_F64)
                sap_colour_kernel<double><<<grid, g.Vb, lds, c->stream>>>(g, (const double2 *)c->U64,
                                                                          (const double2 *)c->A64, (const double2 *)b,
                                                                          (double2 *)z, col, mr, sre, sim);
            else
                sap_colour_kernel<float><<<grid, g.Vb, lds, c->stream>>>(g, (const float2 *)c->U32,
                                                                         (const float2 *)c->A32, (const float2 *)b,
                                                                         (float2 *)z, col, mr, (float)sre, (float)sim);
            int rc = hip_check(c, hipGetLastError(), "sap kernel");
            if (rc) return rc;
        }
    return MGDD_OK;
}

}  // namespace mgdd
