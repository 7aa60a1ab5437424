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

// v from lane (lane ^ X) of the same quad, X = 1 or 2: a DPP quad permutation
// ([1,0,3,2] or [2,3,0,1]) for FP32, a cross-lane shuffle for FP64
template <int X> __device__ inline float quad_xor(float v) {
    constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
}
template <int X> __device__ inline double quad_xor(double v) { return __shfl_xor(v, X, 64); }

// deterministic block-wide sum of three values: an XOR butterfly inside each
// 64-lane wave (every lane ends with the same bits), then the per-wave sums
// added in wave order by every thread.
// TRAIL = false leaves out the closing barrier: for callers that pass a
// barrier of their own before red is written again
template <typename T, bool TRAIL = true> __device__ inline Red3<T> block_sum3(Red3<T> v, T *red) {
#pragma unroll
    for (int m = 32; m >= 4; m >>= 1) {
        v.a += __shfl_xor(v.a, m, 64);
        v.b += __shfl_xor(v.b, m, 64);
        v.c += __shfl_xor(v.c, m, 64);
    }
    v.a += quad_xor<2>(v.a);
    v.b += quad_xor<2>(v.b);
    v.c += quad_xor<2>(v.c);
    v.a += quad_xor<1>(v.a);
    v.b += quad_xor<1>(v.b);
    v.c += quad_xor<1>(v.c);
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
    if (TRAIL) __syncthreads();
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

// ---------------------------------------------------------------- four lanes per site
//
// Lane m = threadIdx & 3 of a site handles the two hops along direction m,
// the rows of the clover term that belong to spin m, and owns spin m
// (components 3m..3m+2) of r, rho, e and q. The hop partial sums of the four
// lanes are combined by a two-step reduce-scatter over lane pairs (xor 2,
// then xor 1), so that every spin's sum is formed by one lane in a fixed
// order. The spin projection is branch-free: in the chiral basis
// gamma_mu = [[0, B],[B^H, 0]] with (B l)_s = beta_s l_pi(s), pi a swap for
// x, y and the identity for z, t, and beta_s in {+-1, +-i}.
struct Proj {
    bool swap;
    float2 b0, b1;  // beta_0, beta_1 (exact in any precision)
};

// beta_0 = -i (x, z), -1 (y, t); beta_1 = -i (x), +1 (y), +i (z), -1 (t);
// written as arithmetic of mu (a table of constants indexed by a lane value
// would be placed in scratch memory)
__device__ inline Proj proj_of(int mu) {
    Proj p;
    const int odd = mu & 1, hi = (mu >> 1) & 1;
    p.swap = mu < 2;
    p.b0 = make_float2(odd ? -1.f : 0.f, odd ? 0.f : -1.f);
    p.b1 = make_float2(odd ? (float)(1 - 2 * hi) : 0.f, odd ? 0.f : (float)(2 * hi - 1));
    return p;
}

template <typename T> __device__ inline C<T> cmulp(float2 beta, C<T> v) {
    return mk<T>((T)beta.x * v.x - (T)beta.y * v.y, (T)beta.x * v.y + (T)beta.y * v.x);
}
template <typename T> __device__ inline C<T> cmulpc(float2 beta, C<T> v) {  // conj(beta) v
    return mk<T>((T)beta.x * v.x + (T)beta.y * v.y, (T)beta.x * v.y - (T)beta.y * v.x);
}

// acc += (1 -+ gamma_mu) U^(H) psi for a runtime direction (FWD: 1 - gamma, U)
template <typename T, bool FWD>
__device__ inline void hop_rt(C<T> *acc, const Proj &p, const C<T> *u, const C<T> *psi) {
    C<T> h0[3], h1[3], w0[3], w1[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        C<T> l0 = psi[6 + a], l1 = psi[9 + a];
        C<T> bl0 = cmulp<T>(p.b0, p.swap ? l1 : l0);
        C<T> bl1 = cmulp<T>(p.b1, p.swap ? l0 : l1);
        h0[a] = FWD ? csub(psi[a], bl0) : cadd(psi[a], bl0);
        h1[a] = FWD ? csub(psi[3 + a], bl1) : cadd(psi[3 + a], bl1);
    }
    su3_mv<T, !FWD>(u, h0, w0);
    su3_mv<T, !FWD>(u, h1, w1);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc[a] = cadd(acc[a], w0[a]);
        acc[3 + a] = cadd(acc[3 + a], w1[a]);
        // (B^H w)_s = conj(beta_pi(s)) w_pi(s); forward subtracts, backward adds
        C<T> bw0 = p.swap ? cmulpc<T>(p.b1, w1[a]) : cmulpc<T>(p.b0, w0[a]);
        C<T> bw1 = p.swap ? cmulpc<T>(p.b0, w0[a]) : cmulpc<T>(p.b1, w1[a]);
        acc[6 + a] = FWD ? csub(acc[6 + a], bw0) : cadd(acc[6 + a], bw0);
        acc[9 + a] = FWD ? csub(acc[9 + a], bw1) : cadd(acc[9 + a], bw1);
    }
}

// Per-lane constants of the spin projection along the lane's direction, for
// the hops inside the block (rho in LDS). With beta in {+-1, +-i},
// beta v = (sx * v'.x, sy * v'.y) where v' = v with real and imaginary parts
// exchanged when beta is imaginary (directions x and z): that exchange is
// done by the LDS addresses (the two halves of a complex are read as two
// floats), and the spin permutation pi (x, y) too, so that a projected
// component costs two FMAs.
struct ProjLds {
    int ox, oy;          // float offsets of the parts read as (x, y): (1, 0) when exchanged
    int src[2];          // LDS component block of l_pi(s): 6 + 3 pi(s)
    float sx[2], sy[2];  // signs of beta_s
    float cx[2], cy[2];  // signs of conj(beta_pi(t)) for the lower spins t
    bool swp, rot;
};

__device__ inline ProjLds proj_lds_of(int mu, const Proj &p) {
    ProjLds q;
    q.rot = !(mu & 1);
    q.swp = p.swap;
    q.ox = q.rot ? 1 : 0;
    q.oy = 1 - q.ox;
    const float2 bs[2] = {p.b0, p.b1};
#pragma unroll
    for (int s = 0; s < 2; s++) {
        q.src[s] = 6 + 3 * (q.swp ? 1 - s : s);
        q.sx[s] = q.rot ? -bs[s].y : bs[s].x;
        q.sy[s] = q.rot ? bs[s].y : bs[s].x;
    }
#pragma unroll
    for (int t = 0; t < 2; t++) {
        const float2 bp = q.swp ? bs[1 - t] : bs[t];   // beta_pi(t), conjugated below
        q.cx[t] = q.rot ? bp.y : bp.x;
        q.cy[t] = q.rot ? -bp.y : bp.x;
    }
    return q;
}

// h = (1 -+ gamma_mu) psi projected to its upper half (FWD: 1 - gamma):
// h_s = u_s -+ beta_s l_pi(s), psi read from the LDS field rho (component
// stride RS) at site i
template <bool FWD>
__device__ inline void project_lds(const float *rf, int RS, int i, const ProjLds &q, float2 *h) {
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float2 u = ((const float2 *)rf)[(3 * s + a) * RS + i];
            const int li = ((q.src[s] + a) * RS + i) * 2;
            const float lx = rf[li + q.ox], ly = rf[li + q.oy];
            h[3 * s + a] = FWD ? make_float2(u.x - q.sx[s] * lx, u.y - q.sy[s] * ly)
                               : make_float2(u.x + q.sx[s] * lx, u.y + q.sy[s] * ly);
        }
}

// sum of a 12-component partial over the 4 lanes of a site, returned for
// spin m only (3 components) in out
template <typename T> __device__ inline void reduce_scatter4(const C<T> *acc, int m, C<T> *out) {
    C<T> kept[2][3];
    const bool hi = m & 2;
#pragma unroll
    for (int k = 0; k < 2; k++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            C<T> mine = hi ? acc[(2 + k) * 3 + c] : acc[k * 3 + c];
            C<T> send = hi ? acc[k * 3 + c] : acc[(2 + k) * 3 + c];
            C<T> recv = mk<T>(quad_xor<2>(send.x), quad_xor<2>(send.y));
            kept[k][c] = cadd(mine, recv);
        }
    const bool odd = m & 1;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        C<T> mine = odd ? kept[1][c] : kept[0][c];
        C<T> send = odd ? kept[0][c] : kept[1][c];
        C<T> recv = mk<T>(quad_xor<1>(send.x), quad_xor<1>(send.y));
        out[c] = cadd(mine, recv);
    }
}

// rows of spin m of the clover block of chirality m/2: y = A x, x = the 6
// components of that chirality
template <typename T>
__device__ inline void clover_rows(const FieldView<T> &A, unsigned aoff, int d, int m, const C<T> *x, C<T> *y,
                                   unsigned salt) {
    T a[36];
#pragma unroll
    for (int k = 0; k < 18; k++) {
        C<T> v = A.ld_lane(k, d, aoff, salt);
        a[2 * k] = v.x;
        a[2 * k + 1] = v.y;
    }
    // rows r0..r0+2 with r0 = 3 (m & 1): every entry is picked by a select
    // between the two compile-time candidates, so no array index depends on
    // the lane
    const bool up = m & 1;
#pragma unroll
    for (int rr = 0; rr < 3; rr++) {
        C<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int j = 0; j < 6; j++) {
            C<T> e0, e1;
            {
                const int i = rr;
                if (j == i) e0 = mk<T>(a[i], (T)0);
                else if (i < j) e0 = mk<T>(a[hpack(i, j)], a[hpack(i, j) + 1]);
                else e0 = mk<T>(a[hpack(j, i)], -a[hpack(j, i) + 1]);
            }
            {
                const int i = 3 + rr;
                if (j == i) e1 = mk<T>(a[i], (T)0);
                else if (i < j) e1 = mk<T>(a[hpack(i, j)], a[hpack(i, j) + 1]);
                else e1 = mk<T>(a[hpack(j, i)], -a[hpack(j, i) + 1]);
            }
            cfma(acc, up ? e1 : e0, x[j]);
        }
        y[rr] = acc;
    }
}

// The forward links of the block's sites (4 x 9 complex per site) are staged
// in LDS once, next to rho: every hop inside the block (forward: the site's
// own link; backward: the neighbour's forward link) reads its link from LDS.
// With links + rho resident a workgroup takes about 100 KB of LDS, so one
// block runs per CU and the clover term re-read at every MR step stays in
// the XCD's L2.
template <typename T, int VB>
__global__ __launch_bounds__(1024) void sap4_kernel(Geom g, const C<T> *__restrict__ Up, const C<T> *__restrict__ Ap,
                                                    const C<T> *__restrict__ b, C<T> *__restrict__ z, int colour,
                                                    int mr, T sre, T sim) {
    extern __shared__ unsigned char smem[];
    // the block volume as a compile-time constant: every LDS offset of a
    // component or link entry becomes an immediate of the LDS instruction
    constexpr int Vb = VB;
    // component strides padded by 4 complex numbers, so that the four lanes
    // of a site (different components or directions, same site) fall in
    // different LDS banks
    const int RS = Vb + 4, MS = 9 * Vb + 4;
    C<T> *rho_lds = (C<T> *)smem;                        // [12][RS]
    C<T> *lnk_lds = rho_lds + 12 * RS;                   // [4][MS]: direction m, entry k at m MS + k Vb
    T *red = (T *)(lnk_lds + 4 * MS);                    // [3 * waves]
    const size_t V = g.V;
    const int pos = (colour ? g.ncol0 : 0) + xcd_block(gridDim.x);
    const int m = threadIdx.x & 3, l = threadIdx.x >> 2;
    const int d = (pos << g.lgVb) + l;
    const size_t roff = (size_t)blockIdx.y * 12 * V;
    // one uniform descriptor for all links and one for the clover term; the
    // lane's direction / chirality enters through the 32-bit vector offset
    const FieldView<T> Uall(Up, V, 36), Aall(Ap, V, 36);
    const unsigned uoff = (unsigned)m * 9u * Uall.cs, aoff = (unsigned)(m >> 1) * 18u * Aall.cs;
    const FieldView<T> bf(b + roff, V, 12), zf(z + roff, V, 12);
    const C<T> shift = mk<T>(sre, sim);
    const Proj pr = proj_of(m);

    // neighbours along the lane's direction m, with every array index a
    // compile-time constant (a lane-dependent index into a private array
    // would put the array in scratch memory)
    int x[4];
    local_coords(g, l, x);
    int nf, nbk, lnf, lnb;
    {
        int xm = 0, lbm = 0, nbm = 0;
#pragma unroll
        for (int mu = 0; mu < 4; mu++)
            if (mu == m) { xm = x[mu]; lbm = g.lb[mu]; nbm = g.nb[mu]; }
        const int bm = 1 << lbm;
        const bool wrap = nbm == 1;
        int yf = xm + 1, yb = xm - 1;
        const bool fin = yf < bm, bin = yb >= 0;       // stays in the block without wrapping
        const int yfw = yf & (bm - 1), ybw = (yb + bm) & (bm - 1);
        int xf[4], xb[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            xf[mu] = mu == m ? yfw : x[mu];
            xb[mu] = mu == m ? ybw : x[mu];
        }
        const int lf = local_index(g, xf), lb = local_index(g, xb);
        lnf = (fin || wrap) ? lf : -1;
        lnb = (bin || wrap) ? lb : -1;
        const int pf = fin ? pos : g.blk_nbr[pos * 8 + 2 * m];
        const int pb = bin ? pos : g.blk_nbr[pos * 8 + 2 * m + 1];
        nf = (pf << g.lgVb) + lf;
        nbk = (pb << g.lgVb) + lb;
    }
    const int ch = m >> 1;  // chirality of spin m

    // r = b - (D - shift) z, spin m. The site's forward link is loaded and
    // staged in LDS, and both neighbour spinors are requested before the
    // barrier that publishes the links; the backward hop then takes its link
    // from LDS when the neighbour is in the block (each link leaves memory once).
    C<T> rho[3], e[3], q[3];
    {
        C<T> acc[12], psi[12], psb[12], u[9];
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = mk<T>(0, 0);
#pragma unroll
        for (int k = 0; k < 9; k++) u[k] = Uall.ld_lane(k, d, uoff);
        load_spinor<T>(zf, nf, psi);
        load_spinor<T>(zf, nbk, psb);
#pragma unroll
        for (int k = 0; k < 9; k++) lnk_lds[m * MS + k * Vb + l] = u[k];
        __syncthreads();
        hop_rt<T, true>(acc, pr, u, psi);
        if (lnb >= 0) {
#pragma unroll
            for (int k = 0; k < 9; k++) u[k] = lnk_lds[m * MS + k * Vb + lnb];
        } else {
#pragma unroll
            for (int k = 0; k < 9; k++) u[k] = Uall.ld_lane(k, nbk, uoff);
        }
        hop_rt<T, false>(acc, pr, u, psb);
        C<T> hs[3], zc[6], az[3], zs[3], bs[3];
        reduce_scatter4<T>(acc, m, hs);
#pragma unroll
        for (int c = 0; c < 6; c++) zc[c] = zf.ld_lane(c, d, 6u * ch * zf.cs);
        clover_rows<T>(Aall, aoff, d, m, zc, az, 0);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            zs[c] = zc[(m & 1) * 3 + c];
            bs[c] = bf.ld_lane(c, d, 3u * m * bf.cs);
            C<T> dz = csub(csub(az[c], cscale(hs[c], (T)0.5)), cmul(shift, zs[c]));
            rho[c] = csub(bs[c], dz);
            e[c] = mk<T>(0, 0);
            rho_lds[(3 * m + c) * RS + l] = rho[c];
        }
    }
    __syncthreads();

    const float *rf = (const float *)rho_lds;
    const ProjLds pq = proj_lds_of(m, pr);
    for (int it = 0; it < mr; it++) {
        const unsigned salt = opaque_zero();
        // the two hops along the lane's direction: w_f = U h_f, w_b = U^H h_b
        // (upper halves); the lower halves are -B^H w_f + B^H w_b = B^H (w_b - w_f)
        C<T> acc[12], h[6], u[9], wf[6], wb[6];
#pragma unroll
        for (int k = 0; k < 6; k++) wf[k] = wb[k] = mk<T>(0, 0);
        if (lnf >= 0) {
            project_lds<true>(rf, RS, lnf, pq, h);
#pragma unroll
            for (int k = 0; k < 9; k++) u[k] = lnk_lds[m * MS + k * Vb + l];
            su3_mv<T, false>(u, h, wf);
            su3_mv<T, false>(u, h + 3, wf + 3);
        }
        if (lnb >= 0) {
            project_lds<false>(rf, RS, lnb, pq, h);
#pragma unroll
            for (int k = 0; k < 9; k++) u[k] = lnk_lds[m * MS + k * Vb + lnb];
            su3_mv<T, true>(u, h, wb);
            su3_mv<T, true>(u, h + 3, wb + 3);
        }
#pragma unroll
        for (int k = 0; k < 6; k++) acc[k] = cadd(wf[k], wb[k]);
#pragma unroll
        for (int t = 0; t < 2; t++)
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const C<T> d0 = csub(wb[a], wf[a]), d1 = csub(wb[3 + a], wf[3 + a]);
                const C<T> src = pq.swp ? (t ? d0 : d1) : (t ? d1 : d0);
                acc[6 + 3 * t + a] = mk<T>(pq.cx[t] * (pq.rot ? src.y : src.x), pq.cy[t] * (pq.rot ? src.x : src.y));
            }
        C<T> hs[3], xc[6], ax[3];
        reduce_scatter4<T>(acc, m, hs);
#pragma unroll
        for (int c = 0; c < 6; c++) xc[c] = rho_lds[(6 * ch + c) * RS + l];
        clover_rows<T>(Aall, aoff, d, m, xc, ax, salt);
        Red3<T> part{0, 0, 0};
#pragma unroll
        for (int c = 0; c < 3; c++) {
            q[c] = csub(csub(ax[c], cscale(hs[c], (T)0.5)), cmul(shift, rho[c]));
            part.a += q[c].x * q[c].x + q[c].y * q[c].y;
            part.b += q[c].x * rho[c].x + q[c].y * rho[c].y;   // conj(q) rho
            part.c += q[c].x * rho[c].y - q[c].y * rho[c].x;
        }
        // the barrier after the rho update below (or the end of the loop) comes
        // before any thread writes red again
        Red3<T> s = block_sum3<T, false>(part, red);
        if (s.a == (T)0) break;
        const T inv = (T)1 / s.a;
        C<T> alpha = mk<T>(s.b * inv, s.c * inv);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            cfma(e[c], alpha, rho[c]);
            rho[c] = csub(rho[c], cmul(alpha, q[c]));
        }
        if (it + 1 < mr) {
#pragma unroll
            for (int c = 0; c < 3; c++) rho_lds[(3 * m + c) * RS + l] = rho[c];
            __syncthreads();
        }
    }
#pragma unroll
    for (int c = 0; c < 3; c++) zf.st_lane(c, d, 3u * m * zf.cs, cadd(zf.ld_lane(c, d, 3u * m * zf.cs), e[c]));
}

// ---------------------------------------------------------------- two lanes per site
//
// Lane h = threadIdx & 1 of a site owns chirality h (spins 2h and 2h + 1:
// components 6h .. 6h + 5) of r, rho, e and q, applies that chirality's 6 x 6
// block of the clover term, and does the hops along directions 2h and 2h + 1
// (x and y for h = 0, z and t for h = 1). Its hop partial sum has all 12
// components; one exchange with the other lane of the site (a DPP quad
// permutation) leaves each lane the sum for its chirality. The links are
// special unitary (checked at ingest), so the block's forward links are
// staged in LDS as their first two rows and row 2 is rebuilt where it is used:
// rho and the links then take about 73 KB of LDS for a 4^4 block, and with at
// most 128 VGPRs per lane two blocks run on one CU at a time, one block's
// memory phase overlapping the other's MR steps.
//
// The spin projection has no lane-dependent branch: with gamma_mu =
// [[0, B_mu], [B_mu^H, 0]] and (B l)_s = beta_s l_pi(s), the lane's first
// direction (x or z) has beta = (-i, -i sig) and its second (y or t)
// beta = (-1, sig), sig = +1 for h = 0 and -1 for h = 1; pi swaps the two
// spins for x and y (h = 0) and is the identity for z and t (h = 1). The
// swap enters through LDS addresses and two selects per component.

// h = (1 -+ gamma) psi projected to its upper half (FWD: 1 - gamma) for the
// lane's first (FIRST) or second direction; u: upper spins of psi, la / lb:
// the lower spins l_pi(0), l_pi(1)
template <bool FIRST, bool FWD>
__device__ inline void project2(const float2 *u, const float2 *la, const float2 *lb, float sig, float2 *h) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const float2 u0 = u[a], u1 = u[3 + a], p = la[a], q = lb[a];
        if (FIRST) {          // beta l = (-i l_a, -i sig l_b)
            h[a] = FWD ? make_float2(u0.x - p.y, u0.y + p.x) : make_float2(u0.x + p.y, u0.y - p.x);
            h[3 + a] = FWD ? make_float2(fmaf(-sig, q.y, u1.x), fmaf(sig, q.x, u1.y))
                           : make_float2(fmaf(sig, q.y, u1.x), fmaf(-sig, q.x, u1.y));
        } else {              // beta l = (-l_a, sig l_b)
            h[a] = FWD ? make_float2(u0.x + p.x, u0.y + p.y) : make_float2(u0.x - p.x, u0.y - p.y);
            h[3 + a] = FWD ? make_float2(fmaf(-sig, q.x, u1.x), fmaf(-sig, q.y, u1.y))
                           : make_float2(fmaf(sig, q.x, u1.x), fmaf(sig, q.y, u1.y));
        }
    }
}

// w = U h (FWD) or U^H h on the two colour vectors of h, then up += w and
// L_t -+= conj(beta_t) w_t (the lower spins, kept in pi order: lower spin s
// receives L_pi(s)); forward hops subtract, backward hops add
template <bool FIRST, bool FWD>
__device__ inline void accumulate_hop(const float2 *u, const float2 *h, float sig, float2 *up, float2 *L) {
    float2 w[6];
    su3_mv<float, !FWD>(u, h, w);
    su3_mv<float, !FWD>(u, h + 3, w + 3);
#pragma unroll
    for (int a = 0; a < 6; a++) up[a] = cadd(up[a], w[a]);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const float2 w0 = w[a], w1 = w[3 + a];
        // FIRST: conj(beta) = (i, i sig); second: (-1, sig)
        const float2 c0 = FIRST ? make_float2(-w0.y, w0.x) : make_float2(-w0.x, -w0.y);
        const float2 c1 = FIRST ? make_float2(-sig * w1.y, sig * w1.x) : make_float2(sig * w1.x, sig * w1.y);
        L[a] = FWD ? csub(L[a], c0) : cadd(L[a], c0);
        L[3 + a] = FWD ? csub(L[3 + a], c1) : cadd(L[3 + a], c1);
    }
}

// rows 0 and 1 of a link from LDS ([6][LS] entries of its direction), row 2 rebuilt
template <int LS> __device__ inline void link_from_lds(const float2 *lk, int site, float sign, float2 *u) {
#pragma unroll
    for (int k = 0; k < 6; k++) u[k] = lk[k * LS + site];
    su3_row2<float>(u, sign);
}

// the spinor at `site` of a field in LDS ([12][RS]): upper spins, and the
// lower spins in pi order (component blocks src0, src1 chosen per lane)
template <int RS>
__device__ inline void spinor_from_lds(const float2 *rl, int site, int src0, int src1, float2 *u, float2 *la, float2 *lb) {
#pragma unroll
    for (int c = 0; c < 6; c++) u[c] = rl[c * RS + site];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        la[a] = rl[(src0 + a) * RS + site];
        lb[a] = rl[(src1 + a) * RS + site];
    }
}

// the same from a field in memory (device site dn; FV: FP32 or half storage)
template <typename FV>
__device__ inline void spinor_from_field(const FV &f, int dn, int src0, int src1, float2 *u, float2 *la,
                                         float2 *lb) {
#pragma unroll
    for (int c = 0; c < 6; c++) u[c] = f.ld(c, dn);
    // src0, src1 in {6, 9}: the lane's choice enters through the vector offset
#pragma unroll
    for (int a = 0; a < 3; a++) {
        la[a] = f.ld_lane(a, dn, (unsigned)src0 * f.cs);
        lb[a] = f.ld_lane(a, dn, (unsigned)src1 * f.cs);
    }
}

// c ? a : b on values (a select of two array elements' addresses would keep
// the arrays in scratch memory)
__device__ inline float2 sel2(bool c, float2 a, float2 b) { return make_float2(c ? a.x : b.x, c ? a.y : b.y); }

// the lane's chirality of the hop sum: lane 0 keeps the upper spins and sends
// its lower sums (kept in swapped order) to lane 1; lane 1 keeps the lower
// spins and sends its upper sums
__device__ inline void exchange_chirality(bool h, const float2 *up, const float2 *L, float2 *hs) {
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const int kp = k < 3 ? k + 3 : k - 3;
        const float2 send = sel2(h, up[k], L[kp]);
        const float2 mine = sel2(h, L[k], up[k]);
        hs[k] = make_float2(mine.x + quad_xor<1>(send.x), mine.y + quad_xor<1>(send.y));
    }
}

// the lane's hops whose neighbour lies in the block: the neighbour's spinor
// from the LDS field fl ([12][RS]), links from LDS (rows 0 and 1 of each
// site's forward links, [4][6][LS]); up / L accumulate as in accumulate_hop
template <int RS, int LS>
__device__ inline void block_hops(const float2 *fl, const float2 *lnk, int h, int l, const int *lnf, const int *lnb,
                                  int src0, int src1, float sig, float sgf, float sgb, float2 *up, float2 *L) {
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const float2 *lk = lnk + (2 * h + i) * 6 * LS;
        const float sf = i ? sgf : 1.f, sb = i ? sgb : 1.f;
        float2 u[9], ps[6], la[3], lb[3], hh[6];
        if (lnf[i] >= 0) {
            spinor_from_lds<RS>(fl, lnf[i], src0, src1, ps, la, lb);
            link_from_lds<LS>(lk, l, sf, u);
            if (i == 0) {
                project2<true, true>(ps, la, lb, sig, hh);
                accumulate_hop<true, true>(u, hh, sig, up, L);
            } else {
                project2<false, true>(ps, la, lb, sig, hh);
                accumulate_hop<false, true>(u, hh, sig, up, L);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (lnb[i] >= 0) {
            spinor_from_lds<RS>(fl, lnb[i], src0, src1, ps, la, lb);
            link_from_lds<LS>(lk, lnb[i], sb, u);
            if (i == 0) {
                project2<true, false>(ps, la, lb, sig, hh);
                accumulate_hop<true, false>(u, hh, sig, up, L);
            } else {
                project2<false, false>(ps, la, lb, sig, hh);
                accumulate_hop<false, false>(u, hh, sig, up, L);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// S: storage of the spinor fields b and z (float, or _Float16: half-precision
// storage with the same FP32 arithmetic, z rounded once when it is stored)
template <int VB, typename S = float>
__global__ __launch_bounds__(2 * VB) __attribute__((amdgpu_waves_per_eu(4))) void sapc_kernel(
    Geom g, const float2 *__restrict__ Up, const float2 *__restrict__ Ap, const void *__restrict__ b,
    void *__restrict__ z, int colour, int mr, float sre, float sim, int antiperiodic) {
    using FV = typename F32Store<S>::view;
    extern __shared__ unsigned char smem[];
    constexpr int Vb = VB, RS = VB + 4, LS = VB + 2;
    float2 *rho_lds = (float2 *)smem;                   // [12][RS]
    float2 *lnk = rho_lds + 12 * RS;                    // [4][6][LS]: rows 0, 1 of each site's forward links
    float *red = (float *)(lnk + 24 * LS);              // [3 * waves]
    const size_t V = g.V;
    const int pos = (colour ? g.ncol0 : 0) + xcd_block(gridDim.x);
    const int h = threadIdx.x & 1, l = threadIdx.x >> 1;
    const int d = (pos << g.lgVb) + l;
    const size_t roff = (size_t)blockIdx.y * 12 * V * F32Store<S>::ESZ;   // bytes
    const FieldView<float> Uall(Up, V, 36), Aall(Ap, V, 36);
    const FV bf((const float2 *)((const char *)b + roff), V, 12), zf((const float2 *)((const char *)z + roff), V, 12);
    const unsigned aoff = (unsigned)h * 18u * Aall.cs, coff = (unsigned)h * 6u * zf.cs;
    const bool swp = h == 0;
    const float sig = h ? -1.f : 1.f;
    const int src0 = swp ? 9 : 6, src1 = swp ? 6 : 9;   // LDS component blocks of l_pi(0), l_pi(1)
    const float2 shift = make_float2(sre, sim);

    // neighbours along the lane's two directions mu = 2h + i (every private
    // array index a compile-time constant)
    int x[4];
    local_coords(g, l, x);
    int nf[2], nbk[2], lnf[2], lnb[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const int m = 2 * h + i;
        int xm = 0, lbm = 0, nbm = 0;
#pragma unroll
        for (int mu = 0; mu < 4; mu++)
            if (mu == m) { xm = x[mu]; lbm = g.lb[mu]; nbm = g.nb[mu]; }
        const int bm = 1 << lbm;
        const bool wrap = nbm == 1;
        const int yf = xm + 1, yb = xm - 1;
        const bool fin = yf < bm, bin = yb >= 0;
        int xf[4], xb[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            xf[mu] = mu == m ? (yf & (bm - 1)) : x[mu];
            xb[mu] = mu == m ? ((yb + bm) & (bm - 1)) : x[mu];
        }
        const int lf = local_index(g, xf), lbk = local_index(g, xb);
        lnf[i] = (fin || wrap) ? lf : -1;
        lnb[i] = (bin || wrap) ? lbk : -1;
        const int pf = fin ? pos : g.blk_nbr[pos * 8 + 2 * m];
        const int pb = bin ? pos : g.blk_nbr[pos * 8 + 2 * m + 1];
        nf[i] = (pf << g.lgVb) + lf;
        nbk[i] = (pb << g.lgVb) + lbk;
    }
    // signs of the rebuilt time links (second direction of lane 1): -1 on the
    // link across the antiperiodic time boundary
    float sgf = 1.f, sgb = 1.f;
    {
        const int t = (int)((g.blk_coord[pos] >> 24) << g.lb[3]) + x[3];
        if (antiperiodic && h == 1 && t == g.L[3] - 1) sgf = -1.f;
        if (antiperiodic && h == 1 && t == 0) sgb = -1.f;
    }

    // stage rows 0 and 1 of the site's forward links of the lane's
    // directions, and the lane's chirality of z, in LDS. The data this
    // workgroup reads or writes once (links, z, b) goes through the caches
    // with the non-temporal policy, so that the clover rows, which every MR
    // step reads again, stay in L2 (20 % fewer bytes from memory)
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const unsigned uo = (unsigned)(2 * h + i) * 9u * Uall.cs;
        float2 *lk = lnk + (2 * h + i) * 6 * LS;
#pragma unroll
        for (int k = 0; k < 6; k++) lk[k * LS + l] = Uall.template ld_lane<true>(k, d, uo);
    }
#pragma unroll
    for (int c = 0; c < 6; c++) rho_lds[(6 * h + c) * RS + l] = zf.template ld_lane<true>(c, d, coff);
    __syncthreads();

    // r = b - (D - shift) z on the lane's chirality: the hops inside the
    // block from LDS, then those that leave it (spinor and, backward, link
    // from memory)
    float2 rho[6], e[6];
    {
        // half of the clover rows before the hops, as in the MR steps below
        float2 ap0[18];
#pragma unroll
        for (int k = 0; k < 9; k++) ap0[k] = Aall.ld_lane(k, d, aoff);
        float2 up[6], L[6];
#pragma unroll
        for (int k = 0; k < 6; k++) up[k] = L[k] = make_float2(0.f, 0.f);
        block_hops<RS, LS>(rho_lds, lnk, h, l, lnf, lnb, src0, src1, sig, sgf, sgb, up, L);
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const float sf = i ? sgf : 1.f, sb = i ? sgb : 1.f;
            float2 u[9], ps[6], la[3], lb[3], hh[6];
            if (lnf[i] < 0) {
                spinor_from_field(zf, nf[i], src0, src1, ps, la, lb);
                link_from_lds<LS>(lnk + (2 * h + i) * 6 * LS, l, sf, u);
                if (i == 0) {
                    project2<true, true>(ps, la, lb, sig, hh);
                    accumulate_hop<true, true>(u, hh, sig, up, L);
                } else {
                    project2<false, true>(ps, la, lb, sig, hh);
                    accumulate_hop<false, true>(u, hh, sig, up, L);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            if (lnb[i] < 0) {
                spinor_from_field(zf, nbk[i], src0, src1, ps, la, lb);
                const unsigned uo = (unsigned)(2 * h + i) * 9u * Uall.cs;
#pragma unroll
                for (int k = 0; k < 6; k++) u[k] = Uall.ld_lane(k, nbk[i], uo);
                su3_row2<float>(u, sb);
                if (i == 0) {
                    project2<true, false>(ps, la, lb, sig, hh);
                    accumulate_hop<true, false>(u, hh, sig, up, L);
                } else {
                    project2<false, false>(ps, la, lb, sig, hh);
                    accumulate_hop<false, false>(u, hh, sig, up, L);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        float2 hs[6], zc[6], az[6];
        exchange_chirality(h, up, L, hs);
#pragma unroll
        for (int c = 0; c < 6; c++) zc[c] = rho_lds[(6 * h + c) * RS + l];
#pragma unroll
        for (int k = 9; k < 18; k++) ap0[k] = Aall.ld_lane(k, d, aoff);
        herm6_mv<float>(ap0, zc, az);
#pragma unroll
        for (int c = 0; c < 6; c++) {
            const float2 bs = bf.template ld_lane<true>(c, d, coff);
            const float2 dz = csub(csub(az[c], cscale(hs[c], 0.5f)), cmul(shift, zc[c]));
            rho[c] = csub(bs, dz);
            e[c] = make_float2(0.f, 0.f);
        }
    }
    // every lane has read z from LDS before rho replaces it
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 6; c++) rho_lds[(6 * h + c) * RS + l] = rho[c];
    __syncthreads();

    for (int it = 0; it < mr; it++) {
        const unsigned salt = opaque_zero();
        float2 up[6], L[6];
#pragma unroll
        for (int k = 0; k < 6; k++) up[k] = L[k] = make_float2(0.f, 0.f);
        // half of the clover rows (from L2) are loaded before the hops,
        // which hide their latency (all 18 would not fit the registers)
        float2 ap[18];
#pragma unroll
        for (int k = 0; k < 9; k++) ap[k] = Aall.ld_lane(k, d, aoff, salt);
        block_hops<RS, LS>(rho_lds, lnk, h, l, lnf, lnb, src0, src1, sig, sgf, sgb, up, L);
        float2 hs[6], ax[6], q[6];
        exchange_chirality(h, up, L, hs);
#pragma unroll
        for (int k = 9; k < 18; k++) ap[k] = Aall.ld_lane(k, d, aoff, salt);
        herm6_mv<float>(ap, rho, ax);
        Red3<float> part{0, 0, 0};
#pragma unroll
        for (int c = 0; c < 6; c++) {
            q[c] = csub(csub(ax[c], cscale(hs[c], 0.5f)), cmul(shift, rho[c]));
            part.a += q[c].x * q[c].x + q[c].y * q[c].y;
            part.b += q[c].x * rho[c].x + q[c].y * rho[c].y;   // conj(q) rho
            part.c += q[c].x * rho[c].y - q[c].y * rho[c].x;
        }
        // the barrier after the rho update below (or the end of the loop) comes
        // before any thread writes red again
        Red3<float> sm = block_sum3<float, false>(part, red);
        if (sm.a == 0.f) break;
        const float inv = 1.f / sm.a;
        const float2 alpha = make_float2(sm.b * inv, sm.c * inv);
#pragma unroll
        for (int c = 0; c < 6; c++) {
            cfma(e[c], alpha, rho[c]);
            rho[c] = csub(rho[c], cmul(alpha, q[c]));
        }
        if (it + 1 < mr) {
#pragma unroll
            for (int c = 0; c < 6; c++) rho_lds[(6 * h + c) * RS + l] = rho[c];
            __syncthreads();
        }
    }
#pragma unroll
    for (int c = 0; c < 6; c++)
        zf.template st_lane<true>(c, d, coff, cadd(zf.template ld_lane<true>(c, d, coff), e[c]));
}

}  // namespace

int launch_sap_colour(Ctx *c, int prec, int nrhs, int col, int mr, double sre, double sim, const void *b, void *z) {
    const Geom &g = c->g;
    if (g.Vb < 64 || g.Vb > 256 || (g.Vb & (g.Vb - 1)))
        return fail(c, MGDD_ESHAPE, "the Schwarz kernel needs a block volume of 64, 128 or 256");
    const int nblocks = col ? g.nblocks - g.ncol0 : g.ncol0;
    if (nblocks == 0) return MGDD_OK;
    size_t lds = (prec == MGDD_F64 ? 16 : 8) * 12 * (size_t)g.Vb + (prec == MGDD_F64 ? 8 : 4) * 3 * (g.Vb / 64);
    // four lanes per site with the block's links staged in LDS (FP32)
    const size_t lds4 = 8 * (12 * ((size_t)g.Vb + 4) + 4 * (9 * (size_t)g.Vb + 4)) + 4 * 3 * (4 * g.Vb / 64);
    // two lanes per site, the links' first two rows staged (special unitary links)
    const size_t ldsc = 8 * (12 * ((size_t)g.Vb + 4) + 24 * ((size_t)g.Vb + 2)) + 4 * 3 * (2 * g.Vb / 64);
    dim3 grid(nblocks, nrhs);
    const bool two_ok = c->links_su3 && ldsc <= c->lds_max, four_ok = lds4 <= c->lds_max;
    // lanes per site of the FP32 kernels: the context's choice, else automatic
    int lanes = c->sap_lanes ? c->sap_lanes : two_ok ? 2 : four_ok ? 4 : 1;
    if (prec == MGDD_F64) lanes = 1;
    if (prec == MGDD_F16 && lanes != 2)
        return fail(c, MGDD_EINVAL,
                    "half-precision spinor storage in the Schwarz sweep runs on the two-lanes-per-site kernel");
    if ((lanes == 2 && !two_ok) || (lanes == 4 && !four_ok))
        return fail(c, MGDD_ESHAPE,
                    lanes == 2 ? "the two-lanes-per-site Schwarz kernel needs special unitary links and the block's "
                                 "link rows in LDS"
                               : "the four-lanes-per-site Schwarz kernel needs the block's links in LDS");
    const int slot = kt_begin(c);
    if ((prec == MGDD_F32 || prec == MGDD_F16) && lanes == 2) {
        const int anti = c->t_antiperiodic ? 1 : 0;
#define SAPC(VB, S)                                                                                               \
    sapc_kernel<VB, S><<<grid, 2 * VB, ldsc, c->stream>>>(g, (const float2 *)c->U32, (const float2 *)c->A32, b, z, \
                                                          col, mr, (float)sre, (float)sim, anti)
        if (prec == MGDD_F32) {
            if (g.Vb == 256) SAPC(256, float);
            else if (g.Vb == 128) SAPC(128, float);
            else SAPC(64, float);
        } else {
            if (g.Vb == 256) SAPC(256, _Float16);
            else if (g.Vb == 128) SAPC(128, _Float16);
            else SAPC(64, _Float16);
        }
#undef SAPC
    } else if (prec == MGDD_F64) {
        sap_colour_kernel<double><<<grid, g.Vb, lds, c->stream>>>(g, (const double2 *)c->U64, (const double2 *)c->A64,
                                                                  (const double2 *)b, (double2 *)z, col, mr, sre, sim);
    } else if (lanes == 4) {
#define SAP4(VB)                                                                                               \
    sap4_kernel<float, VB><<<grid, 4 * VB, lds4, c->stream>>>(g, (const float2 *)c->U32, (const float2 *)c->A32,  \
                                                              (const float2 *)b, (float2 *)z, col, mr, (float)sre, \
                                                              (float)sim)
        if (g.Vb == 256) SAP4(256);
        else if (g.Vb == 128) SAP4(128);
        else SAP4(64);   // the only other power of two in range
#undef SAP4
    } else {
        sap_colour_kernel<float><<<grid, g.Vb, lds, c->stream>>>(g, (const float2 *)c->U32, (const float2 *)c->A32,
                                                                 (const float2 *)b, (float2 *)z, col, mr, (float)sre,
                                                                 (float)sim);
    }
    // per site of the colour: links (two rows each on the two-lanes kernel,
    // which rebuilds the third) and clover term once per launch; z in, b in
    // and z out per field (the halo comes from cache). FP16: FP32 links.
    const double lc = prec == MGDD_F64 ? 1152.0 : lanes == 2 ? 480.0 : 576.0, sp = 3.0 * 12 * csize(prec);
    kt_end(c, slot, KF_SAP, prec, (double)nblocks * g.Vb * nrhs, (double)nblocks * g.Vb * (lc + sp * nrhs));
    return hip_check(c, hipGetLastError(), "sap kernel");
}

int launch_sap(Ctx *c, int prec, int nrhs, int nsweeps, int mr, double sre, double sim, const void *b, void *z) {
    for (int s = 0; s < nsweeps; s++)
        for (int col = 0; col < 2; col++) {
            int rc = launch_sap_colour(c, prec, nrhs, col, mr, sre, sim, b, z);
            if (rc) return rc;
        }
    return MGDD_OK;
}

}  // namespace mgdd
