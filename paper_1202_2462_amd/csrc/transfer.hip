// Aggregation interpolation (Section 3): P from test vectors by a local
// orthonormalisation per (aggregate, chirality), restriction P^H,
// prolongation P, and the coarse operator D_c = P^H D P built column by
// column from the terms of D (self term plus the hops that cross each face of
// an aggregate) followed by a restriction. The coarse stencil apply lives here
// as well.
#include "stencil.h"
#include "transfer.h"
#include "coarse.h"
#include "level2.h"

namespace mgdd {

namespace {

constexpr int TPB = 256;

template <typename T> __device__ inline T wsum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// sum of (a, b) over the workgroup, identical in every thread (fixed order)
__device__ inline double2 block_sum2(double a, double b, double *red) {
    a = wsum(a);
    b = wsum(b);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[2 * w] = a; red[2 * w + 1] = b; }
    __syncthreads();
    double A = 0, B = 0;
    for (int i = 0; i < nw; i++) { A += red[2 * i]; B += red[2 * i + 1]; }
    __syncthreads();
    return make_double2(A, B);
}

// ---------------------------------------------------------------- P: local modified Gram-Schmidt
//
// One workgroup per (aggregate, chirality); the (6 * Va) x N block of the test
// vectors is orthonormalised in place, in column order, so that P^H P = 1 on
// the block with a positive real diagonal of R (the unique thin QR).
__global__ __launch_bounds__(TPB) void build_P_kernel(int V, int Va, int N, const int *__restrict__ agg_sites,
                                                      double2 *__restrict__ P, int *__restrict__ flag) {
    __shared__ double red[2 * (TPB / 64)];
    const int a = blockIdx.x, chi = blockIdx.y;
    const int *sites = agg_sites + (size_t)a * Va;
    const size_t fs = (size_t)12 * V;  // field stride
    for (int k = 0; k < N; k++) {
        double2 *w = P + (size_t)k * fs;
        double n0 = 0;
        for (int l = threadIdx.x; l < Va; l += blockDim.x)
            for (int c = 6 * chi; c < 6 * chi + 6; c++) {
                double2 v = w[(size_t)c * V + sites[l]];
                n0 += v.x * v.x + v.y * v.y;
            }
        n0 = block_sum2(n0, 0, red).x;
        for (int j = 0; j < k; j++) {
            const double2 *q = P + (size_t)j * fs;
            double ra = 0, rb = 0;
            for (int l = threadIdx.x; l < Va; l += blockDim.x)
                for (int c = 6 * chi; c < 6 * chi + 6; c++) {
                    size_t e = (size_t)c * V + sites[l];
                    double2 qv = q[e], wv = w[e];
                    ra += qv.x * wv.x + qv.y * wv.y;
                    rb += qv.x * wv.y - qv.y * wv.x;
                }
            double2 r = block_sum2(ra, rb, red);
            for (int l = threadIdx.x; l < Va; l += blockDim.x)
                for (int c = 6 * chi; c < 6 * chi + 6; c++) {
                    size_t e = (size_t)c * V + sites[l];
                    w[e] = csub(w[e], cmul(r, q[e]));
                }
        }
        double nn = 0;
        for (int l = threadIdx.x; l < Va; l += blockDim.x)
            for (int c = 6 * chi; c < 6 * chi + 6; c++) {
                double2 v = w[(size_t)c * V + sites[l]];
                nn += v.x * v.x + v.y * v.y;
            }
        nn = block_sum2(nn, 0, red).x;
        double rkk = sqrt(nn);
        if (!(rkk > 1e-12 * sqrt(n0)) || n0 == 0.0) {
            if (threadIdx.x == 0) atomicExch(flag, 1);
            rkk = 1.0;
        }
        double inv = 1.0 / rkk;
        for (int l = threadIdx.x; l < Va; l += blockDim.x)
            for (int c = 6 * chi; c < 6 * chi + 6; c++) {
                size_t e = (size_t)c * V + sites[l];
                w[e] = cscale(w[e], inv);
            }
    }
}

// The same orthonormalisation for aggregates of at most TPB sites, one thread
// per site holding the 6 components of the column being orthonormalised in
// registers: each step loads one earlier column once, and each sum over the
// block takes one barrier (two alternating LDS slots). Per-thread sums, the
// butterfly and the order over waves are those of build_P_kernel.
__device__ inline double2 block_sum2_1(double a, double b, double *red) {
    a = wsum(a);
    b = wsum(b);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[2 * w] = a; red[2 * w + 1] = b; }
    __syncthreads();
    double A = 0, B = 0;
    for (int i = 0; i < nw; i++) { A += red[2 * i]; B += red[2 * i + 1]; }
    return make_double2(A, B);
}

__global__ __launch_bounds__(TPB) void build_P_reg_kernel(int V, int Va, int N, const int *__restrict__ agg_sites,
                                                          double2 *__restrict__ P, int *__restrict__ flag) {
    __shared__ double red[2][2 * (TPB / 64)];
    const int a = blockIdx.x, chi = blockIdx.y;
    const bool active = (int)threadIdx.x < Va;
    const int d = active ? agg_sites[(size_t)a * Va + threadIdx.x] : 0;
    const size_t fs = (size_t)12 * V;  // field stride
    int slot = 0;
    for (int k = 0; k < N; k++) {
        double2 *wp = P + (size_t)k * fs;
        double2 w[6];
        double n0 = 0;
#pragma unroll
        for (int c = 0; c < 6; c++) {
            w[c] = active ? wp[(size_t)(6 * chi + c) * V + d] : make_double2(0, 0);
            n0 += w[c].x * w[c].x + w[c].y * w[c].y;
        }
        n0 = block_sum2_1(n0, 0, red[slot]).x;
        slot ^= 1;
        double2 q[6], qn[6];
#pragma unroll
        for (int c = 0; c < 6; c++) q[c] = active && k > 0 ? P[(size_t)(6 * chi + c) * V + d] : make_double2(0, 0);
        for (int j = 0; j < k; j++) {
            // prefetch column j + 1 while column j is used
            const double2 *qp = P + (size_t)(j + 1 < k ? j + 1 : j) * fs;
#pragma unroll
            for (int c = 0; c < 6; c++) qn[c] = active ? qp[(size_t)(6 * chi + c) * V + d] : make_double2(0, 0);
            double ra = 0, rb = 0;
#pragma unroll
            for (int c = 0; c < 6; c++) {
                ra += q[c].x * w[c].x + q[c].y * w[c].y;
                rb += q[c].x * w[c].y - q[c].y * w[c].x;
            }
            const double2 r = block_sum2_1(ra, rb, red[slot]);
            slot ^= 1;
#pragma unroll
            for (int c = 0; c < 6; c++) {
                w[c] = csub(w[c], cmul(r, q[c]));
                q[c] = qn[c];
            }
        }
        double nn = 0;
#pragma unroll
        for (int c = 0; c < 6; c++) nn += w[c].x * w[c].x + w[c].y * w[c].y;
        nn = block_sum2_1(nn, 0, red[slot]).x;
        slot ^= 1;
        double rkk = sqrt(nn);
        if (!(rkk > 1e-12 * sqrt(n0)) || n0 == 0.0) {
            if (threadIdx.x == 0) atomicExch(flag, 1);
            rkk = 1.0;
        }
        const double inv = 1.0 / rkk;
        if (active) {
#pragma unroll
            for (int c = 0; c < 6; c++) wp[(size_t)(6 * chi + c) * V + d] = cscale(w[c], inv);
        }
    }
}

// ---------------------------------------------------------------- restriction c = P^H f
//
// One workgroup per (aggregate, field). out[a * ostride + r * rstride + chi * N + k].
// The workgroups of the nrhs fields of one aggregate are consecutive and on
// one XCD, so the aggregate's columns of P come from HBM once per launch and
// from L2 for the other fields. T: arithmetic and coarse precision; SP, SF:
// storage of P and of the fine field (T, or half precision with T = float).
template <typename T, typename SP = T, typename SF = T>
__global__ __launch_bounds__(TPB) void restrict_kernel(int V, int Va, int N, const int *__restrict__ agg_sites,
                                                       const C<SP> *__restrict__ P, const C<SF> *__restrict__ f,
                                                       C<T> *__restrict__ out, size_t ostride, size_t rstride,
                                                       int nrhs, int ks) {
    extern __shared__ unsigned char smem[];
    T *red = (T *)smem;  // [waves][N][4]
    const int wg = xcd_block(gridDim.x);
    // ks workgroups per (aggregate, field), each for a contiguous range of k
    const int part = wg % ks, af = wg / ks;
    const int a = af / nrhs, r = af % nrhs;
    const int kper = (N + ks - 1) / ks, kb = part * kper, ke = kb + kper < N ? kb + kper : N;
    const int *sites = agg_sites + (size_t)a * Va;
    const size_t fs = (size_t)12 * V;
    const C<SF> *fr = f + (size_t)r * fs;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    auto wide = [](auto v) { return mk<T>((T)v.x, (T)v.y); };
    // one site per thread when Va <= blockDim (the field values stay in registers)
    C<T> f0[12];
    const bool one = Va <= (int)blockDim.x;
    if (one) {
        int d = threadIdx.x < Va ? sites[threadIdx.x] : 0;
#pragma unroll
        for (int c = 0; c < 12; c++) f0[c] = threadIdx.x < Va ? wide(fr[(size_t)c * V + d]) : mk<T>(0, 0);
    }
    for (int k = kb; k < ke; k++) {
        const C<SP> *pk = P + (size_t)k * fs;
        T p0 = 0, p1 = 0, p2 = 0, p3 = 0;
        for (int l = threadIdx.x; l < Va; l += blockDim.x) {
            int d = sites[l];
#pragma unroll
            for (int c = 0; c < 12; c++) {
                C<T> pv = wide(pk[(size_t)c * V + d]), fv = one ? f0[c] : wide(fr[(size_t)c * V + d]);
                T re = pv.x * fv.x + pv.y * fv.y, im = pv.x * fv.y - pv.y * fv.x;
                if (c < 6) { p0 += re; p1 += im; } else { p2 += re; p3 += im; }
            }
        }
        p0 = wsum(p0); p1 = wsum(p1); p2 = wsum(p2); p3 = wsum(p3);
        if (lane == 0) {
            T *o = red + ((size_t)w * N + k) * 4;
            o[0] = p0; o[1] = p1; o[2] = p2; o[3] = p3;
        }
    }
    __syncthreads();
    const int nw = blockDim.x >> 6;
    for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
        int chi = i / N, k = i % N;
        if (k < kb || k >= ke) continue;
        T re = 0, im = 0;
        for (int q = 0; q < nw; q++) {
            re += red[((size_t)q * N + k) * 4 + 2 * chi];
            im += red[((size_t)q * N + k) * 4 + 2 * chi + 1];
        }
        out[(size_t)a * ostride + (size_t)r * rstride + i] = mk<T>(re, im);
    }
}

// ---------------------------------------------------------------- prolongation f = P c
//
// One thread per (site, field), the fields of one site in consecutive threads:
// they read the same entries of P, so P comes from HBM once per launch.
// T: arithmetic and coarse precision; SP, SF: storage of P and of the fine
// field (rounded once to nearest even when half precision).
template <typename T, typename SP = T, typename SF = T>
__global__ __launch_bounds__(TPB) void prolong_kernel(int V, int Vc, int N, const int *__restrict__ site_agg,
                                                      const C<SP> *__restrict__ P, const C<T> *__restrict__ cin,
                                                      C<SF> *__restrict__ f, int nrhs) {
    const size_t i = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= (size_t)V * nrhs) return;
    const int r = (int)(i % nrhs), d = (int)(i / nrhs);
    const int a = site_agg[d];
    const size_t fs = (size_t)12 * V;
    const C<T> *x = cin + ((size_t)r * Vc + a) * 2 * N;
    C<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = mk<T>(0, 0);
    for (int k = 0; k < N; k++) {
        const C<SP> *pk = P + (size_t)k * fs;
        C<T> x0 = x[k], x1 = x[N + k];
#pragma unroll
        for (int c = 0; c < 12; c++) {
            const C<SP> pv = pk[(size_t)c * V + d];
            cfma(acc[c], mk<T>((T)pv.x, (T)pv.y), c < 6 ? x0 : x1);
        }
    }
    C<SF> *fr = f + (size_t)r * fs;
#pragma unroll
    for (int c = 0; c < 12; c++) fr[(size_t)c * V + d] = mk<SF>((SF)acc[c].x, (SF)acc[c].y);
}

// ---------------------------------------------------------------- terms of D for one column of D_c
//
// For the prolonged unit vector P_j (test vector k restricted to chirality
// chi), W_0 = A P_j - 1/2 (hops that stay inside the aggregate) and, for each
// face direction dd = 1 + 2 mu (+mu) or 2 + 2 mu (-mu), W_dd = the single hop of
// D that leaves the aggregate through that face (zero elsewhere). Written as 9
// fine fields [dd][12][V].
template <int MU, bool FWD>
__device__ inline void face_term(const LinkViews<double> &U, const FieldView<double> &pj, int chi, int d, int dn,
                                 bool crosses, double2 *self, double2 *Wdir, size_t V) {
    double2 psi[12], u[9], t[12];
    load_spinor<double>(pj, dn, psi);
#pragma unroll
    for (int c = 0; c < 12; c++) {
        if ((c >= 6) != (chi != 0)) psi[c] = make_double2(0, 0);
        t[c] = make_double2(0, 0);
    }
    load_link<double, MU>(U, FWD ? d : dn, u);
    hop<double, MU, FWD>(t, u, psi);
    FieldView<double> w(Wdir, V, 12);
#pragma unroll
    for (int c = 0; c < 12; c++) {
        if (crosses) {
            w.st(c, d, cscale(t[c], -0.5));
        } else {
            self[c] = cadd(self[c], t[c]);
            w.st(c, d, make_double2(0, 0));
        }
    }
}

__global__ __launch_bounds__(TPB) void dc_terms_kernel(Geom g, AggGeom ag, const double2 *__restrict__ Up,
                                                       const double2 *__restrict__ Ap, const double2 *__restrict__ Pk,
                                                       int chi, double2 *__restrict__ W) {
    const int d = blockIdx.x * TPB + threadIdx.x;
    if (d >= g.V) return;
    const size_t V = g.V;
    int X[4], nbr[8];
    site_coords(g, d, X);
    site_neighbours(g, d, nbr);
    LinkViews<double> U(Up, V);
    CloverViews<double> A(Ap, V);
    FieldView<double> pj(Pk, V, 12);
    double2 self[12], psi[12], ap[12];
#pragma unroll
    for (int c = 0; c < 12; c++) self[c] = make_double2(0, 0);
    bool last[4], first[4];
#pragma unroll
    for (int m = 0; m < 4; m++) {
        int r = X[m] % ag.a[m];
        last[m] = r == ag.a[m] - 1;   // the +m hop leaves the aggregate
        first[m] = r == 0;            // the -m hop leaves the aggregate
    }
    const size_t fs = (size_t)12 * V;
    face_term<0, true>(U, pj, chi, d, nbr[0], last[0], self, W + 1 * fs, V);
    face_term<0, false>(U, pj, chi, d, nbr[1], first[0], self, W + 2 * fs, V);
    face_term<1, true>(U, pj, chi, d, nbr[2], last[1], self, W + 3 * fs, V);
    face_term<1, false>(U, pj, chi, d, nbr[3], first[1], self, W + 4 * fs, V);
    face_term<2, true>(U, pj, chi, d, nbr[4], last[2], self, W + 5 * fs, V);
    face_term<2, false>(U, pj, chi, d, nbr[5], first[2], self, W + 6 * fs, V);
    face_term<3, true>(U, pj, chi, d, nbr[6], last[3], self, W + 7 * fs, V);
    face_term<3, false>(U, pj, chi, d, nbr[7], first[3], self, W + 8 * fs, V);
    // self term: A P_j - 1/2 (hops that stay inside the aggregate)
    load_spinor<double>(pj, d, psi);
#pragma unroll
    for (int c = 0; c < 12; c++) if ((c >= 6) != (chi != 0)) psi[c] = make_double2(0, 0);
    clover_mv<double>(A, d, psi, ap);
    FieldView<double> w0(W, V, 12);
#pragma unroll
    for (int c = 0; c < 12; c++) w0.st(c, d, csub(ap[c], cscale(self[c], 0.5)));
}

// Fallback for aggregates with an extent of 1 in some direction (a site then
// lies on both faces of that direction): one workgroup per (aggregate a,
// column j = (chi', k')), one thread per site x of a: the thread forms the 9
// terms of D applied to the prolonged unit vector P e_j at x (self term:
// clover plus the hops that stay in a; one face term per direction, nonzero
// on that face only), then projects all 9 on every P_k(x) of both
// chiralities in one pass over P. Block layout [a][dir][col][row].
template <int MU, bool FWD>
__device__ inline void term_hop(const LinkViews<double> &U, const FieldView<double> &pj, int chi, int d, int dn,
                                double2 *acc) {
    double2 psi[12], u[9];
    load_spinor<double>(pj, dn, psi);
#pragma unroll
    for (int c = 0; c < 12; c++)
        if ((c >= 6) != (chi != 0)) psi[c] = make_double2(0, 0);
    load_link<double, MU>(U, FWD ? d : dn, u);
    hop<double, MU, FWD>(acc, u, psi);
}

// the hop of one direction: into the face term when it leaves the aggregate
// (scaled by -1/2), else added to the self sum
template <int MU, bool FWD>
__device__ inline void term_into(const LinkViews<double> &U, const FieldView<double> &pj, int chi, int d, int dn,
                                 bool crosses, double2 *self, double2 *face) {
    double2 t[12];
#pragma unroll
    for (int c = 0; c < 12; c++) t[c] = make_double2(0, 0);
    term_hop<MU, FWD>(U, pj, chi, d, dn, t);
#pragma unroll
    for (int c = 0; c < 12; c++) {
        face[c] = crosses ? cscale(t[c], -0.5) : make_double2(0, 0);
        self[c] = crosses ? self[c] : cadd(self[c], t[c]);
    }
}

__global__ __launch_bounds__(256) void dc_build_thin_kernel(Geom g, AggGeom ag, int N, int Va, const int *__restrict__ agg_sites,
                                                       const double2 *__restrict__ Up, const double2 *__restrict__ Ap,
                                                       const double2 *__restrict__ P, double2 *__restrict__ Dc,
                                                       int nwg) {
    extern __shared__ double dred[];  // reduction space (see below)
    const int n2 = 2 * N;
    const int w = xcd_block(nwg);
    const int a = w / n2, j = w % n2, chi = j / N, kk = j % N;
    const size_t V = g.V;
    const int l = threadIdx.x;
    const bool active = l < Va;
    double2 wt[9][12];
#pragma unroll
    for (int t = 0; t < 9; t++)
#pragma unroll
        for (int c = 0; c < 12; c++) wt[t][c] = make_double2(0, 0);
    int d = 0;
    if (active) {
        d = agg_sites[(size_t)a * Va + l];
        int X[4], nbr[8];
        site_coords(g, d, X);
        site_neighbours(g, d, nbr);
        LinkViews<double> U(Up, V);
        CloverViews<double> A(Ap, V);
        FieldView<double> pj(P + (size_t)kk * 12 * V, V, 12);
        double2 self[12];
#pragma unroll
        for (int c = 0; c < 12; c++) self[c] = make_double2(0, 0);
        bool last[4], first[4];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            int r = X[m] % ag.a[m];
            last[m] = r == ag.a[m] - 1;   // the +m hop leaves the aggregate
            first[m] = r == 0;            // the -m hop leaves the aggregate
        }
        term_into<0, true>(U, pj, chi, d, nbr[0], last[0], self, wt[1]);
        term_into<0, false>(U, pj, chi, d, nbr[1], first[0], self, wt[2]);
        term_into<1, true>(U, pj, chi, d, nbr[2], last[1], self, wt[3]);
        term_into<1, false>(U, pj, chi, d, nbr[3], first[1], self, wt[4]);
        term_into<2, true>(U, pj, chi, d, nbr[4], last[2], self, wt[5]);
        term_into<2, false>(U, pj, chi, d, nbr[5], first[2], self, wt[6]);
        term_into<3, true>(U, pj, chi, d, nbr[6], last[3], self, wt[7]);
        term_into<3, false>(U, pj, chi, d, nbr[7], first[3], self, wt[8]);
        double2 psi[12], ap[12];
        load_spinor<double>(pj, d, psi);
#pragma unroll
        for (int c = 0; c < 12; c++)
            if ((c >= 6) != (chi != 0)) psi[c] = make_double2(0, 0);
        clover_mv<double>(A, d, psi, ap);
#pragma unroll
        for (int c = 0; c < 12; c++) wt[0][c] = csub(ap[c], cscale(self[c], 0.5));
    }
    // projections onto the N test-vector columns of aggregate a: for each k
    // every thread writes its 36 partial products (9 terms x re/im x two row
    // chiralities) to LDS, then S threads per product add the partials in a
    // fixed order (a tree through LDS costs fewer instructions than 36
    // cross-lane reductions per wave)
    const int nthr = blockDim.x, S = nthr / 36 > 0 ? nthr / 36 : 1;
    double *red = dred;                         // [36][nthr]
    double *p2 = red + 36 * nthr;               // [36][S]
    double *res = p2 + 36 * S;                  // [N][36]
    for (int k = 0; k < N; k++) {
        double2 pk[12];
        if (active) {
            FieldView<double> fk(P + (size_t)k * 12 * V, V, 12);
            load_spinor<double>(fk, d, pk);
        } else {
#pragma unroll
            for (int c = 0; c < 12; c++) pk[c] = make_double2(0, 0);
        }
#pragma unroll
        for (int t = 0; t < 9; t++) {
            double p[4] = {0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < 12; c++) {
                double re = pk[c].x * wt[t][c].x + pk[c].y * wt[t][c].y;
                double im = pk[c].x * wt[t][c].y - pk[c].y * wt[t][c].x;
                p[c < 6 ? 0 : 2] += re;
                p[c < 6 ? 1 : 3] += im;
            }
#pragma unroll
            for (int q = 0; q < 4; q++) red[(t * 4 + q) * nthr + threadIdx.x] = p[q];
        }
        __syncthreads();
        if ((int)threadIdx.x < 36 * S) {
            const int q = threadIdx.x / S, sidx = threadIdx.x % S;
            double acc = 0;
            for (int i = sidx; i < nthr; i += S) acc += red[q * nthr + i];
            p2[q * S + sidx] = acc;
        }
        __syncthreads();
        if (threadIdx.x < 36) {
            double acc = 0;
            for (int sidx = 0; sidx < S; sidx++) acc += p2[threadIdx.x * S + sidx];
            res[k * 36 + threadIdx.x] = acc;
        }
    }
    __syncthreads();
    const size_t blk = (size_t)n2 * n2;
    for (int e = threadIdx.x; e < 9 * n2; e += blockDim.x) {
        int t = e / n2, i = e % n2;
        int rchi = i / N, k = i % N;
        const double *o = res + (size_t)k * 36 + t * 4;
        Dc[((size_t)a * 9 + t) * blk + (size_t)j * n2 + i] = make_double2(o[2 * rchi], o[2 * rchi + 1]);
    }
}

// D_c for aggregates of at most 256 sites with every extent >= 2: one
// workgroup per (aggregate a, column j = (chi', k'), row chirality h), one
// thread per site x of a. With extents >= 2 a site lies on at most one face
// per direction, so the thread keeps five 6-component terms: the h half of
// the self term (clover block h on P_j, which is zero unless h = chi', minus
// 1/2 the hops that stay in a) and, per direction mu, the h half of -1/2 the
// hop that leaves a through the face the site lies on (zero inside). For
// each k the products with the h half of P_k(x) give 10 partial sums per
// thread; each wave spreads them into its 18 sums (self, + face and - face of
// each direction, re and im) through a wave-private LDS tile, read back by 54
// lanes in three fixed row ranges, so the k loop has no workgroup barrier.
// The per-wave sums are added in wave order at the end.
constexpr int DCB_COLS = 18;   // per-wave sums for one k
constexpr int DCB_LD = 65;     // tile row length in doubles (64 lanes + 1: no bank conflicts)

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one hop of D on P_j (test vector restricted to chirality chi), all 12
// components, without the factor -1/2
template <int MU, bool FWD>
__device__ inline void col_hop(const LinkViews<double> &U, const FieldView<double> &pj, int chi, int d, int dn,
                               double2 *t) {
    double2 psi[12], u[9];
#pragma unroll
    for (int c = 0; c < 12; c++) {
        t[c] = make_double2(0, 0);
        psi[c] = ((c >= 6) == (chi != 0)) ? pj.ld(c, dn) : make_double2(0, 0);
    }
    load_link<double, MU>(U, FWD ? d : dn, u);
    hop<double, MU, FWD>(t, u, psi);
}

// both hops of direction MU: the one that leaves the aggregate (at most one
// when the extent is >= 2) into face, the others into self (h halves)
template <int MU>
__device__ inline void col_dir(const LinkViews<double> &U, const FieldView<double> &pj, int chi, int h, int d,
                               const int *nbr, bool last, bool first, double2 *self, double2 *face) {
    double2 t[12];
    col_hop<MU, true>(U, pj, chi, d, nbr[2 * MU], t);
#pragma unroll
    for (int c = 0; c < 6; c++) {
        const double2 v = h ? t[6 + c] : t[c];
        if (last) face[c] = cscale(v, -0.5);
        else self[c] = cadd(self[c], v);
    }
    col_hop<MU, false>(U, pj, chi, d, nbr[2 * MU + 1], t);
#pragma unroll
    for (int c = 0; c < 6; c++) {
        const double2 v = h ? t[6 + c] : t[c];
        if (first) face[c] = cscale(v, -0.5);
        else self[c] = cadd(self[c], v);
    }
}

__global__ __launch_bounds__(256) void dc_build_kernel(Geom g, AggGeom ag, int N, int Va, const int *__restrict__ agg_sites,
                                                       const double2 *__restrict__ Up, const double2 *__restrict__ Ap,
                                                       const double2 *__restrict__ P, double2 *__restrict__ Dc,
                                                       int nwg) {
    extern __shared__ double dsm[];
    const int n2 = 2 * N;
    const int w = xcd_block(nwg);
    const int h = w & 1, j = (w >> 1) % n2, a = (w >> 1) / n2, chi = j / N, kk = j % N;
    const size_t V = g.V;
    const int l = threadIdx.x, lane = l & 63, wave = l >> 6, nw = blockDim.x >> 6;
    const bool active = l < Va;
    double2 wt[5][6];
#pragma unroll
    for (int s = 0; s < 5; s++)
#pragma unroll
        for (int c = 0; c < 6; c++) wt[s][c] = make_double2(0, 0);
    bool last[4] = {false, false, false, false}, first[4] = {false, false, false, false};
    int d = 0;
    if (active) {
        d = agg_sites[(size_t)a * Va + l];
        int X[4], nbr[8];
        site_coords(g, d, X);
        site_neighbours(g, d, nbr);
        LinkViews<double> U(Up, V);
        FieldView<double> pj(P + (size_t)kk * 12 * V, V, 12);
#pragma unroll
        for (int m = 0; m < 4; m++) {
            const int r = X[m] % ag.a[m];
            last[m] = r == ag.a[m] - 1;   // the +m hop leaves the aggregate
            first[m] = r == 0;            // the -m hop leaves the aggregate
        }
        double2 self[6];
#pragma unroll
        for (int c = 0; c < 6; c++) self[c] = make_double2(0, 0);
        col_dir<0>(U, pj, chi, h, d, nbr, last[0], first[0], self, wt[1]);
        col_dir<1>(U, pj, chi, h, d, nbr, last[1], first[1], self, wt[2]);
        col_dir<2>(U, pj, chi, h, d, nbr, last[2], first[2], self, wt[3]);
        col_dir<3>(U, pj, chi, h, d, nbr, last[3], first[3], self, wt[4]);
        double2 ap[6];
#pragma unroll
        for (int c = 0; c < 6; c++) ap[c] = make_double2(0, 0);
        if (h == chi) {   // the clover term is block diagonal in chirality
            FieldView<double> ab(Ap + (size_t)h * 18 * V, V, 18);   // packed block h
            double2 pa[18], in[6];
#pragma unroll
            for (int q = 0; q < 18; q++) pa[q] = ab.ld(q, d);
#pragma unroll
            for (int c = 0; c < 6; c++) in[c] = pj.ld(6 * h + c, d);
            herm6_mv<double>(pa, in, ap);
        }
#pragma unroll
        for (int c = 0; c < 6; c++) wt[0][c] = csub(ap[c], cscale(self[c], 0.5));
    }
    double *tile = dsm + (size_t)wave * DCB_COLS * DCB_LD;   // [18][65], this wave only
    double *outw = dsm + (size_t)nw * DCB_COLS * DCB_LD;     // [N][nw][18]
    const int col = lane % DCB_COLS, part = lane / DCB_COLS, r0 = 22 * part;
    double2 pk[6];
    {
        FieldView<double> f0(P, V, 12);
#pragma unroll
        for (int c = 0; c < 6; c++) pk[c] = active ? f0.ld(6 * h + c, d) : make_double2(0, 0);
    }
    for (int k = 0; k < N; k++) {
        double2 pn[6];
        const bool more = active && k + 1 < N;
        FieldView<double> fn(P + (size_t)(more ? k + 1 : k) * 12 * V, V, 12);
#pragma unroll
        for (int c = 0; c < 6; c++) pn[c] = more ? fn.ld(6 * h + c, d) : make_double2(0, 0);
        double s[5][2];
#pragma unroll
        for (int q = 0; q < 5; q++) {
            double re = 0, im = 0;
#pragma unroll
            for (int c = 0; c < 6; c++) {
                re += pk[c].x * wt[q][c].x + pk[c].y * wt[q][c].y;
                im += pk[c].x * wt[q][c].y - pk[c].y * wt[q][c].x;
            }
            s[q][0] = re;
            s[q][1] = im;
        }
        tile[0 * DCB_LD + lane] = s[0][0];
        tile[1 * DCB_LD + lane] = s[0][1];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            tile[(2 + 4 * m) * DCB_LD + lane] = last[m] ? s[1 + m][0] : 0.0;
            tile[(3 + 4 * m) * DCB_LD + lane] = last[m] ? s[1 + m][1] : 0.0;
            tile[(4 + 4 * m) * DCB_LD + lane] = first[m] ? s[1 + m][0] : 0.0;
            tile[(5 + 4 * m) * DCB_LD + lane] = first[m] ? s[1 + m][1] : 0.0;
        }
        wave_sync();
        double acc = 0;
        if (lane < 3 * DCB_COLS) {
#pragma unroll
            for (int q = 0; q < 22; q++)
                if (r0 + q < 64) acc += tile[col * DCB_LD + r0 + q];
        }
        const double a1 = __shfl(acc, lane + DCB_COLS, 64), a2 = __shfl(acc, lane + 2 * DCB_COLS, 64);
        if (lane < DCB_COLS) outw[((size_t)k * nw + wave) * DCB_COLS + lane] = (acc + a1) + a2;
        wave_sync();
#pragma unroll
        for (int c = 0; c < 6; c++) pk[c] = pn[c];
    }
    __syncthreads();
    const size_t blk = (size_t)n2 * n2;
    for (int e = threadIdx.x; e < 9 * N; e += blockDim.x) {
        const int t = e / N, k = e % N;
        const int c0 = t == 0 ? 0 : 2 + 2 * (t - 1);   // + face of mu: 2 + 4 mu, - face: 4 + 4 mu
        double re = 0, im = 0;
        for (int q = 0; q < nw; q++) {
            const double *o = outw + ((size_t)k * nw + q) * DCB_COLS + c0;
            re += o[0];
            im += o[1];
        }
        Dc[((size_t)a * 9 + t) * blk + (size_t)j * n2 + (size_t)h * N + k] = make_double2(re, im);
    }
}

// ---------------------------------------------------------------- coarse stencil y = D_c x
//
// One workgroup of 1024 threads per (coarse site, right-hand side): the 9 2N
// products of each row are split over floor(1024 / 2N) thread sets
// (dc_row_partial), whose partial rows are then added in set order. Blocks
// are stored column-major, B[a][dir][col][row], so consecutive threads read
// consecutive rows of one column.
template <typename T>
__global__ __launch_bounds__(1024) void coarse_apply_kernel(int Vc, int N, const int *__restrict__ cnbr,
                                                            const C<T> *__restrict__ Dc, const C<T> *__restrict__ x,
                                                            C<T> *__restrict__ y) {
    const int a = blockIdx.x, r = blockIdx.y;
    const int n2 = 2 * N;
    __shared__ C<T> xs[9 * 64];
    __shared__ C<T> part[1024];
    const C<T> *xr = x + (size_t)r * Vc * n2;
    for (int e = threadIdx.x; e < 9 * n2; e += blockDim.x) xs[e] = xr[(size_t)cnbr[a * 9 + e / n2] * n2 + e % n2];
    __syncthreads();
    dc_row_partial<T>(Dc + (size_t)a * 9 * n2 * n2, xs, n2, part);
    __syncthreads();
    const int i = threadIdx.x, nparts = blockDim.x / n2;
    if (i < n2) {
        C<T> acc = mk<T>(0, 0);
        for (int q = 0; q < nparts; q++) acc = cadd(acc, part[q * n2 + i]);
        y[((size_t)r * Vc + a) * n2 + i] = acc;
    }
}

// D_c applied to many right-hand sides on the matrix cores. Per coarse site
// a the product is Y = sum_dir B_dir X_nbr(dir), a (2N x 2N) by (2N x R)
// complex matrix product for R right-hand sides, done as real 16x16x4 MFMA
// tiles: Re Y += Re B Re X - Im B Im X, Im Y += Re B Im X + Im B Re X.
// A wave owns output rows 16t .. 16t+15 of one coarse site for one tile of
// 16 right-hand sides; its A operand (rows of B_dir, column-major blocks)
// streams from HBM, its B operand (4 consecutive entries of 16 neighbour
// vectors) comes through the caches, which the row tiles of a site share.
// Rows and columns past 2N and right-hand sides past nrhs enter as zeros and
// are not written.
template <typename T> struct MfmaTypes;
// Operands of both: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k.
// Result register v of lane l holds D[row][l % 16] with row = 4 (l / 16) + v
// (FP32) or row = 4 v + l / 16 (FP64).
template <> struct MfmaTypes<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int v, int kq) { return 4 * kq + v; }
};
template <> struct MfmaTypes<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int v, int kq) { return 4 * v + kq; }
};

template <typename T>
__global__ __launch_bounds__(64) void coarse_apply_mfma_kernel(int Vc, int N, int nrhs, int ntiles,
                                                               const int *__restrict__ cnbr,
                                                               const C<T> *__restrict__ Dc,
                                                               const C<T> *__restrict__ x, C<T> *__restrict__ y) {
    using M = MfmaTypes<T>;
    // one wave per (coarse site, row tile, rhs tile); the row tiles of one
    // site are consecutive waves on one XCD, so that they share its L2
    const int w = xcd_block(gridDim.x);
    const int t = w % ntiles, a = w / ntiles, r0 = blockIdx.y * 16;
    const int n2 = 2 * N;
    const int lane = threadIdx.x;
    const int row = t * 16 + (lane & 15), kq = lane >> 4, rl = lane & 15;
    const bool rhs_ok = r0 + rl < nrhs;
    // four independent accumulator chains (Re and Im, two each), so that
    // consecutive MFMAs do not wait for each other's results
    typename M::v4 re0 = {0, 0, 0, 0}, im0 = {0, 0, 0, 0}, re1 = {0, 0, 0, 0}, im1 = {0, 0, 0, 0};
    const C<T> *B = Dc + (size_t)a * 9 * n2 * n2;
    const int nq = (n2 + 3) >> 2;   // k-steps of 4 columns per direction (n2 <= 64)
    for (int dd = 0; dd < 9; dd++) {
        const C<T> *Bd = B + (size_t)dd * n2 * n2;
        const C<T> *xd = x + ((size_t)(r0 + rl) * Vc + cnbr[a * 9 + dd]) * n2;
        // all operands of this direction first, so that their loads overlap
        C<T> av[16], bv[16];
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int j = 4 * q + kq;
            const bool kin = q < nq && j < n2;
            av[q] = (kin && row < n2) ? Bd[(size_t)j * n2 + row] : mk<T>(0, 0);
            bv[q] = (kin && rhs_ok) ? xd[j] : mk<T>(0, 0);
        }
#pragma unroll
        for (int q = 0; q < 16; q++) {
            if (q < nq) {
                re0 = M::mma(av[q].x, bv[q].x, re0);
                im0 = M::mma(av[q].x, bv[q].y, im0);
                re1 = M::mma(-av[q].y, bv[q].y, re1);
                im1 = M::mma(av[q].y, bv[q].x, im1);
            }
        }
    }
    if (!rhs_ok) return;
    const typename M::v4 re = re0 + re1, im = im0 + im1;
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int i = t * 16 + M::row(v, kq);
        if (i < n2) y[((size_t)(r0 + rl) * Vc + a) * n2 + i] = mk<T>(re[v], im[v]);
    }
}

template <typename T>
__global__ void dc_to_f32(int Vc, int n2, const double2 *__restrict__ src, C<T> *__restrict__ dst) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t n = (size_t)Vc * 9 * n2 * n2;
    if (e < n) dst[e] = mk<T>((T)src[e].x, (T)src[e].y);
}

// FP32 copy of the self block and the four forward-hop blocks of every
// coarse site, [Vc][5][col][row] (block q: direction 0 for q = 0, the +mu hop
// 1 + 2 mu for q = 1 + mu)
__global__ void dc_compact_f32(int Vc, int n2, const double2 *__restrict__ src, float2 *__restrict__ dst) {
    const size_t blk = (size_t)n2 * n2;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)Vc * 5 * blk) return;
    const size_t a = e / (5 * blk), r = e % (5 * blk);
    const int q = (int)(r / blk);
    const int t = q == 0 ? 0 : 2 * q - 1;
    const double2 v = src[(a * 9 + t) * blk + r % blk];
    dst[e] = make_float2((float)v.x, (float)v.y);
}

static int coarse_to_f32(Ctx *c) {
    Level1 &L1 = c->c;
    const int n2 = 2 * L1.N;
    const size_t blk = (size_t)n2 * n2, n = (size_t)L1.Vc * 9 * blk, nh = (size_t)L1.Vc * 5 * blk;
    dc_to_f32<float><<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(L1.Vc, n2, (const double2 *)L1.Dc64,
                                                                        (float2 *)L1.Dc32);
    dc_compact_f32<<<(unsigned)((nh + 255) / 256), 256, 0, c->stream>>>(L1.Vc, n2, (const double2 *)L1.Dc64,
                                                                      (float2 *)L1.Dh32);
    return hip_check(c, hipGetLastError(), "D_c convert");
}

}  // namespace

// ---------------------------------------------------------------- host side

// from this many right-hand sides on, D_c is applied on the matrix cores
static int MFMA_MIN_RHS = 4;

// Order in which the coarse GMRES step visits the coarse sites. A site reads
// the forward blocks of its four backward neighbours again (the compact FP32
// D_c), so these should still be in the L2 of its XCD, and the XCDs take
// contiguous eighths of the order. Lexicographic order leaves the z and t
// neighbours far behind; here the sites go in 4-D tiles, time fastest within
// a tile, the tiles in lexicographic order. The spatial extents of a tile are
// 4, 3 or 2, whichever divides the coarse extent first; in time, when 8
// divides the time extent, it is one eighth of it (so that each XCD's range
// is a whole number of time slices, their tiles complete: at 12^3 x 24
// coarse sites, 4 x 4 x 4 x 3 tiles cut the coarse step's reads from memory
// by 5 % and its time by about 3 %, where 4^4 tiles gained nothing), else 4,
// 3 or 2 as in space.
static std::vector<int> coarse_visit_order(const int *Lc) {
    int e[4], nt[4];
    for (int m = 0; m < 4; m++) {
        e[m] = Lc[m] % 4 == 0 ? 4 : Lc[m] % 3 == 0 ? 3 : Lc[m] % 2 == 0 ? 2 : 1;
        if (m == 3 && Lc[3] % 8 == 0) e[3] = Lc[3] / 8;
        nt[m] = Lc[m] / e[m];
    }
    const int vt = e[0] * e[1] * e[2] * e[3], ntiles = nt[0] * nt[1] * nt[2] * nt[3];
    std::vector<int> order;
    order.reserve((size_t)vt * ntiles);
    for (int tile = 0; tile < ntiles; tile++) {
        int tc[4], r = tile;
        for (int m = 0; m < 4; m++) { tc[m] = r % nt[m]; r /= nt[m]; }
        for (int i = 0; i < vt; i++) {
            int x[4], q = i;
            x[3] = q % e[3]; q /= e[3];   // time fastest
            for (int m = 0; m < 3; m++) { x[m] = q % e[m]; q /= e[m]; }
            int y[4];
            for (int m = 0; m < 4; m++) y[m] = tc[m] * e[m] + x[m];
            order.push_back(y[0] + Lc[0] * (y[1] + Lc[1] * (y[2] + Lc[2] * y[3])));
        }
    }
    return order;
}

int transfer_setup(Ctx *c, const int *agg, int N) {
    Level1 &L1 = c->c;
    const Geom &g = c->g;
    for (int m = 0; m < 4; m++)
        if (agg[m] <= 0 || g.L[m] % agg[m]) return fail(c, MGDD_ESHAPE, "aggregates must divide the lattice");
    int Va = agg[0] * agg[1] * agg[2] * agg[3];
    if (N <= 0 || N > 32) return fail(c, MGDD_EINVAL, "number of test vectors must be in 1..32");
    if (N > 6 * Va) return fail(c, MGDD_ERANK, "more test vectors than dof per aggregate and chirality");
    int Lc[4];
    for (int m = 0; m < 4; m++) Lc[m] = g.L[m] / agg[m];
    int Vc = Lc[0] * Lc[1] * Lc[2] * Lc[3];
    bool same = L1.agg_sites && L1.N == N && L1.Vc == Vc;
    for (int m = 0; m < 4 && same; m++) same = L1.agg[m] == agg[m];
    if (same) return MGDD_OK;
    // free the previous level (and the third level built on it)
    level2_free(c);
    void *old[] = {L1.P64, L1.P32, L1.P16, L1.Dc64, L1.Dc32, L1.Dh32, L1.cnbr, L1.corder, L1.agg_sites, L1.site_agg,
                   L1.tv64};
    (void)hipStreamSynchronize(c->stream);
    for (void *p : old) dfree(c, p);
    L1 = Level1();
    // tables: fine sites of each aggregate (local lexicographic order), aggregate of each site
    std::vector<int> agg_sites((size_t)Vc * Va), site_agg(g.V), cnbr((size_t)Vc * 9);
    std::vector<uint32_t> coord;
    std::vector<int> bn, lp;
    Geom hg{};
    int block[4] = {1 << g.lb[0], 1 << g.lb[1], 1 << g.lb[2], 1 << g.lb[3]};
    geometry_tables(g.L, block, hg, coord, bn, &lp);
    hg.blk_coord = coord.data();
    hg.blk_nbr = bn.data();
    hg.pos_of_lex = lp.data();
    std::vector<int> dev_of_lex(g.V);
    for (int d = 0; d < g.V; d++) dev_of_lex[lex_of(hg, d)] = d;
    for (int a = 0; a < Vc; a++) {
        int t = a, ac[4];
        for (int m = 0; m < 4; m++) { ac[m] = t % Lc[m]; t /= Lc[m]; }
        int l = 0;
        for (int x3 = 0; x3 < agg[3]; x3++)
            for (int x2 = 0; x2 < agg[2]; x2++)
                for (int x1 = 0; x1 < agg[1]; x1++)
                    for (int x0 = 0; x0 < agg[0]; x0++) {
                        int X[4] = {ac[0] * agg[0] + x0, ac[1] * agg[1] + x1, ac[2] * agg[2] + x2, ac[3] * agg[3] + x3};
                        int s = X[0] + g.L[0] * (X[1] + g.L[1] * (X[2] + g.L[2] * X[3]));
                        int d = dev_of_lex[s];
                        agg_sites[(size_t)a * Va + l++] = d;
                        site_agg[d] = a;
                    }
        cnbr[(size_t)a * 9] = a;
        for (int m = 0; m < 4; m++)
            for (int dir = 0; dir < 2; dir++) {
                int y[4] = {ac[0], ac[1], ac[2], ac[3]};
                y[m] = (y[m] + (dir == 0 ? 1 : -1) + Lc[m]) % Lc[m];
                cnbr[(size_t)a * 9 + 1 + 2 * m + dir] = y[0] + Lc[0] * (y[1] + Lc[1] * (y[2] + Lc[2] * y[3]));
            }
    }
    size_t fsz = (size_t)N * 12 * g.V;
    size_t dsz = (size_t)Vc * 9 * 4 * N * N;
    L1.P64 = dalloc(c, fsz * 16);
    L1.tv64 = dalloc(c, fsz * 16);
    L1.P32 = dalloc(c, fsz * 8);
    L1.P16 = dalloc(c, fsz * 4);
    L1.Dc64 = dalloc(c, dsz * 16);
    L1.Dc32 = dalloc(c, dsz * 8);
    L1.Dh32 = dalloc(c, dsz / 9 * 5 * 8);
    L1.cnbr = (int *)dalloc(c, cnbr.size() * sizeof(int));
    const std::vector<int> corder = coarse_visit_order(Lc);
    L1.corder = (int *)dalloc(c, corder.size() * sizeof(int));
    L1.agg_sites = (int *)dalloc(c, agg_sites.size() * sizeof(int));
    L1.site_agg = (int *)dalloc(c, site_agg.size() * sizeof(int));
    if (!L1.P64 || !L1.tv64 || !L1.P32 || !L1.P16 || !L1.Dc64 || !L1.Dc32 || !L1.Dh32 || !L1.cnbr || !L1.corder ||
        !L1.agg_sites || !L1.site_agg)
        return MGDD_ENOMEM;
    int rc = hip_check(c, hipMemcpy(L1.cnbr, cnbr.data(), cnbr.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
    if (!rc) rc = hip_check(c, hipMemcpy(L1.corder, corder.data(), corder.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
    if (!rc) rc = hip_check(c, hipMemcpy(L1.agg_sites, agg_sites.data(), agg_sites.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
    if (!rc) rc = hip_check(c, hipMemcpy(L1.site_agg, site_agg.data(), site_agg.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
    if (rc) return rc;
    for (int m = 0; m < 4; m++) { L1.agg[m] = agg[m]; L1.Lc[m] = Lc[m]; }
    L1.Vc = Vc;
    L1.Va = Va;
    L1.N = N;
    return MGDD_OK;
}

int launch_build_P(Ctx *c, const void *tv64) {
    Level1 &L1 = c->c;
    const Geom &g = c->g;
    size_t fsz = (size_t)L1.N * 12 * g.V;
    int rc = hip_check(c, hipMemcpyAsync(L1.P64, tv64, fsz * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
    if (!rc && tv64 != L1.tv64)
        rc = hip_check(c, hipMemcpyAsync(L1.tv64, tv64, fsz * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
    if (rc) return rc;
    int *flag = (int *)ensure_scratch(c, sizeof(int));
    if (!flag) return MGDD_ENOMEM;
    rc = hip_check(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream), "memset");
    if (rc) return rc;
    if (L1.Va <= TPB)
        build_P_reg_kernel<<<dim3(L1.Vc, 2), TPB, 0, c->stream>>>(g.V, L1.Va, L1.N, L1.agg_sites, (double2 *)L1.P64,
                                                                  flag);
    else
        build_P_kernel<<<dim3(L1.Vc, 2), TPB, 0, c->stream>>>(g.V, L1.Va, L1.N, L1.agg_sites, (double2 *)L1.P64, flag);
    rc = hip_check(c, hipGetLastError(), "build_P kernel");
    if (rc) return rc;
    int hflag = 0;
    rc = hip_check(c, hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (rc) return rc;
    if (hflag) return fail(c, MGDD_ERANK, "test vectors are rank deficient on some aggregate");
    rc = launch_convert(c, MGDD_F64, MGDD_F32, fsz, L1.P64, L1.P32);
    if (!rc) rc = launch_convert(c, MGDD_F64, MGDD_F16, fsz, L1.P64, L1.P16);
    return rc;
}

int launch_restrict_ex(Ctx *c, int prec, int nrhs, const void *P, const void *fine, void *out, size_t ostride,
                       size_t rstride) {
    const Level1 &L1 = c->c;
    size_t lds = (size_t)(TPB / 64) * L1.N * 4 * (prec == MGDD_F64 ? 8 : 4);
    // few (aggregate, field) pairs: split the test vectors over up to 4
    // workgroups each, so that the launch fills the chip
    int ks = 1;
    while (ks < 4 && ks < L1.N && (size_t)L1.Vc * nrhs * ks < 1024) ks *= 2;
    const unsigned grid = (unsigned)L1.Vc * (unsigned)nrhs * (unsigned)ks;
    if (prec == MGDD_F64)
        restrict_kernel<double><<<grid, TPB, lds, c->stream>>>(c->g.V, L1.Va, L1.N, L1.agg_sites, (const double2 *)P,
                                                               (const double2 *)fine, (double2 *)out, ostride, rstride,
                                                               nrhs, ks);
    else if (prec == MGDD_F32)
        restrict_kernel<float><<<grid, TPB, lds, c->stream>>>(c->g.V, L1.Va, L1.N, L1.agg_sites, (const float2 *)P,
                                                              (const float2 *)fine, (float2 *)out, ostride, rstride,
                                                              nrhs, ks);
    else   // half-precision fine field and P, FP32 coarse field
        restrict_kernel<float, _Float16, _Float16><<<grid, TPB, lds, c->stream>>>(
            c->g.V, L1.Va, L1.N, L1.agg_sites, (const half_cx *)P, (const half_cx *)fine, (float2 *)out, ostride,
            rstride, nrhs, ks);
    return hip_check(c, hipGetLastError(), "restrict kernel");
}

int launch_restrict(Ctx *c, int prec, int nrhs, const void *fine, void *coarse) {
    const Level1 &L1 = c->c;
    size_t n2 = 2 * (size_t)L1.N;
    return launch_restrict_ex(c, prec, nrhs, prec == MGDD_F64 ? L1.P64 : prec == MGDD_F32 ? L1.P32 : L1.P16, fine,
                              coarse, n2, n2 * L1.Vc);
}

int launch_prolong(Ctx *c, int prec, int nrhs, const void *coarse, void *fine) {
    const Level1 &L1 = c->c;
    size_t n = (size_t)c->g.V * nrhs;
    unsigned nwg = (unsigned)((n + TPB - 1) / TPB);
    if (prec == MGDD_F64)
        prolong_kernel<double><<<nwg, TPB, 0, c->stream>>>(c->g.V, L1.Vc, L1.N, L1.site_agg, (const double2 *)L1.P64,
                                                           (const double2 *)coarse, (double2 *)fine, nrhs);
    else if (prec == MGDD_F32)
        prolong_kernel<float><<<nwg, TPB, 0, c->stream>>>(c->g.V, L1.Vc, L1.N, L1.site_agg, (const float2 *)L1.P32,
                                                          (const float2 *)coarse, (float2 *)fine, nrhs);
    else   // FP32 coarse field, half-precision P and fine field
        prolong_kernel<float, _Float16, _Float16><<<nwg, TPB, 0, c->stream>>>(
            c->g.V, L1.Vc, L1.N, L1.site_agg, (const half_cx *)L1.P16, (const float2 *)coarse, (half_cx *)fine, nrhs);
    return hip_check(c, hipGetLastError(), "prolong kernel");
}

int launch_coarse_build(Ctx *c) {
    Level1 &L1 = c->c;
    const Geom &g = c->g;
    const int N = L1.N, n2 = 2 * N;
    bool thin = false;
    for (int m = 0; m < 4; m++) thin = thin || L1.agg[m] < 2;
    if (L1.Va <= 256) {
        AggGeom ag{};
        for (int m = 0; m < 4; m++) ag.a[m] = L1.agg[m];
        int threads = ((L1.Va + 63) / 64) * 64;
        if (!thin) {
            const int nwg = L1.Vc * n2 * 2;
            const size_t lds = ((size_t)(threads / 64) * DCB_COLS * DCB_LD + (size_t)N * (threads / 64) * DCB_COLS) *
                               sizeof(double);
            dc_build_kernel<<<nwg, threads, lds, c->stream>>>(g, ag, N, L1.Va, L1.agg_sites, (const double2 *)c->U64,
                                                               (const double2 *)c->A64, (const double2 *)L1.P64,
                                                               (double2 *)L1.Dc64, nwg);
        } else {
            const int nwg = L1.Vc * n2;
            const int S = threads / 36 > 0 ? threads / 36 : 1;
            size_t lds = ((size_t)36 * threads + 36 * S + (size_t)36 * N) * sizeof(double);
            dc_build_thin_kernel<<<nwg, threads, lds, c->stream>>>(g, ag, N, L1.Va, L1.agg_sites,
                                                                    (const double2 *)c->U64, (const double2 *)c->A64,
                                                                    (const double2 *)L1.P64, (double2 *)L1.Dc64, nwg);
        }
        int rc = hip_check(c, hipGetLastError(), "D_c build kernel");
        if (rc) return rc;
        return coarse_to_f32(c);
    }
    // aggregates of more than 256 sites: terms of each column as 9 fine
    // fields, then a restriction of those fields
    double2 *W = (double2 *)ensure_scratch(c, (size_t)9 * 12 * g.V * 16);
    if (!W) return MGDD_ENOMEM;
    AggGeom ag{};
    for (int m = 0; m < 4; m++) ag.a[m] = L1.agg[m];
    unsigned nwg = (unsigned)((g.V + TPB - 1) / TPB);
    const size_t blk = (size_t)n2 * n2;
    for (int chi = 0; chi < 2; chi++)
        for (int k = 0; k < N; k++) {
            int j = chi * N + k;
            dc_terms_kernel<<<nwg, TPB, 0, c->stream>>>(g, ag, (const double2 *)c->U64, (const double2 *)c->A64,
                                                       (const double2 *)L1.P64 + (size_t)k * 12 * g.V, chi, W);
            int rc = hip_check(c, hipGetLastError(), "D_c terms kernel");
            if (rc) return rc;
            // column j of the 9 blocks of every coarse site: out[a][dd][j][row]
            rc = launch_restrict_ex(c, MGDD_F64, 9, L1.P64, W, (double2 *)L1.Dc64 + (size_t)j * n2, 9 * blk, blk);
            if (rc) return rc;
        }
    return coarse_to_f32(c);
}

int launch_stencil_apply(Ctx *c, const StencilOp &op, int prec, int nrhs, const void *in, void *out) {
    if (nrhs >= MFMA_MIN_RHS) {
        const int ntiles = (2 * op.N + 15) / 16;
        dim3 grid(op.V * ntiles, (nrhs + 15) / 16);
        if (prec == MGDD_F64)
            coarse_apply_mfma_kernel<double><<<grid, 64, 0, c->stream>>>(
                op.V, op.N, nrhs, ntiles, op.nbr, (const double2 *)op.D64, (const double2 *)in, (double2 *)out);
        else
            coarse_apply_mfma_kernel<float><<<grid, 64, 0, c->stream>>>(
                op.V, op.N, nrhs, ntiles, op.nbr, (const float2 *)op.D32, (const float2 *)in, (float2 *)out);
        return hip_check(c, hipGetLastError(), "coarse apply kernel (MFMA)");
    }
    dim3 grid(op.V, nrhs);
    if (prec == MGDD_F64)
        coarse_apply_kernel<double><<<grid, 1024, 0, c->stream>>>(op.V, op.N, op.nbr, (const double2 *)op.D64,
                                                                 (const double2 *)in, (double2 *)out);
    else
        coarse_apply_kernel<float><<<grid, 1024, 0, c->stream>>>(op.V, op.N, op.nbr, (const float2 *)op.D32,
                                                                (const float2 *)in, (float2 *)out);
    return hip_check(c, hipGetLastError(), "coarse apply kernel");
}

int launch_coarse_apply(Ctx *c, int prec, int nrhs, const void *in, void *out) {
    return launch_stencil_apply(c, level1_op(c), prec, nrhs, in, out);
}

}  // namespace mgdd
