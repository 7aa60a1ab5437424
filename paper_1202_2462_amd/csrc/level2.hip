// Third level of the hierarchy (Section 3: the two-level construction applied
// to the coarse equation D_c x = r_c): aggregates of coarse sites, P2 from
// N2 coarse test vectors, restriction P2^H and prolongation P2, and
// D_cc = P2^H D_c P2 as a 9-point stencil on the level-3 lattice. Coarse
// vectors are [rhs][coarse site][chirality][N1]; level-3 vectors
// [rhs][level-3 site][chirality][N2]. P2 is N2 coarse vectors; each piece
// (aggregate, chirality) of it is orthonormal.
#include <vector>

#include "level2.h"

namespace mgdd {

namespace {

constexpr int TPB = 256;

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// sum over the workgroup, same value returned to every thread (fixed order)
__device__ inline double block_sum_d(double v, double *red) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    v = wave_sum_d(v);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0;
    for (int q = 0; q < nw; q++) s += red[q];
    return s;
}

// One workgroup per (level-3 site A, chirality chi): modified Gram-Schmidt
// of the N2 pieces (Va2 coarse sites x N1 dof) in column order. A piece
// whose norm drops below 1e-12 of its original norm sets *flag.
__global__ __launch_bounds__(TPB) void build_P2_kernel(int Vc, int N1, int N2, int Va2, const int *__restrict__ sites,
                                                       double2 *__restrict__ P2, int *__restrict__ flag) {
    __shared__ double red[TPB / 64];
    const int A = blockIdx.x, chi = blockIdx.y;
    const int ne = Va2 * N1;
    const size_t vs = (size_t)Vc * 2 * N1;   // one coarse vector
    auto idx = [&](int e) { return ((size_t)sites[(size_t)A * Va2 + e / N1] * 2 + chi) * N1 + e % N1; };
    for (int k = 0; k < N2; k++) {
        double2 *pk = P2 + (size_t)k * vs;
        double n0 = 0;
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            double2 v = pk[idx(e)];
            n0 += v.x * v.x + v.y * v.y;
        }
        n0 = block_sum_d(n0, red);
        for (int j = 0; j < k; j++) {
            const double2 *pj = P2 + (size_t)j * vs;
            double re = 0, im = 0;
            for (int e = threadIdx.x; e < ne; e += blockDim.x) {
                double2 a = pj[idx(e)], b = pk[idx(e)];
                re += a.x * b.x + a.y * b.y;
                im += a.x * b.y - a.y * b.x;
            }
            re = block_sum_d(re, red);
            im = block_sum_d(im, red);
            for (int e = threadIdx.x; e < ne; e += blockDim.x) {
                double2 a = pj[idx(e)], b = pk[idx(e)];
                pk[idx(e)] = make_double2(b.x - (re * a.x - im * a.y), b.y - (re * a.y + im * a.x));
            }
        }
        double nn = 0;
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            double2 v = pk[idx(e)];
            nn += v.x * v.x + v.y * v.y;
        }
        nn = block_sum_d(nn, red);
        if (!(nn > 1e-24 * n0) || !(nn > 0)) {
            if (threadIdx.x == 0) atomicOr(flag, 1);
            nn = 1.0;
        }
        const double s = 1.0 / sqrt(nn);
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            double2 v = pk[idx(e)];
            pk[idx(e)] = make_double2(v.x * s, v.y * s);
        }
    }
}

// out[r][A][chi][k] = sum over the piece (A, chi) of conj(P2[k]) c[r]: one
// workgroup per (A, r), one thread per output (chi, k)
template <typename T>
__global__ __launch_bounds__(TPB) void restrict2_kernel(int Vc, int Vcc, int N1, int N2, int Va2,
                                                        const int *__restrict__ sites, const C<T> *__restrict__ P2,
                                                        const C<T> *__restrict__ c, C<T> *__restrict__ out) {
    const int A = blockIdx.x, r = blockIdx.y;
    const size_t vs = (size_t)Vc * 2 * N1;
    const C<T> *cr = c + (size_t)r * vs;
    for (int q = threadIdx.x; q < 2 * N2; q += blockDim.x) {
        const int chi = q / N2, k = q % N2;
        const C<T> *pk = P2 + (size_t)k * vs;
        C<T> acc = mk<T>(0, 0);
        for (int l = 0; l < Va2; l++) {
            const size_t base = ((size_t)sites[(size_t)A * Va2 + l] * 2 + chi) * N1;
            for (int i = 0; i < N1; i++) cfmac(acc, pk[base + i], cr[base + i]);
        }
        out[((size_t)r * Vcc + A) * 2 * N2 + q] = acc;
    }
}

// out[r][a][chi][i] = sum_k P2[k][a][chi][i] cc[r][A(a)][chi][k]
template <typename T>
__global__ __launch_bounds__(TPB) void prolong2_kernel(int Vc, int Vcc, int N1, int N2, const int *__restrict__ site_agg,
                                                       const C<T> *__restrict__ P2, const C<T> *__restrict__ cc,
                                                       C<T> *__restrict__ out, int nrhs) {
    const size_t vs = (size_t)Vc * 2 * N1;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= vs * nrhs) return;
    const int r = (int)(e / vs);
    const size_t el = e % vs;
    const int a = (int)(el / (2 * N1)), chi = (int)((el / N1) % 2);
    const C<T> *ccr = cc + ((size_t)r * Vcc + site_agg[a]) * 2 * N2 + (size_t)chi * N2;
    C<T> acc = mk<T>(0, 0);
    for (int k = 0; k < N2; k++) cfma(acc, P2[(size_t)k * vs + el], ccr[k]);
    out[e] = acc;
}

// D_cc column (chi', k') of level-3 site B, all 9 blocks. Phase 1, one
// thread per (coarse site l of B, row i of its 2 N1): W[dout][l][i] = sum
// over the hops d of D_c into site a (a' = nbr(a, d)) of the class dout
// (0 when a' is reached without crossing B's face in direction d, else d)
// of (D_c[a][d] P2[k'] restricted to a' and chirality chi')[i]. Phase 2, one
// thread per (dout, row (chi, k)): the projection onto P2[k] on B, chi.
__global__ __launch_bounds__(1024) void dcc_build_kernel(int Vc, int N1, int N2, int Va2, const int *__restrict__ Lc,
                                                         const int *__restrict__ agg2, const int *__restrict__ sites,
                                                         const int *__restrict__ cnbr, const double2 *__restrict__ Dc,
                                                         const double2 *__restrict__ P2, double2 *__restrict__ Dcc) {
    extern __shared__ double2 W[];   // [9][Va2][2 N1]
    const int B = blockIdx.x, col = blockIdx.y;
    const int chic = col / N2, kc = col % N2;
    const int n1 = 2 * N1, n3 = 2 * N2;
    const size_t vs = (size_t)Vc * n1;
    for (int t = threadIdx.x; t < Va2 * n1; t += blockDim.x) {
        const int l = t / n1, i = t % n1;
        const int a = sites[(size_t)B * Va2 + l];
        int x[4], rem = a;
        for (int m = 0; m < 4; m++) { x[m] = rem % Lc[m]; rem /= Lc[m]; }
        double2 acc[9];
#pragma unroll
        for (int q = 0; q < 9; q++) acc[q] = make_double2(0, 0);
#pragma unroll
        for (int d = 0; d < 9; d++) {
            int dout = 0;
            if (d > 0) {
                const int mu = (d - 1) / 2, s = (d - 1) % 2;
                const int rr = x[mu] % agg2[mu];
                const bool crosses = s == 0 ? rr == agg2[mu] - 1 : rr == 0;
                dout = crosses ? d : 0;
            }
            const int ap = cnbr[(size_t)a * 9 + d];
            const double2 *blk = Dc + ((size_t)a * 9 + d) * n1 * n1;   // [col][row]
            const double2 *pv = P2 + (size_t)kc * vs + ((size_t)ap * 2 + chic) * N1;
            double2 s2 = make_double2(0, 0);
            for (int j = 0; j < N1; j++) cfma(s2, blk[(size_t)(chic * N1 + j) * n1 + i], pv[j]);
#pragma unroll
            for (int q = 0; q < 9; q++)
                if (q == dout) acc[q] = cadd(acc[q], s2);
        }
#pragma unroll
        for (int q = 0; q < 9; q++) W[((size_t)q * Va2 + l) * n1 + i] = acc[q];
    }
    __syncthreads();
    const size_t blk3 = (size_t)n3 * n3;
    for (int t = threadIdx.x; t < 9 * n3; t += blockDim.x) {
        const int dout = t / n3, row = t % n3, chi = row / N2, k = row % N2;
        const double2 *pk = P2 + (size_t)k * vs;
        double2 acc = make_double2(0, 0);
        for (int l = 0; l < Va2; l++) {
            const int a = sites[(size_t)B * Va2 + l];
            const double2 *pr = pk + ((size_t)a * 2 + chi) * N1;
            const double2 *wr = W + ((size_t)dout * Va2 + l) * n1 + (size_t)chi * N1;
            for (int i = 0; i < N1; i++) cfmac(acc, pr[i], wr[i]);
        }
        Dcc[((size_t)B * 9 + dout) * blk3 + (size_t)col * n3 + row] = acc;
    }
}

// Colour step of the level-2 Schwarz smoother (Algorithm 2.1 on D_c): one
// workgroup per block of coarse sites (blocks of one colour, blockIdx.y the
// right-hand side), one thread per (site l of the block, row i of its 2 N1).
// r = b - D_c z on the block (all nine terms), then MR(mr) on the block
// operator (terms whose neighbour lies in the block; lnbr < 0 otherwise)
// from e = 0 with rho in LDS, and z += e.
// sum_j B[j n1] x[j] over j < n1 (one row of a column-major 2N x 2N block
// times x) in two interleaved FMA chains, so that loads overlap
template <typename T>
__device__ inline C<T> row_dot(const C<T> *__restrict__ B, const C<T> *x, int n1) {
    C<T> a0 = mk<T>(0, 0), a1 = mk<T>(0, 0);
    int j = 0;
#pragma unroll 4
    for (; j + 1 < n1; j += 2) {
        cfma(a0, B[(size_t)j * n1], x[j]);
        cfma(a1, B[(size_t)(j + 1) * n1], x[j + 1]);
    }
    if (j < n1) cfma(a0, B[(size_t)j * n1], x[j]);
    return cadd(a0, a1);
}

template <typename T>
__global__ __launch_bounds__(1024) void sap2_kernel(int Vc, int N1, int Vb2, int blk0, const int *__restrict__ bsites,
                                                    const int *__restrict__ lnbr, const int *__restrict__ gnbr,
                                                    const C<T> *__restrict__ Dc, const C<T> *__restrict__ b,
                                                    C<T> *__restrict__ z, int mr) {
    extern __shared__ unsigned char smem2[];
    const int n1 = 2 * N1;
    C<T> *rho = (C<T> *)smem2;                 // [Vb2][n1]
    double *red = (double *)(rho + Vb2 * n1);  // [3 * waves]
    const int blk = blk0 + blockIdx.x, r = blockIdx.y;
    const int t = threadIdx.x, l = t / n1, i = t % n1;
    const bool act = l < Vb2;
    const size_t vs = (size_t)Vc * n1;
    const C<T> *br = b + (size_t)r * vs;
    C<T> *zr = z + (size_t)r * vs;
    int a = 0;
    if (act) a = bsites[(size_t)blk * Vb2 + l];
    // residual
    C<T> rv = mk<T>(0, 0);
    if (act) {
        C<T> acc = mk<T>(0, 0);
        for (int d = 0; d < 9; d++) {
            const int ap = gnbr[((size_t)blk * Vb2 + l) * 9 + d];
            const C<T> *B = Dc + ((size_t)a * 9 + d) * n1 * n1 + i;
            acc = cadd(acc, row_dot<T>(B, zr + (size_t)ap * n1, n1));
        }
        rv = csub(br[(size_t)a * n1 + i], acc);
        rho[l * n1 + i] = rv;
    }
    C<T> e = mk<T>(0, 0);
    __syncthreads();
    const int wv = t >> 6, lane = t & 63, nw = blockDim.x >> 6;
    for (int it = 0; it < mr; it++) {
        C<T> q = mk<T>(0, 0);
        if (act) {
            for (int d = 0; d < 9; d++) {
                const int ln = lnbr[((size_t)blk * Vb2 + l) * 9 + d];
                if (ln < 0) continue;
                const C<T> *B = Dc + ((size_t)a * 9 + d) * n1 * n1 + i;
                q = cadd(q, row_dot<T>(B, rho + ln * n1, n1));
            }
        }
        double p0 = (double)q.x * q.x + (double)q.y * q.y;
        double p1 = (double)q.x * rv.x + (double)q.y * rv.y;   // conj(q) rho
        double p2 = (double)q.x * rv.y - (double)q.y * rv.x;
        p0 = wave_sum_d(p0);
        p1 = wave_sum_d(p1);
        p2 = wave_sum_d(p2);
        if (lane == 0) { red[3 * wv] = p0; red[3 * wv + 1] = p1; red[3 * wv + 2] = p2; }
        __syncthreads();
        double s0 = 0, s1 = 0, s2 = 0;
        for (int k = 0; k < nw; k++) { s0 += red[3 * k]; s1 += red[3 * k + 1]; s2 += red[3 * k + 2]; }
        if (s0 == 0.0) break;
        const C<T> alpha = mk<T>((T)(s1 / s0), (T)(s2 / s0));
        cfma(e, alpha, rv);
        rv = csub(rv, cmul(alpha, q));
        __syncthreads();   // every thread has read rho and red
        if (act) rho[l * n1 + i] = rv;
        __syncthreads();
    }
    if (act) zr[(size_t)a * n1 + i] = cadd(zr[(size_t)a * n1 + i], e);
}

template <typename T>
__global__ void to_f32_kernel(size_t n, const double2 *__restrict__ src, C<T> *__restrict__ dst) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = mk<T>((T)src[e].x, (T)src[e].y);
}

int upload(Ctx *c, int **dst, const std::vector<int> &v) {
    *dst = (int *)dalloc(c, v.size() * sizeof(int) + 4);
    if (!*dst) return MGDD_ENOMEM;
    return hip_check(c, hipMemcpy(*dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
}

}  // namespace

void level2_free(Ctx *c, bool keep_blocks) {
    Level2 &L2 = c->c2;
    void *old[] = {L2.P2_64, L2.P2_32, L2.Dcc64, L2.Dcc32, L2.cnbr2, L2.agg2_sites, L2.site_agg2, L2.geo, L2.tv2_64};
    (void)hipStreamSynchronize(c->stream);
    for (void *p : old) dfree(c, p);
    Level2 fresh;
    if (keep_blocks) {   // the Schwarz block tables depend on the coarse lattice only
        fresh.blk_sites = L2.blk_sites;
        fresh.blk_lnbr = L2.blk_lnbr;
        fresh.blk_nbr = L2.blk_nbr;
        for (int m = 0; m < 4; m++) fresh.blk[m] = L2.blk[m];
        fresh.nblk = L2.nblk;
        fresh.ncol0 = L2.ncol0;
        fresh.Vb2 = L2.Vb2;
    } else {
        for (void *p : {(void *)L2.blk_sites, (void *)L2.blk_lnbr, (void *)L2.blk_nbr}) dfree(c, p);
    }
    L2 = fresh;
}

// tables of the level-3 lattice for aggregates agg2 of coarse sites and N2 test vectors
int level2_setup(Ctx *c, const int *agg2, int N2) {
    const Level1 &L1 = c->c;
    Level2 &L2 = c->c2;
    if (!L1.ready) return fail(c, MGDD_ENOTREADY, "no coarse level (build P first)");
    for (int m = 0; m < 4; m++)
        if (agg2[m] <= 0 || L1.Lc[m] % agg2[m]) return fail(c, MGDD_ESHAPE, "level-2 aggregates must divide the coarse lattice");
    const int Va2 = agg2[0] * agg2[1] * agg2[2] * agg2[3];
    if (N2 <= 0 || N2 > 32) return fail(c, MGDD_EINVAL, "number of level-2 test vectors must be in 1..32");
    if (N2 > Va2 * L1.N) return fail(c, MGDD_ERANK, "more level-2 test vectors than dof per aggregate and chirality");
    int Lcc[4];
    for (int m = 0; m < 4; m++) Lcc[m] = L1.Lc[m] / agg2[m];
    const int Vcc = Lcc[0] * Lcc[1] * Lcc[2] * Lcc[3];
    bool same = L2.agg2_sites && L2.N2 == N2 && L2.N1 == L1.N && L2.Vcc == Vcc;
    for (int m = 0; m < 4 && same; m++) same = L2.agg[m] == agg2[m];
    if (same) return MGDD_OK;
    level2_free(c, true);
    const int Vc = L1.Vc;
    std::vector<int> sites((size_t)Vcc * Va2), site_agg(Vc), cnbr((size_t)Vcc * 9), lc(L1.Lc, L1.Lc + 4),
        ag(agg2, agg2 + 4);
    std::vector<int> fill(Vcc, 0);
    for (int a = 0; a < Vc; a++) {   // coarse sites in lexicographic order
        int t = a, x[4];
        for (int m = 0; m < 4; m++) { x[m] = t % L1.Lc[m]; t /= L1.Lc[m]; }
        int X[4];
        for (int m = 0; m < 4; m++) X[m] = x[m] / agg2[m];
        const int A = X[0] + Lcc[0] * (X[1] + Lcc[1] * (X[2] + Lcc[2] * X[3]));
        sites[(size_t)A * Va2 + fill[A]++] = a;
        site_agg[a] = A;
    }
    for (int A = 0; A < Vcc; A++) {
        int t = A, y0[4];
        for (int m = 0; m < 4; m++) { y0[m] = t % Lcc[m]; t /= Lcc[m]; }
        cnbr[(size_t)A * 9] = A;
        for (int m = 0; m < 4; m++)
            for (int dir = 0; dir < 2; dir++) {
                int y[4] = {y0[0], y0[1], y0[2], y0[3]};
                y[m] = (y[m] + (dir == 0 ? 1 : -1) + Lcc[m]) % Lcc[m];
                cnbr[(size_t)A * 9 + 1 + 2 * m + dir] = y[0] + Lcc[0] * (y[1] + Lcc[1] * (y[2] + Lcc[2] * y[3]));
            }
    }
    const int N1 = L1.N;
    const size_t vs = (size_t)Vc * 2 * N1, dsz = (size_t)Vcc * 9 * 4 * N2 * N2;
    L2.P2_64 = dalloc(c, vs * N2 * 16);
    L2.P2_32 = dalloc(c, vs * N2 * 8);
    L2.tv2_64 = dalloc(c, vs * N2 * 16);
    L2.Dcc64 = dalloc(c, dsz * 16);
    L2.Dcc32 = dalloc(c, dsz * 8);
    if (!L2.P2_64 || !L2.P2_32 || !L2.tv2_64 || !L2.Dcc64 || !L2.Dcc32) return MGDD_ENOMEM;
    int rc = upload(c, &L2.agg2_sites, sites);
    if (!rc) rc = upload(c, &L2.site_agg2, site_agg);
    if (!rc) rc = upload(c, &L2.cnbr2, cnbr);
    std::vector<int> geo(lc);
    geo.insert(geo.end(), ag.begin(), ag.end());
    if (!rc) rc = upload(c, &L2.geo, geo);
    if (rc) return rc;
    for (int m = 0; m < 4; m++) { L2.agg[m] = agg2[m]; L2.Lcc[m] = Lcc[m]; }
    L2.Vcc = Vcc;
    L2.Va2 = Va2;
    L2.N2 = N2;
    L2.N1 = N1;
    return MGDD_OK;
}

int launch_build_P2(Ctx *c, const void *tv2) {
    Level2 &L2 = c->c2;
    const Level1 &L1 = c->c;
    const size_t vs = (size_t)L1.Vc * 2 * L2.N1;
    int rc = hip_check(c, hipMemcpyAsync(L2.P2_64, tv2, vs * L2.N2 * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
    if (!rc && tv2 != L2.tv2_64)
        rc = hip_check(c, hipMemcpyAsync(L2.tv2_64, tv2, vs * L2.N2 * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
    int *flag = (int *)ensure_scratch(c, sizeof(int));
    if (!flag) return MGDD_ENOMEM;
    if (!rc) rc = hip_check(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream), "memset");
    if (rc) return rc;
    build_P2_kernel<<<dim3(L2.Vcc, 2), TPB, 0, c->stream>>>(L1.Vc, L2.N1, L2.N2, L2.Va2, L2.agg2_sites,
                                                            (double2 *)L2.P2_64, flag);
    rc = hip_check(c, hipGetLastError(), "build_P2 kernel");
    int hflag = 0;
    if (!rc) rc = hip_check(c, hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (rc) return rc;
    if (hflag) return fail(c, MGDD_ERANK, "level-2 test vectors are rank deficient on some aggregate");
    const size_t np = vs * L2.N2;
    to_f32_kernel<float><<<(unsigned)((np + 255) / 256), 256, 0, c->stream>>>(np, (const double2 *)L2.P2_64,
                                                                              (float2 *)L2.P2_32);
    return hip_check(c, hipGetLastError(), "convert");
}

int launch_dcc_build(Ctx *c) {
    Level2 &L2 = c->c2;
    const Level1 &L1 = c->c;
    const int n1 = 2 * L2.N1, n3 = 2 * L2.N2;
    const size_t lds = (size_t)9 * L2.Va2 * n1 * sizeof(double2);
    if (lds > c->lds_max) return fail(c, MGDD_ESHAPE, "level-2 aggregate too large for the D_cc build");
    dim3 grid(L2.Vcc, n3);
    const int *geo = L2.geo;
    dcc_build_kernel<<<grid, 1024, lds, c->stream>>>(L1.Vc, L2.N1, L2.N2, L2.Va2, geo, geo + 4, L2.agg2_sites,
                                                     L1.cnbr, (const double2 *)L1.Dc64, (const double2 *)L2.P2_64,
                                                     (double2 *)L2.Dcc64);
    int rc = hip_check(c, hipGetLastError(), "D_cc build kernel");
    if (rc) return rc;
    const size_t nd = (size_t)L2.Vcc * 9 * n3 * n3;
    to_f32_kernel<float><<<(unsigned)((nd + 255) / 256), 256, 0, c->stream>>>(nd, (const double2 *)L2.Dcc64,
                                                                              (float2 *)L2.Dcc32);
    rc = hip_check(c, hipGetLastError(), "convert");
    if (!rc) L2.ready = true;
    return rc;
}

// blocks of the level-2 Schwarz smoother on the coarse lattice
int level2_sap_setup(Ctx *c, const int *block2) {
    const Level1 &L1 = c->c;
    Level2 &L2 = c->c2;
    if (!L1.ready) return fail(c, MGDD_ENOTREADY, "no coarse level (build P first)");
    bool same = L2.blk_sites != nullptr;
    for (int m = 0; m < 4 && same; m++) same = L2.blk[m] == block2[m];
    if (same) return MGDD_OK;
    int nb[4], Vb2 = 1;
    for (int m = 0; m < 4; m++) {
        if (block2[m] <= 0 || L1.Lc[m] % block2[m])
            return fail(c, MGDD_ESHAPE, "level-2 Schwarz blocks must divide the coarse lattice");
        nb[m] = L1.Lc[m] / block2[m];
        if (nb[m] > 1 && nb[m] % 2) return fail(c, MGDD_ESHAPE, "level-2 Schwarz block counts must be even or 1");
        Vb2 *= block2[m];
    }
    if (Vb2 * 2 * L1.N > 1024) return fail(c, MGDD_ESHAPE, "level-2 Schwarz block too large (sites x 2N > 1024)");
    const int nblk = nb[0] * nb[1] * nb[2] * nb[3];
    // block order: colour 0 first, lexicographic within a colour
    std::vector<int> order, pos(nblk);
    for (int col = 0; col < 2; col++)
        for (int q = 0; q < nblk; q++) {
            int t = q, s = 0;
            for (int m = 0; m < 4; m++) { s += t % nb[m]; t /= nb[m]; }
            if (s % 2 == col) order.push_back(q);
        }
    int ncol0 = 0;
    for (int q = 0; q < nblk; q++) {
        int t = order[q], s = 0;
        for (int m = 0; m < 4; m++) { s += t % nb[m]; t /= nb[m]; }
        if (s % 2 == 0) ncol0++;
        pos[order[q]] = q;
    }
    std::vector<int> bsites((size_t)nblk * Vb2), lnbr((size_t)nblk * Vb2 * 9), gnbr((size_t)nblk * Vb2 * 9);
    std::vector<int> blk_of(L1.Vc), loc_of(L1.Vc), fill(nblk, 0);
    const int *Lc = L1.Lc;
    for (int a = 0; a < L1.Vc; a++) {
        int t = a, x[4];
        for (int m = 0; m < 4; m++) { x[m] = t % Lc[m]; t /= Lc[m]; }
        int bx[4];
        for (int m = 0; m < 4; m++) bx[m] = x[m] / block2[m];
        const int q = pos[bx[0] + nb[0] * (bx[1] + nb[1] * (bx[2] + nb[2] * bx[3]))];
        const int l = fill[q]++;
        bsites[(size_t)q * Vb2 + l] = a;
        blk_of[a] = q;
        loc_of[a] = l;
    }
    std::vector<int> cn((size_t)L1.Vc * 9);
    int rc = hip_check(c, hipMemcpy(cn.data(), L1.cnbr, cn.size() * sizeof(int), hipMemcpyDeviceToHost), "copy");
    if (rc) return rc;
    for (int q = 0; q < nblk; q++)
        for (int l = 0; l < Vb2; l++) {
            const int a = bsites[(size_t)q * Vb2 + l];
            for (int d = 0; d < 9; d++) {
                const int ap = cn[(size_t)a * 9 + d];
                gnbr[((size_t)q * Vb2 + l) * 9 + d] = ap;
                lnbr[((size_t)q * Vb2 + l) * 9 + d] = blk_of[ap] == q ? loc_of[ap] : -1;
            }
        }
    for (void *p : {(void *)L2.blk_sites, (void *)L2.blk_lnbr, (void *)L2.blk_nbr}) dfree(c, p);
    L2.blk_sites = L2.blk_lnbr = L2.blk_nbr = nullptr;
    rc = upload(c, &L2.blk_sites, bsites);
    if (!rc) rc = upload(c, &L2.blk_lnbr, lnbr);
    if (!rc) rc = upload(c, &L2.blk_nbr, gnbr);
    if (rc) return rc;
    for (int m = 0; m < 4; m++) L2.blk[m] = block2[m];
    L2.nblk = nblk;
    L2.ncol0 = ncol0;
    L2.Vb2 = Vb2;
    return MGDD_OK;
}

int launch_sap2(Ctx *c, int prec, int nrhs, int nsweeps, int mr, const void *b, void *z) {
    const Level1 &L1 = c->c;
    const Level2 &L2 = c->c2;
    const int n1 = 2 * L1.N, threads = ((L2.Vb2 * n1 + 63) / 64) * 64;
    const size_t lds = (size_t)L2.Vb2 * n1 * csize(prec) + 3 * 8 * (threads / 64);
    for (int s = 0; s < nsweeps; s++)
        for (int col = 0; col < 2; col++) {
            const int nbl = col ? L2.nblk - L2.ncol0 : L2.ncol0;
            if (nbl == 0) continue;
            dim3 grid(nbl, nrhs);
            const int blk0 = col ? L2.ncol0 : 0;
            if (prec == MGDD_F64)
                sap2_kernel<double><<<grid, threads, lds, c->stream>>>(L1.Vc, L1.N, L2.Vb2, blk0, L2.blk_sites,
                                                                       L2.blk_lnbr, L2.blk_nbr,
                                                                       (const double2 *)L1.Dc64, (const double2 *)b,
                                                                       (double2 *)z, mr);
            else
                sap2_kernel<float><<<grid, threads, lds, c->stream>>>(L1.Vc, L1.N, L2.Vb2, blk0, L2.blk_sites,
                                                                      L2.blk_lnbr, L2.blk_nbr, (const float2 *)L1.Dc32,
                                                                      (const float2 *)b, (float2 *)z, mr);
            int rc = hip_check(c, hipGetLastError(), "level-2 Schwarz kernel");
            if (rc) return rc;
        }
    return MGDD_OK;
}

int launch_restrict2(Ctx *c, int prec, int nrhs, const void *in, void *out) {
    const Level2 &L2 = c->c2;
    dim3 grid(L2.Vcc, nrhs);
    if (prec == MGDD_F64)
        restrict2_kernel<double><<<grid, TPB, 0, c->stream>>>(c->c.Vc, L2.Vcc, L2.N1, L2.N2, L2.Va2, L2.agg2_sites,
                                                              (const double2 *)L2.P2_64, (const double2 *)in,
                                                              (double2 *)out);
    else
        restrict2_kernel<float><<<grid, TPB, 0, c->stream>>>(c->c.Vc, L2.Vcc, L2.N1, L2.N2, L2.Va2, L2.agg2_sites,
                                                             (const float2 *)L2.P2_32, (const float2 *)in,
                                                             (float2 *)out);
    return hip_check(c, hipGetLastError(), "restrict2 kernel");
}

int launch_prolong2(Ctx *c, int prec, int nrhs, const void *in, void *out) {
    const Level2 &L2 = c->c2;
    const size_t n = (size_t)c->c.Vc * 2 * L2.N1 * nrhs;
    const unsigned nwg = (unsigned)((n + 255) / 256);
    if (prec == MGDD_F64)
        prolong2_kernel<double><<<nwg, 256, 0, c->stream>>>(c->c.Vc, L2.Vcc, L2.N1, L2.N2, L2.site_agg2,
                                                            (const double2 *)L2.P2_64, (const double2 *)in,
                                                            (double2 *)out, nrhs);
    else
        prolong2_kernel<float><<<nwg, 256, 0, c->stream>>>(c->c.Vc, L2.Vcc, L2.N1, L2.N2, L2.site_agg2,
                                                           (const float2 *)L2.P2_32, (const float2 *)in,
                                                           (float2 *)out, nrhs);
    return hip_check(c, hipGetLastError(), "prolong2 kernel");
}

}  // namespace mgdd
