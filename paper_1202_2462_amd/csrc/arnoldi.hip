// Arnoldi process on the coarse operator D_c for the fixed-step coarse GMRES
// (Section 4), in three kernels per step for nb right-hand sides at once:
//
//   apply:  v_j = w_j / ||w_j||  (the norm from the previous step's partial
//           sums), y = D_c v_j, and partial sums of <v_i, y> per coarse site;
//   orth:   h1 = <V, y> (summing the partials), y <- y - V h1, and partial
//           sums of <v_i, y>;
//   reorth: h2 = <V, y>, y <- y - V h2, and partial sums of ||y||^2.
//
// This is classical Gram-Schmidt with one re-orthogonalisation, the same
// arithmetic as the general solver path, with the normalisation and the dot
// products folded into the kernels that produce their operands. The coarse
// vectors are small (2N complex per coarse site), so the step count of
// launches, not bandwidth, decides the time. Every sum runs in a fixed order,
// and every workgroup that needs a coefficient adds the same partials in the
// same order, so results are deterministic.
#include "blas.h"
#include "coarse.h"
#include "transfer.h"

namespace mgdd {

namespace {

constexpr int TPB = 512;   // threads of the orthogonalisation and dot-product kernels (8 waves)
constexpr int APB = 1024;  // threads of the apply kernel: the 9 2N products of a site over many threads
constexpr int KMAX = 16;   // basis vectors of the coarse Arnoldi: at most 15 coarse GMRES steps
constexpr int VMAX = 16;   // basis vectors of one fused Gram-Schmidt pass

struct VecList {
    const void *p[VMAX];
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// out[q] = sum_{g < np} part[q * np + g] for q < nq, one wave per q (lanes
// take g = lane, lane + 64, ... in order, then a butterfly); the result is
// left in red[q] (LDS). Called by every thread of the workgroup.
__device__ inline void sum_partials(const double2 *__restrict__ part, int nq, int np, double2 *red) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int q = wv; q < nq; q += nw) {
        double a = 0, b = 0;
        for (int g = lane; g < np; g += 64) {
            double2 v = part[(size_t)q * np + g];
            a += v.x;
            b += v.y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) red[q] = make_double2(a, b);
    }
    __syncthreads();
}

// apply step. Grid (Vc, nb), 1024 threads share the 9 2N products of y(a)
// (dc_row_partial); wave 0 then forms y(a), row i in lane i, and wave k
// the dot product of basis vector k at site a with it. HC: Dc holds the
// compact blocks [Vc][5] (self and forward hops); the backward hops are the
// conjugate transposes of the forward hops of the four backward neighbours
// (dch_row_partial). Those blocks are the ones the neighbours read for their
// own forward hops, so that only 5 of the 9 blocks per site have to come from
// memory when the cache holds the rest.
template <typename T, bool HC = false>
__global__ __launch_bounds__(APB) void arnoldi_apply_kernel(int Vc, int N, const int *__restrict__ cnbr,
                                                            const int *__restrict__ order,
                                                            const C<T> *__restrict__ Dc, const C<T> *__restrict__ w,
                                                            const double2 *__restrict__ npart, int nnp, VecList V,
                                                            int j, C<T> *__restrict__ vj, C<T> *__restrict__ y,
                                                            double2 *__restrict__ part1, double2 *__restrict__ nr) {
    // consecutive entries of the visiting order on one XCD: the neighbours'
    // blocks and vectors are read again from that XCD's L2
    const int l = xcd_block(Vc), a = order ? order[l] : l, sg = blockIdx.y, nb = gridDim.y;
    const int n2 = 2 * N;
    const size_t so = (size_t)sg * Vc * n2;
    __shared__ double2 red[1];
    __shared__ C<T> xs[9 * 64];
    __shared__ C<T> part[APB];
    __shared__ C<T> partb[HC ? APB : 1];
    sum_partials(npart + (size_t)sg * nnp, 1, nnp, red);
    const double nn = red[0].x;
    const T sc = (T)(nn > 0 ? 1.0 / sqrt(nn) : 0.0);
    if (nr && a == 0 && threadIdx.x == 0) nr[sg] = make_double2(nn, 0);
    for (int e = threadIdx.x; e < 9 * n2; e += blockDim.x) {
        const int dd = e / n2, jj = e % n2;
        // HC term order: self, forward hops (directions 1, 3, 5, 7), backward
        const int dir = !HC ? dd : dd == 0 ? 0 : dd <= 4 ? 2 * dd - 1 : 2 * dd - 8;
        C<T> v = w[so + (size_t)cnbr[a * 9 + dir] * n2 + jj];
        xs[e] = mk<T>(v.x * sc, v.y * sc);
    }
    const size_t blk = (size_t)n2 * n2;
    __syncthreads();
    if (HC) {
        const C<T> *Fb[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) Fb[mu] = Dc + ((size_t)cnbr[a * 9 + 2 + 2 * mu] * 5 + 1 + mu) * blk;
        dch_row_partial<T>(Dc + (size_t)a * 5 * blk, Fb, xs, n2, part, partb);
    } else {
        dc_row_partial<T>(Dc + (size_t)a * 9 * blk, xs, n2, part);
    }
    __syncthreads();
    // wave 0 forms y(a) (row i in lane i) and stores it with v_j(a)
    __shared__ C<T> ys[64];
    if (threadIdx.x < 64) {
        const int i = threadIdx.x, nparts = APB / n2;
        C<T> yv = mk<T>(0, 0);
        if (i < n2) {
            for (int q = 0; q < nparts; q++) yv = cadd(yv, part[q * n2 + i]);
            if (HC)
                for (int q = 0; q < nparts; q++) yv = cadd(yv, partb[q * n2 + i]);
            y[so + (size_t)a * n2 + i] = yv;
            vj[so + (size_t)a * n2 + i] = xs[i];   // v_j at this site (direction 0 is the site itself)
        }
        ys[i] = yv;
    }
    __syncthreads();
    // dot products <v_k(a), y(a)>, k <= j: wave k (a second round for k >= 16)
    const int i = threadIdx.x & 63;
    for (int k0 = threadIdx.x >> 6; k0 <= j; k0 += APB / 64) {
        const int k = __builtin_amdgcn_readfirstlane(k0);   // one basis vector per wave: a scalar pointer
        C<T> xv = mk<T>(0, 0);
        if (i < n2) xv = k < j ? ((const C<T> *)V.p[k])[so + (size_t)a * n2 + i] : xs[i];
        const C<T> yv = ys[i];
        double2 d = make_double2(0, 0);
        cfmac(d, make_double2((double)xv.x, (double)xv.y), make_double2((double)yv.x, (double)yv.y));
        const double re = wave_sum(d.x), im = wave_sum(d.y);
        if (i == 0) part1[((size_t)k * nb + sg) * Vc + a] = make_double2(re, im);
    }
}

// orth / reorth step: y <- y - sum_k coef_k v_k over k < nk, coef summed from
// pin (npin partials per coefficient); then partial sums of <v_k, y> (or of
// ||y||^2 when last) per workgroup into pout; workgroup 0 stores the
// coefficients in hout[k * nb + segment]. Grid (G, nb).
template <typename T, int NV>
__global__ __launch_bounds__(TPB) void arnoldi_orth_kernel(size_t n, VecList V, int nk, const double2 *__restrict__ pin,
                                                           int npin, C<T> *__restrict__ y, double2 *__restrict__ pout,
                                                           int last, double2 *__restrict__ hout) {
    const int sg = blockIdx.y, nb = gridDim.y, G = gridDim.x, g = blockIdx.x;
    const size_t so = (size_t)sg * n;
    __shared__ double2 coef[NV];
    __shared__ double red[TPB / 64][2 * NV];
    // the thread's first element (the only one when G * TPB >= n) is loaded
    // before the coefficients are summed: both loads are in flight together
    const size_t e0 = (size_t)g * TPB + threadIdx.x;
    C<T> y0 = mk<T>(0, 0), v0[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) v0[k] = mk<T>(0, 0);
    if (e0 < n) {
        y0 = y[so + e0];
#pragma unroll
        for (int k = 0; k < NV; k++)
            if (k < nk) v0[k] = ((const C<T> *)V.p[k])[so + e0];
    }
    // pin is laid out [k][segment][partial]. One wave per coefficient (wave
    // w takes k = w and w + 8): lane u adds the partials u, u + 64, ...
    // (four independent loads at a time), then a butterfly.
    for (int k = threadIdx.x >> 6; k < NV; k += TPB / 64) {
        const int u = threadIdx.x & 63;
        double a0 = 0, b0 = 0, a1 = 0, b1 = 0;
        if (k < nk) {
            const double2 *pk = pin + ((size_t)k * nb + sg) * npin;
            int q = u;
            for (; q + 192 < npin; q += 256) {
                const double2 v0 = pk[q], v1 = pk[q + 64], v2 = pk[q + 128], v3 = pk[q + 192];
                a0 += v0.x + v2.x;
                b0 += v0.y + v2.y;
                a1 += v1.x + v3.x;
                b1 += v1.y + v3.y;
            }
            for (; q < npin; q += 64) {
                a0 += pk[q].x;
                b0 += pk[q].y;
            }
        }
        const double a = wave_sum(a0 + a1), b = wave_sum(b0 + b1);
        if (k < nk && u == 0) coef[k] = make_double2(a, b);
    }
    __syncthreads();
    if (hout && g == 0 && (int)threadIdx.x < nk) hout[(size_t)threadIdx.x * nb + sg] = coef[threadIdx.x];
    const int nout = last ? 1 : nk;
    double2 acc[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) acc[k] = make_double2(0, 0);
    auto element = [&](size_t e, const C<T> yv, const C<T> *vv) {
        double2 r = make_double2((double)yv.x, (double)yv.y);
#pragma unroll
        for (int k = 0; k < NV; k++)
            if (k < nk) cfma(r, cneg(coef[k]), make_double2((double)vv[k].x, (double)vv[k].y));
        const C<T> rt = mk<T>((T)r.x, (T)r.y);
        y[so + e] = rt;
        const double2 rd = make_double2((double)rt.x, (double)rt.y);
        if (last) {
            acc[0].x += rd.x * rd.x + rd.y * rd.y;
        } else {
#pragma unroll
            for (int k = 0; k < NV; k++)
                if (k < nk) cfmac(acc[k], make_double2((double)vv[k].x, (double)vv[k].y), rd);
        }
    };
    if (e0 < n) element(e0, y0, v0);
    for (size_t e = e0 + (size_t)G * TPB; e < n; e += (size_t)G * TPB) {
        C<T> vv[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) vv[k] = k < nk ? ((const C<T> *)V.p[k])[so + e] : mk<T>(0, 0);
        element(e, y[so + e], vv);
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        if (k < nout) {
            double a = wave_sum(acc[k].x), b = wave_sum(acc[k].y);
            if (lane == 0) { red[wv][2 * k] = a; red[wv][2 * k + 1] = b; }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nout) {
        const int k = threadIdx.x;
        double a = 0, b = 0;
        for (int q = 0; q < TPB / 64; q++) { a += red[q][2 * k]; b += red[q][2 * k + 1]; }
        pout[((size_t)k * nb + sg) * G + g] = make_double2(a, b);
    }
}

// partial sums of <v_k, w> per workgroup: pout[(k * nb + segment) * G + g]
template <typename T, int NV>
__global__ __launch_bounds__(TPB) void dot_partials_kernel(size_t n, VecList V, int nk, const C<T> *__restrict__ w,
                                                           double2 *__restrict__ pout) {
    const int sg = blockIdx.y, nb = gridDim.y, G = gridDim.x, g = blockIdx.x;
    const size_t so = (size_t)sg * n;
    __shared__ double red[TPB / 64][2 * NV];
    double2 acc[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) acc[k] = make_double2(0, 0);
    for (size_t e = (size_t)g * TPB + threadIdx.x; e < n; e += (size_t)G * TPB) {
        const C<T> wv = w[so + e];
        const double2 wd = make_double2((double)wv.x, (double)wv.y);
#pragma unroll
        for (int k = 0; k < NV; k++) {
            if (k < nk) {
                C<T> v = ((const C<T> *)V.p[k])[so + e];
                cfmac(acc[k], make_double2((double)v.x, (double)v.y), wd);
            }
        }
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        if (k < nk) {
            double a = wave_sum(acc[k].x), b = wave_sum(acc[k].y);
            if (lane == 0) { red[wv][2 * k] = a; red[wv][2 * k + 1] = b; }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nk) {
        const int k = threadIdx.x;
        double a = 0, b = 0;
        for (int q = 0; q < TPB / 64; q++) { a += red[q][2 * k]; b += red[q][2 * k + 1]; }
        pout[((size_t)k * nb + sg) * G + g] = make_double2(a, b);
    }
}

// partial sums of ||x||^2 per workgroup: pout[segment * G + g]
template <typename T>
__global__ __launch_bounds__(TPB) void norm_partials_kernel(size_t n, const C<T> *__restrict__ x,
                                                            double2 *__restrict__ pout) {
    const int sg = blockIdx.y, G = gridDim.x, g = blockIdx.x;
    __shared__ double red[TPB / 64];
    double acc = 0;
    for (size_t e = (size_t)g * TPB + threadIdx.x; e < n; e += (size_t)G * TPB) {
        C<T> v = x[(size_t)sg * n + e];
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0;
        for (int q = 0; q < TPB / 64; q++) a += red[q];
        pout[(size_t)sg * G + g] = make_double2(a, 0);
    }
}

// out[q] = sum_g part[q * np + g], in a fixed order: thread t adds the
// entries t, t + NT, ..., then the waves' sums are added in wave order. NT =
// 64 for a few hundred partials, 1024 for one per coarse site (tens of
// thousands: one wave would wait on hundreds of dependent loads)
template <int NT>
__global__ __launch_bounds__(NT) void sum_kernel(int np, const double2 *__restrict__ part, double2 *__restrict__ out) {
    __shared__ double2 red[NT / 64];
    const int q = blockIdx.x, t = threadIdx.x;
    double a = 0, b = 0;
    for (int g = t; g < np; g += NT) {
        double2 v = part[(size_t)q * np + g];
        a += v.x;
        b += v.y;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (NT == 64) {
        if (t == 0) out[q] = make_double2(a, b);
        return;
    }
    if ((t & 63) == 0) red[t >> 6] = make_double2(a, b);
    __syncthreads();
    if (t == 0) {
        double2 s = make_double2(0, 0);
        for (int w = 0; w < NT / 64; w++) {
            s.x += red[w].x;
            s.y += red[w].y;
        }
        out[q] = s;
    }
}

// one element per thread up to 256 workgroups: these passes are short and
// latency-bound, but every workgroup of a pass first adds up the previous
// pass's per-workgroup partial sums, so fewer of them save more (at 12^3 x 24
// coarse sites with N = 20 an orthogonalisation pass took 66 us with 1024
// workgroups, 57 us with 512, 52 us with 256)
inline int orth_grid(size_t n) {
    size_t g = (n + TPB - 1) / TPB;
    return (int)(g < 1 ? 1 : g > 256 ? 256 : g);
}

}  // namespace

size_t coarse_arnoldi_scratch(const StencilOp &op, int m, int nb) {
    const size_t n = (size_t)op.V * 2 * op.N;
    const size_t G = orth_grid(n);
    return ((size_t)(m + 1) * nb * op.V + 3 * (size_t)(m + 1) * nb * G + 2 * (size_t)(m + 1) * nb) * 16 + 4096;
}

// m Arnoldi steps on D_c from b for nb segments. V: m + 1 basis vectors
// (written); work0, work1: two coarse vectors (nb segments each); scratch:
// coarse_arnoldi_scratch bytes. Outputs: H1, H2 (column j at j (m + 1) nb,
// entry [i][segment]) and NR (NR[j nb + segment] = squared norm of the
// j-th unnormalised vector, j = 0 .. m).
int launch_coarse_arnoldi(Ctx *c, const StencilOp &op, int p, int m, int nb, const void *b, void *const *V,
                          void *work0, void *work1, void *scratch, double2 *H1, double2 *H2, double2 *NR) {
    const int Vc = op.V, N = op.N;
    const size_t n = (size_t)Vc * 2 * N;
    const int G = orth_grid(n);
    if (m + 1 > KMAX) return fail(c, MGDD_EINVAL, "too many coarse GMRES steps for the fused Arnoldi kernels");
    double2 *part1 = (double2 *)scratch;                              // [k][s][Vc]
    double2 *part1s = part1 + (size_t)(m + 1) * nb * Vc;             // [k][s] (summed, large Vc)
    double2 *part2 = part1s + (size_t)(m + 1) * nb;                   // [k][s][G]
    double2 *part3 = part2 + (size_t)(m + 1) * nb * G;                // [s][G]
    const bool presum = Vc > 1024;
    dim3 gorth(G, nb);
#define NORMP(T) norm_partials_kernel<T><<<gorth, TPB, 0, c->stream>>>(n, (const C<T> *)b, part3)
    if (p == MGDD_F64) NORMP(double); else NORMP(float);
#undef NORMP
    int rc = hip_check(c, hipGetLastError(), "arnoldi");
    void *work[2] = {work0, work1};
    const void *w = b;
    for (int j = 0; j < m && !rc; j++) {
        VecList vl{};
        for (int k = 0; k <= j; k++) vl.p[k] = V[k];
        void *y = work[j & 1];
        dim3 gapp(Vc, nb);
        // the norm of w: summed once here when every workgroup of the apply
        // would otherwise add many partials, else by each workgroup
        const double2 *np = part3;
        int nnp = G;
        double2 *nrj = NR + (size_t)j * nb;
        if ((size_t)G * Vc > ((size_t)1 << 20)) {
            sum_kernel<64><<<nb, 64, 0, c->stream>>>(G, part3, nrj);
            np = nrj;
            nnp = 1;
            nrj = nullptr;
        }
#define APPLY(T, HC, D, LDS)                                                                                       \
    arnoldi_apply_kernel<T, HC><<<gapp, APB, LDS, c->stream>>>(Vc, N, op.nbr, op.order, (const C<T> *)(D), (const C<T> *)w, \
                                                               np, nnp, vl, j, (C<T> *)V[j], (C<T> *)y, part1, nrj)
        // algorithmic bytes: the blocks once per launch (5 per coarse site when
        // compact, else 9), per right-hand side w read, y and v_j written and
        // the j earlier basis vectors read for the dot products
        const bool compact = p == MGDD_F32 && op.H32;
        const double cs = p == MGDD_F64 ? 16.0 : 8.0, n2d = 2.0 * N;
        const double abytes = (double)Vc * ((compact ? 5.0 : 9.0) * n2d * n2d * cs + nb * (3.0 + j) * n2d * cs);
        const int slot = kt_begin(c);
        if (p == MGDD_F64) APPLY(double, false, op.D64, 0);
        else if (compact) APPLY(float, true, op.H32, 0);
        else APPLY(float, false, op.D32, 0);
        kt_end(c, slot, KF_COARSE, p, (double)Vc * nb, abytes);
#undef APPLY
        const double2 *pin = part1;
        int npin = Vc;
        if (presum) {
            sum_kernel<1024><<<(j + 1) * nb, 1024, 0, c->stream>>>(Vc, part1, part1s);
            pin = part1s;
            npin = 1;
        }
        double2 *h1 = H1 + (size_t)j * (m + 1) * nb, *h2 = H2 + (size_t)j * (m + 1) * nb;
#define ORTH(T, PIN, NPIN, POUT, LAST, HOUT) \
    arnoldi_orth_kernel<T, KMAX><<<gorth, TPB, 0, c->stream>>>(n, vl, j + 1, PIN, NPIN, (C<T> *)y, POUT, LAST, HOUT)
        if (p == MGDD_F64) {
            ORTH(double, pin, npin, part2, 0, h1);
            ORTH(double, part2, G, part3, 1, h2);
        } else {
            ORTH(float, pin, npin, part2, 0, h1);
            ORTH(float, part2, G, part3, 1, h2);
        }
#undef ORTH
        rc = hip_check(c, hipGetLastError(), "arnoldi");
        w = y;
    }
    if (!rc) {
        sum_kernel<64><<<nb, 64, 0, c->stream>>>(G, part3, NR + (size_t)m * nb);
        rc = hip_check(c, hipGetLastError(), "arnoldi");
    }
    return rc;
}

// Least-squares step of a GMRES cycle of m <= LSQ_MAX_STEPS steps on the
// device, one workgroup (one wave) per right-hand side s. The (m+1) x m
// Hessenberg matrix (column j: h1 + h2 in rows 0..j, sqrt(nr[j+1]) in row
// j+1) is cut at the first zero subdiagonal entry (k columns) and reduced
// to upper triangular form by Givens rotations: lane 0 forms rotation j from
// column j and applies it to g = beta e_1, the lanes owning the later
// columns apply it to theirs. y then solves the triangular system (lane 0,
// back substitution), coef[i][s] = y_i for i < k and 0 for the rest; all 0
// when beta = sqrt(nr[0]) is 0. A non-finite beta or y sets *status (if
// given) to 1.
__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }

__global__ __launch_bounds__(64) void hessenberg_lsq_kernel(int m, int nb, const double2 *__restrict__ h1,
                                                            const double2 *__restrict__ h2,
                                                            const double2 *__restrict__ nr, double2 *__restrict__ coef,
                                                            int *__restrict__ status) {
    __shared__ double2 R[LSQ_MAX_STEPS][LSQ_MAX_STEPS + 2];   // [column][row]
    __shared__ double2 g[LSQ_MAX_STEPS + 1], y[LSQ_MAX_STEPS];
    __shared__ double rot_c;
    __shared__ double2 rot_s;
    const int s = blockIdx.x, l = threadIdx.x;
    const double beta = sqrt(nr[s].x);
    if (!(beta > 0.0) || !isfinite(beta)) {   // zero start vector: x = 0
        if (l < m) coef[(size_t)l * nb + s] = make_double2(0, 0);
        if (l == 0 && status && !isfinite(beta)) *status = 1;
        return;
    }
    int k = m;
    for (int j = 0; j < m; j++) {
        const double v = nr[(size_t)(j + 1) * nb + s].x;
        if (l == 0 && status && isnan(v)) *status = 1;
        if (!(v > 0.0)) { k = j + 1; break; }
    }
    if (l < k) {
        const size_t cj = (size_t)l * (m + 1) * nb;
        for (int i = 0; i <= l; i++) {
            const double2 a = h1[cj + (size_t)i * nb + s], b = h2[cj + (size_t)i * nb + s];
            R[l][i] = make_double2(a.x + b.x, a.y + b.y);
        }
        R[l][l + 1] = make_double2(sqrt(fmax(nr[(size_t)(l + 1) * nb + s].x, 0.0)), 0.0);
    }
    if (l <= k) g[l] = make_double2(l == 0 ? beta : 0.0, 0.0);
    __syncthreads();
    for (int j = 0; j < k; j++) {
        if (l == 0) {
            const double2 a = R[j][j], b = R[j][j + 1];
            const double aa = hypot(a.x, a.y), bb = hypot(b.x, b.y);
            double cr;
            double2 sr, rho;
            if (bb == 0.0) {
                cr = 1.0; sr = make_double2(0, 0); rho = a;
            } else if (aa == 0.0) {
                cr = 0.0; sr = make_double2(1, 0); rho = b;
            } else {
                const double r = hypot(aa, bb);
                const double2 ph = make_double2(a.x / aa, a.y / aa);
                cr = aa / r;
                const double2 t = zmul(ph, zconj(b));
                sr = make_double2(t.x / r, t.y / r);
                rho = make_double2(ph.x * r, ph.y * r);
            }
            R[j][j] = rho;
            R[j][j + 1] = make_double2(0, 0);
            const double2 gj = g[j];
            g[j] = make_double2(cr * gj.x, cr * gj.y);
            const double2 t = zmul(zconj(sr), gj);
            g[j + 1] = make_double2(-t.x, -t.y);
            rot_c = cr;
            rot_s = sr;
        }
        __syncthreads();
        if (l > j && l < k) {
            const double cr = rot_c;
            const double2 sr = rot_s, a = R[l][j], b = R[l][j + 1];
            const double2 u = zmul(sr, b), v = zmul(zconj(sr), a);
            R[l][j] = make_double2(cr * a.x + u.x, cr * a.y + u.y);
            R[l][j + 1] = make_double2(cr * b.x - v.x, cr * b.y - v.y);
        }
        __syncthreads();
    }
    if (l == 0) {
        bool ok = true;
        for (int i = k - 1; i >= 0; i--) {
            double2 t = g[i];
            for (int q = i + 1; q < k; q++) {
                const double2 u = zmul(R[q][i], y[q]);
                t = make_double2(t.x - u.x, t.y - u.y);
            }
            const double2 d = R[i][i];
            const double dn = d.x * d.x + d.y * d.y;
            const double2 yi = make_double2((t.x * d.x + t.y * d.y) / dn, (t.y * d.x - t.x * d.y) / dn);
            y[i] = yi;
            ok = ok && isfinite(yi.x) && isfinite(yi.y);
        }
        if (!ok && status) *status = 1;
    }
    __syncthreads();
    if (l < m) coef[(size_t)l * nb + s] = l < k ? y[l] : make_double2(0, 0);
}

// The same two passes for up to 64 vectors (the long Arnoldi runs of the
// setup's second part), in chunks of 16 vectors inside the kernels: the dot
// partials of each chunk are reduced and written before the next chunk.
constexpr int LMAX = 64;

struct VecList64 {
    const void *p[LMAX];
};

template <typename T>
__device__ inline void chunk_partials(const double2 (&acc)[16], int nq, int q0, int nb, int sg, int G, int g,
                                      double (*red)[32], double2 *__restrict__ pout) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 16; q++) {
        if (q < nq) {
            const double a = wave_sum(acc[q].x), b = wave_sum(acc[q].y);
            if (lane == 0) { red[wv][2 * q] = a; red[wv][2 * q + 1] = b; }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nq) {
        const int q = threadIdx.x;
        double a = 0, b = 0;
        for (int u = 0; u < TPB / 64; u++) { a += red[u][2 * q]; b += red[u][2 * q + 1]; }
        pout[((size_t)(q0 + q) * nb + sg) * G + g] = make_double2(a, b);
    }
    __syncthreads();
}

// partial sums of <v_k, w> per workgroup, k < nk <= 64: pout[(k * nb + segment) * G + g]
template <typename T>
__global__ __launch_bounds__(TPB) void dot_partials_long_kernel(size_t n, VecList64 V, int nk,
                                                                const C<T> *__restrict__ w,
                                                                double2 *__restrict__ pout) {
    const int sg = blockIdx.y, nb = gridDim.y, G = gridDim.x, g = blockIdx.x;
    const size_t so = (size_t)sg * n;
    __shared__ double red[TPB / 64][32];
    for (int q0 = 0; q0 < nk; q0 += 16) {
        const int nq = nk - q0 < 16 ? nk - q0 : 16;
        double2 acc[16];
#pragma unroll
        for (int q = 0; q < 16; q++) acc[q] = make_double2(0, 0);
        for (size_t e = (size_t)g * TPB + threadIdx.x; e < n; e += (size_t)G * TPB) {
            const C<T> wv = w[so + e];
            const double2 wd = make_double2((double)wv.x, (double)wv.y);
#pragma unroll
            for (int q = 0; q < 16; q++) {
                if (q < nq) {
                    const C<T> v = ((const C<T> *)V.p[q0 + q])[so + e];
                    cfmac(acc[q], make_double2((double)v.x, (double)v.y), wd);
                }
            }
        }
        chunk_partials<T>(acc, nq, q0, nb, sg, G, g, red, pout);
    }
}

// y <- y - sum_k coef_k v_k over k < nk <= 64, coef summed from pin (npin
// partials each, [k][segment][partial]); then the partials of <v_k, y> (or of
// ||y||^2 when last) per workgroup into pout
template <typename T>
__global__ __launch_bounds__(TPB) void orth_long_kernel(size_t n, VecList64 V, int nk, const double2 *__restrict__ pin,
                                                        int npin, C<T> *__restrict__ y, double2 *__restrict__ pout,
                                                        int last) {
    const int sg = blockIdx.y, nb = gridDim.y, G = gridDim.x, g = blockIdx.x;
    const size_t so = (size_t)sg * n;
    __shared__ double2 coef[LMAX];
    __shared__ double red[TPB / 64][32];
    // one wave per coefficient (wave w takes k = w, w + 8, ...): lane u adds
    // the partials u, u + 64, ... in order, then a butterfly
    for (int k = threadIdx.x >> 6; k < nk; k += TPB / 64) {
        const int u = threadIdx.x & 63;
        const double2 *pk = pin + ((size_t)k * nb + sg) * npin;
        double a = 0, b = 0;
        for (int q = u; q < npin; q += 64) {
            a += pk[q].x;
            b += pk[q].y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (u == 0) coef[k] = make_double2(a, b);
    }
    __syncthreads();
    double nacc = 0;
    for (size_t e = (size_t)g * TPB + threadIdx.x; e < n; e += (size_t)G * TPB) {
        const C<T> yv = y[so + e];
        double2 r = make_double2((double)yv.x, (double)yv.y);
        for (int q0 = 0; q0 < nk; q0 += 16) {
#pragma unroll
            for (int q = 0; q < 16; q++) {
                if (q0 + q < nk) {
                    const C<T> v = ((const C<T> *)V.p[q0 + q])[so + e];
                    cfma(r, cneg(coef[q0 + q]), make_double2((double)v.x, (double)v.y));
                }
            }
        }
        const C<T> rt = mk<T>((T)r.x, (T)r.y);
        y[so + e] = rt;
        nacc += (double)rt.x * rt.x + (double)rt.y * rt.y;
    }
    if (last) {
        double2 acc[16];
#pragma unroll
        for (int q = 0; q < 16; q++) acc[q] = make_double2(q == 0 ? nacc : 0.0, 0);
        chunk_partials<T>(acc, 1, 0, nb, sg, G, g, red, pout);
        return;
    }
    for (int q0 = 0; q0 < nk; q0 += 16) {
        const int nq = nk - q0 < 16 ? nk - q0 : 16;
        double2 acc[16];
#pragma unroll
        for (int q = 0; q < 16; q++) acc[q] = make_double2(0, 0);
        for (size_t e = (size_t)g * TPB + threadIdx.x; e < n; e += (size_t)G * TPB) {
            const C<T> yv = y[so + e];   // this thread's own updated element
            const double2 yd = make_double2((double)yv.x, (double)yv.y);
#pragma unroll
            for (int q = 0; q < 16; q++) {
                if (q < nq) {
                    const C<T> v = ((const C<T> *)V.p[q0 + q])[so + e];
                    cfmac(acc[q], make_double2((double)v.x, (double)v.y), yd);
                }
            }
        }
        chunk_partials<T>(acc, nq, q0, nb, sg, G, g, red, pout);
    }
}

size_t fused_cgs2_red_doubles(size_t n, int k, int nb) {
    return 2 * (2 * (size_t)k + 1) * nb * (size_t)orth_grid(n) + 16;
}

// Classical Gram-Schmidt with one re-orthogonalisation of w against the k
// vectors V (nb segments of length n each) in three passes over memory:
// dot partials; subtract the first projection (coefficients summed first)
// with the dot partials of the second; subtract the second with the partials
// of the squared norm. Outputs: h1[i][s], h2[i][s], nrm[s] (device).
int fused_cgs2(Ctx *c, int p, size_t n, int nb, void *const *V, int k, void *w, double2 *h1, double2 *h2,
               double2 *nrm) {
    if (k < 1 || k > LMAX) return fail(c, MGDD_EINVAL, "fused Gram-Schmidt: bad vector count");
    const int G = orth_grid(n);
    double2 *part = (double2 *)ensure_red(c, fused_cgs2_red_doubles(n, k, nb));
    if (!part) return MGDD_ENOMEM;
    double2 *part2 = part + (size_t)k * nb * G;
    if (k > VMAX) {
        VecList64 vl{};
        for (int i = 0; i < k; i++) vl.p[i] = V[i];
        dim3 grid(G, nb);
#define CGSL(T)                                                                                                   \
    do {                                                                                                          \
        dot_partials_long_kernel<T><<<grid, TPB, 0, c->stream>>>(n, vl, k, (const C<T> *)w, part);                 \
        sum_kernel<64><<<k * nb, 64, 0, c->stream>>>(G, part, h1);                                                    \
        orth_long_kernel<T><<<grid, TPB, 0, c->stream>>>(n, vl, k, h1, 1, (C<T> *)w, part2, 0);                   \
        sum_kernel<64><<<k * nb, 64, 0, c->stream>>>(G, part2, h2);                                                   \
        orth_long_kernel<T><<<grid, TPB, 0, c->stream>>>(n, vl, k, h2, 1, (C<T> *)w, part, 1);                    \
        sum_kernel<64><<<nb, 64, 0, c->stream>>>(G, part, nrm);                                                       \
    } while (0)
        if (p == MGDD_F64) CGSL(double); else CGSL(float);
#undef CGSL
        return hip_check(c, hipGetLastError(), "fused Gram-Schmidt");
    }
    VecList vl{};
    for (int i = 0; i < k; i++) vl.p[i] = V[i];
    dim3 grid(G, nb);
#define CGS(T, NV)                                                                                                 \
    do {                                                                                                           \
        dot_partials_kernel<T, NV><<<grid, TPB, 0, c->stream>>>(n, vl, k, (const C<T> *)w, part);                  \
        sum_kernel<64><<<k * nb, 64, 0, c->stream>>>(G, part, h1);                                                     \
        arnoldi_orth_kernel<T, NV><<<grid, TPB, 0, c->stream>>>(n, vl, k, h1, 1, (C<T> *)w, part2, 0, nullptr);  \
        sum_kernel<64><<<k * nb, 64, 0, c->stream>>>(G, part2, h2);                                                    \
        arnoldi_orth_kernel<T, NV><<<grid, TPB, 0, c->stream>>>(n, vl, k, h2, 1, (C<T> *)w, part, 1, nullptr);   \
        sum_kernel<64><<<nb, 64, 0, c->stream>>>(G, part, nrm);                                                        \
    } while (0)
    if (p == MGDD_F64) {
        if (k <= 4) CGS(double, 4); else if (k <= 8) CGS(double, 8); else CGS(double, 16);
    } else {
        if (k <= 4) CGS(float, 4); else if (k <= 8) CGS(float, 8); else CGS(float, 16);
    }
#undef CGS
    return hip_check(c, hipGetLastError(), "fused Gram-Schmidt");
}

int launch_hessenberg_lsq(Ctx *c, int m, int nb, const double2 *h1, const double2 *h2, const double2 *nr, double2 *coef,
                          int *status) {
    if (m < 1 || m > LSQ_MAX_STEPS) return fail(c, MGDD_EINVAL, "device least squares: bad step count");
    hessenberg_lsq_kernel<<<nb, 64, 0, c->stream>>>(m, nb, h1, h2, nr, coef, status);
    return hip_check(c, hipGetLastError(), "least squares");
}

}  // namespace mgdd
