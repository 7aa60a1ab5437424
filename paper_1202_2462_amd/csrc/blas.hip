// Level-1 kernels on flat complex arrays for the Krylov methods: multi-dot
// products (several vectors against one, in one pass over memory), linear
// combinations y = beta y + alpha sum_i c_i x_i with the coefficients read
// from device memory (so that Gram-Schmidt needs no host round trip), and
// scaling. Every operation works on nseg independent segments of length n at
// once (the right-hand sides of a batched solve, segment s at offset s * n
// of every array; coefficients and results indexed [i][s]); the segment is
// the second grid dimension. Reductions are deterministic: a fixed grid for a
// given length, a fixed butterfly inside each wave, per-workgroup partials
// summed in a fixed order by a second kernel. Sums are accumulated in double.
#include "blas.h"

namespace mgdd {

namespace {

constexpr int TPB = 256;

inline int red_grid(size_t n) {
    size_t g = (n + TPB * 4 - 1) / (TPB * 4);
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (int)g;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// part[i * nwg + wg] = sum over the elements of workgroup wg of conj(x_i) w.
// (A single-kernel variant in which the last workgroup adds the partials
// needs a device-scope release by every workgroup, which writes back L2 on
// every XCD and made the kernel five times slower; a second small kernel
// adds the partials instead.)
template <typename TX, typename TW, int NV, typename PL = PtrList>
__global__ __launch_bounds__(TPB) void multidot_kernel(size_t n, PL xs, int nvec, const C<TW> *__restrict__ w,
                                                       double2 *__restrict__ part) {
    __shared__ double red[TPB / 64][2 * NV];
    double2 acc[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) acc[i] = make_double2(0, 0);
    // slots past nvec read the last vector again (from cache) and their sums
    // are dropped: the loads of one element carry no branches between them and
    // are all in flight at once
    const C<TX> *xp[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) xp[i] = (const C<TX> *)xs.p[i < nvec ? i : nvec - 1];
    const size_t stride = (size_t)gridDim.x * TPB, so = (size_t)blockIdx.y * n;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n; e += stride) {
        C<TW> wv = w[so + e];
        double2 wd = make_double2((double)wv.x, (double)wv.y);
        C<TX> xv[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) xv[i] = xp[i][so + e];
#pragma unroll
        for (int i = 0; i < NV; i++) cfmac(acc[i], make_double2((double)xv[i].x, (double)xv[i].y), wd);
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        if (i < nvec) {
            double a = wave_sum(acc[i].x), b = wave_sum(acc[i].y);
            if (lane == 0) { red[wv][2 * i] = a; red[wv][2 * i + 1] = b; }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nvec) {
        int i = threadIdx.x;
        double a = 0, b = 0;
        for (int k = 0; k < TPB / 64; k++) { a += red[k][2 * i]; b += red[k][2 * i + 1]; }
        part[((size_t)i * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = make_double2(a, b);
    }
}

// out[q] = sum_k part[q * nwg + k] (q = i * nseg + s): one 64-lane wave per q,
// lane l adding the partials k = l, l + 64, ... in order, then a butterfly.
__global__ __launch_bounds__(64) void finish_kernel(int nwg, const double2 *__restrict__ part, double2 *__restrict__ out) {
    const int i = blockIdx.x, lane = threadIdx.x;
    double a = 0, b = 0;
    for (int k = lane; k < nwg; k += 64) {
        double2 v = part[(size_t)i * nwg + k];
        a += v.x;
        b += v.y;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) out[i] = make_double2(a, b);
}

// y = beta y + alpha sum_i coef[i] x_i
// (coefficient of vector i for segment s: coef[i * cstride + s])
template <typename TX, typename TY, int NV>
__global__ __launch_bounds__(TPB) void lincomb_kernel(size_t n, PtrList xs, int nvec, const double2 *__restrict__ coef,
                                                      int cstride, double alpha, double beta, C<TY> *__restrict__ y) {
    double2 c[NV];
#pragma unroll
    for (int i = 0; i < NV; i++)
        c[i] = i < nvec ? cscale(coef[(size_t)i * cstride + blockIdx.y], alpha) : make_double2(0, 0);
    // slots past nvec read the last vector again (from cache) with
    // coefficient 0, so that no branch separates the loads of one element
    const C<TX> *xp[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) xp[i] = (const C<TX> *)xs.p[i < nvec ? i : (nvec > 0 ? nvec - 1 : 0)];
    const size_t stride = (size_t)gridDim.x * TPB, so = (size_t)blockIdx.y * n;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n; e += stride) {
        double2 acc = make_double2(0, 0);
        if (beta != 0.0) {
            C<TY> yv = y[so + e];
            acc = make_double2(beta * (double)yv.x, beta * (double)yv.y);
        }
        if (nvec > 0) {
            C<TX> xv[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) xv[i] = xp[i][so + e];
#pragma unroll
            for (int i = 0; i < NV; i++) cfma(acc, c[i], make_double2((double)xv[i].x, (double)xv[i].y));
        }
        y[so + e] = mk<TY>((TY)acc.x, (TY)acc.y);
    }
}

// y <- y - sum_i coef[i * nseg + s] x_i, then the partial sums of the new y
// against every x_i (mode 0) or of ||y||^2 (mode 1) per workgroup into part, laid out as
// multidot's: one pass over the x_i instead of a lincomb and a multidot (the
// later passes of classical Gram-Schmidt). The update arithmetic is that of
// lincomb_kernel.
template <typename T, int NV>
__global__ __launch_bounds__(TPB) void update_dot_kernel(size_t n, PtrList xs, int nvec,
                                                         const double2 *__restrict__ coef, C<T> *__restrict__ y,
                                                         int mode, double2 *__restrict__ part) {
    const int norm_only = mode == 1;
    __shared__ double red[TPB / 64][2 * NV];
    double2 c[NV], acc[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) {
        c[i] = i < nvec ? cscale(coef[(size_t)i * gridDim.y + blockIdx.y], -1.0) : make_double2(0, 0);
        acc[i] = make_double2(0, 0);
    }
    // slots past nvec: the last vector again with coefficient 0 (see lincomb)
    const C<T> *xp[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) xp[i] = (const C<T> *)xs.p[i < nvec ? i : nvec - 1];
    const size_t stride = (size_t)gridDim.x * TPB, so = (size_t)blockIdx.y * n;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n; e += stride) {
        C<T> yv = y[so + e];
        double2 u = make_double2(1.0 * (double)yv.x, 1.0 * (double)yv.y);
        C<T> xr[NV];
        double2 xv[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) xr[i] = xp[i][so + e];
#pragma unroll
        for (int i = 0; i < NV; i++) {
            xv[i] = make_double2((double)xr[i].x, (double)xr[i].y);
            cfma(u, c[i], xv[i]);
        }
        const C<T> un = mk<T>((T)u.x, (T)u.y);
        y[so + e] = un;
        const double2 ud = make_double2((double)un.x, (double)un.y);
        if (norm_only) {
            cfmac(acc[0], ud, ud);
        } else {
#pragma unroll
            for (int i = 0; i < NV; i++) cfmac(acc[i], xv[i], ud);
        }
    }
    const int nout = norm_only ? 1 : nvec;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        if (i < nout) {
            double a = wave_sum(acc[i].x), b = wave_sum(acc[i].y);
            if (lane == 0) { red[wv][2 * i] = a; red[wv][2 * i + 1] = b; }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nout) {
        int i = threadIdx.x;
        double a = 0, b = 0;
        for (int k = 0; k < TPB / 64; k++) { a += red[k][2 * i]; b += red[k][2 * i + 1]; }
        part[((size_t)i * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = make_double2(a, b);
    }
}

struct PtrListW {
    const void *p[WIDE];
};

// The two passes of the outer Gram-Schmidt step with a lagged second pass
// (see blas.h). G lanes per element (fewer accumulators per lane than one
// lane per element with all the vectors: more waves in flight), each a group
// of 64 / G lanes of a wave; lane l of group g takes element l of the wave's
// range and the vectors g NG ... g NG + NG - 1, NV = G NG vector slots; the
// launcher fills the slots past nvec with vectors that group 0's lanes read
// at the same element (no extra memory traffic), and their coefficients are
// 0 or their sums dropped, so that no branch separates the loads.
//
// Pass A: partial sums of <x_i, w> (q = i) and <x_i, v> (q = nvec + i) per
// workgroup into part, laid out as multidot's.
template <int NG, int G>
__global__ __launch_bounds__(TPB) void dots2_kernel(size_t n, PtrListW xs, int nvec, const double2 *__restrict__ w,
                                                    const double2 *__restrict__ v, double2 *__restrict__ part) {
    constexpr int LG = 64 / G, NV = NG * G;
    __shared__ double red[TPB / 64][4 * NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, grp = lane / LG, gl = lane % LG;
    const double2 *xp[NG];
#pragma unroll
    for (int i = 0; i < NG; i++) xp[i] = (const double2 *)xs.p[grp * NG + i];
    double2 aw[NG], av[NG];
#pragma unroll
    for (int i = 0; i < NG; i++) aw[i] = av[i] = make_double2(0, 0);
    const size_t per = TPB / G, stride = (size_t)gridDim.x * per, so = (size_t)blockIdx.y * n;
    for (size_t e = (size_t)blockIdx.x * per + wv * LG + gl; e < n; e += stride) {
        const double2 wd = w[so + e], vd = v[so + e];
        double2 xv[NG];
#pragma unroll
        for (int i = 0; i < NG; i++) xv[i] = xp[i][so + e];
#pragma unroll
        for (int i = 0; i < NG; i++) {
            cfmac(aw[i], xv[i], wd);
            cfmac(av[i], xv[i], vd);
        }
    }
#pragma unroll
    for (int i = 0; i < NG; i++) {
        double a = aw[i].x, b = aw[i].y, c = av[i].x, d = av[i].y;
#pragma unroll
        for (int m = LG / 2; m >= 1; m >>= 1) {
            a += __shfl_xor(a, m, 64);
            b += __shfl_xor(b, m, 64);
            c += __shfl_xor(c, m, 64);
            d += __shfl_xor(d, m, 64);
        }
        const int q = grp * NG + i;
        if (gl == 0 && q < nvec) {
            red[wv][2 * q] = a;
            red[wv][2 * q + 1] = b;
            red[wv][2 * (NV + q)] = c;
            red[wv][2 * (NV + q) + 1] = d;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * nvec) {
        const int q = threadIdx.x, slot = q < nvec ? q : NV + q - nvec;
        double a = 0, b = 0;
        for (int k = 0; k < TPB / 64; k++) { a += red[k][2 * slot]; b += red[k][2 * slot + 1]; }
        part[((size_t)q * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = make_double2(a, b);
    }
}

// Pass B, for the vectors i0 ... i0 + nvec - 1 of ntot, with the coefficients
// of segment s at coef[q * nseg + s] (q = 0: a, 1: c, 2 + i: -s_i,
// 2 + ntot + i: -t_i):
//   v <- v + sum_i (-s_i) x_i,  w <- w + sum_i (-t_i) x_i,
// and in the last launch (last != 0) then v <- a v, w <- w + c v and the
// partial sums of ||w||^2 per workgroup into part.
template <int NG, int G>
__global__ __launch_bounds__(TPB) void dcgs_update_kernel(size_t n, PtrListW xs, int nvec, int i0, int ntot,
                                                          const double2 *__restrict__ coef, int last,
                                                          double2 *__restrict__ v, double2 *__restrict__ w,
                                                          double2 *__restrict__ part) {
    constexpr int LG = 64 / G, NV = NG * G;
    __shared__ double2 cs[2 * NV + 2];
    __shared__ double red[TPB / 64];
    const int nseg = gridDim.y, sg = blockIdx.y;
    if ((int)threadIdx.x < 2 * NV) {
        const int i = threadIdx.x % NV, q = 2 + ((int)threadIdx.x >= NV ? ntot : 0) + i0 + i;
        cs[threadIdx.x] = i < nvec ? coef[(size_t)q * nseg + sg] : make_double2(0, 0);
    }
    if (threadIdx.x == 0) {
        cs[2 * NV] = last ? coef[sg] : make_double2(1, 0);
        cs[2 * NV + 1] = last ? coef[(size_t)nseg + sg] : make_double2(0, 0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, grp = lane / LG, gl = lane % LG;
    const double2 *xp[NG];
#pragma unroll
    for (int i = 0; i < NG; i++) xp[i] = (const double2 *)xs.p[grp * NG + i];
    const double a = cs[2 * NV].x;
    const double2 cv = cs[2 * NV + 1];
    double accn = 0;
    const size_t per = TPB / G, stride = (size_t)gridDim.x * per, so = (size_t)blockIdx.y * n;
    for (size_t e = (size_t)blockIdx.x * per + wv * LG + gl; e < n; e += stride) {
        const double2 vd = v[so + e], wd = w[so + e];
        double2 xv[NG];
#pragma unroll
        for (int i = 0; i < NG; i++) xv[i] = xp[i][so + e];
        double2 uv = make_double2(0, 0), uw = make_double2(0, 0);
#pragma unroll
        for (int i = 0; i < NG; i++) {
            cfma(uv, cs[grp * NG + i], xv[i]);
            cfma(uw, cs[NV + grp * NG + i], xv[i]);
        }
#pragma unroll
        for (int m = LG; m < 64; m <<= 1) {
            uv = make_double2(uv.x + __shfl_xor(uv.x, m, 64), uv.y + __shfl_xor(uv.y, m, 64));
            uw = make_double2(uw.x + __shfl_xor(uw.x, m, 64), uw.y + __shfl_xor(uw.y, m, 64));
        }
        if (grp == 0) {
            const double2 vn = cscale(cadd(vd, uv), a);
            double2 wn = cadd(wd, uw);
            cfma(wn, cv, vn);
            v[so + e] = vn;
            w[so + e] = wn;
            accn += wn.x * wn.x + wn.y * wn.y;
        }
    }
    if (!last) return;
    const double s = wave_sum(accn);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int k = 0; k < TPB / 64; k++) t += red[k];
        part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = make_double2(t, 0);
    }
}

// y = s * x with s = alpha * coef[0] (coef on the device), or
// s = alpha / sqrt(re nrm2[0]) (0 when that is 0) when inv_norm, or s = alpha
// when coef == nullptr; x and y may alias
template <typename TX, typename TY>
__global__ __launch_bounds__(TPB) void scale_kernel(size_t n, const C<TX> *x, const double2 *__restrict__ coef,
                                                    double2 alpha, int inv_norm, C<TY> *y) {
    double2 s = alpha;
    if (coef && inv_norm) {
        double nn = sqrt(coef[blockIdx.y].x);
        s = nn > 0 ? cscale(alpha, 1.0 / nn) : make_double2(0, 0);
    } else if (coef) {
        s = cmul(coef[blockIdx.y], alpha);
    }
    const size_t stride = (size_t)gridDim.x * TPB, so = (size_t)blockIdx.y * n;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n; e += stride) {
        C<TX> xv = x[so + e];
        double2 v = cmul(s, make_double2((double)xv.x, (double)xv.y));
        y[so + e] = mk<TY>((TY)v.x, (TY)v.y);
    }
}

// coef[0] = 1 / sqrt(re(v[0])) (normalisation from a squared norm)
__global__ void rsqrt_kernel(const double2 *v, double2 *coef) {
    double n = sqrt(v[0].x);
    coef[0] = make_double2(n > 0 ? 1.0 / n : 0.0, 0.0);
}

// ---- tall-skinny products of vector sets (bootstrap setup, FP64)
//
// gram: part[wg][i][j] = sum over the workgroup's elements of conj(x_i) y_j.
// Elements are processed in tiles of gt (a power of two, sized on the host
// so that the tiles fit the dynamic LDS); the tiles of x (and of y unless y
// is x) go through LDS, one row of gt + 1 per vector (the padding puts the rows
// that the threads of a wave read at one element in different banks). The
// output is cut into 4x4 blocks (only those with
// bi <= bj when y is x: the rest is the conjugate transpose); thread t owns
// block t % nblk for the elements e = t / nblk, t / nblk + ngroups, ... of
// each tile, so that up to 256 threads work also when there are few blocks;
// the ngroups partial blocks are added in group order at the end.
constexpr int GMAX = 64;   // vectors per set

struct PtrList64 {
    const void *p[GMAX];
};

template <bool ROWS>   // ROWS: tiles of at least 64 elements, loaded one vector row per wave
__global__ __launch_bounds__(256) void gram_kernel(size_t n, PtrList64 xs, int nx, PtrList64 ys, int ny, int sym,
                                                   int gt, double2 *__restrict__ part) {
    extern __shared__ double2 sm[];   // x and y tiles ([vector][gt + 1]); reused for the group reduction
    const int ld = gt + 1;
    const double2 *yt = sym ? sm : sm + (size_t)nx * ld;
    const int tx = (nx + 3) / 4, ty = (ny + 3) / 4;
    const int nblk = sym ? tx * (tx + 1) / 2 : tx * ty;
    int ngroups = 1;
    while (ngroups < 8 && 2 * ngroups * nblk <= (int)blockDim.x) ngroups *= 2;
    const int t = threadIdx.x, blk = t % nblk, grp = t / nblk;
    const bool owner = t < nblk * ngroups;
    const int nload = sym ? nx : nx + ny;
    int bi = 0, bj = 0;
    if (sym) {   // blk -> (bi, bj), bi <= bj, row by row
        int r = blk;
        while (r >= tx - bi) { r -= tx - bi; bi++; }
        bj = bi + r;
    } else {
        bi = blk / ty;
        bj = blk % ty;
    }
    // rows past the set read row 0 (their products are never stored)
    int xr[4], yr[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        xr[a] = 4 * bi + a < nx ? 4 * bi + a : 0;
        yr[a] = 4 * bj + a < ny ? 4 * bj + a : 0;
    }
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = make_double2(0, 0);
    const size_t ntile = (n + gt - 1) / gt;
    for (size_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const size_t e0 = tile * gt;
        if (ROWS) {
            // one vector row per wave at a time: the row index, and so the
            // vector's pointer, is the same in every lane (a scalar load)
            for (int v0 = t >> 6; v0 < nload; v0 += blockDim.x >> 6) {
                const int v = __builtin_amdgcn_readfirstlane(v0);
                const double2 *src = v < nx ? (const double2 *)xs.p[v] : (const double2 *)ys.p[v - nx];
                for (int e = t & 63; e < gt; e += 64) sm[v * ld + e] = e0 + e < n ? src[e0 + e] : make_double2(0, 0);
            }
        } else {
            // short rows: several rows per wave, the pointer per lane
            for (int q = t; q < nload * gt; q += blockDim.x) {
                const int v = q / gt, e = q - v * gt;
                double2 val = make_double2(0, 0);
                if (e0 + e < n)
                    val = v < nx ? ((const double2 *)xs.p[v])[e0 + e] : ((const double2 *)ys.p[v - nx])[e0 + e];
                sm[v * ld + e] = val;
            }
        }
        __syncthreads();
        if (owner) {
            for (int e = grp; e < gt; e += ngroups) {
                double2 xv[4], yv[4];
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    xv[a] = sm[xr[a] * ld + e];
                    yv[a] = yt[yr[a] * ld + e];
                }
#pragma unroll
                for (int a = 0; a < 4; a++)
#pragma unroll
                    for (int b = 0; b < 4; b++) cfmac(acc[a][b], xv[a], yv[b]);
            }
        }
        __syncthreads();
    }
    // add the groups' partial blocks in group order (through LDS)
    if (ngroups > 1) {
        double2 *red = sm;   // [nblk * ngroups][16]
        if (owner) {
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) red[t * 16 + 4 * a + b] = acc[a][b];
        }
        __syncthreads();
        if (t < nblk) {
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    double2 v = red[t * 16 + 4 * a + b];
                    for (int gq = 1; gq < ngroups; gq++) {
                        const double2 w = red[(gq * nblk + t) * 16 + 4 * a + b];
                        v.x += w.x;
                        v.y += w.y;
                    }
                    acc[a][b] = v;
                }
        }
    }
    if (t >= nblk) return;
    double2 *pw = part + (size_t)blockIdx.x * nx * ny;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int i = 4 * bi + a, j = 4 * bj + b;
            if (i < nx && j < ny) pw[(size_t)i * ny + j] = acc[a][b];
        }
}

// out[q] = sum_wg part[wg][q], q = i ny + j, one workgroup per q: thread t
// adds the partials wg = t, t + 256, ... in order, then the workgroup sum in a
// fixed order; with sym only the blocks with bi <= bj were formed, the others
// are the conjugates of their transposes
__global__ __launch_bounds__(256) void gram_finish_kernel(int nwg, int nx, int ny, int sym,
                                                          const double2 *__restrict__ part, double2 *__restrict__ out) {
    __shared__ double red[2 * 4];
    const int q = blockIdx.x;
    const int i = q / ny, j = q % ny;
    const bool mirror = sym && (i / 4) > (j / 4);
    const int src = mirror ? j * ny + i : q;
    double a = 0, b = 0;
    for (int w = threadIdx.x; w < nwg; w += blockDim.x) {
        const double2 v = part[(size_t)w * nx * ny + src];
        a += v.x;
        b += v.y;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        a += __shfl_xor(a, m, 64);
        b += __shfl_xor(b, m, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[2 * wv] = a; red[2 * wv + 1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double A = 0, B = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) { A += red[2 * k]; B += red[2 * k + 1]; }
        out[q] = make_double2(A, mirror ? -B : B);
    }
}

// y_k = sum_{i < nx} M[i * ny + k] x_i for k < ny, one element per thread
// with the nx inputs of the element in registers (nx <= XMAX), so y may be x
// itself (ny == nx, in place); M is read from LDS, the outputs formed in
// chunks of 8. With upper set M is upper triangular and the zero terms below
// its diagonal are skipped (the same sums, about half the work).
template <int XMAX>
__global__ __launch_bounds__(256) void transform_reg_kernel(size_t n, PtrList64 xs, int nx,
                                                            const double2 *__restrict__ M, int ny, PtrList64 ys,
                                                            int upper) {
    extern __shared__ double2 tsm[];   // M [nx * ny]
    for (int q = threadIdx.x; q < nx * ny; q += blockDim.x) tsm[q] = M[q];
    __syncthreads();
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double2 xv[XMAX];
#pragma unroll
        for (int i = 0; i < XMAX; i++) xv[i] = i < nx ? ((const double2 *)xs.p[i])[e] : make_double2(0, 0);
        for (int k0 = 0; k0 < ny; k0 += 8) {
            double2 acc[8];
#pragma unroll
            for (int kk = 0; kk < 8; kk++) acc[kk] = make_double2(0, 0);
#pragma unroll
            for (int i = 0; i < XMAX; i++) {
                if (i < nx && (!upper || i < k0 + 8)) {   // upper: M[i][k] = 0 for i > k
#pragma unroll
                    for (int kk = 0; kk < 8; kk++)
                        if (k0 + kk < ny) cfma(acc[kk], tsm[i * ny + k0 + kk], xv[i]);
                }
            }
#pragma unroll
            for (int kk = 0; kk < 8; kk++)
                if (k0 + kk < ny) ((double2 *)ys.p[k0 + kk])[e] = acc[kk];
        }
    }
}

// the same product with the ny <= YMAX outputs of an element in registers and
// its inputs streamed once (each read before any output of the element is
// written, so y may alias x)
template <int YMAX>
__global__ __launch_bounds__(256) void transform_stream_kernel(size_t n, PtrList64 xs, int nx,
                                                               const double2 *__restrict__ M, int ny, PtrList64 ys) {
    extern __shared__ double2 tsm[];   // M [nx * ny]
    for (int q = threadIdx.x; q < nx * ny; q += blockDim.x) tsm[q] = M[q];
    __syncthreads();
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double2 acc[YMAX];
#pragma unroll
        for (int k = 0; k < YMAX; k++) acc[k] = make_double2(0, 0);
#pragma unroll 4
        for (int i = 0; i < nx; i++) {
            const double2 x = ((const double2 *)xs.p[i])[e];
#pragma unroll
            for (int k = 0; k < YMAX; k++)
                if (k < ny) cfma(acc[k], tsm[i * ny + k], x);
        }
#pragma unroll
        for (int k = 0; k < YMAX; k++)
            if (k < ny) ((double2 *)ys.p[k])[e] = acc[k];
    }
}

// the same product for nx > 40, over tiles of GT elements through LDS: the
// tile of every x_i is read into LDS before any output of the tile is
// written, so y may be x itself (ny == nx, in place).
constexpr int GT = 32;     // elements per tile

__global__ __launch_bounds__(256) void transform_kernel(size_t n, PtrList64 xs, int nx, const double2 *__restrict__ M,
                                                        int ny, PtrList64 ys) {
    extern __shared__ double2 tsm[];
    double2 *Ms = tsm;                                  // [nx * ny]
    double2 (*xt)[GT] = (double2 (*)[GT])(tsm + nx * ny);   // [nx][GT]
    const int t = threadIdx.x;
    for (int q = t; q < nx * ny; q += blockDim.x) Ms[q] = M[q];
    const size_t ntile = (n + GT - 1) / GT;
    const int e = t % GT, k0 = t / GT, kstep = blockDim.x / GT;
    for (size_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const size_t e0 = tile * GT;
        __syncthreads();
        for (int q = t; q < nx * GT; q += blockDim.x) {
            const int v = q / GT, ee = q % GT;
            xt[v][ee] = e0 + ee < n ? ((const double2 *)xs.p[v])[e0 + ee] : make_double2(0, 0);
        }
        __syncthreads();
        if (e0 + e < n) {
            for (int k = k0; k < ny; k += kstep) {
                double2 acc = make_double2(0, 0);
                for (int i = 0; i < nx; i++) cfma(acc, Ms[i * ny + k], xt[i][e]);
                ((double2 *)ys.p[k])[e0 + e] = acc;
            }
        }
    }
}

int lin_grid(size_t n) {
    size_t g = (n + TPB - 1) / TPB;
    if (g > 8192) g = 8192;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

int blas_multidot(Ctx *c, int px, int pw, size_t n, const void *const *xs, int nvec, const void *w, double2 *out,
                  int nseg) {
    int nwg = red_grid(n);
    double2 *part = (double2 *)ensure_red(c, (size_t)2 * MAXV * nseg * nwg + 16);
    if (!part) return MGDD_ENOMEM;
    for (int i0 = 0; i0 < nvec; i0 += MAXV) {
        int nv = nvec - i0 < MAXV ? nvec - i0 : MAXV;
        PtrList pl{};
        for (int i = 0; i < nv; i++) pl.p[i] = xs[i0 + i];
        dim3 grid(nwg, nseg);
#define MD1(TX, TW, NB) multidot_kernel<TX, TW, NB><<<grid, TPB, 0, c->stream>>>(n, pl, nv, (const C<TW> *)w, part)
#define MD(TX, TW)                                                                                                    \
    do {                                                                                                              \
        if (nv <= 4) MD1(TX, TW, 4); else if (nv <= 8) MD1(TX, TW, 8); else MD1(TX, TW, MAXV);                         \
    } while (0)
        if (px == MGDD_F64 && pw == MGDD_F64) MD(double, double);
        else if (px == MGDD_F32 && pw == MGDD_F32) MD(float, float);
        else if (px == MGDD_F32 && pw == MGDD_F64) MD(float, double);
        else MD(double, float);
#undef MD
#undef MD1
        finish_kernel<<<nv * nseg, 64, 0, c->stream>>>(nwg, part, out + (size_t)i0 * nseg);
        int rc = hip_check(c, hipGetLastError(), "multidot");
        if (rc) return rc;
    }
    return MGDD_OK;
}

int blas_lincomb(Ctx *c, int px, int py, size_t n, const void *const *xs, int nvec, const double2 *coef, double alpha,
                 double beta, void *y, int nseg) {
    int nwg = lin_grid(n);
    dim3 grid(nwg, nseg);
    if (nvec == 0) {
        if (beta == 1.0) return MGDD_OK;
        PtrList pl{};
#define LC(TX, TY) lincomb_kernel<TX, TY, 1><<<grid, TPB, 0, c->stream>>>(n, pl, 0, coef, nseg, alpha, beta, (C<TY> *)y)
        if (py == MGDD_F64) LC(double, double); else LC(float, float);
        return hip_check(c, hipGetLastError(), "lincomb");
    }
    for (int i0 = 0; i0 < nvec; i0 += MAXV) {
        int nv = nvec - i0 < MAXV ? nvec - i0 : MAXV;
        PtrList pl{};
        for (int i = 0; i < nv; i++) pl.p[i] = xs[i0 + i];
        double b = i0 == 0 ? beta : 1.0;
#define LC3(TX, TY, NB) lincomb_kernel<TX, TY, NB><<<grid, TPB, 0, c->stream>>>(n, pl, nv, coef + (size_t)i0 * nseg, \
                                                                                 nseg, alpha, b, (C<TY> *)y)
#define LC2(TX, TY)                                                                                                   \
    do {                                                                                                              \
        if (nv <= 4) LC3(TX, TY, 4); else if (nv <= 8) LC3(TX, TY, 8); else LC3(TX, TY, MAXV);                         \
    } while (0)
        if (px == MGDD_F64 && py == MGDD_F64) LC2(double, double);
        else if (px == MGDD_F32 && py == MGDD_F32) LC2(float, float);
        else if (px == MGDD_F32 && py == MGDD_F64) LC2(float, double);
        else if (px == MGDD_F16 && py == MGDD_F64) LC2(_Float16, double);
        else LC2(double, float);
#undef LC3
#undef LC2
#undef LC
        int rc = hip_check(c, hipGetLastError(), "lincomb");
        if (rc) return rc;
    }
    return MGDD_OK;
}

int blas_update_dot(Ctx *c, int p, size_t n, const void *const *xs, int nvec, const double2 *coef, void *y,
                    double2 *out, int norm_only, int nseg) {
    const int mode = norm_only ? 1 : 0;
    if (nvec < 1 || nvec > MAXV) return fail(c, MGDD_EINVAL, "update_dot: bad vector count");
    // about two elements per thread: every load of the update in flight at once
    size_t g = (n + 2 * TPB - 1) / (2 * TPB);
    const int nwg = (int)(g > 4096 ? 4096 : g < 1 ? 1 : g);
    double2 *part = (double2 *)ensure_red(c, (size_t)2 * MAXV * nseg * nwg + 16);
    if (!part) return MGDD_ENOMEM;
    PtrList pl{};
    for (int i = 0; i < nvec; i++) pl.p[i] = xs[i];
    dim3 grid(nwg, nseg);
#define UD1(T, NB) update_dot_kernel<T, NB><<<grid, TPB, 0, c->stream>>>(n, pl, nvec, coef, (C<T> *)y, mode, part)
#define UD(T)                                                                                                         \
    do {                                                                                                              \
        if (nvec <= 4) UD1(T, 4); else if (nvec <= 8) UD1(T, 8); else UD1(T, MAXV);                                    \
    } while (0)
    if (p == MGDD_F64) UD(double); else UD(float);
#undef UD
#undef UD1
    const int nout = mode == 1 ? 1 : nvec;
    finish_kernel<<<nout * nseg, 64, 0, c->stream>>>(nwg, part, out);
    return hip_check(c, hipGetLastError(), "update_dot");
}

// pointer list of one launch of the lagged Gram-Schmidt kernels: vectors
// i0 ... i0 + nv - 1, the slots past nv filled as the kernels expect (the
// vector group 0 reads in that slot, else the first one, else fill)
static PtrListW dcgs_slots(const void *const *xs, int i0, int nv, int NG, const void *fill) {
    PtrListW pl{};
    for (int q = 0; q < WIDE; q++) {
        const int r = q % NG;
        pl.p[q] = q < nv ? xs[i0 + q] : r < nv ? xs[i0 + r] : nv > 0 ? xs[i0] : fill;
    }
    return pl;
}

static int dcgs_grid(size_t n, int G) {
    size_t g = (n + TPB / G - 1) / (TPB / G);
    return (int)(g > 4096 ? 4096 : g < 1 ? 1 : g);
}

int blas_dots2(Ctx *c, size_t n, const void *const *xs, int nvec, const void *w, const void *v, double2 *out_w,
               double2 *out_v, int nseg) {
    if (nvec < 1) return fail(c, MGDD_EINVAL, "dots2: bad vector count");
    for (int i0 = 0; i0 < nvec; i0 += WIDE) {
        const int nv = nvec - i0 < WIDE ? nvec - i0 : WIDE;
        const int G = nv <= 8 ? 1 : nv <= 16 ? 2 : 4, NG = nv <= 4 ? 4 : 8;
        const int nwg = dcgs_grid(n, G);
        double2 *part = (double2 *)ensure_red(c, (size_t)4 * WIDE * nseg * nwg + 16);
        if (!part) return MGDD_ENOMEM;
        const PtrListW pl = dcgs_slots(xs, i0, nv, NG, w);
        dim3 grid(nwg, nseg);
#define D2(NGT, GT)     dots2_kernel<NGT, GT><<<grid, TPB, 0, c->stream>>>(n, pl, nv, (const double2 *)w, (const double2 *)v, part)
        if (nv <= 4) D2(4, 1); else if (nv <= 8) D2(8, 1); else if (nv <= 16) D2(8, 2); else D2(8, 4);
#undef D2
        finish_kernel<<<nv * nseg, 64, 0, c->stream>>>(nwg, part, out_w + (size_t)i0 * nseg);
        finish_kernel<<<nv * nseg, 64, 0, c->stream>>>(nwg, part + (size_t)nv * nseg * nwg, out_v + (size_t)i0 * nseg);
        int rc = hip_check(c, hipGetLastError(), "dots2");
        if (rc) return rc;
    }
    return MGDD_OK;
}

int blas_dcgs_update(Ctx *c, size_t n, const void *const *xs, int nvec, const double2 *coef, void *v, void *w,
                     double2 *nrm, int nseg) {
    if (nvec < 0) return fail(c, MGDD_EINVAL, "dcgs_update: bad vector count");
    int i0 = 0;
    do {
        const int nv = nvec - i0 < WIDE ? nvec - i0 : WIDE, last = i0 + nv >= nvec;
        const int G = nv <= 8 ? 1 : nv <= 16 ? 2 : 4, NG = nv <= 4 ? 4 : 8;
        const int nwg = dcgs_grid(n, G);
        double2 *part = (double2 *)ensure_red(c, (size_t)2 * nseg * nwg + 16);
        if (!part) return MGDD_ENOMEM;
        const PtrListW pl = dcgs_slots(xs, i0, nv, NG, v);
        dim3 grid(nwg, nseg);
#define DU(NGT, GT)                                                                                                      dcgs_update_kernel<NGT, GT><<<grid, TPB, 0, c->stream>>>(n, pl, nv, i0, nvec, coef, last, (double2 *)v,                                                                      (double2 *)w, part)
        if (nv <= 4) DU(4, 1); else if (nv <= 8) DU(8, 1); else if (nv <= 16) DU(8, 2); else DU(8, 4);
#undef DU
        if (last) finish_kernel<<<nseg, 64, 0, c->stream>>>(nwg, part, nrm);
        int rc = hip_check(c, hipGetLastError(), "dcgs_update");
        if (rc) return rc;
        i0 += nv;
    } while (i0 < nvec);
    return MGDD_OK;
}

static int scale_launch(Ctx *c, int px, int py, size_t n, const void *x, const double2 *coef, double2 alpha,
                        int inv_norm, void *y, int nseg) {
    dim3 grid(lin_grid(n), nseg);
    if (px == MGDD_F64 && py == MGDD_F64)
        scale_kernel<double, double><<<grid, TPB, 0, c->stream>>>(n, (const double2 *)x, coef, alpha, inv_norm, (double2 *)y);
    else if (px == MGDD_F32 && py == MGDD_F32)
        scale_kernel<float, float><<<grid, TPB, 0, c->stream>>>(n, (const float2 *)x, coef, alpha, inv_norm, (float2 *)y);
    else if (px == MGDD_F64)
        scale_kernel<double, float><<<grid, TPB, 0, c->stream>>>(n, (const double2 *)x, coef, alpha, inv_norm, (float2 *)y);
    else
        scale_kernel<float, double><<<grid, TPB, 0, c->stream>>>(n, (const float2 *)x, coef, alpha, inv_norm, (double2 *)y);
    return hip_check(c, hipGetLastError(), "scale");
}

int blas_scale(Ctx *c, int px, int py, size_t n, const void *x, const double2 *coef, double2 alpha, void *y, int nseg) {
    return scale_launch(c, px, py, n, x, coef, alpha, 0, y, nseg);
}

int blas_normalize(Ctx *c, int px, int py, size_t n, const void *x, const double2 *nrm2, void *y, int nseg) {
    return scale_launch(c, px, py, n, x, nrm2, make_double2(1, 0), 1, y, nseg);
}

int blas_gram(Ctx *c, size_t n, const void *const *xs, int nx, const void *const *ys, int ny, double2 *out) {
    if (nx < 1 || ny < 1 || nx > GMAX || ny > GMAX) return fail(c, MGDD_EINVAL, "gram: bad vector count");
    PtrList64 px{}, py{};
    for (int i = 0; i < nx; i++) px.p[i] = xs[i];
    for (int j = 0; j < ny; j++) py.p[j] = ys[j];
    int sym = nx == ny;
    for (int i = 0; i < nx && sym; i++) sym = xs[i] == ys[i];
    // tile length: the loaded rows fill at most 40 KB of LDS, or the space
    // the group reduction needs anyway when that is larger
    const int nload = sym ? nx : nx + ny;
    const int tx = (nx + 3) / 4, ty = (ny + 3) / 4;
    const int nblk = sym ? tx * (tx + 1) / 2 : tx * ty;
    int ngroups = 1;
    while (ngroups < 8 && 2 * ngroups * nblk <= 256) ngroups *= 2;
    const size_t red_bytes = ngroups > 1 ? (size_t)nblk * ngroups * 16 * sizeof(double2) : 0;
    const size_t cap = red_bytes > 40960 ? red_bytes : 40960;
    int gt = 128;
    while (gt > 8 && (size_t)nload * (gt + 1) * sizeof(double2) > cap) gt >>= 1;
    size_t lds = (size_t)nload * (gt + 1) * sizeof(double2);
    if (red_bytes > lds) lds = red_bytes;
    const size_t ntile = (n + gt - 1) / gt;
    const int nwg = (int)(ntile < 2048 ? ntile : 2048);
    double2 *part = (double2 *)ensure_red(c, (size_t)2 * nwg * nx * ny + 16);
    if (!part) return MGDD_ENOMEM;
    if (gt >= 64)
        gram_kernel<true><<<nwg, 256, lds, c->stream>>>(n, px, nx, py, ny, sym, gt, part);
    else
        gram_kernel<false><<<nwg, 256, lds, c->stream>>>(n, px, nx, py, ny, sym, gt, part);
    gram_finish_kernel<<<nx * ny, 256, 0, c->stream>>>(nwg, nx, ny, sym, part, out);
    return hip_check(c, hipGetLastError(), "gram");
}

int blas_transform(Ctx *c, size_t n, const void *const *xs, int nx, const double2 *M, int ny, void *const *ys,
                   int upper) {
    if (nx < 1 || ny < 1 || nx > GMAX || ny > GMAX) return fail(c, MGDD_EINVAL, "transform: bad vector count");
    PtrList64 px{}, py{};
    for (int i = 0; i < nx; i++) px.p[i] = xs[i];
    for (int j = 0; j < ny; j++) py.p[j] = ys[j];
    // every kernel below reads all inputs of an element before it writes an
    // output of that element, and each element belongs to one thread (or, in
    // the tiled form, one tile staged in LDS): outputs may alias inputs
    const size_t nb = (n + 255) / 256;
    const int nwg = (int)(nb < 8192 ? nb : 8192);
    const size_t lds = (size_t)nx * ny * sizeof(double2);
    if (ny <= 24) {   // outputs in registers, inputs streamed
        transform_stream_kernel<24><<<nwg, 256, lds, c->stream>>>(n, px, nx, M, ny, py);
        return hip_check(c, hipGetLastError(), "transform");
    }
    if (nx <= 40) {   // inputs in registers
        if (nx <= 16)
            transform_reg_kernel<16><<<nwg, 256, lds, c->stream>>>(n, px, nx, M, ny, py, upper);
        else if (nx <= 24)
            transform_reg_kernel<24><<<nwg, 256, lds, c->stream>>>(n, px, nx, M, ny, py, upper);
        else if (nx <= 32)
            transform_reg_kernel<32><<<nwg, 256, lds, c->stream>>>(n, px, nx, M, ny, py, upper);
        else
            transform_reg_kernel<40><<<nwg, 256, lds, c->stream>>>(n, px, nx, M, ny, py, upper);
        return hip_check(c, hipGetLastError(), "transform");
    }
    const size_t ntile = (n + GT - 1) / GT;
    const int nwt = (int)(ntile < 4096 ? ntile : 4096);
    const size_t ldt = ((size_t)nx * ny + (size_t)nx * GT) * sizeof(double2);
    transform_kernel<<<nwt, 256, ldt, c->stream>>>(n, px, nx, M, ny, py);
    return hip_check(c, hipGetLastError(), "transform");
}

// y = gamma_5 x on fields [rhs][12][V]: in the chiral basis gamma_5 =
// diag(1, 1, -1, -1) in spin, so components 6..11 (spins 2, 3) change sign
template <typename T> __global__ void gamma5_kernel(size_t V, size_t n, const C<T> *__restrict__ x, C<T> *y) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const C<T> v = x[e];
    y[e] = ((e / V) % 12) >= 6 ? mk<T>(-v.x, -v.y) : v;
}

int blas_gamma5(Ctx *c, int p, size_t V, int nrhs, const void *x, void *y) {
    const size_t n = 12 * V * (size_t)nrhs;
    const unsigned nwg = (unsigned)((n + 255) / 256);
    if (p == MGDD_F64) gamma5_kernel<double><<<nwg, 256, 0, c->stream>>>(V, n, (const double2 *)x, (double2 *)y);
    else gamma5_kernel<float><<<nwg, 256, 0, c->stream>>>(V, n, (const float2 *)x, (float2 *)y);
    return hip_check(c, hipGetLastError(), "gamma5");
}

int blas_rsqrt(Ctx *c, const double2 *v, double2 *coef) {
    rsqrt_kernel<<<1, 1, 0, c->stream>>>(v, coef);
    return hip_check(c, hipGetLastError(), "rsqrt");
}

}  // namespace mgdd
