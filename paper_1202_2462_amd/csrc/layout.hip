// Layout kernels: canonical <-> device fields, gauge-field ingest (links with
// the antiperiodic time boundary folded in), and the clover term.
#include "mgdd_internal.h"

namespace mgdd {

namespace {

constexpr int TPB = 256;

inline unsigned nblk(size_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

template <typename T>
__global__ void pack_kernel(Geom g, int nrhs, const double2 *__restrict__ canon, C<T> *__restrict__ dst) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)nrhs * g.V) return;
    int rhs = (int)(i / g.V), d = (int)(i % g.V);
    int s = lex_of(g, d);
    const double2 *src = canon + ((size_t)rhs * g.V + s) * 12;
    C<T> *o = dst + (size_t)rhs * 12 * g.V + d;
    for (int k = 0; k < 12; k++) {   // one rounding from FP64 to the storage precision
        C<T> v;
        v.x = (T)src[k].x;
        v.y = (T)src[k].y;
        o[(size_t)k * g.V] = v;
    }
}

template <typename T>
__global__ void unpack_kernel(Geom g, int nrhs, const C<T> *__restrict__ src, double2 *__restrict__ canon) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)nrhs * g.V) return;
    int rhs = (int)(i / g.V), d = (int)(i % g.V);
    int s = lex_of(g, d);
    double2 *o = canon + ((size_t)rhs * g.V + s) * 12;
    const C<T> *in = src + (size_t)rhs * 12 * g.V + d;
    for (int k = 0; k < 12; k++) {
        C<T> v = in[(size_t)k * g.V];
        o[k] = make_double2((double)v.x, (double)v.y);
    }
}

// (to half precision: one rounding, to nearest even, from FP64 or FP32)
template <typename S, typename D>
__global__ void convert_kernel(size_t n, const C<S> *__restrict__ src, C<D> *__restrict__ dst) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = mk<D>((D)src[i].x, (D)src[i].y);
}

// ---------------------------------------------------------------- gauge ingest

__global__ void links_kernel(Geom g, const double2 *__restrict__ Uc, double2 *__restrict__ U64, float2 *__restrict__ U32,
                             int *__restrict__ bad, int antiperiodic) {
    int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= g.V) return;
    int X[4];
    site_coords(g, d, X);
    int s = X[0] + g.L[0] * (X[1] + g.L[1] * (X[2] + g.L[2] * X[3]));
    for (int mu = 0; mu < 4; mu++) {
        // antiperiodic in t: the hop across the time boundary carries a sign
        double sg = (antiperiodic && mu == 3 && X[3] == g.L[3] - 1) ? -1.0 : 1.0;
        double2 r[9];
        for (int k = 0; k < 9; k++) {
            double2 u = Uc[((size_t)s * 4 + mu) * 9 + k];
            if (!isfinite(u.x) || !isfinite(u.y)) atomicOr(bad, 2);
            r[k] = u;
            u.x *= sg;
            u.y *= sg;
            U64[((size_t)mu * 9 + k) * g.V + d] = u;
            U32[((size_t)mu * 9 + k) * g.V + d] = make_float2((float)u.x, (float)u.y);
        }
        // a special unitary link has row 2 = conj(row 0 x row 1): the stencil
        // kernels then read rows 0 and 1 only (flag 4 when some link is not)
        for (int a = 0; a < 3; a++) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            const double2 x = csub(cmul(r[b], r[3 + c]), cmul(r[c], r[3 + b]));
            if (fabs(x.x - r[6 + a].x) > 1e-12 || fabs(-x.y - r[6 + a].y) > 1e-12) atomicOr(bad, 4);
        }
    }
}

struct M3 { double2 m[9]; };

// t <- t u, one row of t at a time
__device__ inline void m3_mul_into(M3 &t, const M3 &u) {
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const double2 r0 = t.m[i * 3], r1 = t.m[i * 3 + 1], r2 = t.m[i * 3 + 2];
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double2 acc = make_double2(0, 0);
            cfma(acc, r0, u.m[j]);
            cfma(acc, r1, u.m[3 + j]);
            cfma(acc, r2, u.m[6 + j]);
            t.m[i * 3 + j] = acc;
        }
    }
}
__device__ inline M3 m3_dag(const M3 &a) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) c.m[i * 3 + j] = make_double2(a.m[j * 3 + i].x, -a.m[j * 3 + i].y);
    return c;
}

struct Lex {
    int L[4];
    __device__ int idx(const int *x) const { return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3])); }
};

__device__ inline M3 load_link(const double2 *Uc, const Lex &lx, const int *x, int mu) {
    M3 u;
    const double2 *p = Uc + ((size_t)lx.idx(x) * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; k++) u.m[k] = p[k];
    return u;
}

// F_{mu nu}(x) = (Q - Q^H)/8 from the clover of four plaquettes at x (with
// the periodic links, before the time-boundary sign is folded in: the sign
// cancels in every closed loop).
// (mu, nu compile-time constants: every index into the coordinate arrays is
// one, so that they stay in registers)
template <int mu, int nu>
__device__ __forceinline__ M3 field_strength(const double2 *Uc, const Lex &lx, const int *x) {
    auto sh = [&](const int *a, int m, int s, int *b) {
#pragma unroll
        for (int k = 0; k < 4; k++) b[k] = k == m ? (a[k] + s + lx.L[k]) % lx.L[k] : a[k];
    };
    int xpm[4], xpn[4], xmm[4], xmn[4], xmm_pn[4], xmm_mn[4], xmn_pm[4];
    sh(x, mu, 1, xpm); sh(x, nu, 1, xpn); sh(x, mu, -1, xmm); sh(x, nu, -1, xmn);
    sh(xmm, nu, 1, xmm_pn); sh(xmm, nu, -1, xmm_mn); sh(xmn, mu, 1, xmn_pm);
    // the leaves one after another, each a chain of products from the left
    // added to Q as it is formed; a scheduling barrier after every product
    // keeps the compiler from loading the sixteen links at once (its registers
    // would then spill): one link in flight per thread, many threads per CU
    M3 Q;
#pragma unroll
    for (int k = 0; k < 9; k++) Q.m[k] = make_double2(0, 0);
    // link (at y, direction m), conjugated when dag
    auto step = [&](M3 &t, bool first, const int *y, int m, bool dag) {
        const M3 u = dag ? m3_dag(load_link(Uc, lx, y, m)) : load_link(Uc, lx, y, m);
        if (first) t = u; else m3_mul_into(t, u);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto add = [&](const M3 &t) {
#pragma unroll
        for (int k = 0; k < 9; k++) Q.m[k] = cadd(Q.m[k], t.m[k]);
    };
    M3 t;
    // x -> x+mu -> x+mu+nu -> x+nu -> x
    step(t, true, x, mu, false); step(t, false, xpm, nu, false); step(t, false, xpn, mu, true); step(t, false, x, nu, true);
    add(t);
    // x -> x+nu -> x+nu-mu -> x-mu -> x
    step(t, true, x, nu, false); step(t, false, xmm_pn, mu, true); step(t, false, xmm, nu, true); step(t, false, xmm, mu, false);
    add(t);
    // x -> x-mu -> x-mu-nu -> x-nu -> x
    step(t, true, xmm, mu, true); step(t, false, xmm_mn, nu, true); step(t, false, xmm_mn, mu, false); step(t, false, xmn, nu, false);
    add(t);
    // x -> x-nu -> x-nu+mu -> x+mu -> x
    step(t, true, xmn, nu, true); step(t, false, xmn, mu, false); step(t, false, xmn_pm, nu, false); step(t, false, x, mu, true);
    add(t);
    M3 F;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double2 a = Q.m[i * 3 + j], b = Q.m[j * 3 + i];
            F.m[i * 3 + j] = make_double2((a.x - b.x) * 0.125, (a.y + b.y) * 0.125);
        }
    return F;
}

// index of the upper off-diagonal entry (i<j) of a packed Hermitian 6x6
__host__ __device__ inline int hpk(int i, int j) { return 6 + 2 * ((i * (11 - i)) / 2 + (j - i - 1)); }

// 6x6 complex inverse by Gauss-Jordan elimination with partial pivoting
__device__ bool inv6(double2 (*a)[6], double2 (*inv)[6]) {
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) inv[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    for (int c = 0; c < 6; c++) {
        int p = c;
        double best = a[c][c].x * a[c][c].x + a[c][c].y * a[c][c].y;
        for (int r = c + 1; r < 6; r++) {
            double v = a[r][c].x * a[r][c].x + a[r][c].y * a[r][c].y;
            if (v > best) { best = v; p = r; }
        }
        if (best == 0.0) return false;
        if (p != c)
            for (int j = 0; j < 6; j++) {
                double2 t = a[c][j]; a[c][j] = a[p][j]; a[p][j] = t;
                t = inv[c][j]; inv[c][j] = inv[p][j]; inv[p][j] = t;
            }
        double2 piv = a[c][c];
        double den = piv.x * piv.x + piv.y * piv.y;
        double2 ip = make_double2(piv.x / den, -piv.y / den);
        for (int j = 0; j < 6; j++) { a[c][j] = cmul(a[c][j], ip); inv[c][j] = cmul(inv[c][j], ip); }
        for (int r = 0; r < 6; r++) {
            if (r == c) continue;
            double2 f = a[r][c];
            for (int j = 0; j < 6; j++) {
                a[r][j] = csub(a[r][j], cmul(f, a[c][j]));
                inv[r][j] = csub(inv[r][j], cmul(f, inv[c][j]));
            }
        }
    }
    return true;
}

// A(x) in the chiral basis: with X = F_yz +- F_xt, Y = F_zx +- F_yt,
// Z = F_xy +- F_zt (upper sign for gamma_5 = +1), the clover sum
// (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu} equals -(i/2)[[Z, X-iY],[X+iY, -Z]]
// on each chirality block, so A = (4+m0) - (i c_sw / 2) [[Z, X-iY],[X+iY,-Z]].
// Stored packed (the upper triangle of each Hermitian block). Two kernels,
// so that few field strengths are live in one thread (the registers of one
// kernel computing all six spill): F_xy and F_zt give Z and with it the two
// diagonal 3x3 blocks (OFFDIAG false); F_yz, F_xt, F_xz and F_yt are added
// one by one into the off-diagonal block X - iY of both chiralities:
// chi 0: F_yz + F_xt + i F_xz - i F_yt, chi 1: F_yz - F_xt + i F_xz + i F_yt.
template <bool OFFDIAG>
__global__ __launch_bounds__(128) void clover_kernel(Geom g, const double2 *__restrict__ Uc, double m0, double csw,
                                                     double2 *__restrict__ A64, float2 *__restrict__ A32) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= g.V) return;
    int X[4];
    site_coords(g, d, X);
    const Lex lx{{g.L[0], g.L[1], g.L[2], g.L[3]}};
    // entry (i, j), i <= j, of block chi: -(i c_sw / 2) B_ij, plus 4 + m0 on the diagonal
    auto am = [&](double2 b, bool diag) {
        double2 v = cscale(ci(b), -0.5 * csw);
        if (diag) v.x += 4.0 + m0;
        return v;
    };
    auto put = [&](int chi, int k, double re, double im) {
        A64[(size_t)(chi * 18 + k) * g.V + d] = make_double2(re, im);
        A32[(size_t)(chi * 18 + k) * g.V + d] = make_float2((float)re, (float)im);
    };
    if (!OFFDIAG) {
        const M3 Fxy = field_strength<0, 1>(Uc, lx, X), Fzt = field_strength<2, 3>(Uc, lx, X);
#pragma unroll
        for (int chi = 0; chi < 2; chi++) {
            const double sg = chi == 0 ? 1.0 : -1.0;
            double dg[6];
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = a; b < 3; b++) {
                    const int k = a * 3 + b;
                    const double2 Zm = make_double2(Fxy.m[k].x + sg * Fzt.m[k].x, Fxy.m[k].y + sg * Fzt.m[k].y);
                    const double2 up = am(Zm, a == b), lo = am(cneg(Zm), a == b);
                    if (a == b) {
                        dg[a] = up.x;
                        dg[3 + a] = lo.x;
                    } else {
                        put(chi, hpk(a, b) / 2, up.x, up.y);
                        put(chi, hpk(3 + a, 3 + b) / 2, lo.x, lo.y);
                    }
                }
#pragma unroll
            for (int k = 0; k < 3; k++) put(chi, k, dg[2 * k], dg[2 * k + 1]);
        }
        return;
    }
    double2 od0[9], od1[9];
    {
        const M3 F = field_strength<1, 2>(Uc, lx, X);
#pragma unroll
        for (int k = 0; k < 9; k++) od0[k] = od1[k] = F.m[k];
    }
    {
        const M3 F = field_strength<0, 3>(Uc, lx, X);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            od0[k] = cadd(od0[k], F.m[k]);
            od1[k] = csub(od1[k], F.m[k]);
        }
    }
    {
        const M3 F = field_strength<0, 2>(Uc, lx, X);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            od0[k] = cadd(od0[k], ci(F.m[k]));
            od1[k] = cadd(od1[k], ci(F.m[k]));
        }
    }
    {
        const M3 F = field_strength<1, 3>(Uc, lx, X);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            od0[k] = csub(od0[k], ci(F.m[k]));
            od1[k] = cadd(od1[k], ci(F.m[k]));
        }
    }
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const int k = a * 3 + b;
            const double2 v0 = am(od0[k], false), v1 = am(od1[k], false);
            put(0, hpk(a, 3 + b) / 2, v0.x, v0.y);
            put(1, hpk(a, 3 + b) / 2, v1.x, v1.y);
        }
}

// packed 6x6 Hermitian block chi of A at site d: the 36 reals of the upper triangle
__device__ inline void load_block(const double2 *__restrict__ A64, size_t V, int chi, int d, double *m) {
#pragma unroll
    for (int k = 0; k < 18; k++) {
        const double2 v = A64[(size_t)(chi * 18 + k) * V + d];
        m[2 * k] = v.x;
        m[2 * k + 1] = v.y;
    }
}

__device__ inline void store_block(double2 *__restrict__ Ai, size_t V, int chi, int d, const double *m) {
#pragma unroll
    for (int k = 0; k < 18; k++) Ai[(size_t)(chi * 18 + k) * V + d] = make_double2(m[2 * k], m[2 * k + 1]);
}

// index of entry (i, j), i >= j, of a packed lower triangle
__host__ __device__ constexpr int lti(int i, int j) { return i * (i + 1) / 2 + j; }

// The inverse of each chiral block of A (Hermitian), one thread per (site,
// block), in registers: the Cholesky factorisation A = L L^H (L lower
// triangular with a positive real diagonal), W = L^-1 row by row in the
// place of L, and A^-1 = W^H W, whose upper triangle is stored packed. A
// block that is not positive definite sets flag 8 (the host then inverts
// every block by Gauss-Jordan elimination with partial pivoting).
__global__ __launch_bounds__(256) void clover_inv_kernel(Geom g, const double2 *__restrict__ A64,
                                                         double2 *__restrict__ Ai, int *__restrict__ bad) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * (size_t)g.V) return;
    const int chi = (int)(t / g.V), d = (int)(t % g.V);
    double m[36];
    load_block(A64, g.V, chi, d, m);
    double2 L[21];
    double wd[6];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        double dj = m[j];
#pragma unroll
        for (int k = 0; k < j; k++) dj -= L[lti(j, k)].x * L[lti(j, k)].x + L[lti(j, k)].y * L[lti(j, k)].y;
        ok = ok && dj > 0.0;
        const double ljj = sqrt(dj > 0.0 ? dj : 1.0);
        wd[j] = 1.0 / ljj;
        L[lti(j, j)] = make_double2(ljj, 0.0);
#pragma unroll
        for (int i = j + 1; i < 6; i++) {
            // A_ij = conj(A_ji), A_ji from the packed upper triangle
            double2 s = make_double2(m[hpk(j, i)], -m[hpk(j, i) + 1]);
#pragma unroll
            for (int k = 0; k < j; k++) s = csub(s, cmul(L[lti(i, k)], make_double2(L[lti(j, k)].x, -L[lti(j, k)].y)));
            L[lti(i, j)] = cscale(s, wd[j]);
        }
    }
    if (!ok) {
        atomicOr(bad, 8);
        return;
    }
    // W = L^-1: W_ij = -(sum_{k=j}^{i-1} L_ik W_kj) / L_ii for j < i, in
    // ascending j (W_ij replaces L_ij, which no later j of the row reads)
#pragma unroll
    for (int i = 0; i < 6; i++) {
#pragma unroll
        for (int j = 0; j < i; j++) {
            double2 s = cmul(L[lti(i, j)], make_double2(wd[j], 0.0));
#pragma unroll
            for (int k = j + 1; k < i; k++) s = cadd(s, cmul(L[lti(i, k)], L[lti(k, j)]));
            L[lti(i, j)] = cscale(s, -wd[i]);
        }
        L[lti(i, i)] = make_double2(wd[i], 0.0);
    }
    // (A^-1)_ij = sum_{k >= j} conj(W_ki) W_kj for i <= j
#pragma unroll
    for (int i = 0; i < 6; i++) {
#pragma unroll
        for (int j = i; j < 6; j++) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = j; k < 6; k++) cfmac(s, L[lti(k, i)], L[lti(k, j)]);
            if (i == j) {
                m[i] = s.x;
            } else {
                m[hpk(i, j)] = s.x;
                m[hpk(i, j) + 1] = s.y;
            }
        }
    }
    store_block(Ai, g.V, chi, d, m);
}

// The same by Gauss-Jordan elimination with partial pivoting (blocks that
// are not positive definite); flag 1 for a singular block.
__global__ void clover_inv_pivot_kernel(Geom g, const double2 *__restrict__ A64, double2 *__restrict__ Ai,
                                        int *__restrict__ bad) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * (size_t)g.V) return;
    const int chi = (int)(t / g.V), d = (int)(t % g.V);
    double m[36];
    load_block(A64, g.V, chi, d, m);
    double2 Am[6][6], Av[6][6];
    for (int i = 0; i < 6; i++) {
        Am[i][i] = make_double2(m[i], 0.0);
        for (int j = i + 1; j < 6; j++) {
            Am[i][j] = make_double2(m[hpk(i, j)], m[hpk(i, j) + 1]);
            Am[j][i] = make_double2(m[hpk(i, j)], -m[hpk(i, j) + 1]);
        }
    }
    if (!inv6(Am, Av)) {
        atomicOr(bad, 1);
        return;
    }
    for (int i = 0; i < 6; i++) m[i] = Av[i][i].x;
    for (int i = 0; i < 6; i++)
        for (int j = i + 1; j < 6; j++) {
            // the inverse of a Hermitian matrix is Hermitian: average the two triangles
            m[hpk(i, j)] = 0.5 * (Av[i][j].x + Av[j][i].x);
            m[hpk(i, j) + 1] = 0.5 * (Av[i][j].y - Av[j][i].y);
        }
    store_block(Ai, g.V, chi, d, m);
}

}  // namespace

// Gaussian random fields from a counter-based generator: SplitMix64 (Steele,
// Lea, Flood, "Fast splittable pseudorandom number generators", 2014) with
// value i of stream `seed` = mix64(seed G + (i + 1) G), G = 0x9E3779B97F4A7C15
// (64-bit wrap-around), a uniform in [0, 1) from its top 53 bits, and the
// Box-Muller transform (1958) of the pair (u1, u2) = (value 2e, value 2e + 1):
// element e = sqrt(-2 ln(1 - u1)) (cos 2 pi u2 + i sin 2 pi u2), e counted in
// the canonical order ((field * V + lexicographic site) * 12 + component).
__device__ inline uint64_t splitmix_value(uint64_t seed, uint64_t i) {
    const uint64_t G = 0x9E3779B97F4A7C15ull;
    uint64_t z = seed * G + (i + 1) * G;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void gaussian_fields_kernel(Geom g, int nf, uint64_t seed, double2 *__restrict__ dst) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)nf * g.V) return;
    const int f = (int)(i / g.V), d = (int)(i % g.V);
    const size_t s = (size_t)lex_of(g, d);
    double2 *o = dst + (size_t)f * 12 * g.V + d;
    for (int k = 0; k < 12; k++) {
        const uint64_t e = ((size_t)f * g.V + s) * 12 + k;
        const double u1 = (double)(splitmix_value(seed, 2 * e) >> 11) * (1.0 / 9007199254740992.0);
        const double u2 = (double)(splitmix_value(seed, 2 * e + 1) >> 11) * (1.0 / 9007199254740992.0);
        const double r = sqrt(-2.0 * log1p(-u1));
        double sn, cs;
        sincos(2.0 * M_PI * u2, &sn, &cs);
        o[(size_t)k * g.V] = make_double2(r * cs, r * sn);
    }
}

int launch_gaussian_fields(Ctx *c, int nf, unsigned long long seed, void *dst) {
    size_t n = (size_t)nf * c->g.V;
    gaussian_fields_kernel<<<nblk(n), TPB, 0, c->stream>>>(c->g, nf, (uint64_t)seed, (double2 *)dst);
    return hip_check(c, hipGetLastError(), "random fields kernel");
}

int launch_pack(Ctx *c, int prec, int nrhs, const double2 *canon, void *dst) {
    size_t n = (size_t)nrhs * c->g.V;
    if (prec == MGDD_F64)
        pack_kernel<double><<<nblk(n), TPB, 0, c->stream>>>(c->g, nrhs, canon, (double2 *)dst);
    else if (prec == MGDD_F32)
        pack_kernel<float><<<nblk(n), TPB, 0, c->stream>>>(c->g, nrhs, canon, (float2 *)dst);
    else
        pack_kernel<_Float16><<<nblk(n), TPB, 0, c->stream>>>(c->g, nrhs, canon, (half_cx *)dst);
    return hip_check(c, hipGetLastError(), "pack kernel");
}

int launch_unpack(Ctx *c, int prec, int nrhs, const void *src, double2 *canon) {
    size_t n = (size_t)nrhs * c->g.V;
    if (prec == MGDD_F64)
        unpack_kernel<double><<<nblk(n), TPB, 0, c->stream>>>(c->g, nrhs, (const double2 *)src, canon);
    else if (prec == MGDD_F32)
        unpack_kernel<float><<<nblk(n), TPB, 0, c->stream>>>(c->g, nrhs, (const float2 *)src, canon);
    else
        unpack_kernel<_Float16><<<nblk(n), TPB, 0, c->stream>>>(c->g, nrhs, (const half_cx *)src, canon);
    return hip_check(c, hipGetLastError(), "unpack kernel");
}

int launch_convert(Ctx *c, int from, int to, size_t n, const void *src, void *dst) {
    if (from == to) return hip_check(c, hipMemcpyAsync(dst, src, n * csize(from), hipMemcpyDeviceToDevice, c->stream), "copy");
#define CONV(S, D) convert_kernel<S, D><<<nblk(n), TPB, 0, c->stream>>>(n, (const C<S> *)src, (C<D> *)dst)
    if (from == MGDD_F64 && to == MGDD_F32) CONV(double, float);
    else if (from == MGDD_F32 && to == MGDD_F64) CONV(float, double);
    else if (from == MGDD_F64 && to == MGDD_F16) CONV(double, _Float16);
    else if (from == MGDD_F32 && to == MGDD_F16) CONV(float, _Float16);
    else if (from == MGDD_F16 && to == MGDD_F32) CONV(_Float16, float);
    else CONV(_Float16, double);
#undef CONV
    return hip_check(c, hipGetLastError(), "convert kernel");
}

int launch_gauge_ingest(Ctx *c, const double2 *Ucanon) {
    int *bad = (int *)ensure_scratch(c, sizeof(int));
    if (!bad) return MGDD_ENOMEM;
    int rc = hip_check(c, hipMemsetAsync(bad, 0, sizeof(int), c->stream), "memset");
    if (rc) return rc;
    links_kernel<<<nblk(c->g.V), TPB, 0, c->stream>>>(c->g, Ucanon, (double2 *)c->U64, (float2 *)c->U32, bad,
                                                 c->t_antiperiodic ? 1 : 0);
    rc = hip_check(c, hipGetLastError(), "links kernel");
    if (rc) return rc;
    clover_kernel<false><<<nblk(c->g.V, 128), 128, 0, c->stream>>>(c->g, Ucanon, c->m0, c->csw, (double2 *)c->A64,
                                                                 (float2 *)c->A32);
    clover_kernel<true><<<nblk(c->g.V, 128), 128, 0, c->stream>>>(c->g, Ucanon, c->m0, c->csw, (double2 *)c->A64,
                                                                (float2 *)c->A32);
    rc = hip_check(c, hipGetLastError(), "clover kernel");
    if (rc) return rc;
    clover_inv_kernel<<<nblk(2 * (size_t)c->g.V), TPB, 0, c->stream>>>(c->g, (const double2 *)c->A64,
                                                                        (double2 *)c->Ainv64, bad);
    rc = hip_check(c, hipGetLastError(), "clover inverse kernel");
    if (rc) return rc;
    int hbad = 0;
    rc = hip_check(c, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy");
    if (rc) return rc;
    rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (rc) return rc;
    if ((hbad & 8) && !(hbad & 2)) {   // some block is not positive definite
        clover_inv_pivot_kernel<<<nblk(2 * (size_t)c->g.V), TPB, 0, c->stream>>>(c->g, (const double2 *)c->A64,
                                                                                  (double2 *)c->Ainv64, bad);
        rc = hip_check(c, hipGetLastError(), "clover inverse kernel");
        if (!rc) rc = hip_check(c, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy");
        if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
        if (rc) return rc;
    }
    c->links_su3 = !(hbad & 4);
    if (hbad & 2) return fail(c, MGDD_ENAN, "gauge field holds NaN or Inf");
    if (hbad & 1) return fail(c, MGDD_EINVAL, "clover term is singular on some site");
    return MGDD_OK;
}

}  // namespace mgdd
