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

__device__ inline M3 m3_mul(const M3 &a, const M3 &b) {
    M3 c;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 acc = make_double2(0, 0);
            for (int k = 0; k < 3; k++) cfma(acc, a.m[i * 3 + k], b.m[k * 3 + j]);
            c.m[i * 3 + j] = acc;
        }
    return c;
}
__device__ inline M3 m3_dag(const M3 &a) {
    M3 c;
    for (int i = 0; i < 3; i++)
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
    for (int k = 0; k < 9; k++) u.m[k] = p[k];
    return u;
}

// F_{mu nu}(x) = (Q - Q^H)/8 from the clover of four plaquettes at x (with
// the periodic links, before the time-boundary sign is folded in: the sign
// cancels in every closed loop).
__device__ M3 field_strength(const double2 *Uc, const Lex &lx, const int *x, int mu, int nu) {
    auto sh = [&](const int *a, int m, int s, int *b) {
        for (int k = 0; k < 4; k++) b[k] = a[k];
        b[m] = (b[m] + s + lx.L[m]) % lx.L[m];
    };
    int xpm[4], xpn[4], xmm[4], xmn[4], xmm_pn[4], xmm_mn[4], xmn_pm[4];
    sh(x, mu, 1, xpm); sh(x, nu, 1, xpn); sh(x, mu, -1, xmm); sh(x, nu, -1, xmn);
    sh(xmm, nu, 1, xmm_pn); sh(xmm, nu, -1, xmm_mn); sh(xmn, mu, 1, xmn_pm);
    M3 Q;
    // x -> x+mu -> x+mu+nu -> x+nu -> x
    M3 l1 = m3_mul(m3_mul(load_link(Uc, lx, x, mu), load_link(Uc, lx, xpm, nu)),
                   m3_mul(m3_dag(load_link(Uc, lx, xpn, mu)), m3_dag(load_link(Uc, lx, x, nu))));
    // x -> x+nu -> x+nu-mu -> x-mu -> x
    M3 l2 = m3_mul(m3_mul(load_link(Uc, lx, x, nu), m3_dag(load_link(Uc, lx, xmm_pn, mu))),
                   m3_mul(m3_dag(load_link(Uc, lx, xmm, nu)), load_link(Uc, lx, xmm, mu)));
    // x -> x-mu -> x-mu-nu -> x-nu -> x
    M3 l3 = m3_mul(m3_mul(m3_dag(load_link(Uc, lx, xmm, mu)), m3_dag(load_link(Uc, lx, xmm_mn, nu))),
                   m3_mul(load_link(Uc, lx, xmm_mn, mu), load_link(Uc, lx, xmn, nu)));
    // x -> x-nu -> x-nu+mu -> x+mu -> x
    M3 l4 = m3_mul(m3_mul(m3_dag(load_link(Uc, lx, xmn, nu)), load_link(Uc, lx, xmn, mu)),
                   m3_mul(load_link(Uc, lx, xmn_pm, nu), m3_dag(load_link(Uc, lx, x, mu))));
    for (int k = 0; k < 9; k++) Q.m[k] = cadd(cadd(l1.m[k], l2.m[k]), cadd(l3.m[k], l4.m[k]));
    M3 F;
    for (int i = 0; i < 3; i++)
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
__global__ void clover_kernel(Geom g, const double2 *__restrict__ Uc, double m0, double csw, double2 *__restrict__ A64,
                              float2 *__restrict__ A32, double2 *__restrict__ Ainv, int *__restrict__ bad) {
    int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= g.V) return;
    int X[4];
    site_coords(g, d, X);
    Lex lx{{g.L[0], g.L[1], g.L[2], g.L[3]}};
    M3 Fxy = field_strength(Uc, lx, X, 0, 1), Fxz = field_strength(Uc, lx, X, 0, 2);
    M3 Fxt = field_strength(Uc, lx, X, 0, 3), Fyz = field_strength(Uc, lx, X, 1, 2);
    M3 Fyt = field_strength(Uc, lx, X, 1, 3), Fzt = field_strength(Uc, lx, X, 2, 3);
    for (int chi = 0; chi < 2; chi++) {
        double sg = chi == 0 ? 1.0 : -1.0;
        double2 B[6][6];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                int k = a * 3 + b;
                double2 Xm = make_double2(Fyz.m[k].x + sg * Fxt.m[k].x, Fyz.m[k].y + sg * Fxt.m[k].y);
                double2 Ym = make_double2(-Fxz.m[k].x + sg * Fyt.m[k].x, -Fxz.m[k].y + sg * Fyt.m[k].y);
                double2 Zm = make_double2(Fxy.m[k].x + sg * Fzt.m[k].x, Fxy.m[k].y + sg * Fzt.m[k].y);
                B[a][b] = Zm;
                B[3 + a][3 + b] = cneg(Zm);
                B[a][3 + b] = csub(Xm, ci(Ym));
                B[3 + a][b] = cadd(Xm, ci(Ym));
            }
        double2 Am[6][6];
        for (int i = 0; i < 6; i++)
            for (int j = 0; j < 6; j++) {
                double2 v = cscale(ci(B[i][j]), -0.5 * csw);
                if (i == j) v.x += 4.0 + m0;
                Am[i][j] = v;
            }
        // packed Hermitian: 6 real diagonal entries then (re, im) of the upper triangle, as 18 pairs
        double m[36];
        for (int i = 0; i < 6; i++) m[i] = Am[i][i].x;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++) {
                m[hpk(i, j)] = Am[i][j].x;
                m[hpk(i, j) + 1] = Am[i][j].y;
            }
        for (int k = 0; k < 18; k++) {
            A64[(size_t)(chi * 18 + k) * g.V + d] = make_double2(m[2 * k], m[2 * k + 1]);
            A32[(size_t)(chi * 18 + k) * g.V + d] = make_float2((float)m[2 * k], (float)m[2 * k + 1]);
        }
        double2 Ai[6][6];
        if (!inv6(Am, Ai)) { atomicOr(bad, 1); continue; }
        for (int i = 0; i < 6; i++) m[i] = Ai[i][i].x;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++) {
                // the inverse of a Hermitian matrix is Hermitian: average the two triangles
                m[hpk(i, j)] = 0.5 * (Ai[i][j].x + Ai[j][i].x);
                m[hpk(i, j) + 1] = 0.5 * (Ai[i][j].y - Ai[j][i].y);
            }
        for (int k = 0; k < 18; k++) Ainv[(size_t)(chi * 18 + k) * g.V + d] = make_double2(m[2 * k], m[2 * k + 1]);
    }
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
    clover_kernel<<<nblk(c->g.V, 128), 128, 0, c->stream>>>(c->g, Ucanon, c->m0, c->csw, (double2 *)c->A64,
                                                          (float2 *)c->A32, (double2 *)c->Ainv64, bad);
    rc = hip_check(c, hipGetLastError(), "clover kernel");
    if (rc) return rc;
    int hbad = 0;
    rc = hip_check(c, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy");
    if (rc) return rc;
    rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (rc) return rc;
    c->links_su3 = !(hbad & 4);
    if (hbad & 2) return fail(c, MGDD_ENAN, "gauge field holds NaN or Inf");
    if (hbad & 1) return fail(c, MGDD_EINVAL, "clover term is singular on some site");
    return MGDD_OK;
}

}  // namespace mgdd
