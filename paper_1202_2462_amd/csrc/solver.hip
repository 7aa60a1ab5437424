// Host-driven solvers on top of the kernels: the fixed-step GMRES on D_c, the
// two-level preconditioner, flexible GMRES (Section 4), plain and even-odd
// GCR (comparators), and the bootstrap setup (Section 3). Vectors stay on the
// device; Gram-Schmidt coefficients are produced and consumed on the device,
// and the host reads back only the small Hessenberg or Gram matrices it needs
// for Givens rotations and eigenproblems.
#include <chrono>
#include <cmath>

#include "blas.h"
#include "dirac.h"
#include "eo.h"
#include "learn.h"
#include "level2.h"
#include "linalg.h"
#include "solver.h"
#include "transfer.h"

namespace mgdd {

using la::cd;

// ---------------------------------------------------------------- workspace

void *Arena::take(size_t bytes) {
    size_t b = (bytes + 255) & ~(size_t)255;
    if (off + b > cap) {
        need = off + b > need ? off + b : need;
        off += b;
        return nullptr;
    }
    void *p = base + off;
    off += b;
    return p;
}

int arena_open(Ctx *c, size_t bytes, Arena &a) {
    if (c->ws_bytes < bytes) {
        if (c->ws) {
            (void)hipStreamSynchronize(c->stream);
            dfree(c, c->ws);
        }
        c->ws = dalloc(c, bytes);
        c->ws_bytes = c->ws ? bytes : 0;
        if (!c->ws) return MGDD_ENOMEM;
    }
    a.base = (char *)c->ws;
    a.cap = c->ws_bytes;
    a.off = 0;
    a.need = 0;
    return MGDD_OK;
}

// Pinned host buffer for scalars (fixed capacity, allocated once per context,
// never moved). Every host write into it follows a stream synchronisation, so
// that no copy queued earlier still reads the old contents.
cd *host_buf(Ctx *c, size_t n) {
    const size_t cap = (size_t)1 << 16;
    if (n > cap) return nullptr;
    if (!c->hbuf) {
        if (hipHostMalloc((void **)&c->hbuf, cap * sizeof(cd), hipHostMallocDefault) != hipSuccess) {
            c->hbuf = nullptr;
            return nullptr;
        }
    }
    return (cd *)c->hbuf;
}

// copies n device double2 to host (synchronous)
static int read_dev(Ctx *c, const double2 *src, size_t n, cd *dst) {
    int rc = hip_check(c, hipMemcpyAsync(dst, src, n * sizeof(double2), hipMemcpyDeviceToHost, c->stream), "read");
    if (rc) return rc;
    return hip_check(c, hipStreamSynchronize(c->stream), "sync");
}

// copies n host values to device (asynchronous; src must stay valid until the
// next synchronisation, which every caller performs before reusing it)
static int write_dev(Ctx *c, const cd *src, size_t n, double2 *dst) {
    return hip_check(c, hipMemcpyAsync(dst, src, n * sizeof(double2), hipMemcpyHostToDevice, c->stream), "write");
}

static bool finite(cd z) { return std::isfinite(z.real()) && std::isfinite(z.imag()); }

// Solves min || beta e1 - H y || for the (k+1) x k upper Hessenberg H (column
// major, ld = ldh) by Givens rotations: y (k values) when y is given; returns
// the minimum, |g_k| after the rotations.
static double hessenberg_lsq(int k, const std::vector<cd> &Hcol, int ldh, double beta, std::vector<cd> *y) {
    std::vector<cd> R((size_t)(k + 1) * k);
    for (int j = 0; j < k; j++)
        for (int i = 0; i <= j + 1; i++) R[(size_t)j * (k + 1) + i] = Hcol[(size_t)j * ldh + i];
    std::vector<cd> g(k + 1, 0.0);
    g[0] = beta;
    for (int j = 0; j < k; j++) {
        cd *col = &R[(size_t)j * (k + 1)];
        // earlier rotations were applied column by column as they were formed
        double c;
        cd s, rho;
        la::givens(col[j], col[j + 1], c, s, rho);
        col[j] = rho;
        col[j + 1] = 0.0;
        cd gj = g[j];
        g[j] = c * gj;
        g[j + 1] = -std::conj(s) * gj;
        for (int l = j + 1; l < k; l++) {
            cd *cl = &R[(size_t)l * (k + 1)];
            cd a = cl[j], b = cl[j + 1];
            cl[j] = c * a + s * b;
            cl[j + 1] = -std::conj(s) * a + c * b;
        }
    }
    if (y) {
        y->assign(k, 0.0);
        for (int i = k - 1; i >= 0; i--) {
            cd s = g[i];
            for (int l = i + 1; l < k; l++) s -= R[(size_t)l * (k + 1) + i] * (*y)[l];
            (*y)[i] = s / R[(size_t)i * (k + 1) + i];
        }
    }
    return std::abs(g[k]);
}

// ---------------------------------------------------------------- Gram-Schmidt steps on the device

// w <- w - V (V^H w), twice (classical Gram-Schmidt with one re-orthogonalisation),
// for each of the nb segments (right-hand sides) independently; h1 and h2
// receive the two coefficient vectors ([i][segment]), nrm the squared norms
// of w after.
static int cgs2(Ctx *c, int p, size_t n, void *const *V, int k, void *w, double2 *h1, double2 *h2, double2 *nrm,
                int nb = 1) {
    // short vectors (the coarse level): three fused passes, launch count
    // matters more than bandwidth there
    if (k <= FUSED_CGS2_MAX && n <= (size_t)1 << 18) return fused_cgs2(c, p, n, nb, V, k, w, h1, h2, nrm);
    // long vectors: the update of each pass and the dot products that follow
    // it share one pass over V
    if (k <= MAXV) {
        int rc = blas_multidot(c, p, p, n, V, k, w, h1, nb);
        if (!rc) rc = blas_update_dot(c, p, n, V, k, h1, w, h2, 0, nb);
        if (!rc) rc = blas_update_dot(c, p, n, V, k, h2, w, nrm, 1, nb);
        return rc;
    }
    int rc = blas_multidot(c, p, p, n, V, k, w, h1, nb);
    if (!rc) rc = blas_lincomb(c, p, p, n, V, k, h1, -1.0, 1.0, w, nb);
    if (!rc) rc = blas_multidot(c, p, p, n, V, k, w, h2, nb);
    if (!rc) rc = blas_lincomb(c, p, p, n, V, k, h2, -1.0, 1.0, w, nb);
    const void *wp = w;
    if (!rc) rc = blas_multidot(c, p, p, n, &wp, 1, w, nrm, nb);
    return rc;
}

// Orthonormalisation of nv FP64 vectors in index order (global
// orthonormalisation): the Q of X = Q R with R upper triangular and a
// positive real diagonal, the result of Gram-Schmidt in index order. Computed
// as Cholesky QR applied twice: G = X^H X (one pass over the vectors),
// G = R^H R on the host, X <- X R^{-1} (one pass, in place); the second
// application removes the loss of orthogonality of the first. When a
// Cholesky factorisation fails or the first R shows X to be ill-conditioned
// (min r_ii < 1e-7 max r_ii), the vectors are orthonormalised one by one with
// two classical Gram-Schmidt passes instead.
// gbuf, mbuf: device space for nv^2 values each; scal: 2 nv + 1 values.
static int orthonormalise(Ctx *c, size_t n, void *const *X, int nv, double2 *gbuf, double2 *mbuf, double2 *scal) {
    if (nv <= 64) {
        bool ok = true;
        for (int pass = 0; pass < 2 && ok; pass++) {
            std::vector<cd> G((size_t)nv * nv);
            int rc = blas_gram(c, n, (const void *const *)X, nv, (const void *const *)X, nv, gbuf);
            if (!rc) rc = read_dev(c, gbuf, (size_t)nv * nv, G.data());
            if (rc) return rc;
            la::Mat R;
            ok = la::cholesky_upper(nv, G, R);
            if (!ok) break;
            if (pass == 0) {
                // Cholesky QR twice is orthonormal to rounding only while
                // cond(X) stays below about u^{-1/2} = 1e8; min r_ii / max r_ii
                // bounds cond(X) from below, so a ratio under 1e-7 takes the
                // Gram-Schmidt path before X is touched
                double dmin = R[0].real(), dmax = R[0].real();
                for (int i = 1; i < nv; i++) {
                    dmin = std::min(dmin, R[(size_t)i * nv + i].real());
                    dmax = std::max(dmax, R[(size_t)i * nv + i].real());
                }
                if (dmin < 1e-7 * dmax) {
                    ok = false;
                    break;
                }
            }
            la::Mat Ri = la::upper_inverse(nv, R);
            cd *hb = host_buf(c, (size_t)nv * nv);
            if (!hb) return fail(c, MGDD_ENOMEM, "pinned buffer");
            for (size_t q = 0; q < (size_t)nv * nv; q++) hb[q] = Ri[q];   // M[i][k] = R^{-1}[i][k]
            rc = write_dev(c, hb, (size_t)nv * nv, mbuf);
            if (!rc) rc = blas_transform(c, n, (const void *const *)X, nv, mbuf, nv, X, 1);
            if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");   // hb is reused
            if (rc) return rc;
        }
        if (ok) return MGDD_OK;
    }
    for (int k = 0; k < nv; k++) {
        int rc = MGDD_OK;
        if (k > 0) {
            rc = cgs2(c, MGDD_F64, n, X, k, X[k], scal, scal + nv, scal + 2 * nv);
        } else {
            const void *x0 = X[0];
            rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &x0, 1, X[0], scal + 2 * nv);
        }
        if (!rc) rc = blas_normalize(c, MGDD_F64, MGDD_F64, n, X[k], scal + 2 * nv, X[k]);
        if (rc) return rc;
    }
    return MGDD_OK;
}

// The end of a GMRES cycle of m steps for nb right-hand sides: the
// Hessenberg matrices (h1 + h2 above the diagonal, sqrt(nr) below; column j
// at j (m + 1) nb, entry [i][segment]) are read back, the small least
// squares problems min ||beta e_1 - H y|| solved on the host (a column whose
// subdiagonal is 0 ends the basis), and x = sum_i y_i basis_i. nr[s] is the
// squared norm of the start vector. One host synchronisation.
static int hessenberg_combine(Ctx *c, int p, int m, int nb, size_t n, const double2 *h1, const double2 *h2,
                              const double2 *nr, double2 *coef, void *const *basis, void *x) {
    const size_t hs = (size_t)(m + 1) * (m + 1) * nb;
    cd *hb = host_buf(c, 2 * hs + (size_t)(m + 1) * nb + (size_t)m * nb);
    if (!hb) return fail(c, MGDD_ENOMEM, "pinned buffer");
    int rc = hip_check(c, hipMemcpyAsync(hb, h1, hs * 16, hipMemcpyDeviceToHost, c->stream), "read");
    if (!rc) rc = hip_check(c, hipMemcpyAsync(hb + hs, h2, hs * 16, hipMemcpyDeviceToHost, c->stream), "read");
    if (!rc) rc = read_dev(c, nr, (size_t)(m + 1) * nb, hb + 2 * hs);
    if (rc) return rc;
    const cd *H1 = hb, *H2 = hb + hs, *NR = hb + 2 * hs;
    cd *yb = hb + 2 * hs + (size_t)(m + 1) * nb;   // [i][s]
    for (size_t q = 0; q < (size_t)m * nb; q++) yb[q] = 0.0;
    std::vector<cd> Hc((size_t)m * (m + 1)), y;
    for (int sg = 0; sg < nb; sg++) {
        const double beta = std::sqrt(NR[sg].real());
        if (!std::isfinite(beta)) return fail(c, MGDD_ENAN, "NaN in the coarse solve");
        if (beta == 0.0) continue;   // x_s = 0
        std::fill(Hc.begin(), Hc.end(), cd(0.0));
        int k = m;
        for (int j = 0; j < m; j++) {
            const size_t cj = (size_t)j * (m + 1) * nb;
            for (int i = 0; i <= j; i++)
                Hc[(size_t)j * (m + 1) + i] = H1[cj + (size_t)i * nb + sg] + H2[cj + (size_t)i * nb + sg];
            double hn = std::sqrt(std::max(NR[(size_t)(j + 1) * nb + sg].real(), 0.0));
            Hc[(size_t)j * (m + 1) + j + 1] = hn;
            if (hn == 0.0) { k = j + 1; break; }
        }
        hessenberg_lsq(k, Hc, m + 1, beta, &y);
        for (int i = 0; i < k; i++) {
            if (!finite(y[i])) return fail(c, MGDD_ENAN, "NaN in the coarse solve");
            yb[(size_t)i * nb + sg] = y[i];
        }
    }
    rc = write_dev(c, yb, (size_t)m * nb, coef);
    if (!rc) rc = blas_lincomb(c, p, p, n, basis, m, coef, 1.0, 0.0, x, nb);
    return rc;
}

// ---------------------------------------------------------------- coarse GMRES

size_t coarse_gmres_bytes(const Ctx *c, int p, int m, int nb) { return stencil_gmres_bytes(level1_op(c), p, m, nb); }

size_t stencil_gmres_bytes(const StencilOp &op, int p, int m, int nb) {
    size_t n = (size_t)op.V * 2 * op.N * nb;
    return (size_t)(m + 3) * (n * csize(p) + 256) + (4 * (size_t)(m + 2) * (m + 2) + 2 * (size_t)(m + 2)) * nb * 16 +
           coarse_arnoldi_scratch(op, m, nb) + 8192;
}

int coarse_gmres(Ctx *c, int p, int m, int nb, const void *b, void *x, Arena &A, int *status) {
    return stencil_gmres(c, level1_op(c), p, m, nb, b, x, A, status);
}

// x_s = GMRES_m(op, b_s) from x = 0, no restart, for nb right-hand sides at
// once (one Krylov basis and one Hessenberg matrix each, shared launches).
// Up to LSQ_MAX_STEPS steps the least-squares step runs on the device and
// the whole cycle is asynchronous (a non-finite result sets *status when
// given); longer cycles solve it on the host (one synchronisation, MGDD_ENAN
// on a non-finite result).
int stencil_gmres(Ctx *c, const StencilOp &op, int p, int m, int nb, const void *b, void *x, Arena &A, int *status) {
    const size_t n = (size_t)op.V * 2 * op.N, cs = csize(p);
    const size_t mark = A.off;
    std::vector<void *> V(m + 1);
    for (int i = 0; i <= m; i++) V[i] = A.take(n * nb * cs);
    void *w = A.take(n * nb * cs);
    const size_t hs = (size_t)(m + 1) * (m + 1) * nb;   // column j at j (m + 1) nb, entry [i][s]
    double2 *h1 = (double2 *)A.take(hs * 16);
    double2 *h2 = (double2 *)A.take(hs * 16);
    double2 *nr = (double2 *)A.take((size_t)(m + 2) * nb * 16);
    double2 *coef = (double2 *)A.take((size_t)(m + 2) * nb * 16);
    if (!coef) return fail(c, MGDD_ENOMEM, "coarse GMRES workspace");
    int rc = MGDD_OK;
    if (m <= ARNOLDI_FUSED_MAX_STEPS) {
        // three fused kernels per Arnoldi step
        void *w2 = A.take(n * nb * cs);
        void *scr = A.take(coarse_arnoldi_scratch(op, m, nb));
        if (!scr) return fail(c, MGDD_ENOMEM, "coarse GMRES workspace");
        rc = launch_coarse_arnoldi(c, op, p, m, nb, b, V.data(), w, w2, scr, h1, h2, nr);
    } else {
        const void *bp = b;
        rc = blas_multidot(c, p, p, n, &bp, 1, b, nr, nb);
        if (!rc) rc = blas_normalize(c, p, p, n, b, nr, V[0], nb);
        for (int j = 0; j < m && !rc; j++) {
            rc = launch_stencil_apply(c, op, p, nb, V[j], w);
            if (!rc) rc = cgs2(c, p, n, V.data(), j + 1, w, h1 + (size_t)j * (m + 1) * nb,
                               h2 + (size_t)j * (m + 1) * nb, nr + (size_t)(j + 1) * nb, nb);
            if (!rc) rc = blas_normalize(c, p, p, n, w, nr + (size_t)(j + 1) * nb, V[j + 1], nb);
        }
    }
    if (rc) return rc;
    if (m <= LSQ_MAX_STEPS) {   // no host round trip
        rc = launch_hessenberg_lsq(c, m, nb, h1, h2, nr, coef, status);
        if (!rc) rc = blas_lincomb(c, p, p, n, V.data(), m, coef, 1.0, 0.0, x, nb);
    } else {
        rc = hessenberg_combine(c, p, m, nb, n, h1, h2, nr, coef, V.data(), x);
    }
    A.off = mark;
    return rc;
}

// ---------------------------------------------------------------- multilevel preconditioner

// the precision of the preconditioner's fine fields in a solve
int solve_prec(const mgdd_solve_params *sp) {
    return sp->precision == MGDD_MIXED ? MGDD_F32 : sp->precision == MGDD_MIXED_F16 ? MGDD_F16 : MGDD_F64;
}

MgOpts mg_opts(const mgdd_solve_params *sp) {
    MgOpts o;
    o.nu = sp->nu;
    o.mr = sp->mr_iters;
    o.cit = sp->coarse_iters;
    o.levels = sp->levels == 3 ? 3 : 2;
    o.k2 = sp->k2;
    o.nu2 = sp->nu2;
    o.mr2 = sp->mr2;
    o.gmres_blocks = sp->block_solver == MGDD_BLOCK_GMRES;
    o.additive = sp->additive != 0;
    return o;
}

static SchwarzOpts smoother_opts(const MgOpts &o) {
    SchwarzOpts so;
    so.nsweeps = o.nu;
    so.k = o.mr;
    so.gmres = o.gmres_blocks;
    so.additive = o.additive;
    return so;
}

static size_t level2_fgmres_bytes(const Ctx *c, int p, const MgOpts &o, int nb) {
    const size_t nc = (size_t)c->c.Vc * 2 * c->c.N * nb, ncc = (size_t)c->c2.Vcc * 2 * c->c2.N2 * nb;
    const size_t cs = csize(p), k = o.k2;
    return (2 * k + 2) * (nc * cs + 256) + 2 * (ncc * cs + 256) + 2 * (k + 1) * (k + 1) * nb * 16 +
           2 * (k + 2) * nb * 16 + 1024 + stencil_gmres_bytes(level2_op(c), p, o.cit, nb) + 8192;
}

// x_s = k2 steps of flexible GMRES on D_c x = b_s from x = 0 (no restart),
// right-preconditioned by M2(v) = SAP2^nu2(D_c, v, z0 = P2 GMRES_cit(D_cc,
// P2^H v)), for nb right-hand sides at once (one basis and Hessenberg matrix
// each, shared launches).
static int level2_fgmres(Ctx *c, int p, const MgOpts &o, int nb, const void *b, void *x, Arena &A) {
    const StencilOp op1 = level1_op(c), op2 = level2_op(c);
    const size_t n = (size_t)op1.V * 2 * op1.N, ncc = (size_t)op2.V * 2 * op2.N, cs = csize(p);
    const int m = o.k2;
    const size_t mark = A.off;
    std::vector<void *> V(m + 1), Z(m);
    for (int i = 0; i <= m; i++) V[i] = A.take(n * nb * cs);
    for (int i = 0; i < m; i++) Z[i] = A.take(n * nb * cs);
    void *w = A.take(n * nb * cs);
    void *cb = A.take(ncc * nb * cs), *cx = A.take(ncc * nb * cs);
    const size_t hs = (size_t)(m + 1) * (m + 1) * nb;
    double2 *h1 = (double2 *)A.take(hs * 16), *h2 = (double2 *)A.take(hs * 16);
    double2 *nr = (double2 *)A.take((size_t)(m + 2) * nb * 16);
    double2 *coef = (double2 *)A.take((size_t)(m + 2) * nb * 16);
    if (!coef) return fail(c, MGDD_ENOMEM, "level-2 FGMRES workspace");
    const void *bp = b;
    int rc = blas_multidot(c, p, p, n, &bp, 1, b, nr, nb);
    if (!rc) rc = blas_normalize(c, p, p, n, b, nr, V[0], nb);
    for (int j = 0; j < m && !rc; j++) {
        rc = launch_restrict2(c, p, nb, V[j], cb);
        if (!rc) rc = stencil_gmres(c, op2, p, o.cit, nb, cb, cx, A);
        if (!rc) rc = launch_prolong2(c, p, nb, cx, Z[j]);
        if (!rc && o.nu2 > 0) rc = launch_sap2(c, p, nb, o.nu2, o.mr2, V[j], Z[j]);
        if (!rc) rc = launch_stencil_apply(c, op1, p, nb, Z[j], w);
        if (!rc) rc = cgs2(c, p, n, V.data(), j + 1, w, h1 + (size_t)j * (m + 1) * nb, h2 + (size_t)j * (m + 1) * nb,
                           nr + (size_t)(j + 1) * nb, nb);
        if (!rc) rc = blas_normalize(c, p, p, n, w, nr + (size_t)(j + 1) * nb, V[j + 1], nb);
    }
    if (!rc && m <= LSQ_MAX_STEPS) {
        rc = launch_hessenberg_lsq(c, m, nb, h1, h2, nr, coef, nullptr);
        if (!rc) rc = blas_lincomb(c, p, p, n, Z.data(), m, coef, 1.0, 0.0, x, nb);
    } else if (!rc) {
        rc = hessenberg_combine(c, p, m, nb, n, h1, h2, nr, coef, Z.data(), x);
    }
    A.off = mark;
    return rc;
}

// the precision of the coarse level under fine precision p: half-precision
// storage of the fine fields keeps the coarse level in FP32
static int coarse_prec(int p) { return p == MGDD_F16 ? MGDD_F32 : p; }

size_t precond_bytes(const Ctx *c, int p, const MgOpts &o, int nb) {
    size_t n = (size_t)12 * c->g.V * nb, nc = (size_t)c->c.Vc * 2 * c->c.N * nb;
    const int pc = coarse_prec(p);
    const size_t inner = o.levels == 3 ? level2_fgmres_bytes(c, pc, o, nb) : coarse_gmres_bytes(c, pc, o.cit, nb);
    return n * 8 + 2 * nc * csize(pc) + inner + schwarz_work_bytes(c, p, nb, smoother_opts(o)) + 4096;
}

// z = SAP^nu(D, r, z0 = P x_c) for nb right-hand sides at once, x_c the
// coarse solve of P^H r: GMRES_cit on D_c (two levels) or the level-2
// flexible GMRES (three levels); r in FP64, z in precision p (MGDD_F16:
// half-precision storage of r's copy, z and P, FP32 arithmetic, the coarse
// level in FP32).
int mg_precond(Ctx *c, int p, int nb, const void *r64, void *z, const MgOpts &o, Arena &A) {
    const size_t n = (size_t)12 * c->g.V * nb, nc = (size_t)c->c.Vc * 2 * c->c.N * nb;
    const size_t mark = A.off;
    const int pc = coarse_prec(p);
    const void *rp = r64;
    int rc = MGDD_OK;
    if (p != MGDD_F64) {
        void *rs = A.take(n * csize(p));
        if (!rs) return fail(c, MGDD_ENOMEM, "preconditioner workspace");
        rc = launch_convert(c, MGDD_F64, p, n, r64, rs);
        rp = rs;
    }
    void *cb = A.take(nc * csize(pc)), *cx = A.take(nc * csize(pc));
    if (!cx) return fail(c, MGDD_ENOMEM, "preconditioner workspace");
    if (!rc) rc = launch_restrict(c, p, nb, rp, cb);
    if (!rc) rc = o.levels == 3 ? level2_fgmres(c, pc, o, nb, cb, cx, A) : coarse_gmres(c, pc, o.cit, nb, cb, cx, A);
    if (!rc) rc = launch_prolong(c, p, nb, cx, z);
    if (!rc && o.nu > 0) {
        const SchwarzOpts so = smoother_opts(o);
        void *work = nullptr;
        if (so.additive && !(work = A.take(schwarz_work_bytes(c, p, nb, so))))
            return fail(c, MGDD_ENOMEM, "preconditioner workspace");
        rc = launch_schwarz(c, p, nb, so, 0.0, 0.0, rp, z, work);
    }
    A.off = mark;
    return rc;
}

// ---------------------------------------------------------------- FGMRES with the two-level preconditioner

// Flexible GMRES(m) for nb right-hand sides at once: each has its own Krylov
// basis, Hessenberg matrix, Givens rotations, restarts and stopping test;
// the preconditioner, D and the Gram-Schmidt kernels run on all of them in
// shared launches. A right-hand side that has converged (or ended its
// cycle) gets zero coefficients, so its vectors stay zero until the next
// restart and its iterate no longer changes.
static int fgmres(Ctx *c, const mgdd_solve_params *sp, int nb, const void *b, void *z, mgdd_solve_stats *st,
                  Arena &A) {
    const int m = sp->restart, p = solve_prec(sp);
    const size_t n = (size_t)12 * c->g.V, cs = csize(p), nn = n * nb;
    std::vector<void *> V(m + 1), Z(m);
    for (int i = 0; i <= m; i++) V[i] = A.take(nn * 16);
    for (int i = 0; i < m; i++) Z[i] = A.take(nn * cs);
    void *w = A.take(nn * 16), *r = A.take(nn * 16);
    // h1, h2 and the norms side by side, in the order of their pinned host
    // copies, so that each Arnoldi step reads them back in one copy
    double2 *h1 = (double2 *)A.take((size_t)(2 * (m + 1) + 1) * nb * 16);
    double2 *h2 = h1 ? h1 + (size_t)(m + 1) * nb : nullptr, *nr = h1 ? h2 + (size_t)(m + 1) * nb : nullptr;
    double2 *coef = (double2 *)A.take((size_t)(2 * m + 2) * nb * 16);
    double2 *pm = (double2 *)A.take((size_t)2 * nb * 16);
    if (!pm) return fail(c, MGDD_ENOMEM, "FGMRES workspace");
    // pinned scalars: [pm 2nb | h1 (m+1)nb | h2 (m+1)nb | norms nb | coefficients (2m+2)nb]
    cd *hb = host_buf(c, (size_t)nb * (4 * (size_t)m + 7));
    if (!hb) return fail(c, MGDD_ENOMEM, "pinned buffer (too many right-hand sides for this restart length)");
    cd *Hb1 = hb + 2 * nb, *Hb2 = Hb1 + (size_t)(m + 1) * nb, *Nb = Hb2 + (size_t)(m + 1) * nb,
       *Cb = Nb + nb;
    for (int sg = 0; sg < nb; sg++) {
        hb[sg] = 1.0;
        hb[nb + sg] = -1.0;
    }
    int rc = write_dev(c, hb, 2 * (size_t)nb, pm);
    const void *bp = b;
    if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &bp, 1, b, nr, nb);
    if (!rc) rc = read_dev(c, nr, nb, Nb);
    if (rc) return rc;
    std::vector<double> bn(nb), hn(nb);
    std::vector<char> active(nb, 1), incycle(nb);
    bool zero_rhs = false;
    for (int sg = 0; sg < nb; sg++) {
        bn[sg] = std::sqrt(Nb[sg].real());
        if (!std::isfinite(bn[sg])) return fail(c, MGDD_ENAN, "right-hand side holds NaN or Inf");
        st[sg].iters = st[sg].restarts = 0;
        st[sg].converged = 0;
        st[sg].relres = 0.0;
        if (bn[sg] == 0.0) {
            st[sg].converged = 1;
            active[sg] = 0;
            zero_rhs = true;
        }
    }
    if (zero_rhs) {   // z_s = 0 for b_s = 0
        for (int sg = 0; sg < nb; sg++) Cb[sg] = active[sg] ? 1.0 : 0.0;
        rc = write_dev(c, Cb, nb, coef);
        if (!rc) rc = blas_scale(c, MGDD_F64, MGDD_F64, n, z, coef, make_double2(1, 0), z, nb);
        if (rc) return rc;
    }
    std::vector<std::vector<cd>> Hc(nb);   // Hessenberg columns as formed (ld m + 1)
    std::vector<double> beta0(nb);
    std::vector<int> k(nb);
    for (;;) {
        // true residuals r = b - D z
        rc = launch_dirac(c, MGDD_F64, nb, z, w);
        const void *bw[2] = {b, w};
        if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, bw, 2, pm, 1.0, 0.0, r, nb);
        const void *rp = r;
        if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &rp, 1, r, nr, nb);
        if (!rc) rc = read_dev(c, nr, nb, Nb);
        if (rc) return rc;
        bool any = false;
        for (int sg = 0; sg < nb; sg++) {
            Cb[sg] = 0.0;
            if (!active[sg]) continue;
            const double rn = std::sqrt(Nb[sg].real());
            if (!std::isfinite(rn)) return fail(c, MGDD_ENAN, "NaN in the residual");
            st[sg].relres = rn / bn[sg];
            if (rn <= sp->tol * bn[sg]) {
                st[sg].converged = 1;
                active[sg] = 0;
            } else if (st[sg].iters >= sp->maxit) {
                active[sg] = 0;
            } else {
                Cb[sg] = 1.0 / rn;
                any = true;
            }
        }
        if (!any) return MGDD_OK;
        rc = write_dev(c, Cb, nb, coef);
        if (!rc) rc = blas_scale(c, MGDD_F64, MGDD_F64, n, r, coef, make_double2(1, 0), V[0], nb);
        if (rc) return rc;
        for (int sg = 0; sg < nb; sg++) {
            incycle[sg] = active[sg];
            Hc[sg].assign((size_t)m * (m + 1), 0.0);
            beta0[sg] = std::sqrt(Nb[sg].real());
            k[sg] = 0;
        }
        int kmax = 0;
        for (int j = 0; j < m; j++) {
            rc = mg_precond(c, p, nb, V[j], Z[j], mg_opts(sp), A);
            if (!rc && p != MGDD_F64) {
                rc = launch_dirac_widen(c, nb, Z[j], w, p);
            } else if (!rc) {
                rc = launch_dirac(c, MGDD_F64, nb, Z[j], w);
            }
            // Gram-Schmidt with the second pass of v_j lagged into this step
            // (V[j] holds v_j after one pass, normalised): pass A,
            // t = V[0..j]^H w and s = V[0..j]^H V[j] in one pass over the basis
            if (!rc) rc = blas_dots2(c, n, V.data(), j + 1, w, V[j], h1, h2, nb);
            if (!rc) rc = read_dev(c, h1, (size_t)2 * (m + 1) * nb, Hb1);
            if (rc) return rc;
            // v_j = (V[j] - V s) / alpha with alpha^2 = ||V[j]||^2 - ||s||^2; column
            // j - 1 gains the component of V[j] in span(V[0..j-1]) (D z_{j-1} =
            // sum h_i v_i + beta V[j]); column j: <v_i, w> (i < j) and
            // <v_j, w> = (t_j - s^H t) / alpha
            for (size_t q = 0; q < (size_t)(2 + 2 * j) * nb; q++) Cb[q] = 0.0;
            for (int sg = 0; sg < nb; sg++) {
                Cb[sg] = 1.0;   // right-hand sides outside the cycle: v and w unchanged
                if (!incycle[sg]) continue;
                const cd *S = Hb2 + sg, *T = Hb1 + sg;
                double s2 = 0.0;
                cd st_ = 0.0;
                for (int i = 0; i < j; i++) {
                    s2 += std::norm(S[(size_t)i * nb]);
                    st_ += std::conj(S[(size_t)i * nb]) * T[(size_t)i * nb];
                }
                const double a2 = S[(size_t)j * nb].real() - s2;
                if (!std::isfinite(a2) || !finite(st_)) return fail(c, MGDD_ENAN, "NaN in the Arnoldi step");
                cd *prev = j > 0 ? &Hc[sg][(size_t)(j - 1) * (m + 1)] : nullptr;
                const double beta = prev ? prev[j].real() : 0.0;
                if (prev)
                    for (int i = 0; i < j; i++) prev[i] += beta * S[(size_t)i * nb];
                if (!(a2 > 0.0)) {   // V[j] lies in span(V[0..j-1]): the cycle ends at column j - 1
                    if (prev) prev[j] = 0.0;
                    incycle[sg] = 0;
                    continue;
                }
                const double alpha = std::sqrt(a2);
                if (prev) prev[j] = beta * alpha;
                cd *col = &Hc[sg][(size_t)j * (m + 1)];
                for (int i = 0; i < j; i++) col[i] = T[(size_t)i * nb];
                col[j] = (T[(size_t)j * nb] - st_) / alpha;
                Cb[sg] = 1.0 / alpha;
                Cb[nb + sg] = -col[j];
                for (int i = 0; i < j; i++) {
                    Cb[(size_t)(2 + i) * nb + sg] = -S[(size_t)i * nb];
                    Cb[(size_t)(2 + j + i) * nb + sg] = -T[(size_t)i * nb];
                }
            }
            // pass B: V[j] <- v_j and w <- w - V[0..j] col (one pass over the
            // basis), ||w||^2; w's own second pass comes with v_{j+1}
            rc = write_dev(c, Cb, (size_t)(2 + 2 * j) * nb, coef);
            if (!rc) rc = blas_dcgs_update(c, n, V.data(), j, coef, V[j], w, nr, nb);
            if (!rc) rc = read_dev(c, nr, nb, Nb);
            if (rc) return rc;
            bool more = false;
            for (int sg = 0; sg < nb; sg++) {
                Cb[sg] = 0.0;
                if (!incycle[sg]) continue;
                const double h = std::sqrt(std::max(Nb[sg].real(), 0.0));
                if (!std::isfinite(h)) return fail(c, MGDD_ENAN, "NaN in the Arnoldi step");
                Hc[sg][(size_t)j * (m + 1) + j + 1] = h;
                st[sg].iters++;
                k[sg] = j + 1;
                kmax = std::max(kmax, j + 1);
                // the residual estimate from the columns so far (the last one
                // still without the second pass of v_{j+1}, a rounding-level change)
                const double est = hessenberg_lsq(j + 1, Hc[sg], m + 1, beta0[sg], nullptr);
                if (est <= sp->tol * bn[sg] || h == 0.0 || st[sg].iters >= sp->maxit) {
                    incycle[sg] = 0;
                } else {
                    Cb[sg] = 1.0 / h;
                    more = true;
                }
            }
            if (!more || j + 1 == m) break;
            rc = write_dev(c, Cb, nb, coef);
            if (!rc) rc = blas_scale(c, MGDD_F64, MGDD_F64, n, w, coef, make_double2(1, 0), V[j + 1], nb);
            if (rc) return rc;
        }
        // R y = g (R upper triangular after the rotations), per right-hand side
        for (size_t q = 0; q < (size_t)kmax * nb; q++) Cb[q] = 0.0;
        for (int sg = 0; sg < nb; sg++) {
            if (!active[sg]) continue;
            const int kk = k[sg];
            std::vector<cd> y;
            hessenberg_lsq(kk, Hc[sg], m + 1, beta0[sg], &y);
            for (int i = 0; i < kk; i++) {
                if (!finite(y[i])) return fail(c, MGDD_ENAN, "NaN in the least-squares solve");
                Cb[(size_t)i * nb + sg] = y[i];
            }
            st[sg].restarts++;
        }
        rc = write_dev(c, Cb, (size_t)kmax * nb, coef);
        if (!rc) rc = blas_lincomb(c, p, MGDD_F64, n, Z.data(), kmax, coef, 1.0, 1.0, z, nb);
        if (rc) return rc;
    }
}

// ---------------------------------------------------------------- GCR (plain and even-odd)

// Operator of a GCR solve: the full D or the even-odd Schur complement.
struct GcrOp {
    Ctx *c;
    bool eo;
    void *t;  // half-field temporary for the Schur complement
    int apply(const void *x, void *y) const {
        if (!eo) return launch_dirac(c, MGDD_F64, 1, x, y);
        int rc = launch_eo(c, 0, 0, 1, x, nullptr, 0.0, 1.0, t);   // t = A_ee^-1 H_eo x
        if (!rc) rc = launch_eo(c, 1, 1, 0, t, x, 1.0, -0.25, y);    // y = A_oo x - 1/4 H_oe t
        return rc;
    }
};

// GCR(m) on op x = rhs from x (in/out), until ||rhs - op x|| <= thr, or maxit.
// Returns the true residual norm in *res.
static int gcr_core(Ctx *c, const GcrOp &op, size_t n, int m, const void *rhs, void *x, double thr, int maxit,
                    int &iters, int &restarts, double *res, Arena &A) {
    const size_t mark = A.off;
    std::vector<void *> P(m), Q(m);
    for (int i = 0; i < m; i++) { P[i] = A.take(n * 16); Q[i] = A.take(n * 16); }
    void *r = A.take(n * 16), *w = A.take(n * 16);
    double2 *b1 = (double2 *)A.take((size_t)m * 16), *b2 = (double2 *)A.take((size_t)m * 16);
    double2 *sc = (double2 *)A.take(128), *pm = (double2 *)A.take(32);
    if (!pm) return fail(c, MGDD_ENOMEM, "GCR workspace");
    cd *hb = host_buf(c, 8);
    if (!hb) return fail(c, MGDD_ENOMEM, "pinned buffer");
    hb[0] = 1.0;
    hb[1] = -1.0;
    int rc = write_dev(c, hb, 2, pm);
    for (;;) {
        if (!rc) rc = op.apply(x, w);
        const void *bw[2] = {rhs, w};
        if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, bw, 2, pm, 1.0, 0.0, r);
        const void *rp = r;
        if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &rp, 1, r, sc);
        if (!rc) rc = read_dev(c, sc, 1, hb + 2);
        if (rc) return rc;
        double rn = std::sqrt(hb[2].real());
        if (!std::isfinite(rn)) return fail(c, MGDD_ENAN, "NaN in the GCR residual");
        *res = rn;
        if (rn <= thr || iters >= maxit) break;
        for (int i = 0; i < m; i++) {
            rc = hip_check(c, hipMemcpyAsync(P[i], r, n * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
            if (!rc) rc = op.apply(P[i], Q[i]);
            for (int pass = 0; pass < 2 && i > 0 && !rc; pass++) {
                double2 *bb = pass ? b2 : b1;
                rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, Q.data(), i, Q[i], bb);
                if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, Q.data(), i, bb, -1.0, 1.0, Q[i]);
                if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, P.data(), i, bb, -1.0, 1.0, P[i]);
            }
            const void *qi = Q[i];
            if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &qi, 1, Q[i], sc);
            if (!rc) rc = blas_normalize(c, MGDD_F64, MGDD_F64, n, P[i], sc, P[i]);
            if (!rc) rc = blas_normalize(c, MGDD_F64, MGDD_F64, n, Q[i], sc, Q[i]);
            if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &qi, 1, r, sc + 2);   // alpha = <q, r>
            const void *pi = P[i];
            if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, &pi, 1, sc + 2, 1.0, 1.0, x);
            if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, &qi, 1, sc + 2, -1.0, 1.0, r);
            if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &rp, 1, r, sc + 3);
            if (!rc) rc = read_dev(c, sc + 3, 1, hb + 3);
            if (rc) return rc;
            iters++;
            double rr = std::sqrt(hb[3].real());
            if (!std::isfinite(rr)) return fail(c, MGDD_ENAN, "NaN in GCR");
            if (rr <= thr || iters >= maxit) break;
        }
        restarts++;
    }
    A.off = mark;
    return rc;
}

static int gcr_solve(Ctx *c, const mgdd_solve_params *sp, const void *b, void *z, mgdd_solve_stats *st, Arena &A) {
    const size_t n = (size_t)12 * c->g.V;
    double2 *sc = (double2 *)A.take(64);
    void *w = A.take(n * 16);
    if (!w) return fail(c, MGDD_ENOMEM, "GCR workspace");
    const void *bp = b;
    cd *hb = host_buf(c, 8);
    int rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &bp, 1, b, sc);
    if (!rc) rc = read_dev(c, sc, 1, hb + 4);
    if (rc) return rc;
    const double bn = std::sqrt(hb[4].real());
    if (!std::isfinite(bn)) return fail(c, MGDD_ENAN, "right-hand side holds NaN or Inf");
    st->iters = st->restarts = 0;
    st->converged = 0;
    if (bn == 0.0) {
        st->converged = 1;
        st->relres = 0;
        return blas_lincomb(c, MGDD_F64, MGDD_F64, n, nullptr, 0, nullptr, 0.0, 0.0, z);
    }
    double res = 0;
    if (sp->solver == MGDD_SOLVER_GCR) {
        GcrOp op{c, false, nullptr};
        rc = gcr_core(c, op, n, sp->restart, b, z, sp->tol * bn, sp->maxit, st->iters, st->restarts, &res, A);
        if (rc) return rc;
        st->relres = res / bn;
        st->converged = res <= sp->tol * bn;
        return MGDD_OK;
    }
    // even-odd: solve the Schur complement on the odd sites, then reconstruct
    const size_t nh = n / 2;
    void *be = A.take(nh * 16), *bo = A.take(nh * 16), *ze = A.take(nh * 16), *zo = A.take(nh * 16);
    void *t = A.take(nh * 16), *bh = A.take(nh * 16), *rfull = A.take(n * 16);
    if (!rfull) return fail(c, MGDD_ENOMEM, "GCR workspace");
    GcrOp op{c, true, t};
    rc = launch_eo_split(c, b, be, bo);
    if (!rc) rc = launch_eo_split(c, z, ze, zo);
    if (!rc) rc = launch_eo(c, 0, 0, 1, nullptr, be, 1.0, 0.0, t);      // t = A_ee^-1 b_e
    if (!rc) rc = launch_eo(c, 1, 0, 0, t, bo, 1.0, 0.5, bh);           // b_hat = b_o + 1/2 H_oe t
    double thr = sp->tol * bn;
    for (;;) {
        if (rc) return rc;
        rc = gcr_core(c, op, nh, sp->restart, bh, zo, thr, sp->maxit, st->iters, st->restarts, &res, A);
        if (!rc) rc = launch_eo(c, 0, 0, 1, zo, be, 1.0, 0.5, ze);      // z_e = A_ee^-1 (b_e + 1/2 H_eo z_o)
        if (!rc) rc = launch_eo_merge(c, ze, zo, z);
        if (!rc) rc = launch_dirac(c, MGDD_F64, 1, z, w);
        // full residual ||b - D z||
        if (!rc) {
            double2 *pm = sc + 2;
            cd *h = host_buf(c, 8);
            h[0] = 1.0;
            h[1] = -1.0;
            rc = write_dev(c, h, 2, pm);
            const void *bw2[2] = {b, w};
            if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, bw2, 2, pm, 1.0, 0.0, rfull);
            const void *rf = rfull;
            if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &rf, 1, rfull, sc);
            if (!rc) rc = read_dev(c, sc, 1, h + 4);
            if (rc) return rc;
            double full = std::sqrt(h[4].real());
            st->relres = full / bn;
            if (full <= sp->tol * bn) { st->converged = 1; return MGDD_OK; }
            if (st->iters >= sp->maxit) return MGDD_OK;
            thr *= 0.1;
        }
    }
}

// ---------------------------------------------------------------- CGN (the paper's comparator)

// CG on D^H D z = D^H b with the residual r = b - D z updated alongside
// (CGNR); D^H = gamma_5 D gamma_5. When the updated residual reaches tol ||b||
// (or maxit is reached) the true residual is recomputed; CG starts again from
// the iterate while it is too large. Two host reads per iteration.
static int cgn_solve(Ctx *c, const mgdd_solve_params *sp, const void *b, void *z, mgdd_solve_stats *st, Arena &A) {
    const size_t V = c->g.V, n = 12 * V;
    double2 *sc = (double2 *)A.take(64), *one = (double2 *)A.take(16);
    void *r = A.take(n * 16), *s = A.take(n * 16), *p = A.take(n * 16), *w = A.take(n * 16);
    if (!w) return fail(c, MGDD_ENOMEM, "CGN workspace");
    cd *hb = host_buf(c, 8);
    if (!hb) return fail(c, MGDD_ENOMEM, "pinned buffer");
    hb[0] = 1.0;
    int rc = write_dev(c, hb, 1, one);
    const void *bp = b;
    if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &bp, 1, b, sc);
    if (!rc) rc = read_dev(c, sc, 1, hb + 4);
    if (rc) return rc;
    const double bn = std::sqrt(hb[4].real());
    if (!std::isfinite(bn)) return fail(c, MGDD_ENAN, "right-hand side holds NaN or Inf");
    st->iters = st->restarts = 0;
    st->converged = 0;
    if (bn == 0.0) {
        st->converged = 1;
        st->relres = 0;
        return blas_lincomb(c, MGDD_F64, MGDD_F64, n, nullptr, 0, nullptr, 0.0, 0.0, z);
    }
    const double thr = sp->tol * bn;
    auto dag = [&](const void *x, void *y) {   // y = gamma_5 D gamma_5 x (w as temporary)
        int e = blas_gamma5(c, MGDD_F64, V, 1, x, w);
        if (!e) e = launch_dirac(c, MGDD_F64, 1, w, y);
        if (!e) e = blas_gamma5(c, MGDD_F64, V, 1, y, y);
        return e;
    };
    auto norm2 = [&](const void *x, double2 *out) {
        const void *xp = x;
        return blas_multidot(c, MGDD_F64, MGDD_F64, n, &xp, 1, x, out);
    };
    for (;;) {
        // true residual
        rc = launch_dirac(c, MGDD_F64, 1, z, w);
        if (!rc) rc = hip_check(c, hipMemcpyAsync(r, b, n * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
        const void *wp = w;
        if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, &wp, 1, one, -1.0, 1.0, r);
        if (!rc) rc = norm2(r, sc);
        if (!rc) rc = read_dev(c, sc, 1, hb + 4);
        if (rc) return rc;
        const double rn = std::sqrt(hb[4].real());
        if (!std::isfinite(rn)) return fail(c, MGDD_ENAN, "NaN in the CGN residual");
        st->relres = rn / bn;
        if (rn <= thr) { st->converged = 1; return MGDD_OK; }
        if (st->iters >= sp->maxit) return MGDD_OK;
        rc = dag(r, s);
        if (!rc) rc = hip_check(c, hipMemcpyAsync(p, s, n * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
        if (!rc) rc = norm2(s, sc);
        if (!rc) rc = read_dev(c, sc, 1, hb + 4);
        if (rc) return rc;
        double ss = hb[4].real();
        while (st->iters < sp->maxit) {
            rc = launch_dirac(c, MGDD_F64, 1, p, w);
            if (!rc) rc = norm2(w, sc);
            if (!rc) rc = read_dev(c, sc, 1, hb + 4);
            if (rc) return rc;
            const double alpha = ss / hb[4].real();
            if (!std::isfinite(alpha)) return fail(c, MGDD_ENAN, "NaN in CGN");
            const void *pp = p, *wq = w;
            rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, &pp, 1, one, alpha, 1.0, z);
            if (!rc) rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, &wq, 1, one, -alpha, 1.0, r);
            st->iters++;
            if (!rc) rc = dag(r, s);
            if (!rc) rc = norm2(r, sc);
            if (!rc) rc = norm2(s, sc + 1);
            if (!rc) rc = read_dev(c, sc, 2, hb + 4);
            if (rc) return rc;
            if (std::sqrt(hb[4].real()) <= thr) break;
            const double ss_new = hb[5].real();
            const void *sq = s;
            rc = blas_lincomb(c, MGDD_F64, MGDD_F64, n, &sq, 1, one, 1.0, ss_new / ss, p);   // p = s + beta p
            if (rc) return rc;
            ss = ss_new;
        }
        st->restarts++;
    }
}

// ---------------------------------------------------------------- solve entry

size_t solve_bytes(const Ctx *c, const mgdd_solve_params *sp, int nb) {
    const size_t n = (size_t)12 * c->g.V;
    const int m = sp->restart;
    if (sp->solver == MGDD_SOLVER_FGMRES_MG) {
        const int p = solve_prec(sp);
        return (size_t)(m + 3) * (n * nb * 16 + 256) + (size_t)m * (n * nb * csize(p) + 256) +
               (3 * (size_t)m + 8) * nb * 16 + precond_bytes(c, p, mg_opts(sp), nb) + 65536;
    }
    return (size_t)(2 * m + 10) * (n * 16 + 256) + 65536;
}

// nb right-hand sides: one batched FGMRES, or GCR one after the other
int solve_batch(Ctx *c, const mgdd_solve_params *sp, int nb, const void *b, void *z, mgdd_solve_stats *st) {
    Arena A;
    const bool batched = sp->solver == MGDD_SOLVER_FGMRES_MG;
    int rc = arena_open(c, solve_bytes(c, sp, batched ? nb : 1), A);
    if (rc) return rc;
    auto t0 = std::chrono::steady_clock::now();
    if (batched) {
        rc = fgmres(c, sp, nb, b, z, st, A);
    } else {
        const size_t fb = (size_t)12 * c->g.V * 16;
        for (int r = 0; r < nb && !rc; r++) {
            A.off = 0;
            if (sp->solver == MGDD_SOLVER_CGN)
                rc = cgn_solve(c, sp, (const char *)b + r * fb, (char *)z + r * fb, &st[r], A);
            else
                rc = gcr_solve(c, sp, (const char *)b + r * fb, (char *)z + r * fb, &st[r], A);
        }
    }
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < nb; r++) st[r].seconds = secs;
    if (A.need) return fail(c, MGDD_ENOMEM, "solver workspace estimate too small");
    if (rc) return rc;
    for (int r = 0; r < nb; r++)
        if (!st[r].converged) return fail(c, MGDD_ENOCONV, "maxit reached before the tolerance");
    return MGDD_OK;
}

// ---------------------------------------------------------------- bootstrap setup

static int arnoldi_host(Ctx *c, int m, const void *v0, std::vector<void *> &Qv, std::vector<cd> &H, int &k, Arena &A) {
    const size_t n = (size_t)c->c.Vc * 2 * c->c.N;
    void *w = A.take(n * 16);
    double2 *h1 = (double2 *)A.take((size_t)(m + 1) * (m + 1) * 16), *h2 = (double2 *)A.take((size_t)(m + 1) * (m + 1) * 16);
    double2 *nr = (double2 *)A.take((size_t)(m + 2) * 16), *coef = (double2 *)A.take((size_t)(m + 2) * 16);
    Qv.resize(m + 1);
    for (int i = 0; i <= m; i++) Qv[i] = A.take(n * 16);
    if (!Qv[m]) return fail(c, MGDD_ENOMEM, "Arnoldi workspace");
    const void *vp = v0;
    int rc = blas_multidot(c, MGDD_F64, MGDD_F64, n, &vp, 1, v0, nr);
    if (!rc) rc = blas_normalize(c, MGDD_F64, MGDD_F64, n, v0, nr, Qv[0]);
    for (int j = 0; j < m && !rc; j++) {
        rc = launch_coarse_apply(c, MGDD_F64, 1, Qv[j], w);
        if (!rc) rc = cgs2(c, MGDD_F64, n, Qv.data(), j + 1, w, h1 + (size_t)j * (m + 1), h2 + (size_t)j * (m + 1), nr + j + 1);
        if (!rc) rc = blas_normalize(c, MGDD_F64, MGDD_F64, n, w, nr + j + 1, Qv[j + 1]);
    }
    if (rc) return rc;
    const size_t hs = (size_t)(m + 1) * (m + 1);
    std::vector<cd> b1(hs), b2(hs), nn(m + 1);
    rc = hip_check(c, hipMemcpyAsync(b1.data(), h1, hs * 16, hipMemcpyDeviceToHost, c->stream), "read");
    if (!rc) rc = hip_check(c, hipMemcpyAsync(b2.data(), h2, hs * 16, hipMemcpyDeviceToHost, c->stream), "read");
    if (!rc) rc = hip_check(c, hipMemcpyAsync(nn.data(), nr, (m + 1) * 16, hipMemcpyDeviceToHost, c->stream), "read");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (rc) return rc;
    if (!(nn[0].real() > 0)) return fail(c, MGDD_EINVAL, "Arnoldi start vector is zero");
    // H (m+1) x m, row-major
    H.assign((size_t)(m + 1) * m, 0.0);
    k = m;
    for (int j = 0; j < m; j++) {
        for (int i = 0; i <= j; i++) H[(size_t)i * m + j] = b1[(size_t)j * (m + 1) + i] + b2[(size_t)j * (m + 1) + i];
        double hn = std::sqrt(std::max(nn[j + 1].real(), 0.0));
        H[(size_t)(j + 1) * m + j] = hn;
        if (hn == 0.0) { k = j + 1; break; }
    }
    return MGDD_OK;
}

// Lattices from this volume on (or any, when the caller sets a chunk) take the
// memory-lean form of the setup: the part-1 sweeps run over chunks of vectors
// (a zero right-hand side and FP32 copies of that many fields instead of N),
// and the second part forms its Gram matrix <D w_i, D w_j> as
// <w_i, D^H D w_j> (D^H = g5 D g5) over chunks of columns instead of holding
// D W. At 48^3 x 96 with 20 test vectors the full form needs more than the
// 288 GB of one GPU.
constexpr int LEAN_SITES = 1 << 22;
constexpr int SETUP_CHUNK = 4;

int bootstrap(Ctx *c, const mgdd_setup_params *sp, const void *rv64, const void *start64) {
    const int N = sp->ntv, p = sp->prec;
    const size_t n = (size_t)12 * c->g.V;
    int rc = transfer_setup(c, sp->agg, N);
    if (rc) return rc;
    const bool lean = sp->chunk > 0 || c->g.V >= LEAN_SITES;
    const int chunk = std::min(sp->chunk > 0 ? sp->chunk : SETUP_CHUNK, 2 * N);   // at most the 2N columns
    const int R = lean ? std::min(N, chunk) : N;   // vectors per part-1 sweep launch
    const size_t nc = (size_t)c->c.Vc * 2 * N;
    const int mA = sp->arnoldi_m > 0 ? sp->arnoldi_m : (int)std::min<size_t>(nc, 2 * (size_t)N + 10);
    // workspace: FP32 sweep copies and the zero right-hand side (R fields each),
    // the N new vectors of the second part, D W (2N fields, or 2 chunk fields
    // in the lean form), the coarse vectors
    const size_t dw_fields = lean ? 2 * (size_t)chunk : 2 * (size_t)N;
    size_t bytes = (p == MGDD_F32 ? (size_t)R * n * 8 + 256 : 0) + (size_t)R * n * csize(p) + 256 +
                   (size_t)N * n * 16 + 256 + dw_fields * n * 16 + 256 + (p == MGDD_F32 ? n * 8 + 256 : 0) +
                   (size_t)(mA + 3 + N) * (nc * 16 + 256) + 64 * (size_t)(mA + 2) * (mA + 2) + (1 << 20);
    Arena A;
    rc = arena_open(c, bytes, A);
    if (rc) return rc;
    // the test vectors are worked on in place in the context's copy, which
    // launch_build_P then keeps (a failed setup leaves the level not ready)
    std::vector<void *> Vt(N);
    void *vt = c->c.tv64;
    void *vs = p == MGDD_F32 ? A.take((size_t)R * n * 8) : nullptr;
    void *zero = A.take((size_t)R * n * csize(p));
    double2 *scal = (double2 *)A.take(4096);
    double2 *gdev = (double2 *)A.take((size_t)4 * N * N * 16 + 256), *ydev = (double2 *)A.take((size_t)4 * N * N * 16 + 256);
    if (!ydev) return fail(c, MGDD_ENOMEM, "setup workspace");
    for (int i = 0; i < N; i++) Vt[i] = (char *)vt + (size_t)i * n * 16;
    if (rv64 == vt) {
        // the caller (the learned setup) has put the starting vectors in place
    } else if (rv64) {
        rc = hip_check(c, hipMemcpyAsync(vt, rv64, (size_t)N * n * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
    } else {
        rc = launch_gaussian_fields(c, N, sp->seed, vt);
    }
    if (!rc) rc = hip_check(c, hipMemsetAsync(zero, 0, (size_t)R * n * csize(p), c->stream), "memset");
    // part 1: nu rounds of (one SAP sweep with b = 0 on all vectors, global MGS)
    for (int it = 0; it < sp->nu && !rc; it++) {
        for (int r0 = 0; r0 < N && !rc; r0 += R) {
            const int nr = std::min(R, N - r0);
            void *vr = Vt[r0];
            if (p == MGDD_F32) {
                rc = launch_convert(c, MGDD_F64, MGDD_F32, (size_t)nr * n, vr, vs);
                if (!rc) rc = launch_sap(c, p, nr, 1, sp->mr_iters, 0.0, 0.0, zero, vs);
                if (!rc) rc = launch_convert(c, MGDD_F32, MGDD_F64, (size_t)nr * n, vs, vr);
            } else {
                rc = launch_sap(c, p, nr, 1, sp->mr_iters, 0.0, 0.0, zero, vr);
            }
        }
        if (!rc) rc = orthonormalise(c, n, Vt.data(), N, gdev, ydev, scal);
    }
    if (!rc) rc = launch_build_P(c, vt);
    if (!rc) rc = launch_coarse_build(c);
    if (rc) return rc;
    // part 2. W = (the nk new vectors, the N current test vectors): the second
    // block is the test vectors themselves, which the final transform replaces
    std::vector<void *> W(2 * N), DW(dw_fields);
    void *wbuf = A.take((size_t)N * n * 16), *dwbuf = A.take(dw_fields * n * 16);
    void *tmp32 = p == MGDD_F32 ? A.take(n * 8) : nullptr;
    std::vector<void *> phi(N);
    void *phib = A.take((size_t)N * nc * 16);   // the coarse Ritz vectors, contiguous
    if (!dwbuf || !phib) return fail(c, MGDD_ENOMEM, "setup workspace");
    for (int i = 0; i < N; i++) phi[i] = (char *)phib + (size_t)i * nc * 16;
    for (size_t i = 0; i < dw_fields; i++) DW[i] = (char *)dwbuf + i * n * 16;
    for (int i = 0; i < N; i++) W[i] = (char *)wbuf + (size_t)i * n * 16;
    for (int rep = 0; rep < sp->n_part2; rep++) {
        const size_t mark = A.off;
        std::vector<void *> Qv;
        std::vector<cd> H;
        int k = 0;
        rc = arnoldi_host(c, mA, start64, Qv, H, k, A);
        if (rc) return rc;
        // harmonic Ritz pairs of D_c for target 0
        la::Mat T((size_t)k * k);
        for (int i = 0; i < k; i++)
            for (int j = 0; j < k; j++) T[(size_t)i * k + j] = H[(size_t)i * mA + j];
        if (k == mA) {
            cd hk = H[(size_t)mA * mA + mA - 1];
            la::Mat HmH((size_t)k * k);
            for (int i = 0; i < k; i++)
                for (int j = 0; j < k; j++) HmH[(size_t)i * k + j] = std::conj(T[(size_t)j * k + i]);
            std::vector<cd> f(k, 0.0);
            f[k - 1] = 1.0;
            if (!la::lu_solve(k, HmH, f)) return fail(c, MGDD_EBREAKDOWN, "singular Hessenberg matrix in the setup");
            for (int i = 0; i < k; i++) T[(size_t)i * k + k - 1] += std::norm(hk) * f[i];
        }
        std::vector<cd> th;
        la::Mat Y;
        if (!la::eig(k, T, th, Y)) return fail(c, MGDD_EBREAKDOWN, "eigenvalue iteration did not converge");
        std::vector<int> order(k);
        for (int i = 0; i < k; i++) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int a, int b) {
            double ma = std::abs(th[a]), mb = std::abs(th[b]);
            if (ma != mb) return ma < mb;
            if (th[a].real() != th[b].real()) return th[a].real() < th[b].real();
            return th[a].imag() < th[b].imag();
        });
        const int nk = std::min(N, k);
        // phi_i = Q y_i / ||Q y_i||, w_i = P phi_i, then iota sweeps of SAP with shift theta_i
        cd *hb = host_buf(c, (size_t)k * nk + 8);
        if (!hb) return fail(c, MGDD_ENOMEM, "pinned buffer");
        for (int i = 0; i < nk; i++)
            for (int j = 0; j < k; j++) hb[(size_t)i * k + j] = Y[(size_t)j * k + order[i]];
        rc = write_dev(c, hb, (size_t)k * nk, ydev);
        for (int i = 0; i < nk && !rc; i++) {
            rc = blas_lincomb(c, MGDD_F64, MGDD_F64, nc, Qv.data(), k, ydev + (size_t)i * k, 1.0, 0.0, phi[i]);
            const void *pp = phi[i];
            if (!rc) rc = blas_multidot(c, MGDD_F64, MGDD_F64, nc, &pp, 1, phi[i], scal);
            if (!rc) rc = blas_normalize(c, MGDD_F64, MGDD_F64, nc, phi[i], scal, phi[i]);
        }
        // w_i = P phi_i for all i in one launch (P read once)
        if (!rc && nk > 0) rc = launch_prolong(c, MGDD_F64, nk, phib, wbuf);
        for (int i = 0; i < nk && !rc; i++) {
            cd lam = th[order[i]];
            if (p == MGDD_F32) {
                if (!rc) rc = launch_convert(c, MGDD_F64, MGDD_F32, n, W[i], tmp32);
                if (!rc) rc = launch_sap(c, p, 1, sp->iota, sp->mr_iters, lam.real(), lam.imag(), zero, tmp32);
                if (!rc) rc = launch_convert(c, MGDD_F32, MGDD_F64, n, tmp32, W[i]);
            } else if (!rc) {
                rc = launch_sap(c, p, 1, sp->iota, sp->mr_iters, lam.real(), lam.imag(), zero, W[i]);
            }
        }
        if (rc) return rc;
        const int nw = nk + N;
        for (int j = 0; j < N; j++) W[nk + j] = Vt[j];
        rc = orthonormalise(c, n, W.data(), nw, gdev, ydev, scal);
        // G[i][j] = <DW_i, DW_j>
        la::Mat Gm((size_t)nw * nw);
        if (!lean) {
            if (!rc && nk > 0) rc = launch_dirac(c, MGDD_F64, nk, wbuf, DW[0]);
            if (!rc) rc = launch_dirac(c, MGDD_F64, N, vt, DW[nk]);
            if (!rc) rc = blas_gram(c, n, (const void *const *)DW.data(), nw, (const void *const *)DW.data(), nw, gdev);
            if (!rc) rc = read_dev(c, gdev, (size_t)nw * nw, Gm.data());
        } else {
            // columns j0 .. j0 + cj - 1 (contiguous, inside one block of W):
            // Y = g5 D g5 D W_j, then <W_i, Y_j> for all i
            std::vector<cd> Gc((size_t)nw * chunk);
            for (int j0 = 0; j0 < nw && !rc;) {
                const int cj = std::min(chunk, (j0 < nk ? nk : nw) - j0);
                void *tmp = DW[0], *Y = DW[chunk];
                rc = launch_dirac(c, MGDD_F64, cj, W[j0], tmp);
                if (!rc) rc = blas_gamma5(c, MGDD_F64, (size_t)c->g.V, cj, tmp, tmp);
                if (!rc) rc = launch_dirac(c, MGDD_F64, cj, tmp, Y);
                if (!rc) rc = blas_gamma5(c, MGDD_F64, (size_t)c->g.V, cj, Y, Y);
                if (!rc) rc = blas_gram(c, n, (const void *const *)W.data(), nw,
                                        (const void *const *)(DW.data() + chunk), cj, gdev);
                if (!rc) rc = read_dev(c, gdev, (size_t)nw * cj, Gc.data());
                for (int i = 0; i < nw && !rc; i++)
                    for (int q = 0; q < cj; q++) Gm[(size_t)i * nw + j0 + q] = Gc[(size_t)i * cj + q];
                j0 += cj;
            }
            // the Hermitian part (the two triangles agree up to rounding)
            for (int i = 0; i < nw && !rc; i++)
                for (int j = i; j < nw; j++) {
                    const cd h = 0.5 * (Gm[(size_t)i * nw + j] + std::conj(Gm[(size_t)j * nw + i]));
                    Gm[(size_t)i * nw + j] = h;
                    Gm[(size_t)j * nw + i] = std::conj(h);
                }
        }
        if (rc) return rc;
        std::vector<double> sig;
        la::Mat Z;
        la::eigh(nw, Gm, sig, Z);
        // V_i = sum_j W_j Z[j][i] for the N smallest eigenpairs (columns of Z)
        hb = host_buf(c, (size_t)nw * N + 8);
        for (int j = 0; j < nw; j++)
            for (int i = 0; i < N; i++) hb[(size_t)j * N + i] = Z[(size_t)j * nw + i];
        rc = write_dev(c, hb, (size_t)nw * N, ydev);
        if (!rc) rc = blas_transform(c, n, (const void *const *)W.data(), nw, ydev, N, Vt.data());
        if (!rc) rc = launch_build_P(c, vt);
        if (!rc) rc = launch_coarse_build(c);
        if (rc) return rc;
        A.off = mark;
    }
    rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (A.need) return fail(c, MGDD_ENOMEM, "setup workspace estimate too small");
    return rc;
}


// ---------------------------------------------------------------- third level setup

// Test vectors of the second level and the third level built from them:
// the fine test vectors taken to the coarse grid with P^H (the first
// min(N, N2)), completed by the caller's random coarse vectors, orthonormalised
// in index order; nu2 rounds of one level-2 Schwarz sweep on D_c v = 0 from
// each vector, each followed by the orthonormalisation; then P2 and D_cc.
// FP64 throughout.
int level2_bootstrap(Ctx *c, const mgdd_level2_params *lp, const void *random2) {
    const Level1 &L1 = c->c;
    c->c2.ready = false;
    int rc = level2_sap_setup(c, lp->block2);
    if (!rc) rc = level2_setup(c, lp->agg2, lp->ntv2);
    if (rc) return rc;
    const int N2 = lp->ntv2, nres = std::min(N2, L1.N);
    if (N2 > nres && !random2) return fail(c, MGDD_EINVAL, "random coarse vectors needed (ntv2 > N)");
    const size_t nc = (size_t)L1.Vc * 2 * L1.N;
    Arena A;
    rc = arena_open(c, 2 * ((size_t)N2 * nc * 16 + 256) + 2 * (size_t)N2 * N2 * 16 + (2 * (size_t)N2 + 1) * 16 + 4096, A);
    if (rc) return rc;
    char *X0 = (char *)A.take((size_t)N2 * nc * 16);
    void *zero = A.take(nc * 16 * N2);
    double2 *gbuf = (double2 *)A.take((size_t)N2 * N2 * 16), *mbuf = (double2 *)A.take((size_t)N2 * N2 * 16);
    double2 *scal = (double2 *)A.take((2 * (size_t)N2 + 1) * 16);
    if (!scal) return fail(c, MGDD_ENOMEM, "level-2 setup workspace");
    std::vector<void *> X(N2);
    for (int k = 0; k < N2; k++) X[k] = X0 + (size_t)k * nc * 16;
    rc = launch_restrict(c, MGDD_F64, nres, L1.tv64, X0);
    if (!rc && N2 > nres)
        rc = hip_check(c, hipMemcpyAsync(X[nres], random2, (size_t)(N2 - nres) * nc * 16, hipMemcpyDeviceToDevice,
                                         c->stream), "copy");
    if (!rc) rc = hip_check(c, hipMemsetAsync(zero, 0, nc * 16 * N2, c->stream), "memset");
    if (!rc) rc = orthonormalise(c, nc, X.data(), N2, gbuf, mbuf, scal);
    for (int r = 0; r < lp->nu2 && !rc; r++) {
        rc = launch_sap2(c, MGDD_F64, N2, 1, lp->mr_iters, zero, X0);
        if (!rc) rc = orthonormalise(c, nc, X.data(), N2, gbuf, mbuf, scal);
    }
    if (!rc) rc = launch_build_P2(c, X0);
    if (!rc) rc = launch_dcc_build(c);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (!rc && A.need) rc = fail(c, MGDD_ENOMEM, "level-2 setup workspace estimate too small");
    return rc;
}

// ---------------------------------------------------------------- learned setup

// The network maps the caller's random vectors to test vectors; the bootstrap
// setup then continues from them (sp->nu part-1 rounds, sp->n_part2 second
// parts), so that with nu = n_part2 = 0 only P and D_c are built from the
// network's vectors. When the network's vectors cannot serve (P rank
// deficient on an aggregate, or NaN / Inf on the way), the plain bootstrap
// setup runs from the caller's random vectors with the same parameters, and
// c->learned_fallback records it.
int setup_learned(Ctx *c, const NetShape &sh, const double2 *W64, const mgdd_setup_params *sp, const void *rv64,
                  const void *start64) {
    const int N = sp->ntv;
    const size_t n = (size_t)12 * c->g.V;
    // the random vectors (the caller's, or drawn from the seeded stream) go
    // to the context's test vectors, and the network maps them there in place,
    // a few at a time (its workspace is that of the chunk, not of all N)
    int rc = transfer_setup(c, sp->agg, N);
    if (rc) return rc;
    void *vt = c->c.tv64;
    if (rv64)
        rc = hip_check(c, hipMemcpyAsync(vt, rv64, (size_t)N * n * 16, hipMemcpyDeviceToDevice, c->stream), "copy");
    else
        rc = launch_gaussian_fields(c, N, sp->seed, vt);
    const int R = std::min(N, 4);
    Arena A;
    if (!rc) rc = arena_open(c, net_forward_bytes(c, sh, R) + 2 * ((size_t)R * n * 8 + 256) + 4096, A);
    void *in32 = rc ? nullptr : A.take((size_t)R * n * 8), *out32 = rc ? nullptr : A.take((size_t)R * n * 8);
    if (!rc && !out32) rc = fail(c, MGDD_ENOMEM, "learned setup workspace");
    for (int i0 = 0; i0 < N && !rc; i0 += R) {
        const int r = std::min(R, N - i0);
        void *vi = (char *)vt + (size_t)i0 * n * 16;
        rc = launch_convert(c, MGDD_F64, MGDD_F32, (size_t)r * n, vi, in32);
        if (!rc) rc = net_forward(c, sh, W64, r, in32, out32, A);
        if (!rc) rc = launch_convert(c, MGDD_F32, MGDD_F64, (size_t)r * n, out32, vi);
    }
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (!rc) rc = bootstrap(c, sp, vt, start64);
    (void)hipStreamSynchronize(c->stream);
    c->learned_fallback = rc == MGDD_ERANK || rc == MGDD_ENAN;
    if (c->learned_fallback) rc = bootstrap(c, sp, rv64, start64);
    return rc;
}

}  // namespace mgdd
