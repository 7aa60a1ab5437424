/*
 * Plain FP64 CPU oracle for the SAP + aggregation multilevel solver of
 * Frommer, Kahl, Krieg, Leder, Rottmann, "Aggregation-based Multilevel Methods
 * for Lattice QCD" (Lattice 2011).
 *
 * TEST INFRASTRUCTURE ONLY. This file is used by the test-suite, by the smoke
 * check and by the CPU timing leg of the benchmark. The GPU library never
 * links, loads or calls it, and it shares no code with the GPU library.
 *
 * Everything here is written from the definitions, one site at a time, with no
 * blocking or fusion: it is meant to be checked against the paper by eye.
 *
 * Canonical layouts (complex double):
 *   site      s = x + Lx*(y + Ly*(z + Lz*t))
 *   gauge     U[s][mu][a][b]              mu = 0,1,2,3 for x,y,z,t
 *   spinor    psi[s][spin][colour]        12 dof per site
 *   clover    A[s][12][12]                row/col index = spin*3 + colour
 *   P         N fine fields P[k][s][spin][colour]
 *   coarse    c[a][chi][k]                a = coarse site (lexicographic on
 *                                         the coarse lattice), chi = 0 for
 *                                         spins 0,1 and 1 for spins 2,3
 *   D_c       Dc[a][dir][2N][2N]          dir 0 = self, 1+2*mu = +mu,
 *                                         2+2*mu = -mu; row/col = chi*N + k
 *
 * Readings of the paper that it follows (the paper names but does not write
 * these down):
 *   - chiral gamma basis: gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 *     gamma_t = [[0,-1],[-1,0]]; gamma_5 = gamma_t gamma_x gamma_y gamma_z
 *     = diag(1,1,-1,-1);
 *   - Wilson-clover operator (Section 1, D = D(U) + m):
 *       (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ eta+ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                                  + eta- (1+gamma_mu) U_mu(x-mu)^H psi(x-mu) ]
 *     with eta = -1 on hops across the time boundary (antiperiodic in t);
 *   - clover term A(x) = (4+m0) + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x),
 *     sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu], F = (Q - Q^H)/8, Q the sum of
 *     the four plaquette leaves at x in the (mu,nu) plane; no trace removed.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define OR_OK 0
#define OR_ESHAPE -2
#define OR_ERANK -3

/* ------------------------------------------------------------ lattice */

static int vol(const int *L) { return L[0] * L[1] * L[2] * L[3]; }

static int site_of(const int *L, const int *x) {
    return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]));
}

static void coords_of(const int *L, int s, int *x) {
    x[0] = s % L[0]; s /= L[0];
    x[1] = s % L[1]; s /= L[1];
    x[2] = s % L[2]; s /= L[2];
    x[3] = s;
}

/* neighbour of s one step in direction mu (dir = +1 or -1), periodic */
static int neighbour(const int *L, int s, int mu, int dir) {
    int x[4];
    coords_of(L, s, x);
    x[mu] = (x[mu] + dir + L[mu]) % L[mu];
    return site_of(L, x);
}

/* sign of a hop from s in direction mu, dir: -1 when it crosses the time boundary */
static double hop_sign(const int *L, int s, int mu, int dir) {
    int x[4];
    if (mu != 3) return 1.0;
    coords_of(L, s, x);
    if (dir > 0 && x[3] == L[3] - 1) return -1.0;
    if (dir < 0 && x[3] == 0) return -1.0;
    return 1.0;
}

/* ------------------------------------------------------------ gamma matrices */

static cplx G[4][4][4];     /* gamma_mu */
static cplx G5[4][4];
static int gamma_ready = 0;

static void build_gamma(void) {
    if (gamma_ready) return;
    const cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(G, 0, sizeof(G));
    for (int k = 0; k < 3; k++)
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) {
                G[k][i][2 + j] = -I * sig[k][i][j];
                G[k][2 + i][j] = I * sig[k][i][j];
            }
    for (int i = 0; i < 2; i++) {
        G[3][i][2 + i] = -1;
        G[3][2 + i][i] = -1;
    }
    /* gamma5 = gamma_t gamma_x gamma_y gamma_z */
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx acc = 0;
            for (int k = 0; k < 4; k++) acc += G[3][i][k] * G[0][k][j];
            t1[i][j] = acc;
        }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx acc = 0;
            for (int k = 0; k < 4; k++) acc += t1[i][k] * G[1][k][j];
            t2[i][j] = acc;
        }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx acc = 0;
            for (int k = 0; k < 4; k++) acc += t2[i][k] * G[2][k][j];
            G5[i][j] = acc;
        }
    gamma_ready = 1;
}

void or_gamma(double *out /* [5][4][4] complex: gamma_x,y,z,t then gamma_5 */) {
    build_gamma();
    cplx *o = (cplx *)out;
    for (int m = 0; m < 4; m++)
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) o[(m * 4 + i) * 4 + j] = G[m][i][j];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) o[(16 + i) * 4 + j] = G5[i][j];
}

/* ------------------------------------------------------------ SU(3) helpers */

static const cplx *link(const cplx *U, int s, int mu) { return U + ((size_t)s * 4 + mu) * 9; }

static void mat_mul(const cplx *a, const cplx *b, cplx *c) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx acc = 0;
            for (int k = 0; k < 3; k++) acc += a[i * 3 + k] * b[k * 3 + j];
            c[i * 3 + j] = acc;
        }
}

static void mat_dag(const cplx *a, cplx *c) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) c[i * 3 + j] = conj(a[j * 3 + i]);
}

/* product of four 3x3 matrices */
static void mat_mul4(const cplx *a, const cplx *b, const cplx *c, const cplx *d, cplx *out) {
    cplx t1[9], t2[9];
    mat_mul(a, b, t1);
    mat_mul(t1, c, t2);
    mat_mul(t2, d, out);
}

/* ------------------------------------------------------------ clover term */

/* Q_{mu nu}(x): sum of the four plaquette leaves in the (mu,nu) plane that
 * start and end at x, all with the same orientation. */
static void clover_leaves(const int *L, const cplx *U, int s, int mu, int nu, cplx *Q) {
    int xpm = neighbour(L, s, mu, +1), xpn = neighbour(L, s, nu, +1);
    int xmm = neighbour(L, s, mu, -1), xmn = neighbour(L, s, nu, -1);
    int xmm_pn = neighbour(L, xmm, nu, +1);
    int xmm_mn = neighbour(L, xmm, nu, -1);
    int xmn_pm = neighbour(L, xmn, mu, +1);
    cplx d1[9], d2[9], leaf[9];
    for (int i = 0; i < 9; i++) Q[i] = 0;

    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H */
    mat_dag(link(U, xpn, mu), d1);
    mat_dag(link(U, s, nu), d2);
    mat_mul4(link(U, s, mu), link(U, xpm, nu), d1, d2, leaf);
    for (int i = 0; i < 9; i++) Q[i] += leaf[i];

    /* U_nu(x) U_mu(x+nu-mu)^H U_nu(x-mu)^H U_mu(x-mu) */
    mat_dag(link(U, xmm_pn, mu), d1);
    mat_dag(link(U, xmm, nu), d2);
    mat_mul4(link(U, s, nu), d1, d2, link(U, xmm, mu), leaf);
    for (int i = 0; i < 9; i++) Q[i] += leaf[i];

    /* U_mu(x-mu)^H U_nu(x-mu-nu)^H U_mu(x-mu-nu) U_nu(x-nu) */
    mat_dag(link(U, xmm, mu), d1);
    mat_dag(link(U, xmm_mn, nu), d2);
    mat_mul4(d1, d2, link(U, xmm_mn, mu), link(U, xmn, nu), leaf);
    for (int i = 0; i < 9; i++) Q[i] += leaf[i];

    /* U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^H */
    mat_dag(link(U, xmn, nu), d1);
    mat_dag(link(U, s, mu), d2);
    mat_mul4(d1, link(U, xmn, mu), link(U, xmn_pm, nu), d2, leaf);
    for (int i = 0; i < 9; i++) Q[i] += leaf[i];
}

/* A(x) = (4 + m0) 1 + c_sw (i/4) sum_{mu != nu} sigma_{mu nu} (x) F_{mu nu}(x) */
void or_clover(const int *L, const double *Ud, double m0, double csw, double *Ad) {
    build_gamma();
    const cplx *U = (const cplx *)Ud;
    cplx *A = (cplx *)Ad;
    int V = vol(L);
    /* sigma_{mu nu} = (i/2)(gamma_mu gamma_nu - gamma_nu gamma_mu) */
    static cplx sigma[4][4][4][4];
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++)
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) {
                    cplx c = 0;
                    for (int k = 0; k < 4; k++) c += G[mu][i][k] * G[nu][k][j] - G[nu][i][k] * G[mu][k][j];
                    sigma[mu][nu][i][j] = 0.5 * I * c;
                }
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++) {
        cplx *As = A + (size_t)s * 144;
        for (int i = 0; i < 144; i++) As[i] = 0;
        for (int i = 0; i < 12; i++) As[i * 12 + i] = 4.0 + m0;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = 0; nu < 4; nu++) {
                if (mu == nu) continue;
                cplx Q[9], F[9];
                clover_leaves(L, U, s, mu, nu, Q);
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) F[a * 3 + b] = (Q[a * 3 + b] - conj(Q[b * 3 + a])) / 8.0;
                for (int al = 0; al < 4; al++)
                    for (int be = 0; be < 4; be++)
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++)
                                As[(al * 3 + a) * 12 + be * 3 + b] +=
                                    csw * (I / 4.0) * sigma[mu][nu][al][be] * F[a * 3 + b];
            }
    }
}

/* ------------------------------------------------------------ Dirac operator */

/* out(s) = ((D - shift) in)(s). When blk >= 0 only neighbours that lie in
 * block blk (of the block decomposition with block sizes B) are used: this is
 * I^T (D - shift) I applied to a field that is zero outside the block. */
static void dirac_site(const int *L, const cplx *U, const cplx *A, cplx shift, const cplx *in, int s,
                       const int *B, int blk, cplx *out) {
    cplx acc[12];
    const cplx *As = A + (size_t)s * 144;
    const cplx *ps = in + (size_t)s * 12;
    for (int i = 0; i < 12; i++) {
        cplx c = 0;
        for (int j = 0; j < 12; j++) c += As[i * 12 + j] * ps[j];
        acc[i] = c - shift * ps[i];
    }
    for (int mu = 0; mu < 4; mu++) {
        for (int dir = 1; dir >= -1; dir -= 2) {
            int y = neighbour(L, s, mu, dir);
            if (blk >= 0) {
                int xy[4], by = 0, stride = 1;
                coords_of(L, y, xy);
                for (int nu = 0; nu < 4; nu++) {
                    by += (xy[nu] / B[nu]) * stride;
                    stride *= L[nu] / B[nu];
                }
                if (by != blk) continue;
            }
            double eta = hop_sign(L, s, mu, dir);
            const cplx *py = in + (size_t)y * 12;
            /* colour part: U_mu(x) psi(x+mu) or U_mu(x-mu)^H psi(x-mu) */
            cplx Upsi[4][3];
            const cplx *Ul = (dir > 0) ? link(U, s, mu) : link(U, y, mu);
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx c = 0;
                    for (int b = 0; b < 3; b++)
                        c += ((dir > 0) ? Ul[a * 3 + b] : conj(Ul[b * 3 + a])) * py[sp * 3 + b];
                    Upsi[sp][a] = c;
                }
            /* spin part: (1 - gamma_mu) forward, (1 + gamma_mu) backward */
            for (int al = 0; al < 4; al++)
                for (int a = 0; a < 3; a++) {
                    cplx c = 0;
                    for (int be = 0; be < 4; be++) {
                        cplx P = (al == be ? 1.0 : 0.0) - (double)dir * G[mu][al][be];
                        c += P * Upsi[be][a];
                    }
                    acc[al * 3 + a] -= 0.5 * eta * c;
                }
        }
    }
    for (int i = 0; i < 12; i++) out[i] = acc[i];
}

void or_dirac(const int *L, const double *Ud, const double *Ad, double shift_re, double shift_im,
              const double *ind, double *outd) {
    build_gamma();
    int V = vol(L);
    cplx shift = shift_re + I * shift_im;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++)
        dirac_site(L, (const cplx *)Ud, (const cplx *)Ad, shift, (const cplx *)ind, s, NULL, -1,
                   (cplx *)outd + (size_t)s * 12);
}

/* ------------------------------------------------------------ SAP (red-black Schwarz) */

/* block index (lexicographic over the block grid) and colour of site s */
static int block_of(const int *L, const int *B, int s, int *colour) {
    int x[4], b = 0, stride = 1, csum = 0;
    coords_of(L, s, x);
    for (int mu = 0; mu < 4; mu++) {
        int bm = x[mu] / B[mu];
        b += bm * stride;
        stride *= L[mu] / B[mu];
        csum += bm;
    }
    if (colour) *colour = csum & 1;
    return b;
}

/* sites of block b in local lexicographic order */
static void block_sites(const int *L, const int *B, int b, int *sites) {
    int nb[4], bc[4];
    for (int mu = 0; mu < 4; mu++) nb[mu] = L[mu] / B[mu];
    bc[0] = b % nb[0]; b /= nb[0];
    bc[1] = b % nb[1]; b /= nb[1];
    bc[2] = b % nb[2]; b /= nb[2];
    bc[3] = b;
    int n = 0, x[4];
    for (int lt = 0; lt < B[3]; lt++)
        for (int lz = 0; lz < B[2]; lz++)
            for (int ly = 0; ly < B[1]; ly++)
                for (int lx = 0; lx < B[0]; lx++) {
                    x[0] = bc[0] * B[0] + lx;
                    x[1] = bc[1] * B[1] + ly;
                    x[2] = bc[2] * B[2] + lz;
                    x[3] = bc[3] * B[3] + lt;
                    sites[n++] = site_of(L, x);
                }
}

int or_sap_check(const int *L, const int *B) {
    for (int mu = 0; mu < 4; mu++) {
        if (B[mu] <= 0 || L[mu] % B[mu]) return OR_ESHAPE;
        int nb = L[mu] / B[mu];
        if (nb > 1 && (nb & 1)) return OR_ESHAPE;
    }
    return OR_OK;
}

/* sum over the sites of a block of conj(x) y */
static cplx block_dot(const int *sites, int Vb, const cplx *x, const cplx *y) {
    cplx acc = 0;
    for (int n = 0; n < Vb; n++)
        for (int i = 0; i < 12; i++) {
            size_t k = (size_t)sites[n] * 12 + i;
            acc += conj(x[k]) * y[k];
        }
    return acc;
}

/* e = approximate solution of the block system I^T (D - shift) I e = I^T r by
 * mr_iters steps of minimal residual from e = 0 (stop if q^H q = 0). rho, q:
 * work fields (only the block's sites are touched). */
static void block_mr(const int *L, const cplx *U, const cplx *A, cplx shift, const int *B, int bb, const int *sites,
                     int Vb, int mr_iters, const cplx *r, cplx *e, cplx *rho, cplx *q) {
    for (int n = 0; n < Vb; n++)
        for (int i = 0; i < 12; i++) {
            size_t k = (size_t)sites[n] * 12 + i;
            rho[k] = r[k];
            e[k] = 0;
        }
    for (int it = 0; it < mr_iters; it++) {
        for (int n = 0; n < Vb; n++) dirac_site(L, U, A, shift, rho, sites[n], B, bb, q + (size_t)sites[n] * 12);
        double qq = 0;
        cplx qr = 0;
        for (int n = 0; n < Vb; n++)
            for (int i = 0; i < 12; i++) {
                size_t k = (size_t)sites[n] * 12 + i;
                qq += creal(conj(q[k]) * q[k]);
                qr += conj(q[k]) * rho[k];
            }
        if (qq == 0.0) break;
        cplx alpha = qr / qq;
        for (int n = 0; n < Vb; n++)
            for (int i = 0; i < 12; i++) {
                size_t k = (size_t)sites[n] * 12 + i;
                e[k] += alpha * rho[k];
                rho[k] -= alpha * q[k];
            }
    }
}

/* e = approximate solution of the same block system by k steps of GMRES from
 * e = 0 (the block solver of the paper's experiments, Section 4): Arnoldi with
 * modified Gram-Schmidt on I^T (D - shift) I started from r / ||r||, stopped
 * early when h_{j+1,j} = 0; y minimises ||beta e_1 - H y|| (Givens rotations
 * applied to the columns as they are formed, then back substitution), and
 * e = sum_i y_i v_i. Vk: k + 1 work fields, w: one more (block sites only). */
static void block_gmres(const int *L, const cplx *U, const cplx *A, cplx shift, const int *B, int bb,
                        const int *sites, int Vb, int k, const cplx *r, cplx *e, cplx **Vk, cplx *w) {
    for (int n = 0; n < Vb; n++)
        for (int i = 0; i < 12; i++) e[(size_t)sites[n] * 12 + i] = 0;
    double beta = sqrt(creal(block_dot(sites, Vb, r, r)));
    if (beta == 0.0 || k < 1) return;
    cplx *H = calloc((size_t)(k + 1) * k, sizeof(cplx));   /* column j at H + j (k + 1) */
    double *cs = calloc(k, sizeof(double));
    cplx *sn = calloc(k, sizeof(cplx)), *g = calloc(k + 1, sizeof(cplx)), *y = calloc(k, sizeof(cplx));
    for (int n = 0; n < Vb; n++)
        for (int i = 0; i < 12; i++) {
            size_t q = (size_t)sites[n] * 12 + i;
            Vk[0][q] = r[q] / beta;
        }
    int kk = k;
    for (int j = 0; j < k; j++) {
        cplx *h = H + (size_t)j * (k + 1);
        for (int n = 0; n < Vb; n++) dirac_site(L, U, A, shift, Vk[j], sites[n], B, bb, w + (size_t)sites[n] * 12);
        for (int i = 0; i <= j; i++) {
            h[i] = block_dot(sites, Vb, Vk[i], w);
            for (int n = 0; n < Vb; n++)
                for (int c = 0; c < 12; c++) {
                    size_t q = (size_t)sites[n] * 12 + c;
                    w[q] -= h[i] * Vk[i][q];
                }
        }
        double hn = sqrt(creal(block_dot(sites, Vb, w, w)));
        h[j + 1] = hn;
        if (hn == 0.0) {
            kk = j + 1;
            break;
        }
        for (int n = 0; n < Vb; n++)
            for (int c = 0; c < 12; c++) {
                size_t q = (size_t)sites[n] * 12 + c;
                Vk[j + 1][q] = w[q] / hn;
            }
    }
    g[0] = beta;
    for (int j = 0; j < kk; j++) {
        cplx *h = H + (size_t)j * (k + 1);
        for (int i = 0; i < j; i++) {   /* earlier rotations on column j */
            cplx a = h[i], b = h[i + 1];
            h[i] = cs[i] * a + sn[i] * b;
            h[i + 1] = -conj(sn[i]) * a + cs[i] * b;
        }
        cplx a = h[j], b = h[j + 1];
        double aa = cabs(a), bb2 = cabs(b);
        if (bb2 == 0.0) {
            cs[j] = 1.0; sn[j] = 0.0;
        } else if (aa == 0.0) {
            cs[j] = 0.0; sn[j] = 1.0; h[j] = b;
        } else {
            double rr = sqrt(aa * aa + bb2 * bb2);
            cs[j] = aa / rr;
            sn[j] = (a / aa) * conj(b) / rr;
            h[j] = (a / aa) * rr;
        }
        h[j + 1] = 0.0;
        cplx gj = g[j];
        g[j] = cs[j] * gj;
        g[j + 1] = -conj(sn[j]) * gj;
    }
    for (int i = kk - 1; i >= 0; i--) {
        cplx t = g[i];
        for (int l = i + 1; l < kk; l++) t -= H[(size_t)l * (k + 1) + i] * y[l];
        y[i] = t / H[(size_t)i * (k + 1) + i];
    }
    for (int i = 0; i < kk; i++)
        for (int n = 0; n < Vb; n++)
            for (int c = 0; c < 12; c++) {
                size_t q = (size_t)sites[n] * 12 + c;
                e[q] += y[i] * Vk[i][q];
            }
    free(H); free(cs); free(sn); free(g); free(y);
}

/* nsweeps applications of a Schwarz method (Section 2) to (D - shift) z = b.
 * additive = 0: red-black multiplicative Schwarz, Algorithm 2.1 (colour 0
 * first; the residual is recomputed before each colour). additive = 1:
 * additive Schwarz (the first error propagator of eq. (2.1)): one residual
 * r = b - (D - shift) z per sweep, every block system solved for it, then z
 * += sum of the block corrections. Block solver: solver = 0 MR(k), 1 GMRES(k),
 * both from e = 0 on I^T (D - shift) I. */
int or_schwarz(const int *L, const double *Ud, const double *Ad, const int *B, int nsweeps, int k, int solver,
               int additive, double shift_re, double shift_im, const double *bd, double *zd) {
    build_gamma();
    if (or_sap_check(L, B)) return OR_ESHAPE;
    const cplx *U = (const cplx *)Ud, *A = (const cplx *)Ad, *b = (const cplx *)bd;
    cplx *z = (cplx *)zd;
    cplx shift = shift_re + I * shift_im;
    int V = vol(L), Vb = B[0] * B[1] * B[2] * B[3], nblk = V / Vb;
    const size_t V12 = (size_t)V * 12;
    cplx *r = calloc(V12, sizeof(cplx)), *e = calloc(V12, sizeof(cplx));
    int nwork = solver == 1 ? k + 2 : 2;
    cplx **work = malloc(sizeof(cplx *) * nwork);
    for (int i = 0; i < nwork; i++) work[i] = calloc(V12, sizeof(cplx));
    int *colour = malloc(sizeof(int) * nblk);
    for (int bb = 0; bb < nblk; bb++) {
        int bc[4], t = bb, csum = 0;
        int nb[4] = {L[0] / B[0], L[1] / B[1], L[2] / B[2], L[3] / B[3]};
        for (int mu = 0; mu < 4; mu++) { bc[mu] = t % nb[mu]; t /= nb[mu]; csum += bc[mu]; }
        colour[bb] = csum & 1;
    }
    const int nsteps = additive ? 1 : 2;
    for (int sweep = 0; sweep < nsweeps; sweep++) {
        for (int c = 0; c < nsteps; c++) {
            /* r <- b - (D - shift) z on the sites of the blocks treated in this step */
#pragma omp parallel for schedule(static)
            for (int s = 0; s < V; s++) {
                int col;
                block_of(L, B, s, &col);
                if (!additive && col != c) continue;
                cplx Dz[12];
                dirac_site(L, U, A, shift, z, s, NULL, -1, Dz);
                for (int i = 0; i < 12; i++) r[(size_t)s * 12 + i] = b[(size_t)s * 12 + i] - Dz[i];
            }
            /* e <- B_i r on every block of this step (blocks touch disjoint sites) */
#pragma omp parallel for schedule(static)
            for (int bb = 0; bb < nblk; bb++) {
                if (!additive && colour[bb] != c) continue;
                int *sites = malloc(sizeof(int) * Vb);
                block_sites(L, B, bb, sites);
                if (solver == 1)
                    block_gmres(L, U, A, shift, B, bb, sites, Vb, k, r, e, work, work[k + 1]);
                else
                    block_mr(L, U, A, shift, B, bb, sites, Vb, k, r, e, work[0], work[1]);
                free(sites);
            }
            /* z <- z + e on the same sites */
#pragma omp parallel for schedule(static)
            for (int s = 0; s < V; s++) {
                int col;
                block_of(L, B, s, &col);
                if (!additive && col != c) continue;
                for (int i = 0; i < 12; i++) z[(size_t)s * 12 + i] += e[(size_t)s * 12 + i];
            }
        }
    }
    for (int i = 0; i < nwork; i++) free(work[i]);
    free(work); free(r); free(e); free(colour);
    return OR_OK;
}

/* nsweeps applications of Red-Black Schwarz (Section 2, Algorithm 2.1) to
 * (D - shift) z = b. Each block system I^T (D - shift) I e = I^T r is
 * approximated by mr_iters steps of minimal residual from e = 0. */
int or_sap(const int *L, const double *Ud, const double *Ad, const int *B, int nsweeps, int mr_iters,
           double shift_re, double shift_im, const double *bd, double *zd) {
    return or_schwarz(L, Ud, Ad, B, nsweeps, mr_iters, 0, 0, shift_re, shift_im, bd, zd);
}

/* block matrix I^T (D - shift) I applied to a field given on the whole lattice
 * (only the sites of block blk are read and written). Used by the tests to
 * build dense block matrices. */
int or_block_apply(const int *L, const double *Ud, const double *Ad, const int *B, int blk, double shift_re,
                   double shift_im, const double *ind, double *outd) {
    build_gamma();
    int V = vol(L), Vb = B[0] * B[1] * B[2] * B[3];
    if (blk < 0 || blk >= V / Vb) return OR_ESHAPE;
    int *sites = malloc(sizeof(int) * Vb);
    block_sites(L, B, blk, sites);
    for (int n = 0; n < Vb; n++)
        dirac_site(L, (const cplx *)Ud, (const cplx *)Ad, shift_re + I * shift_im, (const cplx *)ind, sites[n],
                   B, blk, (cplx *)outd + (size_t)sites[n] * 12);
    free(sites);
    return OR_OK;
}

void or_block_sites(const int *L, const int *B, int blk, int *sites) { block_sites(L, B, blk, sites); }

/* ------------------------------------------------------------ aggregation: P, R = P^H */

/* coarse site and chirality of a fine dof */
static int coarse_site_of(const int *L, const int *Ag, int s) {
    int x[4], Lc[4];
    coords_of(L, s, x);
    for (int mu = 0; mu < 4; mu++) Lc[mu] = L[mu] / Ag[mu];
    int xc[4] = {x[0] / Ag[0], x[1] / Ag[1], x[2] / Ag[2], x[3] / Ag[3]};
    return site_of(Lc, xc);
}

static int chirality_of_spin(int spin) { return spin >= 2; }

/* P from N test vectors (Section 3, aggregation based interpolation): the test
 * vectors are cut up over the aggregates, each aggregate split by chirality so
 * that gamma_5 P = P gamma_5^c, and every piece is orthonormalised by modified
 * Gram-Schmidt in column order (thin QR with positive diagonal of R). */
int or_build_P(const int *L, const int *Ag, int N, const double *vd, double *Pd) {
    for (int mu = 0; mu < 4; mu++)
        if (Ag[mu] <= 0 || L[mu] % Ag[mu]) return OR_ESHAPE;
    int V = vol(L), Va = Ag[0] * Ag[1] * Ag[2] * Ag[3], Vc = V / Va;
    if (N > 6 * Va) return OR_ERANK;
    const cplx *v = (const cplx *)vd;
    cplx *P = (cplx *)Pd;
    memcpy(P, v, sizeof(cplx) * (size_t)N * V * 12);
    int status = OR_OK;
    /* sites of every aggregate: the aggregates form a block decomposition */
    int *sites_all = malloc(sizeof(int) * V);
    for (int a = 0; a < Vc; a++) block_sites(L, Ag, a, sites_all + (size_t)a * Va);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < Vc; a++) {
        const int *sites = sites_all + (size_t)a * Va;
        for (int chi = 0; chi < 2; chi++) {
            for (int k = 0; k < N; k++) {
                cplx *w = P + (size_t)k * V * 12;
                double n0 = 0;
                for (int n = 0; n < Va; n++)
                    for (int sp = 2 * chi; sp < 2 * chi + 2; sp++)
                        for (int c = 0; c < 3; c++) {
                            cplx x = w[(size_t)sites[n] * 12 + sp * 3 + c];
                            n0 += creal(conj(x) * x);
                        }
                for (int j = 0; j < k; j++) {
                    cplx *qj = P + (size_t)j * V * 12;
                    cplx rjk = 0;
                    for (int n = 0; n < Va; n++)
                        for (int sp = 2 * chi; sp < 2 * chi + 2; sp++)
                            for (int c = 0; c < 3; c++) {
                                size_t i = (size_t)sites[n] * 12 + sp * 3 + c;
                                rjk += conj(qj[i]) * w[i];
                            }
                    for (int n = 0; n < Va; n++)
                        for (int sp = 2 * chi; sp < 2 * chi + 2; sp++)
                            for (int c = 0; c < 3; c++) {
                                size_t i = (size_t)sites[n] * 12 + sp * 3 + c;
                                w[i] -= rjk * qj[i];
                            }
                }
                double nn = 0;
                for (int n = 0; n < Va; n++)
                    for (int sp = 2 * chi; sp < 2 * chi + 2; sp++)
                        for (int c = 0; c < 3; c++) {
                            cplx x = w[(size_t)sites[n] * 12 + sp * 3 + c];
                            nn += creal(conj(x) * x);
                        }
                double rkk = sqrt(nn);
                if (!(rkk > 1e-12 * sqrt(n0)) || n0 == 0.0) {
#pragma omp atomic write
                    status = OR_ERANK;
                    rkk = 1.0;
                }
                for (int n = 0; n < Va; n++)
                    for (int sp = 2 * chi; sp < 2 * chi + 2; sp++)
                        for (int c = 0; c < 3; c++) w[(size_t)sites[n] * 12 + sp * 3 + c] /= rkk;
            }
        }
    }
    free(sites_all);
    return status;
}

/* c = P^H r : c[a][chi][k] = sum over the (a,chi) dof of conj(P_k) r */
void or_restrict(const int *L, const int *Ag, int N, const double *Pd, const double *fd, double *cd) {
    int V = vol(L), Vc = V / (Ag[0] * Ag[1] * Ag[2] * Ag[3]);
    const cplx *P = (const cplx *)Pd, *f = (const cplx *)fd;
    cplx *c = (cplx *)cd;
    for (int i = 0; i < Vc * 2 * N; i++) c[i] = 0;
    /* serial over sites: a fixed summation order */
    for (int s = 0; s < V; s++) {
        int a = coarse_site_of(L, Ag, s);
        for (int sp = 0; sp < 4; sp++)
            for (int col = 0; col < 3; col++)
                for (int k = 0; k < N; k++) {
                    size_t i = (size_t)s * 12 + sp * 3 + col;
                    c[((size_t)a * 2 + chirality_of_spin(sp)) * N + k] += conj(P[(size_t)k * V * 12 + i]) * f[i];
                }
    }
}

/* e = P c */
void or_prolong(const int *L, const int *Ag, int N, const double *Pd, const double *cd, double *fd) {
    int V = vol(L);
    const cplx *P = (const cplx *)Pd, *c = (const cplx *)cd;
    cplx *f = (cplx *)fd;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++) {
        int a = coarse_site_of(L, Ag, s);
        for (int sp = 0; sp < 4; sp++)
            for (int col = 0; col < 3; col++) {
                size_t i = (size_t)s * 12 + sp * 3 + col;
                cplx acc = 0;
                for (int k = 0; k < N; k++) acc += P[(size_t)k * V * 12 + i] * c[((size_t)a * 2 + chirality_of_spin(sp)) * N + k];
                f[i] = acc;
            }
    }
}

/* ------------------------------------------------------------ coarse operator D_c = P^H D P */

/* 12x12 matrix of the term of D that couples x to y: term 0 is A(x) (y = x),
 * term 1+2*mu is the forward hop (y = x+mu), term 2+2*mu the backward hop. */
static void dirac_term(const int *L, const cplx *U, const cplx *A, int s, int term, int *y, cplx *M) {
    if (term == 0) {
        *y = s;
        for (int i = 0; i < 144; i++) M[i] = A[(size_t)s * 144 + i];
        return;
    }
    int mu = (term - 1) / 2, dir = ((term - 1) % 2 == 0) ? 1 : -1;
    int t = neighbour(L, s, mu, dir);
    *y = t;
    double eta = hop_sign(L, s, mu, dir);
    const cplx *Ul = (dir > 0) ? link(U, s, mu) : link(U, t, mu);
    for (int al = 0; al < 4; al++)
        for (int a = 0; a < 3; a++)
            for (int be = 0; be < 4; be++)
                for (int b = 0; b < 3; b++) {
                    cplx P = (al == be ? 1.0 : 0.0) - (double)dir * G[mu][al][be];
                    cplx Uab = (dir > 0) ? Ul[a * 3 + b] : conj(Ul[b * 3 + a]);
                    M[(al * 3 + a) * 12 + be * 3 + b] = -0.5 * eta * P * Uab;
                }
}

/* D_c = P^H D P as a 9-point stencil on the coarse lattice. A term of D at
 * fine site x in aggregate a goes to the self block when it stays inside a
 * (without crossing a face of a), and otherwise to the block of the face it
 * crosses, whose coarse neighbour is taken periodically. */
int or_coarse_build(const int *L, const int *Ag, int N, const double *Ud, const double *Ad, const double *Pd,
                    double *Dcd) {
    build_gamma();
    for (int mu = 0; mu < 4; mu++)
        if (Ag[mu] <= 0 || L[mu] % Ag[mu]) return OR_ESHAPE;
    const cplx *U = (const cplx *)Ud, *A = (const cplx *)Ad, *P = (const cplx *)Pd;
    cplx *Dc = (cplx *)Dcd;
    int V = vol(L), Va = Ag[0] * Ag[1] * Ag[2] * Ag[3], Vc = V / Va, n2 = 2 * N;
    memset(Dc, 0, sizeof(cplx) * (size_t)Vc * 9 * n2 * n2);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < Vc; a++) {
        int *sites = malloc(sizeof(int) * Va);
        block_sites(L, Ag, a, sites);
        cplx M[144], w[12];
        for (int n = 0; n < Va; n++) {
            int s = sites[n], x[4];
            coords_of(L, s, x);
            for (int term = 0; term < 9; term++) {
                int y, d = 0;
                dirac_term(L, U, A, s, term, &y, M);
                if (term > 0) {
                    int mu = (term - 1) / 2, fwd = ((term - 1) % 2 == 0);
                    int crosses = fwd ? (x[mu] % Ag[mu] == Ag[mu] - 1) : (x[mu] % Ag[mu] == 0);
                    d = crosses ? term : 0;
                }
                cplx *blk = Dc + ((size_t)a * 9 + d) * n2 * n2;
                for (int chi2 = 0; chi2 < 2; chi2++)
                    for (int k2 = 0; k2 < N; k2++) {
                        /* w = M * (P_k2 at y, restricted to chirality chi2) */
                        const cplx *py = P + (size_t)k2 * V * 12 + (size_t)y * 12;
                        for (int i = 0; i < 12; i++) {
                            cplx acc = 0;
                            for (int j = 0; j < 12; j++)
                                if (chirality_of_spin(j / 3) == chi2) acc += M[i * 12 + j] * py[j];
                            w[i] = acc;
                        }
                        for (int chi1 = 0; chi1 < 2; chi1++)
                            for (int k1 = 0; k1 < N; k1++) {
                                const cplx *px = P + (size_t)k1 * V * 12 + (size_t)s * 12;
                                cplx acc = 0;
                                for (int i = 0; i < 12; i++)
                                    if (chirality_of_spin(i / 3) == chi1) acc += conj(px[i]) * w[i];
                                blk[(chi1 * N + k1) * n2 + chi2 * N + k2] += acc;
                            }
                    }
            }
        }
        free(sites);
    }
    return OR_OK;
}

/* y = D_c x, y[a] = sum_dir Dc[a][dir] x[a + dir] (periodic coarse lattice) */
void or_coarse_apply(const int *Lc, int N, const double *Dcd, const double *xd, double *yd) {
    const cplx *Dc = (const cplx *)Dcd, *x = (const cplx *)xd;
    cplx *y = (cplx *)yd;
    int Vc = vol(Lc), n2 = 2 * N;
#pragma omp parallel for schedule(static)
    for (int a = 0; a < Vc; a++) {
        for (int i = 0; i < n2; i++) {
            cplx acc = 0;
            for (int d = 0; d < 9; d++) {
                int b = (d == 0) ? a : neighbour(Lc, a, (d - 1) / 2, ((d - 1) % 2 == 0) ? 1 : -1);
                const cplx *blk = Dc + ((size_t)a * 9 + d) * n2 * n2;
                for (int j = 0; j < n2; j++) acc += blk[i * n2 + j] * x[(size_t)b * n2 + j];
            }
            y[(size_t)a * n2 + i] = acc;
        }
    }
}

int or_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
