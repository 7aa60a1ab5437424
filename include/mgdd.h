/*
 * mgdd.h -- C ABI of the MI355X (gfx950) library for the SAP-preconditioned
 * aggregation multilevel solver of the Wilson-clover Dirac equation
 *     D z = b,   D = D(U) + m
 * after Frommer, Kahl, Krieg, Leder, Rottmann, "Aggregation-based Multilevel
 * Methods for Lattice QCD" (Lattice 2011, arXiv:1202.2462).
 *
 * Conventions of every call
 * -------------------------
 *  - Every call returns MGDD_OK (0) or a negative MGDD_E* code; the text of the
 *    last error of a context is returned by mgdd_last_error(). No C++
 *    exception crosses this boundary.
 *  - Device buffers are plain device pointers owned by the caller (for
 *    example the data pointers of PyTorch tensors); host buffers are plain host
 *    pointers owned by the caller. The library owns the gauge links, the
 *    clover term, P, D_c and its own workspace.
 *  - Work is queued on the HIP stream given to mgdd_create, in order, and is
 *    asynchronous unless a call says otherwise. One context per stream; a
 *    context must not be used from two host threads at once.
 *  - Input and output buffers of one call must not overlap unless a call says
 *    so.
 *
 * Lattice and field layouts
 * -------------------------
 *  Canonical (interchange) layout, complex double:
 *    site    s = x + Lx*(y + Ly*(z + Lz*t))
 *    gauge   U[s][mu][a][b]         mu = 0,1,2,3 for x,y,z,t, SU(3) links
 *    spinor  psi[rhs][s][spin][col] 4 spins x 3 colours = 12 dof per site
 *    coarse  c[rhs][a][chi][k]      a = coarse site (lexicographic on the
 *                                   coarse lattice L/agg), chi = 0 for
 *                                   spins 0,1 (gamma_5 = +1) and 1 for spins
 *                                   2,3, k = test-vector index
 *  Boundary conditions: periodic in x, y, z and antiperiodic in t.
 *  Gamma matrices: chiral basis, gamma_k = [[0,-i s_k],[i s_k,0]],
 *  gamma_t = [[0,-1],[-1,0]], gamma_5 = diag(1,1,-1,-1).
 *  Operator (Section 1 of the paper; clover term named in its abstract):
 *    (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                                          + (1+gamma_mu) U_mu(x-mu)^H psi(x-mu) ]
 *    A(x) = (4+m0) + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x),
 *    F = (Q - Q^H)/8 with Q the four plaquette leaves at x.
 *
 *  Device field layout (what every `void*` field argument points to):
 *    fine field, precision p, nrhs right-hand sides:
 *      [rhs][component 0..11][site'] of complex p  (component = spin*3+col)
 *    where site' is the device site order: lattice blocks of the size given
 *    to mgdd_create in block-major order (all blocks of colour 0 first, then
 *    colour 1, colour = parity of the sum of block coordinates), and inside a
 *    block the sites of even parity first. mgdd_pack / mgdd_unpack convert
 *    between canonical and device layout. Sizes: mgdd_field_bytes().
 *    coarse field: [rhs][a][chi][k] of complex p (the canonical order).
 *  Precision codes: MGDD_F64 (complex double), MGDD_F32 (complex float).
 */
#ifndef MGDD_H
#define MGDD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MGDD_OK = 0,
    MGDD_EINVAL = -1,     /* bad argument (null pointer, bad precision code, ...) */
    MGDD_ESHAPE = -2,     /* lattice / block / aggregate shapes do not fit */
    MGDD_ERANK = -3,      /* test vectors are rank deficient on an aggregate */
    MGDD_ENOTREADY = -4,  /* no gauge field, or no P / D_c yet */
    MGDD_ENOCONV = -5,    /* solver hit maxit; solution and stats are written */
    MGDD_EBREAKDOWN = -6, /* Krylov breakdown that could not be recovered */
    MGDD_ENAN = -7,       /* NaN or Inf met in the input or the iteration */
    MGDD_EHIP = -8,       /* a HIP runtime call failed */
    MGDD_ENOMEM = -9      /* device allocation failed */
};

enum { MGDD_F64 = 0, MGDD_F32 = 1 };

typedef struct mgdd_ctx mgdd_ctx;

/* Context for one lattice. dims = (Lx,Ly,Lz,Lt). block = (bx,by,bz,bt) is the
 * lattice block decomposition of Section 2 used by the Schwarz smoother and
 * by the device site order: every b_mu a power of two >= 2 dividing L_mu,
 * and the number of blocks L_mu/b_mu even or 1 in every direction (a
 * two-colouring in which no two neighbouring blocks share a colour).
 * hip_stream: a hipStream_t (NULL = the default stream). *out receives the
 * context. Errors: MGDD_ESHAPE, MGDD_EINVAL, MGDD_EHIP. */
int mgdd_create(const int dims[4], const int block[4], void *hip_stream, mgdd_ctx **out);

/* Frees everything the context owns. Safe on NULL. */
int mgdd_destroy(mgdd_ctx *ctx);

/* Text of the last error on ctx (never NULL; "" when none). */
const char *mgdd_last_error(const mgdd_ctx *ctx);

/* Bytes of a device field: level 0 = fine lattice, level 1 = coarse lattice
 * of the current P (0 if there is none). */
size_t mgdd_field_bytes(const mgdd_ctx *ctx, int prec, int nrhs, int level);

/* Sets the gauge field and mass of D = D(U) + m (Section 1): U is the
 * canonical host array [V][4][3][3] of complex double (read only, copied).
 * Builds on the device the links in FP64 and FP32 and the clover term
 * A(x) = (4+m0) + c_sw (i/4) sum sigma F (both chiral 6x6 blocks, FP64 and
 * FP32) and the inverse of A on even sites (FP64). Synchronous. Drops any P. */
int mgdd_set_gauge(mgdd_ctx *ctx, const double *U, double m0, double csw);

/* Canonical complex-double fields (nrhs of them, host or device memory as
 * src_on_device says) -> device layout of precision prec (round to nearest
 * for MGDD_F32). Asynchronous for device sources; synchronous for host ones. */
int mgdd_pack(mgdd_ctx *ctx, int prec, int nrhs, const double *src, int src_on_device, void *dst);

/* Device layout -> canonical complex double (host or device). Synchronous for
 * host destinations. */
int mgdd_unpack(mgdd_ctx *ctx, int prec, int nrhs, const void *src, double *dst, int dst_on_device);

/* out = D in for nrhs fields (Section 1, eq. (1.1)); in and out are device
 * fields of precision prec. Asynchronous. */
int mgdd_dirac_apply(mgdd_ctx *ctx, int prec, int nrhs, const void *in, void *out);

/* nsweeps sweeps of Red-Black Schwarz (Section 2, Algorithm 2.1) on
 * (D - shift) z = b, z in/out, over the blocks of mgdd_create; each block
 * system I^T (D - shift) I e = I^T r is approximated by mr_iters minimal
 * residual steps from e = 0 (the shifted block inverses B_j(lambda) of the
 * second setup part use shift = lambda). Asynchronous. */
int mgdd_sap(mgdd_ctx *ctx, int prec, int nrhs, int nsweeps, int mr_iters, double shift_re, double shift_im,
             const void *b, void *z);

#ifdef __cplusplus
}
#endif
#endif
