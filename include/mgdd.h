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
 *  Boundary conditions: periodic in x, y, z; antiperiodic in t unless the
 *  context was created with t_antiperiodic = 0 (then periodic in t).
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
 *  Precision codes: MGDD_F64 (complex double), MGDD_F32 (complex float),
 *    MGDD_F16 (complex stored as two IEEE binary16 values, 4 bytes; a storage
 *    format of fine fields only: accepted by mgdd_field_bytes (level 0),
 *    mgdd_pack, mgdd_unpack, mgdd_dirac_apply, mgdd_sap and mgdd_schwarz
 *    (red-black, MR block solves, special unitary links), mgdd_restrict and
 *    mgdd_prolong (the coarse field then in FP32, P read in half precision)
 *    and mgdd_timing_read, whose arithmetic is FP32; values are rounded to
 *    nearest even when stored).
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

enum { MGDD_F64 = 0, MGDD_F32 = 1, MGDD_F16 = 2 };

typedef struct mgdd_ctx mgdd_ctx;

/* Context for one lattice. dims = (Lx,Ly,Lz,Lt). block = (bx,by,bz,bt) is the
 * lattice block decomposition of Section 2 used by the Schwarz smoother and
 * by the device site order: every b_mu a power of two >= 2 dividing L_mu,
 * and the number of blocks L_mu/b_mu even or 1 in every direction (a
 * two-colouring in which no two neighbouring blocks share a colour). The
 * device site order is built from these blocks (a colour step of the
 * smoother reads one contiguous half of every field), so the Schwarz block
 * of a context is fixed; another block shape needs another context.
 * t_antiperiodic: 1 for antiperiodic boundary conditions in time (the hops
 * across the time boundary carry a sign -1), 0 for periodic ones.
 * The volume is at most 14 913 080 sites (device arrays are addressed with
 * 32-bit byte offsets, 288 bytes per site at most; 48^3 x 96 fits).
 * hip_stream: a hipStream_t (NULL = the default stream). *out receives the
 * context. Errors: MGDD_ESHAPE, MGDD_EINVAL, MGDD_EHIP. */
int mgdd_create(const int dims[4], const int block[4], int t_antiperiodic, void *hip_stream, mgdd_ctx **out);

/* Device memory of the context (links, clover term, P, D_c, workspace)
 * taken from a caller's allocator instead of hipMalloc / hipFree, so that for
 * example PyTorch's caching allocator can own it: alloc(bytes, user) returns
 * a device pointer (aligned to at least 256 bytes) or NULL, free(ptr, user)
 * releases one. Every allocation made after this call goes through the pair
 * and is released through it (by mgdd_release_workspace, by a rebuild of P,
 * or at the latest by mgdd_destroy); earlier allocations keep hipFree.
 * alloc = free = NULL restores hipMalloc / hipFree for later allocations.
 * Both or neither must be given. Errors: MGDD_EINVAL. */
typedef void *(*mgdd_alloc_fn)(size_t bytes, void *user);
typedef void (*mgdd_free_fn)(void *ptr, void *user);
int mgdd_set_allocator(mgdd_ctx *ctx, mgdd_alloc_fn alloc, mgdd_free_fn free_fn, void *user);

/* Thread tiles of the kernels, the knobs an autotuner searches beside the
 * Schwarz block shape (they change the schedule, never the arithmetic of a
 * site beyond the summation order of the FP32 Schwarz kernels):
 *   sap_lanes: lanes per site of the FP32 Schwarz colour kernel (Algorithm
 *     2.1): 0 automatic (2 when the links are special unitary and the
 *     staged links fit in LDS, else 4 when the staged links fit, else 1),
 *     1 (one lane per site, spinors in LDS), 2 (two lanes per site, one per
 *     chirality, rows 0 and 1 of the block's links staged in LDS; needs
 *     special unitary links) or 4 (four lanes per site, the whole links
 *     staged). Half-precision storage runs with 2 lanes only; FP64 sweeps
 *     always use 1.
 *   dirac_stage: Wilson-clover apply with blocks of 256 sites: 0 automatic
 *     (the workgroup's block of spinors staged in LDS), 1 staged, -1 not
 *     staged (every neighbour read from memory).
 * A variant the context cannot run fails at launch with MGDD_ESHAPE.
 * Errors: MGDD_EINVAL (values outside these sets). */
typedef struct {
    int sap_lanes;
    int dirac_stage;
} mgdd_kernel_options;
int mgdd_set_kernel_options(mgdd_ctx *ctx, const mgdd_kernel_options *options);

/* Frees everything the context owns. Safe on NULL. */
int mgdd_destroy(mgdd_ctx *ctx);

/* Text of the last error on ctx (never NULL; "" when none). */
const char *mgdd_last_error(const mgdd_ctx *ctx);

/* Bytes of a device field: level 0 = fine lattice, level 1 = coarse lattice
 * of the current P, level 2 = level-3 lattice of the current P2 (0 if there
 * is none). */
size_t mgdd_field_bytes(const mgdd_ctx *ctx, int prec, int nrhs, int level);

/* Sets the gauge field and mass of D = D(U) + m (Section 1): U is the
 * canonical array [V][4][3][3] of complex double (read only), in host memory
 * or, if src_on_device, in device memory. Builds on the device the links in
 * FP64 and FP32 and the clover term A(x) = (4+m0) + c_sw (i/4) sum sigma F
 * (both chiral 6x6 blocks, FP64 and FP32) and the inverse of A (FP64, for the
 * even-odd comparator). Synchronous. Drops any P. Errors: MGDD_ENAN (NaN or
 * Inf in U, m0 or csw), MGDD_EINVAL (singular clover block). */
int mgdd_set_gauge(mgdd_ctx *ctx, const double *U, int src_on_device, double m0, double csw);

/* Canonical complex-double fields (nrhs of them, host or device memory as
 * src_on_device says) -> device layout of precision prec (round to nearest
 * for MGDD_F32). Asynchronous for device sources; synchronous for host ones. */
int mgdd_pack(mgdd_ctx *ctx, int prec, int nrhs, const double *src, int src_on_device, void *dst);

/* Device layout -> canonical complex double (host or device). Synchronous for
 * host destinations. */
int mgdd_unpack(mgdd_ctx *ctx, int prec, int nrhs, const void *src, double *dst, int dst_on_device);

/* out = D in for nrhs fields (Section 1, eq. (1.1)); in and out are device
 * fields of precision prec (MGDD_F16: half-precision spinors, FP32 links,
 * clover term and arithmetic, the result rounded to half). Asynchronous. */
int mgdd_dirac_apply(mgdd_ctx *ctx, int prec, int nrhs, const void *in, void *out);

/* nsweeps sweeps of Red-Black Schwarz (Section 2, Algorithm 2.1) on
 * (D - shift) z = b, z in/out, over the lattice blocks `block` (NULL: the
 * blocks of mgdd_create; otherwise they must be those blocks, see
 * mgdd_create, else MGDD_ESHAPE); each block system I^T (D - shift) I e =
 * I^T r is approximated by mr_iters minimal residual steps from e = 0 (the
 * shifted block inverses B_j(lambda) of the second setup part use shift =
 * lambda). prec MGDD_F16: b and z in half precision, the sweep in FP32 (z
 * rounded once per colour step when it is stored); needs special unitary
 * links, else MGDD_EINVAL. Asynchronous. */
int mgdd_sap(mgdd_ctx *ctx, int prec, int nrhs, const int block[4], int nsweeps, int mr_iters, double shift_re,
             double shift_im, const void *b, void *z);

/* Schwarz variants of Section 2 and of the paper's experiments (Section 4:
 * 3 GMRES steps per block system). block_solver: MGDD_BLOCK_MR (k steps of
 * minimal residual, as mgdd_sap) or MGDD_BLOCK_GMRES (k = 1..3 steps of GMRES
 * from e = 0 on I^T (D - shift) I: Arnoldi, then the small least-squares
 * problem, per block). additive = 0: red-black multiplicative sweeps
 * (Algorithm 2.1); additive = 1: additive Schwarz (the first propagator of
 * eq. (2.1)): per sweep one residual r = b - D z, every block system solved
 * for it, z += the sum of the corrections (needs shift = 0). block: as for
 * mgdd_sap. b, z: nrhs fields of precision prec, z in/out, not aliased. Uses
 * the context's workspace (additive). Errors: MGDD_EINVAL (bad parameters),
 * MGDD_ESHAPE (block volume outside 64..256, or not the context's blocks),
 * MGDD_ENOTREADY (no gauge field). Asynchronous. */
enum { MGDD_BLOCK_MR = 0, MGDD_BLOCK_GMRES = 1 };
typedef struct {
    int nsweeps;
    int block_iters;       /* k */
    int block_solver;      /* MGDD_BLOCK_MR or MGDD_BLOCK_GMRES */
    int additive;          /* 0 red-black multiplicative, 1 additive */
    double shift_re, shift_im;
} mgdd_schwarz_params;
int mgdd_schwarz(mgdd_ctx *ctx, int prec, int nrhs, const int block[4], const mgdd_schwarz_params *params,
                 const void *b, void *z);

/* ------------------------------------------------------------------ coarse level (Section 3) */

/* Builds the aggregation interpolation P from ntv test vectors (Section 3,
 * "Aggregation Based Interpolation"): the vectors are cut up over the
 * aggregates, which form a block decomposition of extents agg (each dividing
 * L) and are split by chirality (spins 0,1 and 2,3) so that
 * gamma_5 P = P gamma_5^c; each (aggregate, chirality) piece is
 * orthonormalised by modified Gram-Schmidt in column order (P^H P = 1, the
 * unique thin QR with positive diagonal of R). Then builds the coarse operator
 * D_c = P^H D P (a 9-point stencil of 2N x 2N blocks) in FP64, with FP32
 * copies of P and D_c and a half-precision copy of P: every precision is
 * always stored (the FP64 pair serves the plain FP64 solve and the FP64 parts
 * of the setup, the FP32 pair the mixed-precision preconditioner, the half
 * P the half-storage transfers), so there is no storage-precision argument.
 * The FP32 copy of D_c used by the coarse GMRES keeps the self block and the
 * four forward hops of each coarse site; its backward hops are the
 * gamma5^c-conjugate transposes D_c(a, a - mu) = g5c D_c(a - mu, a)^H g5c
 * (D_c is gamma5^c-hermitian because D is gamma5-hermitian and
 * gamma_5 P = P gamma_5^c). test_vectors: ntv FP64 device fields (read only).
 * Synchronous. Errors: MGDD_ERANK (ntv > 6 * vol(agg) or a piece is rank
 * deficient), MGDD_ESHAPE, MGDD_EINVAL (ntv not in 1..32). */
int mgdd_build_P(mgdd_ctx *ctx, const int agg[4], int ntv, const void *test_vectors);

/* Copies the ntv test vectors that define the current P (FP64 device fields)
 * to dst (device, ntv fine FP64 fields). */
int mgdd_get_test_vectors(mgdd_ctx *ctx, void *dst);

/* Checkpoint of the setup (the paper's amortisation of one setup over many
 * solves, Section 4): writes the test vectors that define the current P to
 * a file (a header with lattice, aggregate, ntv, m0, c_sw, payload size and a
 * 64-bit FNV-1a checksum, then the vectors in canonical order, complex
 * double). Synchronous. Errors: MGDD_ENOTREADY (no P), MGDD_EINVAL (file). */
int mgdd_save_setup(mgdd_ctx *ctx, const char *path);

/* Rebuilds P and D_c from a setup file written by mgdd_save_setup for the
 * same lattice (the block shape may differ; the gauge field set on this
 * context is used for D_c). Synchronous. Errors: MGDD_ENOTREADY (no gauge
 * field), MGDD_ESHAPE (another lattice), MGDD_EINVAL (unreadable,
 * truncated or corrupt file: the checksum is verified before anything is
 * changed), and those of mgdd_build_P. */
int mgdd_load_setup(mgdd_ctx *ctx, const char *path);

/* coarse = P^H fine (restriction R = P^H, Section 3); nrhs fields. prec
 * MGDD_F16: fine field and P in half precision, coarse field and arithmetic
 * in FP32. */
int mgdd_restrict(mgdd_ctx *ctx, int prec, int nrhs, const void *fine, void *coarse);

/* fine = P coarse (interpolation, Section 3); nrhs fields. prec MGDD_F16:
 * coarse field FP32, P and the fine field (rounded once) in half precision. */
int mgdd_prolong(mgdd_ctx *ctx, int prec, int nrhs, const void *coarse, void *fine);

/* out = D_c in, D_c = P^H D P (eq. (3.1)); nrhs coarse fields. */
int mgdd_coarse_apply(mgdd_ctx *ctx, int prec, int nrhs, const void *in, void *out);

/* x = approximate D_c^{-1} b by `iters` steps of GMRES from x = 0 without
 * restart (the coarse solve of Section 4 uses 12). nrhs coarse fields, each
 * with its own Krylov basis and Hessenberg matrix, computed together in
 * shared launches; synchronous (one host read of the Hessenberg matrices). */
int mgdd_coarse_solve(mgdd_ctx *ctx, int prec, int nrhs, int iters, const void *b, void *x);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * mgdd_coarse_solve, with every buffer of the solve (Krylov basis, Hessenberg
 * matrices, partial sums, status flag) in a fixed 64 MiB device array of the
 * library instead of the context's workspace; it calls no hipMalloc, hipFree
 * or allocating library routine. One copy of the array exists per GPU and is
 * shared by every context and call on that GPU: calls that overlap on one GPU
 * (two streams, two host threads) race and must not be issued. iters <= 15.
 * Errors: MGDD_EINVAL (more than 15 steps, or the solve would need more than
 * the 64 MiB: (iters + 3) * nrhs coarse fields plus small terms), those of
 * mgdd_coarse_solve. Synchronous. */
int mgdd_coarse_solve_noalloc(mgdd_ctx *ctx, int prec, int nrhs, int iters, const void *b, void *x);

/* Two-level preconditioner (Section 3: smoother and coarse-grid correction
 * alternate): z = P GMRES_iters(D_c, P^H r) followed by nu Schwarz sweeps
 * (mr_iters MR steps per block) on D z = r. r: FP64 fine fields; z: fine
 * fields of precision prec (the precision the preconditioner computes in). */
int mgdd_precondition(mgdd_ctx *ctx, int prec, int nrhs, int nu, int mr_iters, int coarse_iters, const void *r,
                      void *z);

/* ------------------------------------------------------------------ setup and solve */

typedef struct {
    int agg[4];       /* aggregate extents */
    int ntv;          /* number of test vectors N */
    int nu;           /* first part: rounds of one Schwarz sweep (b = 0) + orthonormalisation */
    int iota;         /* second part: shifted Schwarz sweeps on each interpolated Ritz vector */
    int mr_iters;     /* minimal residual steps per block solve */
    int arnoldi_m;    /* Arnoldi steps for the harmonic Ritz pairs; 0 = min(dim D_c, 2N + 10) */
    int n_part2;      /* repetitions of the second part (the paper runs it once) */
    int prec;         /* precision of the Schwarz sweeps: MGDD_F64 or MGDD_F32 */
    int chunk;        /* 0: automatic. Otherwise the memory-lean form with this many
                         vectors per first-part sweep launch and columns per block
                         of the second part's Gram matrix, formed as
                         <w_i, D^H D w_j> without holding D W. Automatic is the full
                         form below 2^22 sites and chunks of 4 from there on. */
    unsigned long long seed;  /* stream of the random vectors drawn by the library when
                                 mgdd_setup_bootstrap gets random_vectors = NULL */
} mgdd_setup_params;

/* Bootstrap setup (Section 3, "Bootstrap Setup"). Part 1: the ntv random
 * fields (random_vectors: ntv FP64 device fields, read only; or NULL: drawn
 * by the library from stream params->seed of the counter-based generator
 * SplitMix64 (Steele, Lea, Flood 2014), value i = mix64(seed G + (i+1) G),
 * G = 0x9E3779B97F4A7C15, uniforms from the top 53 bits, complex Gaussian
 * element e = sqrt(-2 ln(1 - u_2e)) exp(2 pi i u_2e+1), e counted in the
 * canonical order ((field V + site) 12 + component)) get nu rounds of
 * one Schwarz sweep with b = 0, each followed by a global modified
 * Gram-Schmidt in index order; then P and D_c. Part 2 (n_part2 times):
 * harmonic Ritz pairs (lambda_i, phi_i) of D_c (target 0, the ntv of smallest
 * modulus, from arnoldi_m Arnoldi steps started at arnoldi_start: one FP64
 * coarse field, device), w_i = P phi_i smoothed by iota sweeps of Schwarz with
 * block inverses of D - lambda_i, then the 2N vectors {w_i} u {v_j} are
 * orthonormalised and replaced by the N combinations given by the N smallest
 * eigenpairs of the Gram matrix (DV)^H DV; then P and D_c again.
 * Synchronous. */
int mgdd_setup_bootstrap(mgdd_ctx *ctx, const mgdd_setup_params *params, const void *random_vectors,
                         const void *arnoldi_start);

enum { MGDD_SOLVER_FGMRES_MG = 0, MGDD_SOLVER_GCR = 1, MGDD_SOLVER_GCR_EO = 2, MGDD_SOLVER_CGN = 3 };
enum { MGDD_PLAIN_F64 = 0, MGDD_MIXED = 1, MGDD_MIXED_F16 = 2 };

typedef struct {
    int solver;        /* MGDD_SOLVER_* */
    int precision;     /* MGDD_PLAIN_F64, or MGDD_MIXED: the preconditioner (SAP,
                          restriction, prolongation, coarse solve) in FP32, the
                          outer orthogonalisation, true residual and solution
                          update in FP64; or MGDD_MIXED_F16: as MGDD_MIXED with
                          the preconditioner's fine fields (its copy of the
                          residual, the Schwarz iterate, the flexible basis Z)
                          and P stored in half precision, arithmetic in FP32,
                          the coarse level in FP32 (red-black Schwarz with MR
                          block solves and special unitary links only) */
    int restart;       /* Krylov restart length m */
    double tol;        /* stop when ||b - D z|| <= tol ||b|| (true residual, FP64) */
    int maxit;         /* maximal number of outer iterations */
    int coarse_iters;  /* GMRES steps on D_c per preconditioner application */
    int nu;            /* Schwarz sweeps per preconditioner application */
    int mr_iters;      /* MR steps per block solve */
    int levels;        /* 3: three-level preconditioner (needs mgdd_setup_level2 or
                          mgdd_build_P2); 0 or 2: two levels */
    int k2;            /* three levels: flexible GMRES steps on D_c per coarse solve */
    int nu2;           /* three levels: level-2 Schwarz sweeps per application of
                          the level-2 preconditioner */
    int mr2;           /* three levels: MR steps per level-2 block solve */
    int block_solver;  /* smoother's block solves: MGDD_BLOCK_MR (mr_iters MR steps) or
                          MGDD_BLOCK_GMRES (mr_iters = 1..3 GMRES steps) */
    int additive;      /* smoother: 0 red-black multiplicative, 1 additive Schwarz */
} mgdd_solve_params;

typedef struct {
    int iters;         /* outer iterations */
    int restarts;      /* true-residual recomputations */
    int converged;     /* 1 if ||b - D z|| <= tol ||b|| */
    double relres;     /* final ||b - D z|| / ||b|| in FP64 */
    double seconds;    /* wall time of the solve this right-hand side was part of */
} mgdd_solve_stats;

/* Solves D z = b (eq. (1.1)) for nrhs FP64 device fields b; z (FP64 device
 * fields) holds the initial guess on entry and the solution on exit.
 * FGMRES_MG: flexible GMRES(restart) right-preconditioned by the two-level
 * method (Section 4), or with levels = 3 by the three-level method
 * (mgdd_precondition3); coarse_iters is then the GMRES step count on the
 * coarsest operator D_cc. GCR: plain GCR(restart) on D. GCR_EO: GCR(restart) on
 * the even-odd Schur complement, convergence judged on the full system. CGN:
 * conjugate gradients on D^H D z = D^H b (the paper's comparator, Section 4)
 * with the residual b - D z updated alongside; when it reaches the tolerance
 * the true residual is recomputed, and CG starts again from the iterate if
 * it is still too large (counted in restarts); restart is unused.
 * With FGMRES_MG the nrhs right-hand sides are solved together: one Krylov
 * basis, Hessenberg matrix, restart and stopping test each, with D, the
 * preconditioner and the Gram-Schmidt steps applied to all of them in shared
 * launches (a right-hand side that has converged stops changing). If the
 * workspace for all of them does not fit in device memory they are split
 * into smaller batches. GCR, GCR_EO and CGN solve them one after the other.
 * stats: array of nrhs entries (may be NULL). Synchronous. Errors:
 * MGDD_ENOCONV (maxit reached; z and stats written), MGDD_ENAN,
 * MGDD_ENOTREADY (no gauge field; no P for FGMRES_MG; no third level or no
 * level-2 Schwarz blocks for levels = 3). */
int mgdd_solve(mgdd_ctx *ctx, const mgdd_solve_params *params, int nrhs, const void *b, void *z,
               mgdd_solve_stats *stats);

/* ------------------------------------------------------------------ third level
 * Section 3: the two-level construction applied to the coarse equation
 * D_c x = r_c (the paper's recursive extension). Level-2 aggregates are
 * blocks of coarse sites (agg2, dividing the coarse lattice); each is split
 * by the coarse chirality (the first / last N dof of a coarse site) into two
 * pieces of vol(agg2) * N dof. Level-3 vectors: [rhs][level-3 site
 * (lexicographic)][chirality][N2] complex, MGDD_F64 or MGDD_F32
 * (mgdd_field_bytes with level 2). Building P2 or D_c again (mgdd_build_P,
 * mgdd_setup_bootstrap) invalidates the third level. */

/* P2 from ntv2 coarse FP64 test vectors (ntv2 coarse fields, device
 * memory, copied): every (aggregate, chirality) piece orthonormalised in
 * column order (the unique thin QR with a positive diagonal of R), then
 * D_cc = P2^H D_c P2 as a 9-point stencil with 2*ntv2 x 2*ntv2 blocks, built
 * by the local formula (a hop of D_c inside an aggregate goes to the self
 * block, one crossing its face in direction d to block d). Errors:
 * MGDD_ENOTREADY (no P), MGDD_ESHAPE (agg2 does not divide the coarse
 * lattice), MGDD_EINVAL (ntv2 not in 1..32), MGDD_ERANK (rank-deficient
 * piece). Synchronous. */
int mgdd_build_P2(mgdd_ctx *ctx, const int agg2[4], int ntv2, const void *test_vectors2);

/* coarse2 = P2^H coarse; nrhs coarse fields to nrhs level-3 fields. */
int mgdd_restrict2(mgdd_ctx *ctx, int prec, int nrhs, const void *coarse, void *coarse2);

/* coarse = P2 coarse2. */
int mgdd_prolong2(mgdd_ctx *ctx, int prec, int nrhs, const void *coarse2, void *coarse);

/* out = D_cc in on nrhs level-3 fields (in and out must not alias). */
int mgdd_coarse2_apply(mgdd_ctx *ctx, int prec, int nrhs, const void *in, void *out);

/* nsweeps sweeps of the red-black Schwarz method (Algorithm 2.1) on the
 * coarse equation D_c z = b, the smoother of the second level: the coarse
 * lattice is split into blocks of block2 coarse sites (dividing it, with an
 * even number of blocks or one block per direction, at most 1024 / (2N)
 * sites per block); blocks whose block coordinates have an even sum (colour
 * 0) are updated first, then colour 1, each by MR(mr_iters) on the block
 * operator (D_c restricted to the block: hops leaving it dropped) started
 * from a zero correction. b, z: nrhs coarse fields of precision prec, z holds
 * the initial guess on entry and the result on exit (z and b must not
 * alias). Errors: MGDD_ENOTREADY (no P), MGDD_ESHAPE (block2 invalid).
 * Synchronous. */
int mgdd_coarse_sap(mgdd_ctx *ctx, int prec, int nrhs, const int block2[4], int nsweeps, int mr_iters, const void *b,
                    void *z);

/* Three-level preconditioner (Section 3 applied recursively): as
 * mgdd_precondition, with the coarse equation D_c x_c = P^H r solved by k2
 * steps of flexible GMRES from x_c = 0 (no restart), right-preconditioned by
 * the two-level method on D_c: M2(v) = nu2 level-2 Schwarz sweeps (mr2 MR
 * steps per block, the blocks of the last mgdd_setup_level2 or
 * mgdd_coarse_sap call) on D_c y = v from y0 = P2 GMRES_coarse_iters(D_cc,
 * P2^H v). Errors: MGDD_ENOTREADY (no third level; no level-2 blocks while
 * nu2 > 0), MGDD_EINVAL (k2 not in 1..64). Synchronous. */
int mgdd_precondition3(mgdd_ctx *ctx, int prec, int nrhs, int nu, int mr_iters, int k2, int nu2, int mr2,
                       int coarse_iters, const void *r, void *z);

typedef struct {
    int agg2[4];       /* level-2 aggregate in coarse sites (divides the coarse lattice) */
    int ntv2;          /* N2: test vectors of the second level, 1..32 */
    int block2[4];     /* level-2 Schwarz block in coarse sites (as mgdd_coarse_sap) */
    int nu2;           /* smoothing rounds of the test vectors */
    int mr_iters;      /* MR steps per level-2 block solve */
} mgdd_level2_params;

/* Setup of the third level (the recursive part of the bootstrap setup,
 * Section 3): the test vectors of the second level are the fine test vectors
 * P was built from, taken to the coarse grid with P^H (the first min(N,
 * ntv2)), then ntv2 - N of the caller's random coarse vectors when ntv2 > N,
 * orthonormalised in index order; nu2 rounds of one level-2 Schwarz sweep on
 * D_c y = 0 started from each vector, each round followed by the
 * orthonormalisation; then P2 and D_cc as in mgdd_build_P2. FP64 throughout.
 * random2: ntv2 - N FP64 coarse fields in device memory (may be NULL when
 * ntv2 <= N). Errors: those of mgdd_build_P2 and mgdd_coarse_sap,
 * MGDD_EINVAL (random2 missing). Synchronous. */
int mgdd_setup_level2(mgdd_ctx *ctx, const mgdd_level2_params *params, const void *random2);

/* ------------------------------------------------------------------ learned setup
 * Not from the paper: a gauge-covariant network that maps random vectors to
 * test vectors, in place of most iterations of the bootstrap setup (whose
 * test-vector iterations are described in Section 3). Layer l maps
 * widths[l] spinor channels to widths[l+1]:
 *   y[c] = sum_{c', h} W_l[c][c'][h] T_h x[c'],   h = 0..8,
 * with complex scalar weights, T_0 = 1, T_{1+2mu} x(s) = U_mu(s) x(s + mu),
 * T_{2+2mu} x(s) = U_mu(s - mu)^H x(s - mu) (colour hops of the Wilson
 * stencil, antiperiodic in time, every spin alike), so the network commutes
 * with gauge transformations. widths[0] = widths[nlayers] = 1; widths in
 * {1, 2, 4, 8, 16}, neighbouring widths equal, 2x apart, or one of them 1.
 * Weights: device array of complex FP64, layer by layer, [c][c'][h] within
 * a layer (mgdd_net_weight_count entries). Samples: nsamples fine fields of
 * one channel each, MGDD_F32, device layout. */
typedef struct {
    int nlayers;      /* 1..8 */
    int widths[9];
} mgdd_net_shape;

/* number of complex weights (0 for an invalid shape) */
size_t mgdd_net_weight_count(const mgdd_net_shape *shape);

/* out = net(in) for nsamples fields (in and out must not alias).
 * Synchronous. Errors: MGDD_EINVAL (shape), MGDD_ENOTREADY (no gauge field). */
int mgdd_net_apply(mgdd_ctx *ctx, const mgdd_net_shape *shape, const void *weights, int nsamples, const void *in,
                   void *out);

/* Training loss and gradient against the context's current interpolation P
 * (built from bootstrap test vectors of the same gauge field): loss = mean
 * over the samples of ||(1 - P P^H) f||^2 / ||f||^2, f = net(in_s), the
 * part of the output outside the bootstrap's coarse space; grad (device,
 * complex FP64, weight layout, written) = dloss / dconj(W), by
 * back-propagation through the layers (FP32 activations, FP64 weight
 * gradients). Synchronous. Errors: MGDD_ENOTREADY (no P), MGDD_ENAN (zero or
 * non-finite output). */
int mgdd_net_grad(mgdd_ctx *ctx, const mgdd_net_shape *shape, const void *weights, int nsamples, const void *in,
                  double *loss, void *grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected for step
 * >= 1) on the real and imaginary parts of every weight; m and v: device
 * state of the weights' layout, zero before step 1. Asynchronous. */
int mgdd_net_adam(mgdd_ctx *ctx, const mgdd_net_shape *shape, void *weights, const void *grad, void *m, void *v,
                  int step, double lr);

/* Setup with the network: the random vectors (params->ntv FP64 fine
 * fields, or NULL: drawn by the library from stream params->seed as for
 * mgdd_setup_bootstrap) are mapped by the network, a few at a time in the
 * context's test-vector storage, then the bootstrap setup continues
 * from the outputs as from its random vectors (params->nu part-1 rounds,
 * params->n_part2 second parts; with both 0 only P and D_c are built).
 * The plain bootstrap setup is the fallback: when the network's vectors
 * cannot serve (P rank deficient on an aggregate, or NaN / Inf on the way),
 * the bootstrap runs from the caller's random vectors with the same
 * parameters and the call returns its status (mgdd_setup_fallback then
 * returns 1). arnoldi_start may be NULL when n_part2 = 0. Synchronous. */
int mgdd_setup_learned(mgdd_ctx *ctx, const mgdd_net_shape *shape, const void *weights,
                       const mgdd_setup_params *params, const void *random_vectors, const void *arnoldi_start);

/* 1 if the last mgdd_setup_learned on this context fell back to the plain
 * bootstrap setup, else 0 (also for a NULL context). */
int mgdd_setup_fallback(const mgdd_ctx *ctx);

/* Frees the context's solver / setup workspace and staging buffer (they grow
 * on demand and are otherwise kept until mgdd_destroy), for programs that
 * hold many contexts; the next call that needs them allocates them again.
 * Synchronises the context's stream. */
int mgdd_release_workspace(mgdd_ctx *ctx);

/* ------------------------------------------------------------------ kernel timing
 * Instrumentation, not part of the method. While timing is enabled the
 * library brackets every launch of the Wilson-clover kernel
 * (MGDD_KERNEL_DIRAC, used by mgdd_dirac_apply and inside the solvers), of
 * the Schwarz colour kernel (MGDD_KERNEL_SAP, one launch per colour step of
 * Alg. 2.1) and of the coarse operator step of the coarse GMRES
 * (MGDD_KERNEL_COARSE: y = D_c v_j with the dot products of the Arnoldi
 * step, one launch per GMRES step of Section 4) with a pair of HIP events on
 * the context's stream, and adds up the durations per kernel family and
 * precision. Enabling creates a fixed
 * pool of events (owned by the context, released by mgdd_destroy);
 * disabling keeps the totals. The pool is drained with a stream
 * synchronisation when it is full or when the totals are read. */
enum { MGDD_KERNEL_DIRAC = 0, MGDD_KERNEL_SAP = 1, MGDD_KERNEL_COARSE = 2 };

/* on: nonzero to enable, 0 to disable. Errors: MGDD_EHIP (event creation). */
int mgdd_timing_enable(mgdd_ctx *ctx, int on);

/* Totals for one kernel family (MGDD_KERNEL_*) and precision (MGDD_F64,
 * MGDD_F32 or MGDD_F16), after a synchronisation of the context's stream.
 * Outputs (each may be NULL): total_ms = sum of launch durations in
 * milliseconds; site_updates = sum over launches of sites times right-hand
 * sides processed (the sites of one colour for a Schwarz launch, coarse sites
 * for a coarse step); launches = number of launches; alg_bytes = sum over
 * launches of the algorithmic HBM bytes of each launch: links and clover term
 * read once per launch (links as two rows, 4 x 6 complex, when every link is
 * special unitary, else 4 x 9; the clover term 72 reals), the spinors of every
 * right-hand side read and written once. Per site: an FP64 apply of n fields
 * 960 + 384 n (1152 + 384 n with full links), of n FP32 fields 960 + 288 n,
 * of n half fields 960 + 240 n; FP32 480 + 192 n (576 + 192 n), half
 * 480 + 96 n; per site of a Schwarz colour step 480 + 288 n (FP32, two lanes
 * per site), 576 + 288 n (FP32, 1 or 4 lanes), 480 + 144 n (half), 1152 + 576 n
 * (FP64); per coarse site of a coarse step with N test vectors and j earlier
 * basis vectors 5 (2N)^2 blocks (the compact FP32 D_c, else 9) plus
 * (3 + j) 2N values per right-hand side. reset: nonzero to zero these totals
 * afterwards. Errors: MGDD_EINVAL (bad kernel or precision). */
int mgdd_timing_read(mgdd_ctx *ctx, int kernel, int prec, int reset, double *total_ms, double *site_updates,
                     long long *launches, double *alg_bytes);

#ifdef __cplusplus
}
#endif
#endif
