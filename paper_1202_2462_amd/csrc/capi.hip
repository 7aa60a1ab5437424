// C ABI entry points: argument checks, context and workspace management, and
// dispatch to the kernel launchers. No C++ exception leaves this file.
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <cstdint>
#include <fstream>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "learn.h"
#include "level2.h"
#include "mgdd_internal.h"
#include "solver.h"
#include "transfer.h"

// Workspace of mgdd_coarse_solve_noalloc: a fixed device array, one copy on
// every GPU the library runs on, held until the process ends. Host code never
// passes `scratch` itself to a kernel (in host code the name is a stand-in,
// not a device address); it uses the address hipGetSymbolAddress returns for
// the current device, recorded per device when a context is created.
static constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static constexpr int NOALLOC_MAX_DEVICES = 64;
static void *scratch_dev[NOALLOC_MAX_DEVICES];
static std::mutex scratch_mu;

__global__ void zero_int_kernel(int *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

namespace mgdd {

int fail(Ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

int hip_check(Ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return MGDD_OK;
    return fail(c, MGDD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Device allocations go through the caller's allocator when one is set
// (mgdd_set_allocator), else hipMalloc; each remembers how it is released.
void *dalloc(Ctx *c, size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (c->ualloc) {
        p = c->ualloc(bytes, c->uuser);
        if (!p) {
            fail(c, MGDD_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed (caller's allocator)");
            return nullptr;
        }
        c->owned.push_back(Owned{p, c->ufree, c->uuser});
        return p;
    }
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(c, MGDD_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed (hipMalloc)");
        return nullptr;
    }
    c->owned.push_back(Owned{p, nullptr, nullptr});
    return p;
}

void release_owned(const Owned &o) {
    if (o.free_fn) o.free_fn(o.p, o.user);
    else (void)hipFree(o.p);
}

void dfree(Ctx *c, void *p) {
    if (!p) return;
    for (size_t i = 0; i < c->owned.size(); i++)
        if (c->owned[i].p == p) {
            const Owned o = c->owned[i];
            c->owned[i] = c->owned.back();
            c->owned.pop_back();
            release_owned(o);
            return;
        }
}

void *ensure_stage(Ctx *c, size_t bytes) {
    if (c->stage_bytes >= bytes) return c->stage;
    if (c->stage) {
        (void)hipStreamSynchronize(c->stream);
        dfree(c, c->stage);
    }
    c->stage = dalloc(c, bytes);
    c->stage_bytes = c->stage ? bytes : 0;
    return c->stage;
}

void *ensure_scratch(Ctx *c, size_t bytes) {
    if (c->scratch_bytes >= bytes) return c->scratch;
    if (c->scratch) {
        (void)hipStreamSynchronize(c->stream);
        dfree(c, c->scratch);
    }
    c->scratch = dalloc(c, bytes);
    c->scratch_bytes = c->scratch ? bytes : 0;
    return c->scratch;
}

double *ensure_red(Ctx *c, size_t n) {
    if (c->red_doubles >= n) return c->red;
    if (c->red) {
        (void)hipStreamSynchronize(c->stream);
        dfree(c, c->red);
        (void)hipHostFree(c->red_host);
        c->red_host = nullptr;
    }
    c->red = (double *)dalloc(c, n * sizeof(double));
    if (!c->red) return nullptr;
    if (hipHostMalloc((void **)&c->red_host, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        fail(c, MGDD_ENOMEM, "hipHostMalloc failed");
        return nullptr;
    }
    c->red_doubles = n;
    return c->red;
}

// ------------------------------------------------------------------ kernel timing

constexpr int KT_SLOTS = 2048;

int kt_flush(Ctx *c) {
    KTimer &k = c->kt;
    if (k.used == 0) return MGDD_OK;
    int rc = hip_check(c, hipEventSynchronize(k.ev[2 * (k.used - 1) + 1]), "timing");
    for (int i = 0; i < k.used && !rc; i++) {
        float ms = 0;
        rc = hip_check(c, hipEventElapsedTime(&ms, k.ev[2 * i], k.ev[2 * i + 1]), "timing");
        const int f = k.fam[i] / 3, p = k.fam[i] % 3;
        k.ms[f][p] += ms;
        k.usum[f][p] += k.units[i];
        k.bsum[f][p] += k.bytes[i];
        k.launches[f][p]++;
    }
    k.used = 0;
    return rc;
}

int kt_begin(Ctx *c) {
    KTimer &k = c->kt;
    if (!k.on) return -1;
    if (k.used == KT_SLOTS && kt_flush(c)) return -1;
    const int s = k.used++;
    if (hipEventRecord(k.ev[2 * s], c->stream) != hipSuccess) {
        (void)hipGetLastError();
        k.used--;
        return -1;
    }
    return s;
}

void kt_end(Ctx *c, int slot, int family, int prec, double units, double bytes) {
    if (slot < 0) return;
    KTimer &k = c->kt;
    (void)hipEventRecord(k.ev[2 * slot + 1], c->stream);
    k.fam[slot] = family * 3 + prec;
    k.units[slot] = units;
    k.bytes[slot] = bytes;
}

static void kt_release(Ctx *c) {
    for (hipEvent_t e : c->kt.ev) (void)hipEventDestroy(e);
    c->kt.ev.clear();
    c->kt.on = false;
    c->kt.used = 0;
}

static int setup_geometry(Ctx *c, const int *dims, const int *block) {
    std::vector<uint32_t> coord;
    std::vector<int> nbr, lexpos;
    std::string e = geometry_tables(dims, block, c->g, coord, nbr, &lexpos);
    if (!e.empty()) return fail(c, MGDD_ESHAPE, e);
    c->d_blk_coord = (uint32_t *)dalloc(c, coord.size() * sizeof(uint32_t));
    c->d_blk_nbr = (int *)dalloc(c, nbr.size() * sizeof(int));
    int *d_lexpos = (int *)dalloc(c, lexpos.size() * sizeof(int));
    if (!c->d_blk_coord || !c->d_blk_nbr || !d_lexpos) return MGDD_ENOMEM;
    int rc0 = hip_check(c, hipMemcpy(d_lexpos, lexpos.data(), lexpos.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
    if (rc0) return rc0;
    c->g.pos_of_lex = d_lexpos;
    int rc = hip_check(c, hipMemcpy(c->d_blk_coord, coord.data(), coord.size() * sizeof(uint32_t), hipMemcpyHostToDevice), "copy");
    if (rc) return rc;
    rc = hip_check(c, hipMemcpy(c->d_blk_nbr, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
    if (rc) return rc;
    c->g.blk_coord = c->d_blk_coord;
    c->g.blk_nbr = c->d_blk_nbr;
    return MGDD_OK;
}

static bool valid_prec(int p) { return p == MGDD_F64 || p == MGDD_F32; }
// fine fields for storage, layout conversion and the Wilson-clover apply may also be FP16
static bool valid_fine_prec(int p) { return valid_prec(p) || p == MGDD_F16; }

// true when the last error was a failed device allocation (then a smaller
// batch may fit); clears the HIP error state
static bool alloc_failed(Ctx *c) {
    (void)hipGetLastError();
    return c->err.rfind("device allocation", 0) == 0;
}

}  // namespace mgdd

using namespace mgdd;

struct mgdd_ctx {
    Ctx c;
};

#define GUARD_BEGIN try {
#define GUARD_END                                                         \
    }                                                                     \
    catch (const std::bad_alloc &) {                                      \
        return fail(ctx ? &ctx->c : nullptr, MGDD_ENOMEM, "host allocation failed"); \
    }                                                                     \
    catch (...) {                                                         \
        return fail(ctx ? &ctx->c : nullptr, MGDD_EINVAL, "internal error"); \
    }

extern "C" {

int mgdd_create(const int dims[4], const int block[4], int t_antiperiodic, void *hip_stream, mgdd_ctx **out) {
    if (!dims || !block || !out || (t_antiperiodic != 0 && t_antiperiodic != 1)) return MGDD_EINVAL;
    *out = nullptr;
    mgdd_ctx *ctx = nullptr;
    GUARD_BEGIN
    ctx = new mgdd_ctx();
    ctx->c.stream = (hipStream_t)hip_stream;
    ctx->c.t_antiperiodic = t_antiperiodic == 1;
    (void)hipGetDevice(&ctx->c.dev);
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->c.dev) == hipSuccess && v > 0)
            ctx->c.lds_max = (size_t)v;
    }
    int rc = MGDD_OK;
    {
        // device address of the allocation-free workspace on this device
        std::lock_guard<std::mutex> lock(scratch_mu);
        const int dv = ctx->c.dev;
        if (dv < 0 || dv >= NOALLOC_MAX_DEVICES) {
            rc = fail(&ctx->c, MGDD_EINVAL, "device index beyond the supported range");
        } else if (!scratch_dev[dv]) {
            void *p = nullptr;
            rc = hip_check(&ctx->c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the scratch array");
            if (!rc && !p) rc = fail(&ctx->c, MGDD_EHIP, "address of the scratch array is null");
            if (!rc) scratch_dev[dv] = p;
        }
    }
    if (!rc) rc = setup_geometry(&ctx->c, dims, block);
    if (rc) {
        // keep the context so that the caller can read the error, then free it
        std::string msg = ctx->c.err;
        for (const Owned &o : ctx->c.owned) release_owned(o);
        delete ctx;
        fprintf(stderr, "mgdd_create: %s\n", msg.c_str());
        return rc;
    }
    *out = ctx;
    return MGDD_OK;
    GUARD_END
}

int mgdd_set_allocator(mgdd_ctx *ctx, mgdd_alloc_fn alloc, mgdd_free_fn free_fn, void *user) {
    if (!ctx || (alloc == nullptr) != (free_fn == nullptr)) return MGDD_EINVAL;
    ctx->c.ualloc = alloc;
    ctx->c.ufree = free_fn;
    ctx->c.uuser = alloc ? user : nullptr;
    return MGDD_OK;
}

int mgdd_set_kernel_options(mgdd_ctx *ctx, const mgdd_kernel_options *o) {
    if (!ctx || !o) return MGDD_EINVAL;
    const int l = o->sap_lanes, s = o->dirac_stage;
    if ((l != 0 && l != 1 && l != 2 && l != 4) || s < -1 || s > 1)
        return fail(&ctx->c, MGDD_EINVAL, "kernel options: sap_lanes in {0, 1, 2, 4}, dirac_stage in {-1, 0, 1}");
    ctx->c.sap_lanes = l;
    ctx->c.dirac_stage = s;
    return MGDD_OK;
}

int mgdd_destroy(mgdd_ctx *ctx) {
    if (!ctx) return MGDD_OK;
    (void)hipStreamSynchronize(ctx->c.stream);
    kt_release(&ctx->c);
    for (const Owned &o : ctx->c.owned) release_owned(o);
    if (ctx->c.red_host) (void)hipHostFree(ctx->c.red_host);
    if (ctx->c.hbuf) (void)hipHostFree(ctx->c.hbuf);
    delete ctx;
    return MGDD_OK;
}

int mgdd_release_workspace(mgdd_ctx *ctx) {
    if (!ctx) return MGDD_EINVAL;
    Ctx *c = &ctx->c;
    (void)hipStreamSynchronize(c->stream);
    for (void **p : {&c->ws, &c->stage}) {
        if (*p) dfree(c, *p);
        *p = nullptr;
    }
    c->ws_bytes = 0;
    c->stage_bytes = 0;
    return MGDD_OK;
}

const char *mgdd_last_error(const mgdd_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

size_t mgdd_field_bytes(const mgdd_ctx *ctx, int prec, int nrhs, int level) {
    if (!ctx || !valid_fine_prec(prec) || nrhs < 0) return 0;
    if (level == 0) return csize(prec) * fine_elems(&ctx->c, nrhs);
    if (!valid_prec(prec)) return 0;
    if (level == 1 && ctx->c.c.ready) return csize(prec) * (size_t)nrhs * ctx->c.c.Vc * 2 * ctx->c.c.N;
    if (level == 2 && ctx->c.c2.ready) return csize(prec) * (size_t)nrhs * ctx->c.c2.Vcc * 2 * ctx->c.c2.N2;
    return 0;
}

int mgdd_set_gauge(mgdd_ctx *ctx, const double *U, int src_on_device, double m0, double csw) {
    if (!ctx || !U) return MGDD_EINVAL;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    const size_t V = c->g.V;
    if (!std::isfinite(m0) || !std::isfinite(csw)) return fail(c, MGDD_ENAN, "m0 or csw not finite");
    if (!c->U64) {
        c->U64 = dalloc(c, V * 36 * 16);
        c->U32 = dalloc(c, V * 36 * 8);
        c->A64 = dalloc(c, V * 72 * 8);
        c->A32 = dalloc(c, V * 72 * 4);
        c->Ainv64 = dalloc(c, V * 72 * 8);
        if (!c->U64 || !c->U32 || !c->A64 || !c->A32 || !c->Ainv64) return MGDD_ENOMEM;
    }
    c->m0 = m0;
    c->csw = csw;
    c->c.ready = false;
    c->gauge_ready = false;
    const double2 *src = (const double2 *)U;
    int rc = MGDD_OK;
    if (!src_on_device) {
        void *st = ensure_stage(c, V * 36 * 16);
        if (!st) return MGDD_ENOMEM;
        rc = hip_check(c, hipMemcpyAsync(st, U, V * 36 * 16, hipMemcpyHostToDevice, c->stream), "copy gauge");
        if (rc) return rc;
        src = (const double2 *)st;
    }
    rc = launch_gauge_ingest(c, src);
    if (rc) return rc;
    c->gauge_ready = true;
    return MGDD_OK;
    GUARD_END
}

int mgdd_pack(mgdd_ctx *ctx, int prec, int nrhs, const double *src, int src_on_device, void *dst) {
    if (!ctx || !src || !dst || !valid_fine_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    size_t bytes = (size_t)nrhs * 12 * c->g.V * 16;
    const double2 *canon = (const double2 *)src;
    if (!src_on_device) {
        void *st = ensure_stage(c, bytes);
        if (!st) return MGDD_ENOMEM;
        int rc = hip_check(c, hipMemcpyAsync(st, src, bytes, hipMemcpyHostToDevice, c->stream), "copy field");
        if (rc) return rc;
        canon = (const double2 *)st;
    }
    int rc = launch_pack(c, prec, nrhs, canon, dst);
    if (rc) return rc;
    if (!src_on_device) return hip_check(c, hipStreamSynchronize(c->stream), "sync");
    return MGDD_OK;
    GUARD_END
}

int mgdd_unpack(mgdd_ctx *ctx, int prec, int nrhs, const void *src, double *dst, int dst_on_device) {
    if (!ctx || !src || !dst || !valid_fine_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    size_t bytes = (size_t)nrhs * 12 * c->g.V * 16;
    double2 *canon = (double2 *)dst;
    if (!dst_on_device) {
        canon = (double2 *)ensure_stage(c, bytes);
        if (!canon) return MGDD_ENOMEM;
    }
    int rc = launch_unpack(c, prec, nrhs, src, canon);
    if (rc) return rc;
    if (!dst_on_device) {
        rc = hip_check(c, hipMemcpyAsync(dst, canon, bytes, hipMemcpyDeviceToHost, c->stream), "copy field");
        if (rc) return rc;
        return hip_check(c, hipStreamSynchronize(c->stream), "sync");
    }
    return MGDD_OK;
    GUARD_END
}

int mgdd_dirac_apply(mgdd_ctx *ctx, int prec, int nrhs, const void *in, void *out) {
    if (!ctx || !in || !out || !valid_fine_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    if (in == out) return fail(&ctx->c, MGDD_EINVAL, "in and out alias");
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    GUARD_BEGIN
    return launch_dirac(&ctx->c, prec, nrhs, in, out);
    GUARD_END
}

// the Schwarz blocks of a call: NULL or the blocks the device site order was built from
static int check_block(Ctx *c, const int *block) {
    if (!block) return MGDD_OK;
    for (int mu = 0; mu < 4; mu++)
        if (block[mu] != (1 << c->g.lb[mu]))
            return fail(c, MGDD_ESHAPE,
                        "the Schwarz blocks are the blocks of mgdd_create (the device site order is built from "
                        "them); create a context with this block shape");
    return MGDD_OK;
}

int mgdd_sap(mgdd_ctx *ctx, int prec, int nrhs, const int block[4], int nsweeps, int mr_iters, double shift_re,
             double shift_im, const void *b, void *z) {
    if (!ctx || !b || !z || !valid_fine_prec(prec) || nrhs <= 0 || nsweeps < 0 || mr_iters < 0) return MGDD_EINVAL;
    if (b == z) return fail(&ctx->c, MGDD_EINVAL, "b and z alias");
    if (check_block(&ctx->c, block)) return MGDD_ESHAPE;
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    GUARD_BEGIN
    return launch_sap(&ctx->c, prec, nrhs, nsweeps, mr_iters, shift_re, shift_im, b, z);
    GUARD_END
}

int mgdd_schwarz(mgdd_ctx *ctx, int prec, int nrhs, const int block[4], const mgdd_schwarz_params *params,
                 const void *b, void *z) {
    if (!ctx || !params || !b || !z || !valid_fine_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    const mgdd_schwarz_params *q = params;
    if (prec == MGDD_F16 && (q->additive || q->block_solver != MGDD_BLOCK_MR))
        return fail(&ctx->c, MGDD_EINVAL, "half-precision storage: red-black Schwarz with MR block solves only");
    if (b == z) return fail(&ctx->c, MGDD_EINVAL, "b and z alias");
    if (check_block(&ctx->c, block)) return MGDD_ESHAPE;
    if (q->nsweeps < 0 || q->block_iters < 0 || (q->block_solver != MGDD_BLOCK_MR && q->block_solver != MGDD_BLOCK_GMRES))
        return fail(&ctx->c, MGDD_EINVAL, "bad Schwarz parameters");
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    SchwarzOpts o;
    o.nsweeps = q->nsweeps;
    o.k = q->block_iters;
    o.gmres = q->block_solver == MGDD_BLOCK_GMRES;
    o.additive = q->additive != 0;
    Arena A;
    void *work = nullptr;
    const size_t wb = schwarz_work_bytes(c, prec, nrhs, o);
    int rc = MGDD_OK;
    if (wb) {
        rc = arena_open(c, wb, A);
        if (!rc && !(work = A.take(wb))) rc = fail(c, MGDD_ENOMEM, "Schwarz workspace");
    }
    if (!rc) rc = launch_schwarz(c, prec, nrhs, o, q->shift_re, q->shift_im, b, z, work);
    return rc;
    GUARD_END
}

static int need_coarse(mgdd_ctx *ctx) {
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    if (!ctx->c.c.ready) return fail(&ctx->c, MGDD_ENOTREADY, "no interpolation P (call mgdd_build_P or mgdd_setup_bootstrap)");
    return MGDD_OK;
}

int mgdd_build_P(mgdd_ctx *ctx, const int agg[4], int ntv, const void *test_vectors) {
    if (!ctx || !agg || !test_vectors) return MGDD_EINVAL;
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    c->c.ready = false;
    c->c2.ready = false;
    int rc = transfer_setup(c, agg, ntv);
    if (!rc) rc = launch_build_P(c, test_vectors);
    if (!rc) rc = launch_coarse_build(c);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (!rc) c->c.ready = true;
    return rc;
    GUARD_END
}

int mgdd_get_test_vectors(mgdd_ctx *ctx, void *dst) {
    if (!ctx || !dst) return MGDD_EINVAL;
    int rc = need_coarse(ctx);
    if (rc) return rc;
    Ctx *c = &ctx->c;
    return hip_check(c, hipMemcpyAsync(dst, c->c.tv64, (size_t)c->c.N * 12 * c->g.V * 16, hipMemcpyDeviceToDevice,
                                       c->stream), "copy");
}

// ---------------------------------------------------------------- setup checkpoint

namespace {
struct SetupFileHeader {
    char magic[8];        // "MGDDSET1"
    int32_t dims[4];
    int32_t agg[4];
    int32_t ntv;
    int32_t reserved;
    double m0, csw;
    uint64_t payload_bytes;
    uint64_t checksum;    // FNV-1a (64 bit) of the payload
};

uint64_t fnv1a(const unsigned char *p, size_t n, uint64_t h = 1469598103934665603ull) {
    for (size_t i = 0; i < n; i++) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}
}  // namespace

int mgdd_save_setup(mgdd_ctx *ctx, const char *path) {
    if (!ctx || !path) return MGDD_EINVAL;
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    const int N = c->c.N;
    const size_t bytes = (size_t)N * 12 * c->g.V * 16;
    double2 *canon = (double2 *)ensure_stage(c, bytes);
    if (!canon) return MGDD_ENOMEM;
    rc = launch_unpack(c, MGDD_F64, N, c->c.tv64, canon);
    std::vector<unsigned char> host(bytes);
    if (!rc) rc = hip_check(c, hipMemcpyAsync(host.data(), canon, bytes, hipMemcpyDeviceToHost, c->stream), "copy");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (rc) return rc;
    SetupFileHeader h{};
    std::memcpy(h.magic, "MGDDSET1", 8);
    for (int m = 0; m < 4; m++) {
        h.dims[m] = c->g.L[m];
        h.agg[m] = c->c.agg[m];
    }
    h.ntv = N;
    h.m0 = c->m0;
    h.csw = c->csw;
    h.payload_bytes = bytes;
    h.checksum = fnv1a(host.data(), bytes);
    std::ofstream f(path, std::ios::binary | std::ios::trunc);
    if (!f) return fail(c, MGDD_EINVAL, "cannot open the setup file for writing");
    f.write((const char *)&h, sizeof h);
    f.write((const char *)host.data(), (std::streamsize)bytes);
    if (!f) return fail(c, MGDD_EINVAL, "writing the setup file failed");
    return MGDD_OK;
    GUARD_END
}

int mgdd_load_setup(mgdd_ctx *ctx, const char *path) {
    if (!ctx || !path) return MGDD_EINVAL;
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(c, MGDD_EINVAL, "cannot open the setup file");
    SetupFileHeader h{};
    f.read((char *)&h, sizeof h);
    if (!f || std::memcmp(h.magic, "MGDDSET1", 8) != 0) return fail(c, MGDD_EINVAL, "not a setup file");
    for (int m = 0; m < 4; m++)
        if (h.dims[m] != c->g.L[m]) return fail(c, MGDD_ESHAPE, "the setup file is for another lattice");
    const size_t bytes = (size_t)h.ntv * 12 * c->g.V * 16;
    if (h.ntv < 1 || h.ntv > 32 || h.payload_bytes != bytes) return fail(c, MGDD_EINVAL, "corrupt setup file (sizes)");
    std::vector<unsigned char> host(bytes);
    f.read((char *)host.data(), (std::streamsize)bytes);
    if (!f) return fail(c, MGDD_EINVAL, "the setup file is truncated");
    if (fnv1a(host.data(), bytes) != h.checksum) return fail(c, MGDD_EINVAL, "corrupt setup file (checksum)");
    void *st = ensure_stage(c, bytes);
    if (!st) return MGDD_ENOMEM;
    c->c.ready = false;
    c->c2.ready = false;
    int rc = transfer_setup(c, h.agg, h.ntv);
    if (!rc) rc = hip_check(c, hipMemcpyAsync(st, host.data(), bytes, hipMemcpyHostToDevice, c->stream), "copy");
    if (!rc) rc = launch_pack(c, MGDD_F64, h.ntv, (const double2 *)st, c->c.tv64);
    if (!rc) rc = launch_build_P(c, c->c.tv64);
    if (!rc) rc = launch_coarse_build(c);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (!rc) c->c.ready = true;
    return rc;
    GUARD_END
}

int mgdd_restrict(mgdd_ctx *ctx, int prec, int nrhs, const void *fine, void *coarse) {
    if (!ctx || !fine || !coarse || !valid_fine_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    return launch_restrict(&ctx->c, prec, nrhs, fine, coarse);
    GUARD_END
}

int mgdd_prolong(mgdd_ctx *ctx, int prec, int nrhs, const void *coarse, void *fine) {
    if (!ctx || !fine || !coarse || !valid_fine_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    return launch_prolong(&ctx->c, prec, nrhs, coarse, fine);
    GUARD_END
}

int mgdd_coarse_apply(mgdd_ctx *ctx, int prec, int nrhs, const void *in, void *out) {
    if (!ctx || !in || !out || !valid_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    if (in == out) return fail(&ctx->c, MGDD_EINVAL, "in and out alias");
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    return launch_coarse_apply(&ctx->c, prec, nrhs, in, out);
    GUARD_END
}

static int need_level2(mgdd_ctx *ctx) {
    int rc = need_coarse(ctx);
    if (rc) return rc;
    if (!ctx->c.c2.ready) return fail(&ctx->c, MGDD_ENOTREADY, "no third level (call mgdd_build_P2 or mgdd_setup_level2)");
    return MGDD_OK;
}

int mgdd_build_P2(mgdd_ctx *ctx, const int agg2[4], int ntv2, const void *test_vectors2) {
    if (!ctx || !agg2 || !test_vectors2) return MGDD_EINVAL;
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    c->c2.ready = false;
    rc = level2_setup(c, agg2, ntv2);
    if (!rc) rc = launch_build_P2(c, test_vectors2);
    if (!rc) rc = launch_dcc_build(c);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (rc) c->c2.ready = false;
    return rc;
    GUARD_END
}

int mgdd_restrict2(mgdd_ctx *ctx, int prec, int nrhs, const void *coarse, void *coarse2) {
    if (!ctx || !coarse || !coarse2 || !valid_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    int rc = need_level2(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    return launch_restrict2(&ctx->c, prec, nrhs, coarse, coarse2);
    GUARD_END
}

int mgdd_prolong2(mgdd_ctx *ctx, int prec, int nrhs, const void *coarse2, void *coarse) {
    if (!ctx || !coarse || !coarse2 || !valid_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    int rc = need_level2(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    return launch_prolong2(&ctx->c, prec, nrhs, coarse2, coarse);
    GUARD_END
}

int mgdd_coarse2_apply(mgdd_ctx *ctx, int prec, int nrhs, const void *in, void *out) {
    if (!ctx || !in || !out || !valid_prec(prec) || nrhs <= 0) return MGDD_EINVAL;
    if (in == out) return fail(&ctx->c, MGDD_EINVAL, "in and out alias");
    int rc = need_level2(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    return launch_stencil_apply(&ctx->c, level2_op(&ctx->c), prec, nrhs, in, out);
    GUARD_END
}

static int need_level3_solver(mgdd_ctx *ctx, int k2, int nu2, int mr2) {
    if (k2 < 1 || k2 > 64 || nu2 < 0 || mr2 < 0) return fail(&ctx->c, MGDD_EINVAL, "bad level-2 solver parameters");
    int rc = need_level2(ctx);
    if (rc) return rc;
    if (nu2 > 0 && !ctx->c.c2.blk_sites)
        return fail(&ctx->c, MGDD_ENOTREADY, "no level-2 Schwarz blocks (call mgdd_setup_level2 or mgdd_coarse_sap)");
    return MGDD_OK;
}

int mgdd_precondition3(mgdd_ctx *ctx, int prec, int nrhs, int nu, int mr_iters, int k2, int nu2, int mr2,
                       int coarse_iters, const void *r, void *z) {
    if (!ctx || !r || !z || !valid_prec(prec) || nrhs <= 0 || nu < 0 || mr_iters < 0 || coarse_iters < 1)
        return MGDD_EINVAL;
    int rc = need_level3_solver(ctx, k2, nu2, mr2);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    MgOpts o;
    o.nu = nu;
    o.mr = mr_iters;
    o.cit = coarse_iters;
    o.levels = 3;
    o.k2 = k2;
    o.nu2 = nu2;
    o.mr2 = mr2;
    Arena A;
    rc = arena_open(c, precond_bytes(c, prec, o, nrhs), A);
    if (!rc) rc = mg_precond(c, prec, nrhs, r, z, o, A);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (!rc && A.need) rc = fail(c, MGDD_ENOMEM, "preconditioner workspace estimate too small");
    return rc;
    GUARD_END
}

int mgdd_setup_level2(mgdd_ctx *ctx, const mgdd_level2_params *params, const void *random2) {
    if (!ctx || !params || params->nu2 < 0 || params->mr_iters < 0) return MGDD_EINVAL;
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    rc = level2_bootstrap(&ctx->c, params, random2);
    if (rc) ctx->c.c2.ready = false;
    return rc;
    GUARD_END
}

int mgdd_coarse_sap(mgdd_ctx *ctx, int prec, int nrhs, const int block2[4], int nsweeps, int mr_iters, const void *b,
                    void *z) {
    if (!ctx || !block2 || !b || !z || !valid_prec(prec) || nrhs <= 0 || nsweeps < 0 || mr_iters < 0)
        return MGDD_EINVAL;
    if (b == z) return fail(&ctx->c, MGDD_EINVAL, "b and z alias");
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    rc = level2_sap_setup(c, block2);
    if (!rc) rc = launch_sap2(c, prec, nrhs, nsweeps, mr_iters, b, z);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    return rc;
    GUARD_END
}

int mgdd_coarse_solve(mgdd_ctx *ctx, int prec, int nrhs, int iters, const void *b, void *x) {
    if (!ctx || !b || !x || !valid_prec(prec) || nrhs <= 0 || iters < 1 || iters > 1000) return MGDD_EINVAL;
    if (b == x) return fail(&ctx->c, MGDD_EINVAL, "b and x alias");
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    Arena A;
    rc = arena_open(c, coarse_gmres_bytes(c, prec, iters, nrhs) + 256, A);
    int *status = rc ? nullptr : (int *)A.take(sizeof(int));
    if (!rc && !status) rc = fail(c, MGDD_ENOMEM, "coarse solve workspace");
    if (!rc) rc = hip_check(c, hipMemsetAsync(status, 0, sizeof(int), c->stream), "memset");
    if (!rc) rc = coarse_gmres(c, prec, iters, nrhs, b, x, A, status);
    int hstatus = 0;
    if (!rc) rc = hip_check(c, hipMemcpyAsync(&hstatus, status, sizeof(int), hipMemcpyDeviceToHost, c->stream), "read");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (!rc && hstatus) rc = fail(c, MGDD_ENAN, "NaN in the coarse solve");
    return rc;
    GUARD_END
}

int mgdd_coarse_solve_noalloc(mgdd_ctx *ctx, int prec, int nrhs, int iters, const void *b, void *x) {
    if (!ctx || !b || !x || !valid_prec(prec) || nrhs <= 0 || iters < 1) return MGDD_EINVAL;
    if (b == x) return fail(&ctx->c, MGDD_EINVAL, "b and x alias");
    if (iters > ARNOLDI_FUSED_MAX_STEPS || iters > LSQ_MAX_STEPS)
        return fail(&ctx->c, MGDD_EINVAL,
                    "the allocation-free coarse solve takes at most " + std::to_string(ARNOLDI_FUSED_MAX_STEPS) +
                        " GMRES steps");
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    void *base = (c->dev >= 0 && c->dev < NOALLOC_MAX_DEVICES) ? scratch_dev[c->dev] : nullptr;
    if (!base) return fail(c, MGDD_ENOTREADY, "no scratch array on this device");
    const size_t need = coarse_gmres_bytes(c, prec, iters, nrhs) + 256;
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(c, MGDD_EINVAL,
                    "the allocation-free coarse solve needs " + std::to_string(need) + " bytes of scratch, more than its " +
                        std::to_string(NOALLOC_SCRATCH_BYTES) + " (fewer right-hand sides or steps per call)");
    Arena A;
    A.base = (char *)base;
    A.cap = NOALLOC_SCRATCH_BYTES;
    int *status = (int *)A.take(sizeof(int));
    // cleared by a kernel, not by a memset node
    zero_int_kernel<<<1, 64, 0, c->stream>>>(status);
    rc = hip_check(c, hipGetLastError(), "zero kernel");
    if (!rc) rc = coarse_gmres(c, prec, iters, nrhs, b, x, A, status);
    if (!rc && A.need) rc = fail(c, MGDD_EINVAL, "scratch estimate of the coarse solve too small");
    int hstatus = 0;
    if (!rc) rc = hip_check(c, hipMemcpyAsync(&hstatus, status, sizeof(int), hipMemcpyDeviceToHost, c->stream), "read");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (!rc && hstatus) rc = fail(c, MGDD_ENAN, "NaN in the coarse solve");
    return rc;
    GUARD_END
}

int mgdd_precondition(mgdd_ctx *ctx, int prec, int nrhs, int nu, int mr_iters, int coarse_iters, const void *r,
                      void *z) {
    if (!ctx || !r || !z || !valid_prec(prec) || nrhs <= 0 || nu < 0 || mr_iters < 0 || coarse_iters < 1)
        return MGDD_EINVAL;
    int rc = need_coarse(ctx);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    Arena A;
    MgOpts o;
    o.nu = nu;
    o.mr = mr_iters;
    o.cit = coarse_iters;
    rc = arena_open(c, precond_bytes(c, prec, o, nrhs), A);
    if (!rc) rc = mg_precond(c, prec, nrhs, r, z, o, A);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    return rc;
    GUARD_END
}

int mgdd_setup_bootstrap(mgdd_ctx *ctx, const mgdd_setup_params *params, const void *random_vectors,
                         const void *arnoldi_start) {
    if (!ctx || !params || !arnoldi_start) return MGDD_EINVAL;
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    const mgdd_setup_params *sp = params;
    if (!valid_prec(sp->prec) || sp->nu < 0 || sp->iota < 0 || sp->mr_iters < 0 || sp->n_part2 < 0 || sp->arnoldi_m < 0 ||
        sp->chunk < 0)
        return fail(&ctx->c, MGDD_EINVAL, "bad setup parameters");
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    c->c.ready = false;
    c->c2.ready = false;
    int rc = bootstrap(c, sp, random_vectors, arnoldi_start);
    if (!rc) c->c.ready = true;
    return rc;
    GUARD_END
}

// ---------------------------------------------------------------- learned setup

static int net_shape(mgdd_ctx *ctx, const mgdd_net_shape *s, NetShape &sh) {
    if (!s) return MGDD_EINVAL;
    if (s->nlayers < 1 || s->nlayers > NET_MAX_LAYERS) return fail(&ctx->c, MGDD_EINVAL, "network: 1 to 8 layers");
    sh.nlayers = s->nlayers;
    for (int l = 0; l <= s->nlayers; l++) sh.widths[l] = s->widths[l];
    return check_net_shape(&ctx->c, sh);
}

size_t mgdd_net_weight_count(const mgdd_net_shape *shape) {
    if (!shape || shape->nlayers < 1 || shape->nlayers > NET_MAX_LAYERS) return 0;
    NetShape sh;
    sh.nlayers = shape->nlayers;
    for (int l = 0; l <= shape->nlayers; l++) sh.widths[l] = shape->widths[l];
    return net_shape_valid(sh) ? sh.nweights() : 0;
}

int mgdd_net_apply(mgdd_ctx *ctx, const mgdd_net_shape *shape, const void *weights, int nsamples, const void *in,
                   void *out) {
    if (!ctx || !shape || !weights || !in || !out || nsamples <= 0) return MGDD_EINVAL;
    if (in == out) return fail(&ctx->c, MGDD_EINVAL, "in and out alias");
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    NetShape sh;
    int rc = net_shape(ctx, shape, sh);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    Arena A;
    rc = arena_open(c, net_forward_bytes(c, sh, nsamples), A);
    if (!rc) rc = net_forward(c, sh, (const double2 *)weights, nsamples, in, out, A);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    return rc;
    GUARD_END
}

int mgdd_net_grad(mgdd_ctx *ctx, const mgdd_net_shape *shape, const void *weights, int nsamples, const void *in,
                  double *loss, void *grad) {
    if (!ctx || !shape || !weights || !in || !loss || !grad || nsamples <= 0) return MGDD_EINVAL;
    int rc = need_coarse(ctx);
    if (rc) return rc;
    NetShape sh;
    rc = net_shape(ctx, shape, sh);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    Arena A;
    rc = arena_open(c, net_grad_bytes(c, sh, nsamples), A);
    if (!rc) rc = net_grad(c, sh, (const double2 *)weights, nsamples, in, loss, (double2 *)grad, A);
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    return rc;
    GUARD_END
}

int mgdd_net_adam(mgdd_ctx *ctx, const mgdd_net_shape *shape, void *weights, const void *grad, void *m, void *v,
                  int step, double lr) {
    if (!ctx || !shape || !weights || !grad || !m || !v || step < 1 || !(lr > 0)) return MGDD_EINVAL;
    NetShape sh;
    int rc = net_shape(ctx, shape, sh);
    if (rc) return rc;
    GUARD_BEGIN
    return launch_net_adam(&ctx->c, sh.nweights(), (double2 *)weights, (const double2 *)grad, (double2 *)m,
                           (double2 *)v, step, lr, 0.9, 0.999, 1e-8);
    GUARD_END
}

int mgdd_setup_learned(mgdd_ctx *ctx, const mgdd_net_shape *shape, const void *weights,
                       const mgdd_setup_params *params, const void *random_vectors, const void *arnoldi_start) {
    if (!ctx || !shape || !weights || !params) return MGDD_EINVAL;
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    const mgdd_setup_params *sp = params;
    if (!valid_prec(sp->prec) || sp->nu < 0 || sp->iota < 0 || sp->mr_iters < 0 || sp->n_part2 < 0 || sp->arnoldi_m < 0 ||
        sp->chunk < 0)
        return fail(&ctx->c, MGDD_EINVAL, "bad setup parameters");
    if (sp->n_part2 > 0 && !arnoldi_start) return fail(&ctx->c, MGDD_EINVAL, "the second setup part needs a start vector");
    NetShape sh;
    int rc = net_shape(ctx, shape, sh);
    if (rc) return rc;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    c->c.ready = false;
    c->c2.ready = false;
    rc = setup_learned(c, sh, (const double2 *)weights, sp, random_vectors, arnoldi_start);
    if (!rc) c->c.ready = true;
    return rc;
    GUARD_END
}

int mgdd_setup_fallback(const mgdd_ctx *ctx) { return ctx && ctx->c.learned_fallback ? 1 : 0; }

int mgdd_solve(mgdd_ctx *ctx, const mgdd_solve_params *params, int nrhs, const void *b, void *z,
               mgdd_solve_stats *stats) {
    if (!ctx || !params || !b || !z || nrhs <= 0) return MGDD_EINVAL;
    const mgdd_solve_params *sp = params;
    if (sp->restart < 1 || sp->restart > 256 || sp->maxit < 0 || !(sp->tol > 0) ||
        (sp->solver != MGDD_SOLVER_FGMRES_MG && sp->solver != MGDD_SOLVER_GCR && sp->solver != MGDD_SOLVER_GCR_EO &&
         sp->solver != MGDD_SOLVER_CGN) ||
        (sp->precision != MGDD_PLAIN_F64 && sp->precision != MGDD_MIXED && sp->precision != MGDD_MIXED_F16))
        return fail(&ctx->c, MGDD_EINVAL, "bad solve parameters");
    if (!ctx->c.gauge_ready) return fail(&ctx->c, MGDD_ENOTREADY, "no gauge field");
    if (sp->solver == MGDD_SOLVER_FGMRES_MG) {
        int rc = need_coarse(ctx);
        if (rc) return rc;
        if (sp->coarse_iters < 1 || sp->nu < 0 || sp->mr_iters < 0) return fail(&ctx->c, MGDD_EINVAL, "bad solve parameters");
        if ((sp->block_solver != MGDD_BLOCK_MR && sp->block_solver != MGDD_BLOCK_GMRES) ||
            (sp->block_solver == MGDD_BLOCK_GMRES && (sp->mr_iters < 1 || sp->mr_iters > SCHWARZ_GMRES_MAX)))
            return fail(&ctx->c, MGDD_EINVAL, "bad smoother block solver (GMRES takes 1 to 3 steps)");
        if (sp->levels == 3) {
            rc = need_level3_solver(ctx, sp->k2, sp->nu2, sp->mr2);
            if (rc) return rc;
        } else if (sp->levels != 0 && sp->levels != 2) {
            return fail(&ctx->c, MGDD_EINVAL, "levels must be 2 or 3");
        }
    }
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    const size_t n = (size_t)12 * c->g.V * 16;
    std::vector<mgdd_solve_stats> st(nrhs);
    // all right-hand sides in one batched solve; when the workspace for that
    // does not fit in device memory, in batches of half the size, and so on
    int batch = nrhs, result = MGDD_OK;
    for (int r0 = 0; r0 < nrhs;) {
        const int nb = nrhs - r0 < batch ? nrhs - r0 : batch;
        int rc = solve_batch(c, sp, nb, (const char *)b + r0 * n, (char *)z + r0 * n, st.data() + r0);
        if (rc == MGDD_ENOMEM && nb > 1 && alloc_failed(c)) {
            batch = (nb + 1) / 2;
            continue;
        }
        if (rc == MGDD_ENOCONV) result = rc;
        else if (rc) {
            if (stats) std::copy(st.begin(), st.end(), stats);
            return rc;
        }
        r0 += nb;
    }
    if (stats) std::copy(st.begin(), st.end(), stats);
    return result;
    GUARD_END
}

int mgdd_timing_enable(mgdd_ctx *ctx, int on) {
    if (!ctx) return MGDD_EINVAL;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    if (!on) {
        int rc = kt_flush(c);
        c->kt.on = false;
        return rc;
    }
    if (c->kt.ev.empty()) {
        c->kt.ev.resize(2 * KT_SLOTS);
        for (auto &e : c->kt.ev) {
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                e = nullptr;
                kt_release(c);
                return fail(c, MGDD_EHIP, "hipEventCreate failed");
            }
        }
        c->kt.fam.assign(KT_SLOTS, 0);
        c->kt.units.assign(KT_SLOTS, 0.0);
        c->kt.bytes.assign(KT_SLOTS, 0.0);
    }
    c->kt.on = true;
    return MGDD_OK;
    GUARD_END
}

int mgdd_timing_read(mgdd_ctx *ctx, int kernel, int prec, int reset, double *total_ms, double *site_updates,
                     long long *launches, double *alg_bytes) {
    if (!ctx || kernel < 0 || kernel >= KF_COUNT || !valid_fine_prec(prec)) return MGDD_EINVAL;
    GUARD_BEGIN
    Ctx *c = &ctx->c;
    int rc = kt_flush(c);
    if (rc) return rc;
    const int p = prec;
    if (total_ms) *total_ms = c->kt.ms[kernel][p];
    if (site_updates) *site_updates = c->kt.usum[kernel][p];
    if (launches) *launches = c->kt.launches[kernel][p];
    if (alg_bytes) *alg_bytes = c->kt.bsum[kernel][p];
    if (reset) {
        c->kt.ms[kernel][p] = 0;
        c->kt.usum[kernel][p] = 0;
        c->kt.bsum[kernel][p] = 0;
        c->kt.launches[kernel][p] = 0;
    }
    return MGDD_OK;
    GUARD_END
}

}  // extern "C"
