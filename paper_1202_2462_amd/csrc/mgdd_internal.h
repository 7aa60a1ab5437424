// Internal declarations of the gfx950 library: device geometry, complex
// helpers, the context, and the launch entry points of each kernel file.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mgdd.h"

namespace mgdd {

// ------------------------------------------------------------------ complex arithmetic

// complex number stored in half precision (storage only: arithmetic is FP32)
struct alignas(4) half_cx {
    _Float16 x, y;
};

template <typename T> struct cx;
template <> struct cx<double> { using t = double2; };
template <> struct cx<float> { using t = float2; };
template <> struct cx<_Float16> { using t = half_cx; };
template <typename T> using C = typename cx<T>::t;

template <typename T> __host__ __device__ inline C<T> mk(T r, T i) { C<T> z; z.x = r; z.y = i; return z; }
template <typename V> __host__ __device__ inline V cadd(V a, V b) { V z; z.x = a.x + b.x; z.y = a.y + b.y; return z; }
template <typename V> __host__ __device__ inline V csub(V a, V b) { V z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename V> __host__ __device__ inline V cmul(V a, V b) {
    V z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z;
}
// conj(a) * b
template <typename V> __host__ __device__ inline V cmulc(V a, V b) {
    V z; z.x = a.x * b.x + a.y * b.y; z.y = a.x * b.y - a.y * b.x; return z;
}
// acc += a * b, as four fused multiply-adds into the accumulator
template <typename V> __host__ __device__ inline void cfma(V &acc, V a, V b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename V> __host__ __device__ inline void cfmac(V &acc, V a, V b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}
template <typename V, typename S> __host__ __device__ inline V cscale(V a, S s) { V z; z.x = a.x * s; z.y = a.y * s; return z; }
// i * a
template <typename V> __host__ __device__ inline V ci(V a) { V z; z.x = -a.y; z.y = a.x; return z; }
template <typename V> __host__ __device__ inline V cneg(V a) { V z; z.x = -a.x; z.y = -a.y; return z; }

}  // namespace mgdd

#include "geometry.h"

namespace mgdd {

// Remaps the workgroup index so that consecutive ranges of workgroups (and so
// of lattice sites) land on the same XCD: the hardware hands workgroups to the
// 8 XCDs round-robin, each XCD with its own L2.
__host__ __device__ inline int xcd_remap(int b, int nwg) {
    const int q = nwg >> 3, r = nwg & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}
__device__ inline int xcd_block(int nwg) { return xcd_remap(blockIdx.x, nwg); }

// ------------------------------------------------------------------ the context

struct Level1 {  // coarse level of the current P
    bool ready = false;
    int agg[4] = {0, 0, 0, 0};
    int Lc[4] = {0, 0, 0, 0};
    int Vc = 0, Va = 0, N = 0;
    void *P64 = nullptr, *P32 = nullptr;    // N fine fields, device layout
    void *P16 = nullptr;                    // the same in half precision (FP16-storage transfers)
    void *Dc64 = nullptr, *Dc32 = nullptr;  // [Vc][9][2N (col)][2N (row)] complex
    // [Vc][5][2N (col)][2N (row)] FP32: the self block and the forward hops
    // D_c(a, a + mu); the backward hops follow from gamma5^c-hermiticity
    void *Dh32 = nullptr;
    int *cnbr = nullptr;                    // [Vc][9] coarse neighbour (self first)
    int *corder = nullptr;                  // [Vc] order in which the coarse step visits the coarse sites
    int *agg_sites = nullptr;               // [Vc][Va] device site of each local site of an aggregate
    int *site_agg = nullptr;                // [V] aggregate of each device site
    void *tv64 = nullptr;                   // the N test vectors P was built from
};

// Third level: aggregates of coarse sites, P2 from N2 coarse test vectors,
// D_cc = P2^H D_c P2 on the level-3 lattice, and the blocks of the level-2
// Schwarz smoother on the coarse lattice.
struct Level2 {
    bool ready = false;                     // P2 and D_cc built
    int agg[4] = {0, 0, 0, 0}, Lcc[4] = {0, 0, 0, 0};
    int Vcc = 0, Va2 = 0, N2 = 0, N1 = 0;
    void *P2_64 = nullptr, *P2_32 = nullptr;    // [N2][Vc][2 N1] complex (coarse vectors)
    void *Dcc64 = nullptr, *Dcc32 = nullptr;    // [Vcc][9][2N2 (col)][2N2 (row)] complex
    int *cnbr2 = nullptr;                   // [Vcc][9]
    int *agg2_sites = nullptr;              // [Vcc][Va2] coarse sites of each level-3 site
    int *site_agg2 = nullptr;               // [Vc] level-3 site of each coarse site
    int *geo = nullptr;                     // coarse extents Lc[4], then the aggregate shape [4]
    void *tv2_64 = nullptr;                 // the N2 test vectors P2 was built from
    // Schwarz blocks of the level-2 smoother
    int blk[4] = {0, 0, 0, 0};
    int nblk = 0, ncol0 = 0, Vb2 = 0;
    int *blk_sites = nullptr;               // [nblk][Vb2], colour-0 blocks first
    int *blk_lnbr = nullptr;                // [nblk][Vb2][9] local index of the neighbour in the block, or -1
    int *blk_nbr = nullptr;                 // [nblk][Vb2][9] coarse site of the neighbour
};

// Optional timing of kernel families with HIP events on the context's stream:
// each launch is bracketed by an event pair from a fixed pool; durations are
// added up when the pool is full or when the caller reads them.
enum KernelFamily { KF_DIRAC = 0, KF_SAP = 1, KF_COARSE = 2, KF_COUNT = 3 };
struct KTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;      // 2 per slot
    std::vector<int> fam;            // family * 3 + precision code, per used slot
    std::vector<double> units;       // site-rhs updates, per used slot
    std::vector<double> bytes;       // algorithmic bytes, per used slot
    int used = 0;
    double ms[KF_COUNT][3] = {};
    double usum[KF_COUNT][3] = {};
    double bsum[KF_COUNT][3] = {};
    long long launches[KF_COUNT][3] = {};
};

// one device allocation of a context and the routine that releases it
// (hipFree when free_fn is null, else the caller's allocator)
struct Owned {
    void *p;
    mgdd_free_fn free_fn;
    void *user;
};

struct Ctx {
    Geom g{};
    bool t_antiperiodic = true;             // sign -1 on the hops across the time boundary
    hipStream_t stream = nullptr;
    std::string err;
    int dev = 0;
    size_t lds_max = 65536;                 // LDS bytes one workgroup may take
    int sap_lanes = 0;                      // mgdd_kernel_options: 0 automatic, 1, 2, 4
    bool learned_fallback = false;          // the last learned setup fell back to the bootstrap
    int dirac_stage = 0;                    // 0 automatic, 1 staged, -1 not staged
    // geometry tables
    uint32_t *d_blk_coord = nullptr;
    int *d_blk_nbr = nullptr;
    // operator
    bool gauge_ready = false;
    bool links_su3 = false;                 // every link special unitary: row 2 = conj(row 0 x row 1)
    double m0 = 0, csw = 0;
    void *U64 = nullptr, *U32 = nullptr;    // [4][9][V] complex
    void *A64 = nullptr, *A32 = nullptr;    // [36][V] complex pairs (packed Hermitian 6x6 x 2 chiralities)
    void *Ainv64 = nullptr;                 // [36][V] the same for the inverse of A (even-odd)
    Level1 c;
    Level2 c2;
    // workspace
    std::vector<Owned> owned;
    mgdd_alloc_fn ualloc = nullptr;         // caller's allocator (mgdd_set_allocator), or hipMalloc
    mgdd_free_fn ufree = nullptr;
    void *uuser = nullptr;
    void *stage = nullptr;                  // canonical staging buffer
    size_t stage_bytes = 0;
    double *red = nullptr;                  // reduction partials
    size_t red_doubles = 0;
    double *red_host = nullptr;             // pinned
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    void *ws = nullptr;                     // solver / setup workspace
    size_t ws_bytes = 0;
    void *hbuf = nullptr;                   // pinned scalars (see host_buf)
    KTimer kt;
};

int fail(Ctx *c, int code, const std::string &msg);
int hip_check(Ctx *c, hipError_t e, const char *what);
void *dalloc(Ctx *c, size_t bytes);
void dfree(Ctx *c, void *p);
void release_owned(const Owned &o);
void *ensure_stage(Ctx *c, size_t bytes);
void *ensure_scratch(Ctx *c, size_t bytes);
double *ensure_red(Ctx *c, size_t ndoubles);
// kt_begin returns a slot (or -1 when timing is off); kt_end closes it.
int kt_begin(Ctx *c);
void kt_end(Ctx *c, int slot, int family, int prec, double units, double bytes);
int kt_flush(Ctx *c);
inline size_t csize(int prec) { return prec == MGDD_F64 ? 16 : prec == MGDD_F32 ? 8 : 4; }
inline size_t fine_elems(const Ctx *c, int nrhs) { return (size_t)nrhs * 12 * c->g.V; }

// ------------------------------------------------------------------ launchers (one per kernel family)

// layout.hip
int launch_pack(Ctx *c, int prec, int nrhs, const double2 *canon, void *dst);
int launch_unpack(Ctx *c, int prec, int nrhs, const void *src, double2 *canon);
int launch_gauge_ingest(Ctx *c, const double2 *Ucanon);
int launch_convert(Ctx *c, int from, int to, size_t n, const void *src, void *dst);
// nf FP64 Gaussian random fields (device layout) from the counter-based generator of stream seed
int launch_gaussian_fields(Ctx *c, int nf, unsigned long long seed, void *dst);

// dirac.hip
int launch_dirac(Ctx *c, int prec, int nrhs, const void *in, void *out);

// sap.hip: nsweeps red-black sweeps with MR(mr) block solves; one colour step
int launch_sap(Ctx *c, int prec, int nrhs, int nsweeps, int mr, double sre, double sim, const void *b, void *z);
int launch_sap_colour(Ctx *c, int prec, int nrhs, int col, int mr, double sre, double sim, const void *b, void *z);

}  // namespace mgdd
