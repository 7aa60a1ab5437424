// Device building blocks of the Wilson-clover stencil: buffer-resource loads
// from the site-major (structure-of-arrays) layout, the spin-projected hops in
// the chiral basis, and the packed clover term.
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

// ------------------------------------------------------------------ buffer access
//
// Every field is read through a buffer resource (wave-uniform, in SGPRs): the
// per-thread address is one 32-bit VGPR (site offset) and the component offset
// is an SGPR, instead of one 64-bit address pair per load. Reads outside
// num_records return zero and writes there are dropped by the hardware.
using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ inline rsrc_t make_rsrc(const void *p, size_t bytes) {
    unsigned n = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, 0x00020000);
}

template <typename T> struct BIO;
// NT: the non-temporal cache policy (data read or written once: the caches
// evict it first, which keeps data that is read again in them)
template <> struct BIO<float> {
    template <bool NT = false> __device__ static float2 ld(rsrc_t r, unsigned vo, unsigned so) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, NT ? 2 : 0));
    }
    template <bool NT = false> __device__ static void st(float2 v, rsrc_t r, unsigned vo, unsigned so) {
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, vo, so, NT ? 2 : 0);
    }
};
template <> struct BIO<double> {
    template <bool NT = false> __device__ static double2 ld(rsrc_t r, unsigned vo, unsigned so) {
        return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, NT ? 2 : 0));
    }
    template <bool NT = false> __device__ static void st(double2 v, rsrc_t r, unsigned vo, unsigned so) {
        using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, v), r, vo, so, NT ? 2 : 0);
    }
};

// A set of `ncomp` complex components of V sites, stored [comp][V].
template <typename T> struct FieldView {
    rsrc_t r;
    unsigned cs;  // bytes between components
    __device__ FieldView(const C<T> *base, size_t V, int ncomp) {
        r = make_rsrc(base, (size_t)ncomp * V * sizeof(C<T>));
        cs = (unsigned)(V * sizeof(C<T>));
    }
    template <bool NT = false> __device__ C<T> ld(int comp, int site, unsigned salt = 0) const {
        return BIO<T>::template ld<NT>(r, (unsigned)site * (unsigned)sizeof(C<T>), comp * cs + salt);
    }
    template <bool NT = false> __device__ void st(int comp, int site, C<T> v) const {
        BIO<T>::template st<NT>(v, r, (unsigned)site * (unsigned)sizeof(C<T>), comp * cs);
    }
    // load / store with an extra per-lane byte offset (the descriptor and the
    // scalar offset stay wave-uniform; a lane-dependent scalar offset would
    // make the compiler loop over the distinct values)
    template <bool NT = false> __device__ C<T> ld_lane(int comp, int site, unsigned lane_off, unsigned salt = 0) const {
        return BIO<T>::template ld<NT>(r, (unsigned)site * (unsigned)sizeof(C<T>) + lane_off, comp * cs + salt);
    }
    template <bool NT = false> __device__ void st_lane(int comp, int site, unsigned lane_off, C<T> v) const {
        BIO<T>::template st<NT>(v, r, (unsigned)site * (unsigned)sizeof(C<T>) + lane_off, comp * cs);
    }
};

// A set of `ncomp` complex components of V sites stored in half precision
// ([comp][V], 4 bytes per complex), read and written as FP32 complex numbers
// (round to nearest even on the way out).
struct HalfFieldView {
    rsrc_t r;
    unsigned cs;
    __device__ HalfFieldView(const void *base, size_t V, int ncomp) {
        r = make_rsrc(base, (size_t)ncomp * V * 4);
        cs = (unsigned)(V * 4);
    }
    template <bool NT = false> __device__ float2 ld(int comp, int site, unsigned salt = 0) const {
        const half_cx h = __builtin_bit_cast(
            half_cx, __builtin_amdgcn_raw_buffer_load_b32(r, (unsigned)site * 4u, comp * cs + salt, NT ? 2 : 0));
        return make_float2((float)h.x, (float)h.y);
    }
    template <bool NT = false> __device__ void st(int comp, int site, float2 v) const {
        half_cx h;
        h.x = (_Float16)v.x;
        h.y = (_Float16)v.y;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, h), r, (unsigned)site * 4u, comp * cs,
                                              NT ? 2 : 0);
    }
    // with an extra per-lane byte offset, as FieldView's
    template <bool NT = false> __device__ float2 ld_lane(int comp, int site, unsigned lane_off, unsigned salt = 0) const {
        const half_cx h = __builtin_bit_cast(half_cx, __builtin_amdgcn_raw_buffer_load_b32(
                                                          r, (unsigned)site * 4u + lane_off, comp * cs + salt, NT ? 2 : 0));
        return make_float2((float)h.x, (float)h.y);
    }
    template <bool NT = false> __device__ void st_lane(int comp, int site, unsigned lane_off, float2 v) const {
        half_cx h;
        h.x = (_Float16)v.x;
        h.y = (_Float16)v.y;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, h), r, (unsigned)site * 4u + lane_off,
                                              comp * cs, NT ? 2 : 0);
    }
};

// the view of a fine field stored as S (float: FieldView<float>, _Float16:
// HalfFieldView), arithmetic in FP32; ESZ: bytes of one complex value
template <typename S> struct F32Store;
template <> struct F32Store<float> {
    using view = FieldView<float>;
    static constexpr size_t ESZ = 8;
};
template <> struct F32Store<_Float16> {
    using view = HalfFieldView;
    static constexpr size_t ESZ = 4;
};

// FV: FieldView<T>, or HalfFieldView with T = float
template <typename T, typename FV> __device__ inline void load_spinor(const FV &f, int d, C<T> *s) {
#pragma unroll
    for (int k = 0; k < 12; k++) s[k] = f.ld(k, d);
}

// NT: written once (non-temporal cache policy)
template <typename T, bool NT = false, typename FV> __device__ inline void store_spinor(const FV &f, int d, const C<T> *s) {
#pragma unroll
    for (int k = 0; k < 12; k++) f.template st<NT>(k, d, s[k]);
}

// links: one view per direction ([9][V] complex each)
template <typename T> struct LinkViews {
    FieldView<T> u0, u1, u2, u3;
    __device__ LinkViews(const C<T> *U, size_t V)
        : u0(U, V, 9), u1(U + 9 * V, V, 9), u2(U + 18 * V, V, 9), u3(U + 27 * V, V, 9) {}
    template <int MU> __device__ const FieldView<T> &get() const {
        return MU == 0 ? u0 : MU == 1 ? u1 : MU == 2 ? u2 : u3;
    }
};

// row 2 of a special unitary link from rows 0 and 1: u_2a = s conj(u_0b u_1c -
// u_0c u_1b) with (a, b, c) cyclic; s = -1 on the links that carry the
// antiperiodic time-boundary sign (the folded sign makes the determinant -1)
template <typename T> __device__ inline void su3_row2(C<T> *u, T s) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        const C<T> x = csub(cmul(u[b], u[3 + c]), cmul(u[c], u[3 + b]));
        u[6 + a] = mk<T>(s * x.x, -s * x.y);
    }
}

// RECON: the links are special unitary (checked at ingest); rows 0 and 1 are
// read and row 2 is rebuilt (sign: see su3_row2), a third fewer link bytes
template <typename T, int MU, bool RECON = false>
__device__ inline void load_link(const LinkViews<T> &U, int d, C<T> *u, unsigned salt = 0, T sign = 1) {
    const FieldView<T> &f = U.template get<MU>();
#pragma unroll
    for (int k = 0; k < (RECON ? 6 : 9); k++) u[k] = f.ld(k, d, salt);
    if (RECON) su3_row2<T>(u, sign);
}

// A zero the compiler cannot see through: added to the offsets of loads inside
// a loop it keeps them from being hoisted out of the loop (which would hold
// every link of the site in registers for the whole loop).
__device__ inline unsigned opaque_zero() {
    unsigned z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

// clover: two views ([18][V] complex pairs per chirality)
template <typename T> struct CloverViews {
    FieldView<T> a0, a1;
    __device__ CloverViews(const C<T> *A, size_t V) : a0(A, V, 18), a1(A + 18 * V, V, 18) {}
};

// ------------------------------------------------------------------ algebra

// w = U v (colour), or U^H v when DAG
template <typename T, bool DAG> __device__ inline void su3_mv(const C<T> *u, const C<T> *v, C<T> *w) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        C<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int b = 0; b < 3; b++) {
            if (DAG) cfmac(acc, u[b * 3 + a], v[b]);
            else cfma(acc, u[a * 3 + b], v[b]);
        }
        w[a] = acc;
    }
}

// acc += (1 - gamma_mu) U psi  (FWD)   or   acc += (1 + gamma_mu) U^H psi  (!FWD)
// Chiral basis: gamma_mu = [[0, B],[B^H, 0]] with B_k = -i sigma_k, B_t = -1.
// (1 -+ gamma) psi = (h, -+ B^H h) with h = u -+ B l for psi = (u, l).
template <typename T, int MU, bool FWD> __device__ inline void hop(C<T> *acc, const C<T> *u, const C<T> *psi) {
    C<T> h0[3], h1[3], w0[3], w1[3];
    const C<T> *u0 = psi, *u1 = psi + 3, *l0 = psi + 6, *l1 = psi + 9;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (MU == 0) {        // B l = (-i l1, -i l0)
            h0[a] = FWD ? cadd(u0[a], ci(l1[a])) : csub(u0[a], ci(l1[a]));
            h1[a] = FWD ? cadd(u1[a], ci(l0[a])) : csub(u1[a], ci(l0[a]));
        } else if (MU == 1) { // B l = (-l1, l0)
            h0[a] = FWD ? cadd(u0[a], l1[a]) : csub(u0[a], l1[a]);
            h1[a] = FWD ? csub(u1[a], l0[a]) : cadd(u1[a], l0[a]);
        } else if (MU == 2) { // B l = (-i l0, i l1)
            h0[a] = FWD ? cadd(u0[a], ci(l0[a])) : csub(u0[a], ci(l0[a]));
            h1[a] = FWD ? csub(u1[a], ci(l1[a])) : cadd(u1[a], ci(l1[a]));
        } else {              // B l = -l
            h0[a] = FWD ? cadd(u0[a], l0[a]) : csub(u0[a], l0[a]);
            h1[a] = FWD ? cadd(u1[a], l1[a]) : csub(u1[a], l1[a]);
        }
    }
    su3_mv<T, !FWD>(u, h0, w0);
    su3_mv<T, !FWD>(u, h1, w1);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc[a] = cadd(acc[a], w0[a]);
        acc[3 + a] = cadd(acc[3 + a], w1[a]);
        // lower spins: -B^H w (forward) or +B^H w (backward)
        if (MU == 0) {        // B^H w = (i w1, i w0)
            acc[6 + a] = FWD ? csub(acc[6 + a], ci(w1[a])) : cadd(acc[6 + a], ci(w1[a]));
            acc[9 + a] = FWD ? csub(acc[9 + a], ci(w0[a])) : cadd(acc[9 + a], ci(w0[a]));
        } else if (MU == 1) { // B^H w = (w1, -w0)
            acc[6 + a] = FWD ? csub(acc[6 + a], w1[a]) : cadd(acc[6 + a], w1[a]);
            acc[9 + a] = FWD ? cadd(acc[9 + a], w0[a]) : csub(acc[9 + a], w0[a]);
        } else if (MU == 2) { // B^H w = (i w0, -i w1)
            acc[6 + a] = FWD ? csub(acc[6 + a], ci(w0[a])) : cadd(acc[6 + a], ci(w0[a]));
            acc[9 + a] = FWD ? cadd(acc[9 + a], ci(w1[a])) : csub(acc[9 + a], ci(w1[a]));
        } else {              // B^H w = -w
            acc[6 + a] = FWD ? cadd(acc[6 + a], w0[a]) : csub(acc[6 + a], w0[a]);
            acc[9 + a] = FWD ? cadd(acc[9 + a], w1[a]) : csub(acc[9 + a], w1[a]);
        }
    }
}

// Packed Hermitian 6x6: 36 reals = 6 diagonal entries, then (re, im) of the
// upper entries (0,1),(0,2),...,(0,5),(1,2),...,(4,5); stored as 18 pairs.
__host__ __device__ inline int hpack(int i, int j) { return 6 + 2 * ((i * (11 - i)) / 2 + (j - i - 1)); }

template <typename T> __device__ inline void herm6_mv(const C<T> *p /*18 pairs*/, const C<T> *x, C<T> *y) {
    T m[36];
#pragma unroll
    for (int k = 0; k < 18; k++) { m[2 * k] = p[k].x; m[2 * k + 1] = p[k].y; }
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] = cscale(x[i], m[i]);
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i + 1; j < 6; j++) {
            int k = hpack(i, j);
            C<T> aij = mk<T>(m[k], m[k + 1]);
            cfma(y[i], aij, x[j]);
            cfmac(y[j], aij, x[i]);
        }
}

// out = A in for the two chirality blocks of site d. NT: the clover term is
// read once (non-temporal cache policy)
template <typename T, bool NT = false>
__device__ inline void clover_mv(const CloverViews<T> &A, int d, const C<T> *in, C<T> *out, unsigned salt = 0) {
    C<T> p[18];
#pragma unroll
    for (int k = 0; k < 18; k++) p[k] = A.a0.template ld<NT>(k, d, salt);
    herm6_mv<T>(p, in, out);
#pragma unroll
    for (int k = 0; k < 18; k++) p[k] = A.a1.template ld<NT>(k, d, salt);
    herm6_mv<T>(p, in + 6, out + 6);
}

template <typename T, int MU, bool FWD, bool RECON = false, typename FV>
__device__ inline void hop_from(const LinkViews<T> &U, const FV &f, int d, int dn, C<T> *acc, T sign = 1) {
    C<T> psi[12], u[9];
    load_spinor<T>(f, dn, psi);
    load_link<T, MU, RECON>(U, FWD ? d : dn, u, 0, sign);
    hop<T, MU, FWD>(acc, u, psi);
    // keep the scheduler from hoisting the loads of all eight hops at once
    __builtin_amdgcn_sched_barrier(0);
}

// sum over the 8 hops of the Wilson term, without the factor -1/2:
// H psi(x) = sum_mu (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^H psi(x-mu)
// RECON: links rebuilt from two rows; sf, sb: the signs of the forward and
// backward time links of this site (-1 where the hop crosses the
// antiperiodic time boundary)
template <typename T, bool RECON = false, typename FV>
__device__ inline void hop_sum(const LinkViews<T> &U, const FV &f, int d, const int *nbr, C<T> *acc, T sf = 1,
                               T sb = 1) {
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = mk<T>(0, 0);
    hop_from<T, 0, true, RECON>(U, f, d, nbr[0], acc);
    hop_from<T, 0, false, RECON>(U, f, d, nbr[1], acc);
    hop_from<T, 1, true, RECON>(U, f, d, nbr[2], acc);
    hop_from<T, 1, false, RECON>(U, f, d, nbr[3], acc);
    hop_from<T, 2, true, RECON>(U, f, d, nbr[4], acc);
    hop_from<T, 2, false, RECON>(U, f, d, nbr[5], acc);
    hop_from<T, 3, true, RECON>(U, f, d, nbr[6], acc, sf);
    hop_from<T, 3, false, RECON>(U, f, d, nbr[7], acc, sb);
}

// The hop sum for a workgroup that holds the spinors of its own lattice block
// in LDS (sp: [12][NT] complex numbers of type S, the block at device position
// pos, NT sites). The neighbour's spinor is read through a generic pointer
// that points into LDS for a neighbour inside the block and into memory (the
// field in, [12][V]) for one outside it, so that all lanes run the same
// instructions; S is FP64, FP32 or half precision, widened to T on the way.
__device__ inline float2 widen_to(float2 v, float) { return v; }
__device__ inline double2 widen_to(double2 v, double) { return v; }
__device__ inline double2 widen_to(float2 v, double) { return make_double2((double)v.x, (double)v.y); }
__device__ inline double2 widen_to(half_cx v, double) { return make_double2((double)v.x, (double)v.y); }

template <typename T, typename S, int MU, bool FWD, bool RECON, int NT>
__device__ inline void hop_from_staged(const LinkViews<T> &U, const C<S> *in, size_t V, const C<S> *sp, int pos,
                                       int lgVb, int d, int dn, C<T> *acc, T sign) {
    C<T> psi[12], u[9];
    const bool inside = (dn >> lgVb) == pos;
    const C<S> *src = inside ? sp + (dn & (NT - 1)) : in + dn;
    const size_t stride = inside ? (size_t)NT : V;
#pragma unroll
    for (int k = 0; k < 12; k++) psi[k] = widen_to(src[k * stride], T());
    load_link<T, MU, RECON>(U, FWD ? d : dn, u, 0, sign);
    hop<T, MU, FWD>(acc, u, psi);
    __builtin_amdgcn_sched_barrier(0);
}

template <typename T, typename S, bool RECON, int NT>
__device__ inline void hop_sum_staged(const LinkViews<T> &U, const C<S> *in, size_t V, const C<S> *sp, int pos,
                                      int lgVb, int d, const int *nbr, C<T> *acc, T sf, T sb) {
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = mk<T>(0, 0);
    hop_from_staged<T, S, 0, true, RECON, NT>(U, in, V, sp, pos, lgVb, d, nbr[0], acc, (T)1);
    hop_from_staged<T, S, 0, false, RECON, NT>(U, in, V, sp, pos, lgVb, d, nbr[1], acc, (T)1);
    hop_from_staged<T, S, 1, true, RECON, NT>(U, in, V, sp, pos, lgVb, d, nbr[2], acc, (T)1);
    hop_from_staged<T, S, 1, false, RECON, NT>(U, in, V, sp, pos, lgVb, d, nbr[3], acc, (T)1);
    hop_from_staged<T, S, 2, true, RECON, NT>(U, in, V, sp, pos, lgVb, d, nbr[4], acc, (T)1);
    hop_from_staged<T, S, 2, false, RECON, NT>(U, in, V, sp, pos, lgVb, d, nbr[5], acc, (T)1);
    hop_from_staged<T, S, 3, true, RECON, NT>(U, in, V, sp, pos, lgVb, d, nbr[6], acc, sf);
    hop_from_staged<T, S, 3, false, RECON, NT>(U, in, V, sp, pos, lgVb, d, nbr[7], acc, sb);
}

// signs of the time links of site d when they are rebuilt from two rows: -1
// on the link that crosses the antiperiodic time boundary
template <typename T> __device__ inline void time_link_signs(const Geom &g, int d, int antiperiodic, T &sf, T &sb) {
    int X[4];
    site_coords(g, d, X);
    sf = (antiperiodic && X[3] == g.L[3] - 1) ? (T)-1 : (T)1;
    sb = (antiperiodic && X[3] == 0) ? (T)-1 : (T)1;
}

__device__ inline void site_neighbours(const Geom &g, int d, int *nbr) {
    int pos = d >> g.lgVb, l = d & (g.Vb - 1);
    int x[4];
    local_coords(g, l, x);
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        nbr[2 * mu] = neighbour(g, pos, x, mu, +1);
        nbr[2 * mu + 1] = neighbour(g, pos, x, mu, -1);
    }
}

}  // namespace mgdd
