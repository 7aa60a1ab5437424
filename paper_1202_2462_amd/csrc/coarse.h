// Device helper of the coarse stencil y = D_c x at one coarse site, shared by
// the coarse apply kernel and the fused Arnoldi kernel.
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

// The 9 blocks of coarse site a are column-major, B[dir][col][row], so term
// tau = dir * n2 + col of row i sits at B[tau * n2 + i]. A workgroup of
// blockDim.x threads splits the 9 n2 terms into nparts = blockDim.x / n2
// interleaved sets: thread t < nparts n2 takes row i = t % n2 and the terms
// tau = t / n2, t / n2 + nparts, ..., four independent products at a time.
// xs holds the 9 neighbour vectors, xs[tau] = x_{nbr(dir)}[col]. The partial
// row sums go to part[t]; the caller adds part[p * n2 + i] over p in order.
template <typename T>
__device__ inline void dc_row_partial(const C<T> *__restrict__ B, const C<T> *xs, int n2, C<T> *part) {
    const int nparts = blockDim.x / n2;
    const int t = threadIdx.x;
    if (t >= nparts * n2) return;
    const int i = t % n2, p0 = t / n2, nterm = 9 * n2;
    C<T> a0 = mk<T>(0, 0), a1 = a0, a2 = a0, a3 = a0;
    int tau = p0;
    for (; tau + 3 * nparts < nterm; tau += 4 * nparts) {
        const C<T> b0 = B[(size_t)tau * n2 + i], b1 = B[(size_t)(tau + nparts) * n2 + i];
        const C<T> b2 = B[(size_t)(tau + 2 * nparts) * n2 + i], b3 = B[(size_t)(tau + 3 * nparts) * n2 + i];
        cfma(a0, b0, xs[tau]);
        cfma(a1, b1, xs[tau + nparts]);
        cfma(a2, b2, xs[tau + 2 * nparts]);
        cfma(a3, b3, xs[tau + 3 * nparts]);
    }
    for (; tau < nterm; tau += nparts) cfma(a0, B[(size_t)tau * n2 + i], xs[tau]);
    part[t] = cadd(cadd(a0, a1), cadd(a2, a3));
}

// The same row sums from the compact blocks of a gamma5^c-hermitian D_c
// (gamma5^c = +1 on the first N coarse components, -1 on the others, and
// D_c^H = gamma5^c D_c gamma5^c, which P^H D P inherits from D when P keeps
// the chiralities apart): H holds site a's self block and its forward hops
// D_c(a, a + mu) (5 blocks, column-major), Fb[mu] the forward hop
// F_mu = D_c(b_mu, b_mu + mu) of the neighbour b_mu = a - mu, from which
// D_c(a, a - mu)[i][j] = s_i s_j conj(F_mu[j][i]), s = gamma5^c. xs is ordered
// as the terms: self, the four forward neighbours, then the four backward
// ones. The self and forward terms go to part as in dc_row_partial. The
// backward terms are split the other way round, so that the reads of the
// transposed blocks stay contiguous: thread t takes row i = t / nparts and
// the columns j = g, g + nparts, ... (g = t % nparts) of all four blocks,
// row i of F_mu^H being column i of F_mu; its sum goes to partb[g n2 + i].
template <typename T>
__device__ inline void dch_row_partial(const C<T> *__restrict__ H, const C<T> *const *Fb, const C<T> *xs, int n2,
                                       C<T> *part, C<T> *partb) {
    const int nparts = blockDim.x / n2;
    const int t = threadIdx.x;
    if (t >= nparts * n2) return;
    const int i = t % n2, p0 = t / n2, nf = 5 * n2, N = n2 / 2;
    C<T> a0 = mk<T>(0, 0), a1 = a0, a2 = a0, a3 = a0;
    int tau = p0;
    for (; tau + 3 * nparts < nf; tau += 4 * nparts) {
        const C<T> b0 = H[(size_t)tau * n2 + i], b1 = H[(size_t)(tau + nparts) * n2 + i];
        const C<T> b2 = H[(size_t)(tau + 2 * nparts) * n2 + i], b3 = H[(size_t)(tau + 3 * nparts) * n2 + i];
        cfma(a0, b0, xs[tau]);
        cfma(a1, b1, xs[tau + nparts]);
        cfma(a2, b2, xs[tau + 2 * nparts]);
        cfma(a3, b3, xs[tau + 3 * nparts]);
    }
    for (; tau < nf; tau += nparts) cfma(a0, H[(size_t)tau * n2 + i], xs[tau]);
    part[t] = cadd(cadd(a0, a1), cadd(a2, a3));
    // backward hops
    const int ib = t / nparts, g = t % nparts;
    const bool upper = ib < N;
    C<T> b[4] = {mk<T>(0, 0), mk<T>(0, 0), mk<T>(0, 0), mk<T>(0, 0)};
    for (int j = g; j < n2; j += nparts) {
        const T sg = (j < N) == upper ? (T)1 : (T)-1;
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            const C<T> f = Fb[mu][(size_t)ib * n2 + j];
            cfma(b[mu], mk<T>(sg * f.x, -sg * f.y), xs[nf + mu * n2 + j]);
        }
    }
    partb[g * n2 + ib] = cadd(cadd(b[0], b[1]), cadd(b[2], b[3]));
}

}  // namespace mgdd
