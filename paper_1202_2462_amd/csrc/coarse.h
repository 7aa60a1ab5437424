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

}  // namespace mgdd
