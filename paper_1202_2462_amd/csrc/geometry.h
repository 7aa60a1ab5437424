// Lattice geometry of the device site order (host and device code) and the
// host-side construction of its tables.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace mgdd {

// ------------------------------------------------------------------ lattice geometry
//
// Device site order: the lattice is cut into blocks of size b (powers of two,
// b_mu >= 2). Block position pos: all colour-0 blocks (even sum of block
// coordinates) in lexicographic order, then all colour-1 blocks. Inside a
// block, local index l = parity * Vb/2 + (local lexicographic index >> 1).
// Device site index = pos * Vb + l.
struct Geom {
    int L[4];
    int lb[4];       // log2 of block dims
    int nb[4];       // blocks per dimension
    int V, Vb, lgVb, nblocks, ncol0;
    const uint32_t *blk_coord;   // [nblocks] packed block coords of position pos (8 bits each)
    const int *blk_nbr;          // [nblocks][8] position of the neighbour block, dir = 2*mu + (0:+,1:-)
    const int *pos_of_lex;       // [nblocks] position of the block with lexicographic block index b
};

// Device site of the i-th site in lexicographic block order (blocks in
// lexicographic order of their coordinates, sites in device order inside a
// block): kernels that visit every site use this order so that a range of
// consecutive workgroups covers a compact slab of the lattice with both
// colours, and neighbour faces are reused from cache.
__host__ __device__ inline int site_in_lex_block_order(const Geom &g, int i) {
    return (g.pos_of_lex[i >> g.lgVb] << g.lgVb) + (i & (g.Vb - 1));
}

__host__ __device__ inline int local_index(const Geom &g, const int *x) {
    int lex = x[0] + (x[1] << g.lb[0]) + (x[2] << (g.lb[0] + g.lb[1])) + (x[3] << (g.lb[0] + g.lb[1] + g.lb[2]));
    int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    return p * (g.Vb >> 1) + (lex >> 1);
}

__host__ __device__ inline void local_coords(const Geom &g, int l, int *x) {
    int half = g.Vb >> 1;
    int p = l >= half;
    int h = l & (half - 1);
    int sx = g.lb[0] - 1;
    int lxh = h & ((1 << sx) - 1);
    int r = h >> sx;
    x[1] = r & ((1 << g.lb[1]) - 1);
    r >>= g.lb[1];
    x[2] = r & ((1 << g.lb[2]) - 1);
    r >>= g.lb[2];
    x[3] = r;
    x[0] = 2 * lxh + ((p + x[1] + x[2] + x[3]) & 1);
}

__host__ __device__ inline void unpack_block(uint32_t c, int *bc) {
    bc[0] = c & 255; bc[1] = (c >> 8) & 255; bc[2] = (c >> 16) & 255; bc[3] = c >> 24;
}

// global coordinates of device site d
__host__ __device__ inline void site_coords(const Geom &g, int d, int *X) {
    int pos = d >> g.lgVb, l = d & (g.Vb - 1);
    int bc[4];
    unpack_block(g.blk_coord[pos], bc);
    local_coords(g, l, X);
    for (int mu = 0; mu < 4; mu++) X[mu] += bc[mu] << g.lb[mu];
}

// device index of the neighbour of (pos, local coords x) one step in direction
// mu (dir = +1/-1), periodic.
__host__ __device__ inline int neighbour(const Geom &g, int pos, const int *x, int mu, int dir) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    int bmu = 1 << g.lb[mu];
    y[mu] += dir;
    int npos = pos;
    if (y[mu] < 0 || y[mu] >= bmu) {
        y[mu] = (y[mu] + bmu) & (bmu - 1);
        npos = g.blk_nbr[pos * 8 + 2 * mu + (dir > 0 ? 0 : 1)];
    }
    return (npos << g.lgVb) + local_index(g, y);
}

// lexicographic (canonical) site of device site d
__host__ __device__ inline int lex_of(const Geom &g, int d) {
    int X[4];
    site_coords(g, d, X);
    return X[0] + g.L[0] * (X[1] + g.L[1] * (X[2] + g.L[2] * X[3]));
}


// Host construction of the block tables. Checks the shapes: every block
// extent a power of two >= 2 dividing L, the number of blocks per direction
// even or 1 (two-colouring), fewer than 256 blocks per direction.
// coord[pos] and nbr[pos*8 + dir] are filled; returns "" or the error text.
inline std::string geometry_tables(const int *dims, const int *block, Geom &g, std::vector<uint32_t> &coord,
                                   std::vector<int> &nbr, std::vector<int> *lexpos = nullptr) {
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    auto ilog2 = [](int v) { int r = 0; while ((1 << r) < v) r++; return r; };
    for (int mu = 0; mu < 4; mu++) {
        if (dims[mu] <= 0 || block[mu] < 2 || !pow2(block[mu]) || dims[mu] % block[mu])
            return "block dims must be powers of two >= 2 dividing the lattice";
        int nb = dims[mu] / block[mu];
        if (nb > 1 && (nb & 1)) return "number of blocks per direction must be even or 1";
        if (nb > 255) return "more than 255 blocks in one direction";
        g.L[mu] = dims[mu];
        g.lb[mu] = ilog2(block[mu]);
        g.nb[mu] = nb;
    }
    long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    // the kernels address a per-site array with 32-bit byte offsets; the
    // largest are 288 bytes per site (links or clover blocks of all
    // directions in FP32, one chirality's clover block in FP64)
    if (V * 288 >= (1LL << 32)) return "lattice too large (at most 14 913 080 sites)";
    g.V = (int)V;
    g.Vb = block[0] * block[1] * block[2] * block[3];
    g.lgVb = ilog2(g.Vb);
    g.nblocks = g.V / g.Vb;
    coord.clear();
    std::vector<int> pos_of_lex(g.nblocks);
    for (int col = 0; col < 2; col++)
        for (int lex = 0; lex < g.nblocks; lex++) {
            int t = lex, bc[4], s = 0;
            for (int mu = 0; mu < 4; mu++) { bc[mu] = t % g.nb[mu]; t /= g.nb[mu]; s += bc[mu]; }
            if ((s & 1) != col) continue;
            pos_of_lex[lex] = (int)coord.size();
            coord.push_back((uint32_t)bc[0] | ((uint32_t)bc[1] << 8) | ((uint32_t)bc[2] << 16) | ((uint32_t)bc[3] << 24));
            if (col == 0) g.ncol0 = (int)coord.size();
        }
    if (coord.empty() || coord.size() != (size_t)g.nblocks) return "block table construction failed";
    // every colour-0 block comes first; ncol0 counts them
    g.ncol0 = 0;
    for (int p = 0; p < g.nblocks; p++) {
        int bc[4];
        unpack_block(coord[p], bc);
        if (((bc[0] + bc[1] + bc[2] + bc[3]) & 1) == 0) g.ncol0++;
    }
    nbr.assign((size_t)g.nblocks * 8, 0);
    for (int p = 0; p < g.nblocks; p++) {
        int bc[4];
        unpack_block(coord[p], bc);
        for (int mu = 0; mu < 4; mu++)
            for (int dir = 0; dir < 2; dir++) {
                int y[4] = {bc[0], bc[1], bc[2], bc[3]};
                y[mu] = (y[mu] + (dir == 0 ? 1 : -1) + g.nb[mu]) % g.nb[mu];
                int lex = y[0] + g.nb[0] * (y[1] + g.nb[1] * (y[2] + g.nb[2] * y[3]));
                nbr[(size_t)p * 8 + 2 * mu + dir] = pos_of_lex[lex];
            }
    }
    if (lexpos) *lexpos = pos_of_lex;
    return "";
}

}  // namespace mgdd
