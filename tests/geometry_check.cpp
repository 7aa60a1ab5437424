// Host check of the library's device site order (run by tests/test_geometry.py):
// for a set of lattice / block shapes it verifies, on the CPU, that
//  - device index <-> coordinates is a bijection onto [0, V),
//  - every neighbour index lies in [0, V) and is the periodic neighbour,
//  - in-block local neighbour indices (the Schwarz kernel's LDS indices) lie
//    in [0, Vb) and agree with the global neighbour when it is in the block,
//  - the blocks of colour 0 come first and no two neighbouring blocks share a
//    colour,
//  - the XCD workgroup remap is a permutation.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1202_2462_amd/csrc/mgdd_internal.h"

using namespace mgdd;

static int check(const int *dims, const int *block, bool expect_ok) {
    Geom g{};
    std::vector<uint32_t> coord;
    std::vector<int> nbr, lexpos;
    std::string e = geometry_tables(dims, block, g, coord, nbr, &lexpos);
    if (!expect_ok) {
        if (e.empty()) { printf("FAIL: shape accepted but should be rejected\n"); return 1; }
        return 0;
    }
    if (!e.empty()) { printf("FAIL: %s\n", e.c_str()); return 1; }
    g.blk_coord = coord.data();
    g.blk_nbr = nbr.data();
    g.pos_of_lex = lexpos.data();
    std::vector<int> seen(g.V, 0), seen2(g.V, 0);
    for (int i = 0; i < g.V; i++) {
        int d = site_in_lex_block_order(g, i);
        if (d < 0 || d >= g.V || seen2[d]) { printf("FAIL lexicographic block order\n"); return 1; }
        seen2[d] = 1;
    }
    for (int d = 0; d < g.V; d++) {
        int X[4];
        site_coords(g, d, X);
        for (int mu = 0; mu < 4; mu++)
            if (X[mu] < 0 || X[mu] >= g.L[mu]) { printf("FAIL coords out of range\n"); return 1; }
        int s = lex_of(g, d);
        if (s < 0 || s >= g.V || seen[s]) { printf("FAIL not a bijection at %d\n", d); return 1; }
        seen[s] = 1;
        int pos = d >> g.lgVb, l = d & (g.Vb - 1);
        int x[4];
        local_coords(g, l, x);
        if (local_index(g, x) != l) { printf("FAIL local index roundtrip\n"); return 1; }
        int par = (X[0] + X[1] + X[2] + X[3]) & 1;
        if ((l >= g.Vb / 2) != par) { printf("FAIL parity split\n"); return 1; }
        for (int mu = 0; mu < 4; mu++)
            for (int dir = -1; dir <= 1; dir += 2) {
                int n = neighbour(g, pos, x, mu, dir);
                if (n < 0 || n >= g.V) { printf("FAIL neighbour out of range\n"); return 1; }
                int Y[4];
                site_coords(g, n, Y);
                for (int nu = 0; nu < 4; nu++) {
                    int want = nu == mu ? (X[nu] + dir + g.L[nu]) % g.L[nu] : X[nu];
                    if (Y[nu] != want) { printf("FAIL wrong neighbour\n"); return 1; }
                }
                // local neighbour as the Schwarz kernel computes it
                int bm = 1 << g.lb[mu];
                int y[4] = {x[0], x[1], x[2], x[3]};
                y[mu] = x[mu] + dir;
                if (g.nb[mu] == 1) y[mu] = (y[mu] + bm) & (bm - 1);
                if (y[mu] >= 0 && y[mu] < bm) {
                    int ln = local_index(g, y);
                    if (ln < 0 || ln >= g.Vb) { printf("FAIL LDS index\n"); return 1; }
                    if (((n >> g.lgVb) != pos) || (n & (g.Vb - 1)) != ln) { printf("FAIL in-block neighbour\n"); return 1; }
                } else if ((n >> g.lgVb) == pos) {
                    printf("FAIL neighbour outside the block maps into it\n");
                    return 1;
                }
            }
    }
    for (int p = 0; p < g.nblocks; p++) {
        int bc[4];
        unpack_block(coord[p], bc);
        int col = (bc[0] + bc[1] + bc[2] + bc[3]) & 1;
        if ((p < g.ncol0) != (col == 0)) { printf("FAIL colour order\n"); return 1; }
        for (int k = 0; k < 8; k++) {
            int q = nbr[(size_t)p * 8 + k];
            if (q < 0 || q >= g.nblocks) { printf("FAIL block neighbour range\n"); return 1; }
            int bq[4];
            unpack_block(coord[q], bq);
            int cq = (bq[0] + bq[1] + bq[2] + bq[3]) & 1;
            if (q != p && cq == col) { printf("FAIL two neighbouring blocks share a colour\n"); return 1; }
        }
    }
    for (int nwg : {1, 2, 7, 8, 9, 15, 16, 24, 8 * 37, 1000, 1001}) {
        std::vector<int> hit(nwg, 0);
        for (int b = 0; b < nwg; b++) {
            int w = xcd_remap(b, nwg);
            if (w < 0 || w >= nwg || hit[w]) { printf("FAIL xcd remap\n"); return 1; }
            hit[w] = 1;
        }
    }
    return 0;
}

int main() {
    struct Case { int d[4], b[4]; bool ok; };
    const Case cases[] = {
        {{8, 8, 8, 8}, {4, 4, 4, 4}, true},   {{4, 8, 4, 16}, {4, 4, 2, 4}, true},
        {{8, 4, 4, 8}, {2, 4, 4, 2}, true},   {{16, 16, 16, 32}, {4, 4, 4, 4}, true},
        {{4, 4, 4, 4}, {4, 4, 4, 4}, true},   {{2, 2, 2, 2}, {2, 2, 2, 2}, true},
        {{8, 8, 8, 16}, {2, 2, 2, 2}, true},  {{24, 8, 8, 8}, {4, 4, 4, 4}, true},
        {{8, 8, 8, 8}, {3, 4, 4, 4}, false},  {{8, 8, 8, 8}, {1, 4, 4, 4}, false},
        {{12, 8, 8, 8}, {4, 4, 4, 4}, false},
        // the largest workload lattice, and one past the 32-bit offset limit
        {{48, 48, 48, 96}, {4, 4, 4, 4}, true}, {{64, 64, 64, 64}, {4, 4, 4, 4}, false},
    };
    int bad = 0;
    for (const Case &c : cases) {
        int r = check(c.d, c.b, c.ok);
        printf("%s dims %d %d %d %d block %d %d %d %d\n", r ? "FAIL" : "ok", c.d[0], c.d[1], c.d[2], c.d[3], c.b[0],
               c.b[1], c.b[2], c.b[3]);
        bad += r;
    }
    printf(bad ? "GEOMETRY FAILED\n" : "GEOMETRY OK\n");
    return bad ? 1 : 0;
}
