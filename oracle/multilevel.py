"""Third level of the hierarchy, for the oracle (Section 3: the two-level
construction applied recursively to the coarse equation).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py). Plain numpy in FP64 on
the coarse operator D_c of the second level, stored as the oracle stores it:
Dc[a][d][i][j], a coarse site (lexicographic), d = 0 the site itself and
d = 1 + 2 mu + s the neighbour a + mu (s = 0) or a - mu (s = 1), i the row
and j the column of the 2N x 2N block; a coarse vector is c[a][chi][k]
(chirality chi of the coarse gamma_5 = diag(1_N, -1_N), test vector k).

The pieces, each the level-1 construction restated on D_c:
* `coarse_sap`: Algorithm 2.1 on D_c (blocks of coarse sites, red-black,
  MR(k) block solves on the block-restricted D_c);
* `build_P2`: the test vectors cut per (aggregate of coarse sites,
  chirality) and orthonormalised in column order (modified Gram-Schmidt);
* `restrict2`, `prolong2`: P2^H and P2;
* `dcc_build`: D_cc = P2^H D_c P2 as 9 blocks per level-3 site, by the local
  formula (a hop of D_c between coarse sites of the same aggregate goes to
  the self block, one that crosses the aggregate face in direction d to
  block d);
* `level2_test_vectors`: the smoothed fine test vectors taken to the coarse
  grid with P^H (the recursive step of the bootstrap setup, Section 3),
  completed with random coarse vectors when more are asked for, smoothed
  by level-2 SAP sweeps and kept orthonormal;
* `ThreeLevel`: the preconditioner with the coarse equation solved by a
  fixed number of flexible GMRES steps preconditioned by the two-level
  method of the second level.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

import oracle
from oracle.solvers import dot, gmres_fixed, mgs, norm

# --------------------------------------------------------------------------- geometry


def coords(dims, s):
    x = []
    for L in dims:
        x.append(s % L)
        s //= L
    return x


def lex(dims, x):
    s = 0
    for L, xi in zip(reversed(dims), reversed(x)):
        s = s * L + xi
    return s


@lru_cache(maxsize=16)
def coarse_nbr(cdims):
    """nbr[a][d] for the 9 directions of the stencil (d = 0: a itself)."""
    cdims = tuple(cdims)
    V = int(np.prod(cdims))
    nbr = np.zeros((V, 9), dtype=np.int64)
    for a in range(V):
        x = coords(cdims, a)
        nbr[a, 0] = a
        for mu in range(4):
            for s, step in ((0, 1), (1, -1)):
                y = list(x)
                y[mu] = (y[mu] + step) % cdims[mu]
                nbr[a, 1 + 2 * mu + s] = lex(cdims, y)
    return nbr


def apply_Dc(cdims, Dc, x):
    """y = D_c x through the oracle's C stencil."""
    return oracle.coarse_apply(cdims, Dc, x)

# --------------------------------------------------------------------------- level-2 SAP (Algorithm 2.1 on D_c)


def block_of(cdims, block, a):
    x = coords(cdims, a)
    nb = [L // b for L, b in zip(cdims, block)]
    bx = [xi // b for xi, b in zip(x, block)]
    return lex(nb, bx), sum(bx) % 2


def block_apply(cdims, Dc, block, sites, x):
    """I^T D_c I x for the block with the given sites (x, y indexed by site):
    hops that leave the block are dropped; a hop that wraps around a
    direction the block spans entirely stays inside it."""
    nbr = coarse_nbr(tuple(cdims))
    inblk = set(int(a) for a in sites)
    y = {}
    for a in sites:
        acc = np.zeros(Dc.shape[-1], dtype=np.complex128)
        for d in range(9):
            b = int(nbr[a, d])
            if b in inblk:
                acc = acc + Dc[a, d] @ x[b]
        y[int(a)] = acc
    return y


def coarse_sap(cdims, Dc, block, b, z0, nsweeps, mr_iters):
    """nsweeps red-black Schwarz sweeps on D_c z = b from z0 (colour 0, the
    blocks with even sum of block coordinates, first), MR(mr_iters) on each
    block from e = 0 (stop if q^H q = 0)."""
    V = int(np.prod(cdims))
    n2 = Dc.shape[-1]
    z = np.array(z0, dtype=np.complex128).reshape(V, n2).copy()
    bb = np.asarray(b, dtype=np.complex128).reshape(V, n2)
    blocks = {}
    for a in range(V):
        bi, col = block_of(cdims, block, a)
        blocks.setdefault((col, bi), []).append(a)
    for _ in range(nsweeps):
        for colour in (0, 1):
            r = bb - apply_Dc(cdims, Dc, z.reshape(V, 2, n2 // 2)).reshape(V, n2)
            for (col, bi), sites in sorted(blocks.items()):
                if col != colour:
                    continue
                rho = {a: r[a].copy() for a in sites}
                e = {a: np.zeros(n2, dtype=np.complex128) for a in sites}
                for _ in range(mr_iters):
                    q = block_apply(cdims, Dc, block, sites, rho)
                    qq = sum(np.vdot(q[a], q[a]).real for a in sites)
                    if qq == 0.0:
                        break
                    alpha = sum(np.vdot(q[a], rho[a]) for a in sites) / qq
                    for a in sites:
                        e[a] = e[a] + alpha * rho[a]
                        rho[a] = rho[a] - alpha * q[a]
                for a in sites:
                    z[a] = z[a] + e[a]
    return z.reshape(V, 2, n2 // 2)

# --------------------------------------------------------------------------- P2, restriction, prolongation, D_cc


def aggregate_sites(cdims, agg2):
    """sites of every level-2 aggregate (lexicographic over the aggregate
    grid; sites in lexicographic order inside)"""
    V = int(np.prod(cdims))
    na = [L // g for L, g in zip(cdims, agg2)]
    out = [[] for _ in range(int(np.prod(na)))]
    for a in range(V):
        x = coords(cdims, a)
        out[lex(na, [xi // g for xi, g in zip(x, agg2)])].append(a)
    return out


def build_P2(cdims, agg2, tv):
    """P2 from N2 coarse test vectors tv[k][a][chi][i]: for each aggregate and
    chirality, modified Gram-Schmidt of the N2 pieces in column order.
    Returns P2[k][a][chi][i] (zero outside the piece's aggregate and
    chirality is implied by the layout: every entry belongs to one piece)."""
    tv = np.asarray(tv, dtype=np.complex128)
    N2 = tv.shape[0]
    P2 = np.zeros_like(tv)
    for sites in aggregate_sites(cdims, agg2):
        for chi in (0, 1):
            W = [tv[k][sites, chi, :].ravel() for k in range(N2)]
            Q = mgs(W)
            for k in range(N2):
                P2[k][sites, chi, :] = Q[k].reshape(len(sites), -1)
    return P2


def restrict2(cdims, agg2, P2, c):
    """(P2^H c)[A][chi][k] = sum over the sites of A and the N1 dof of
    chirality chi of conj(P2[k]) c"""
    N2 = P2.shape[0]
    aggs = aggregate_sites(cdims, agg2)
    out = np.zeros((len(aggs), 2, N2), dtype=np.complex128)
    for A, sites in enumerate(aggs):
        for chi in (0, 1):
            for k in range(N2):
                out[A, chi, k] = np.vdot(P2[k][sites, chi, :], c[sites, chi, :])
    return out


def prolong2(cdims, agg2, P2, cc):
    """(P2 cc)[a][chi][i] = sum_k P2[k][a][chi][i] cc[A(a)][chi][k]"""
    N2 = P2.shape[0]
    out = np.zeros(P2.shape[1:], dtype=np.complex128)
    for A, sites in enumerate(aggregate_sites(cdims, agg2)):
        for chi in (0, 1):
            for k in range(N2):
                out[sites, chi, :] += P2[k][sites, chi, :] * cc[A, chi, k]
    return out


def dcc_build(cdims, agg2, Dc, P2):
    """D_cc = P2^H D_c P2 as Dcc[B][d][row][col] (the level-1 stencil format):
    the hop of D_c from a' = nbr(a, d) into a (a in aggregate B) goes to the
    self block when a' is reached without crossing B's face in direction d,
    else to block d; rows (chi, k) and columns (chi', k') are pieces of P2."""
    N2 = P2.shape[0]
    N1 = P2.shape[-1]
    ccd = tuple(L // g for L, g in zip(cdims, agg2))
    nbr = coarse_nbr(tuple(cdims))
    Vcc = int(np.prod(ccd))
    Dcc = np.zeros((Vcc, 9, 2 * N2, 2 * N2), dtype=np.complex128)
    V = int(np.prod(cdims))
    for a in range(V):
        x = coords(cdims, a)
        B = lex(ccd, [xi // g for xi, g in zip(x, agg2)])
        for d in range(9):
            if d == 0:
                dout = 0
            else:
                mu, s = (d - 1) // 2, (d - 1) % 2
                r = x[mu] % agg2[mu]
                crosses = (r == agg2[mu] - 1) if s == 0 else (r == 0)
                dout = d if crosses else 0
            ap = int(nbr[a, d])
            blk = Dc[a, d]
            for chi in (0, 1):
                for chj in (0, 1):
                    sub = blk[chi * N1:(chi + 1) * N1, chj * N1:(chj + 1) * N1]
                    # rows: conj(P2[k][a][chi]); columns: P2[k'][ap][chj]
                    L = np.conj(P2[:, a, chi, :])          # (N2, N1)
                    Rm = P2[:, ap, chj, :]                  # (N2, N1)
                    Dcc[B, dout, chi * N2:(chi + 1) * N2, chj * N2:(chj + 1) * N2] += L @ sub @ Rm.T
    return Dcc

# --------------------------------------------------------------------------- setup and cycle


def level2_test_vectors(cdims, Dc, block2, restricted, N2, nu2, mr_iters, random_coarse):
    """Level-2 test vectors: the restricted fine test vectors (first
    min(N1, N2)) then random coarse vectors, nu2 rounds of one level-2 SAP
    sweep with b = 0 on each followed by global MGS in index order."""
    V = [np.array(v, dtype=np.complex128) for v in restricted][:N2]
    extra = N2 - len(V)
    V += [np.array(r, dtype=np.complex128) for r in random_coarse[:extra]]
    V = mgs(V)
    zero = np.zeros_like(V[0])
    for _ in range(nu2):
        V = [coarse_sap(cdims, Dc, block2, zero, v, 1, mr_iters) for v in V]
        V = mgs(V)
    return V


class ThreeLevel:
    """z = SAP^nu(D, r, z0 = P x_c), x_c = FGMRES_k2(D_c, P^H r; M2) from 0,
    M2(r_c) = SAP2^nu2(D_c, r_c, z0 = P2 GMRES_cit(D_cc, P2^H r_c))."""

    def __init__(self, two_level, agg2, block2, tv2, k2=8, nu2=1, mr2=4, cit=12):
        tl = two_level
        self.tl = tl
        self.cdims = tl.cdims
        self.Dc = tl.Dc
        self.agg2, self.block2 = tuple(agg2), tuple(block2)
        self.k2, self.nu2, self.mr2, self.cit = k2, nu2, mr2, cit
        self.P2 = build_P2(self.cdims, self.agg2, np.stack(tv2))
        self.ccdims = tuple(L // g for L, g in zip(self.cdims, self.agg2))
        self.Dcc = dcc_build(self.cdims, self.agg2, self.Dc, self.P2)

    def Dc_apply(self, c):
        return apply_Dc(self.cdims, self.Dc, c)

    def M2(self, rc):
        cc = restrict2(self.cdims, self.agg2, self.P2, rc)
        xcc = gmres_fixed(lambda y: oracle.coarse_apply(self.ccdims, self.Dcc, y), cc, self.cit)
        z0 = prolong2(self.cdims, self.agg2, self.P2, xcc)
        return coarse_sap(self.cdims, self.Dc, self.block2, rc, z0, self.nu2, self.mr2)

    def coarse_solve(self, rc):
        """k2 steps of right-preconditioned flexible GMRES from x = 0, no
        restart (fewer only on exact breakdown)."""
        beta = norm(rc)
        if beta == 0.0:
            return np.zeros_like(rc)
        Vb = [rc / beta]
        Z = []
        H = np.zeros((self.k2 + 1, self.k2), dtype=np.complex128)
        k = self.k2
        for j in range(self.k2):
            Z.append(self.M2(Vb[j]))
            w = self.Dc_apply(Z[j])
            for i in range(j + 1):
                H[i, j] = dot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = norm(w)
            if H[j + 1, j] == 0.0:
                k = j + 1
                break
            Vb.append(w / H[j + 1, j])
        g = np.zeros(k + 1, dtype=np.complex128)
        g[0] = beta
        y = np.linalg.lstsq(H[:k + 1, :k], g, rcond=None)[0]
        x = np.zeros_like(rc)
        for i in range(k):
            x = x + y[i] * Z[i]
        return x

    def precond(self, r):
        tl = self.tl
        z0 = tl.prolong(self.coarse_solve(tl.restrict(r)))
        return tl.op.sap(tl.block, r, z0, tl.nu, tl.mr_iters)
