"""Pin of the oracle's bootstrap setup (Section 3, "Bootstrap Setup"), both
parts, by a step-by-step reconstruction written here from the definitions:

* the Schwarz sweep of Algorithm 2.1 with MR block solves, each block operator
  applied as (D - lambda) on the block's zero-extended vector, restricted to
  the block (hops leaving the block dropped);
* "kept orthonormal": the unique thin QR with a positive diagonal of R (numpy
  QR, signs fixed), which modified Gram-Schmidt in index order computes;
* P per (aggregate, chirality) by the same QR, D_c = P^H D P as a dense
  matrix;
* with as many Arnoldi steps as D_c has rows, the harmonic Ritz pairs for
  target 0 are the exact eigenpairs of D_c (numpy eig), the N of smallest
  modulus;
* the 2N -> N reduction by the N smallest eigenpairs of the Hermitian
  (DV)^H (DV) with V orthonormal (numpy eigh).

Only the Wilson-clover apply of the oracle is used (pinned by the free-field
spectrum and the invariants in test_oracle_dirac.py). The lattice is 4^3 x 8
with 4^4 Schwarz blocks and aggregates and N = 8, so D_c has 2 * 2N = 32 rows
and the oracle's Arnoldi run covers the whole coarse space. Test vectors are
unique up to one phase per vector, which is aligned before comparing. The
same reconstruction with the shift of the second part's sweeps dropped, or
with the wrong eigenpairs kept, is shown to land far away, so a mistake of
either kind in the oracle would fail the comparison."""
from __future__ import annotations

import numpy as np
import pytest

import latgen
from oracle import solvers
from helpers import aligned_difference, random_op

DIMS, BLOCK, N = (4, 4, 4, 8), (4, 4, 4, 4), 8
NU, IOTA, MR = 3, 3, 4


def _coords(dims):
    s = np.arange(int(np.prod(dims)))
    x = s % dims[0]
    y = (s // dims[0]) % dims[1]
    z = (s // (dims[0] * dims[1])) % dims[2]
    t = s // (dims[0] * dims[1] * dims[2])
    return np.stack([x, y, z, t], 1)


def _blocks(dims, block):
    """(lexicographic block index of every site, number of blocks, colour of each block)"""
    X = _coords(dims)
    nb = [d // b for d, b in zip(dims, block)]
    bc = X // np.array(block)
    lex = bc[:, 0] + nb[0] * (bc[:, 1] + nb[1] * (bc[:, 2] + nb[2] * bc[:, 3]))
    nblk = int(np.prod(nb))
    colour = np.zeros(nblk, dtype=int)
    for b in range(nblk):
        colour[b] = int(bc[lex == b][0].sum()) % 2
    return lex, nblk, colour


def _qr(cols):
    """orthonormal Q of the columns with a real positive diagonal of R"""
    Q, R = np.linalg.qr(np.stack(cols, 1))
    d = np.diag(R)
    return Q * (d / np.abs(d))[None, :]


class Dense:
    """The reconstruction, on one operator."""

    def __init__(self, op):
        self.op = op
        self.shape = (int(np.prod(op.dims)), 4, 3)
        self.blk, self.nblk, self.colour = _blocks(op.dims, BLOCK)

    def D(self, v, lam=0.0):
        return self.op.apply(v.reshape(self.shape)).ravel() - lam * v

    def mr(self, mask, r, lam, k):
        """k MR steps on the block operator from e = 0"""
        e = np.zeros_like(r)
        rho = r.copy()
        for _ in range(k):
            q = self.D(rho * mask, lam) * mask
            qq = np.vdot(q, q).real
            if qq == 0.0:
                break
            alpha = np.vdot(q, rho) / qq
            e = e + alpha * rho
            rho = rho - alpha * q
        return e

    def sweep(self, b, z, lam, k):
        """one red-black sweep on (D - lam) z = b, colour 0 first"""
        site_mask = [np.repeat(self.blk == i, 12).astype(float) for i in range(self.nblk)]
        for c in (0, 1):
            r = b - self.D(z, lam)
            corr = np.zeros_like(z)
            for i in range(self.nblk):
                if self.colour[i] == c:
                    corr = corr + self.mr(site_mask[i], r * site_mask[i], lam, k)
            z = z + corr
        return z

    def prolongator(self, V, agg):
        """dense P (rows: fine dof, columns: (aggregate, chirality, k))"""
        ablk, na, _ = _blocks(self.op.dims, agg)
        n = V[0].size
        P = np.zeros((n, na * 2 * N), dtype=np.complex128)
        spin = np.tile(np.repeat(np.arange(4), 3), n // 12)
        site = np.repeat(np.arange(n // 12), 12)
        for a in range(na):
            for chi in (0, 1):
                rows = np.nonzero((ablk[site] == a) & ((spin >= 2) == bool(chi)))[0]
                Q = _qr([v[rows] for v in V])
                P[rows, a * 2 * N + chi * N: a * 2 * N + (chi + 1) * N] = Q
        return P

    def bootstrap(self, rnd, agg, drop_shift=False, largest_ritz=False, largest_gram=False):
        zero = np.zeros(rnd[0].size, dtype=np.complex128)
        V = [np.asarray(v, dtype=np.complex128).ravel() for v in rnd]
        for _ in range(NU):
            V = [self.sweep(zero, v, 0.0, MR) for v in V]
            Q = _qr(V)
            V = [Q[:, i] for i in range(N)]
        P = self.prolongator(V, agg)
        DP = np.stack([self.D(P[:, j]) for j in range(P.shape[1])], 1)
        Dc = P.conj().T @ DP
        theta, Phi = np.linalg.eig(Dc)
        order = sorted(range(len(theta)), key=lambda i: (abs(theta[i]), theta[i].real, theta[i].imag))
        if largest_ritz:
            order = order[::-1]
        order = order[:N]
        W = []
        for i in order:
            w = P @ (Phi[:, i] / np.linalg.norm(Phi[:, i]))
            lam = 0.0 if drop_shift else theta[i]
            for _ in range(IOTA):
                w = self.sweep(zero, w, lam, MR)
            W.append(w)
        Q = _qr(W + V)
        DW = np.stack([self.D(Q[:, j]) for j in range(2 * N)], 1)
        G = DW.conj().T @ DW
        sig, Y = np.linalg.eigh(G)
        keep = slice(N, 2 * N) if largest_gram else slice(0, N)
        return (Q @ Y[:, keep]).T, theta[order], sig


def problem():
    op = random_op(DIMS, seed=17, eps=0.5, m0=0.05, csw=1.0)
    rnd = latgen.gaussian_fields(DIMS, N, 50)
    nc = (np.prod(DIMS) // np.prod(BLOCK)) * 2 * N
    start = latgen.gaussian_vector(int(nc), 51)
    return op, rnd, start, int(nc)


@pytest.mark.slow
def test_bootstrap_matches_step_by_step_reconstruction():
    op, rnd, start, nc = problem()
    assert nc == 32
    tv_or, _ = solvers.bootstrap(op, BLOCK, BLOCK, N, NU, IOTA, MR, rnd, start, m_arnoldi=nc)
    dense = Dense(op)
    tv, theta, sig = dense.bootstrap(rnd, BLOCK)
    # premise: no tie where the N smallest eigenvalues of the Gram matrix are
    # cut off, so the kept space is unique (the Ritz cut: test below)
    assert sig[N] - sig[N - 1] > 1e-6 * sig[-1]
    diff = aligned_difference(tv_or, tv)
    print("bootstrap: oracle vs reconstruction", diff, "smallest Ritz values", np.abs(theta))
    assert diff < 1e-10
    # the oracle's output is orthonormal and ||D v_i|| ascends
    G = np.array([[np.vdot(a, b) for b in tv_or] for a in tv_or])
    assert np.max(np.abs(G - np.eye(N))) < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("mistake", ["drop_shift", "largest_ritz", "largest_gram"])
def test_bootstrap_reconstruction_detects_mistakes(mistake):
    """The comparison above is sensitive to the mistakes it is meant to catch:
    the reconstruction with one of them differs from the oracle by far more
    than its bar."""
    op, rnd, start, nc = problem()
    tv_or, _ = solvers.bootstrap(op, BLOCK, BLOCK, N, NU, IOTA, MR, rnd, start, m_arnoldi=nc)
    tv_bad, _, _ = Dense(op).bootstrap(rnd, BLOCK, **{mistake: True})
    diff = aligned_difference(tv_or, tv_bad)
    print(mistake, diff)
    assert diff > 1e-3


@pytest.mark.slow
def test_ritz_cut_is_unique():
    """The N-th and (N+1)-th smallest |eigenvalues| of D_c after the first
    part differ clearly (D_c is gamma_5^c-Hermitian, so its eigenvalues come in
    complex-conjugate pairs of equal modulus; a cut through a pair would make
    the choice of Ritz pairs depend on rounding)."""
    op, rnd, start, nc = problem()
    _, tl = solvers.bootstrap(op, BLOCK, BLOCK, N, NU, IOTA, MR, rnd, start, n_part2=0)
    Dc = np.stack([tl.coarse_apply(e.reshape(-1, 2, N)).ravel() for e in np.eye(nc, dtype=np.complex128)], 1)
    ev = np.sort(np.abs(np.linalg.eigvals(Dc)))
    print("|theta|", ev[:N + 2])
    assert ev[N] - ev[N - 1] > 1e-4 * ev[N]
