"""Krylov solvers, two-level preconditioner and bootstrap setup of the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py). Plain numpy in FP64 on top
of the C site-loop operators; small dense problems use numpy.linalg as a step
(least squares, eigenvalues), with no blocking or reordering beyond the
algorithms as stated.
"""
from __future__ import annotations

import numpy as np

from . import (BLOCK_MR, block_apply, build_P, clover, coarse_apply, coarse_build, coarse_dims, dirac, gamma, prolong,
               restrict, sap, schwarz)


def dot(a, b) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm(a) -> float:
    return float(np.sqrt(np.vdot(a.ravel(), a.ravel()).real))


def mgs(vectors):
    """Modified Gram-Schmidt in index order (global orthonormalisation)."""
    out = []
    for v in vectors:
        w = np.array(v, dtype=np.complex128, copy=True)
        for q in out:
            w = w - dot(q, w) * q
        n = norm(w)
        if n == 0.0:
            raise ValueError("mgs: linearly dependent vectors")
        out.append(w / n)
    return out


# --------------------------------------------------------------------- GMRES

def arnoldi(apply, v0, m, reorth=False):
    """m steps of Arnoldi with modified Gram-Schmidt. Returns (V list, H[(k+1), k], k)
    where k <= m is the number of steps done (k < m on an exact breakdown).
    reorth: a second Gram-Schmidt pass per step (its coefficients added to
    H), so that V stays orthonormal to rounding even when the Krylov space
    fills the whole space; the same H and V in exact arithmetic."""
    beta = norm(v0)
    V = [v0 / beta]
    H = np.zeros((m + 1, m), dtype=np.complex128)
    for j in range(m):
        w = apply(V[j])
        for _ in range(2 if reorth else 1):
            for i in range(j + 1):
                h = dot(V[i], w)
                H[i, j] += h
                w = w - h * V[i]
        H[j + 1, j] = norm(w)
        if H[j + 1, j] == 0.0:
            return V, H[: j + 2, : j + 1], j + 1
        V.append(w / H[j + 1, j].real)
    return V, H, m


def gmres_fixed(apply, b, m):
    """GMRES from x0 = 0 with exactly m Arnoldi steps (fewer only on an exact
    breakdown), no restart; the coarse solve of Section 4 uses m = 12."""
    beta = norm(b)
    if beta == 0.0:
        return np.zeros_like(b)
    V, H, k = arnoldi(apply, b, m)
    rhs = np.zeros(H.shape[0], dtype=np.complex128)
    rhs[0] = beta
    y = np.linalg.lstsq(H[: k + 1, :k], rhs[: k + 1], rcond=None)[0]
    x = np.zeros_like(b)
    for i in range(k):
        x = x + y[i] * V[i]
    return x


# --------------------------------------------------------------------- FGMRES and GCR

class Stats:
    def __init__(self):
        self.iters = 0
        self.restarts = 0
        self.history = []
        self.converged = False
        self.relres = np.inf


def fgmres(applyD, precond, b, m, tol, maxit, z0=None):
    """Right-preconditioned flexible GMRES(m) with a true-residual restart;
    stops when ||b - D z|| <= tol ||b||."""
    st = Stats()
    z = np.zeros_like(b) if z0 is None else np.array(z0, dtype=np.complex128, copy=True)
    bn = norm(b)
    if bn == 0.0:
        st.converged, st.relres = True, 0.0
        return np.zeros_like(b), st
    while True:
        r = b - applyD(z)
        beta = norm(r)
        st.relres = beta / bn
        st.history.append(st.relres)
        if beta <= tol * bn:
            st.converged = True
            return z, st
        if st.iters >= maxit:
            return z, st
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        k = 0
        for j in range(m):
            Z.append(precond(V[j]))
            w = applyD(Z[j])
            for i in range(j + 1):
                H[i, j] = dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = norm(w)
            k = j + 1
            st.iters += 1
            rhs = np.zeros(k + 1, dtype=np.complex128)
            rhs[0] = beta
            y, *_ = np.linalg.lstsq(H[: k + 1, :k], rhs, rcond=None)
            est = norm(rhs - H[: k + 1, :k] @ y)
            st.history.append(est / bn)
            if est <= tol * bn or H[j + 1, j] == 0.0 or st.iters >= maxit:
                break
            V.append(w / H[j + 1, j].real)
        for i in range(k):
            z = z + y[i] * Z[i]
        st.restarts += 1


def gcr(applyD, b, m, tol, maxit, z0=None, precond=None, check=None):
    """GCR(m): p = M r, q = D p orthogonalised against the earlier q of the
    cycle (p updated alike), z += alpha p, r -= alpha q; the stored directions are
    dropped every m steps and r is recomputed there. `check(z)` returns the
    residual norm that decides convergence (default: the recursive one)."""
    st = Stats()
    z = np.zeros_like(b) if z0 is None else np.array(z0, dtype=np.complex128, copy=True)
    bn = norm(b)
    if bn == 0.0:
        st.converged, st.relres = True, 0.0
        return z, st
    r = b - applyD(z)
    while True:
        ps, qs = [], []
        for _ in range(m):
            rn = norm(r)
            st.relres = rn / bn
            st.history.append(st.relres)
            if rn <= tol * bn or st.iters >= maxit:
                break
            p = r.copy() if precond is None else precond(r)
            q = applyD(p)
            for pj, qj in zip(ps, qs):
                beta = dot(qj, q)
                q = q - beta * qj
                p = p - beta * pj
            qn = norm(q)
            q, p = q / qn, p / qn
            alpha = dot(q, r)
            z = z + alpha * p
            r = r - alpha * q
            ps.append(p)
            qs.append(q)
            st.iters += 1
        r = b - applyD(z)
        true = norm(r) if check is None else check(z)
        st.relres = true / bn
        st.restarts += 1
        if true <= tol * bn:
            st.converged = True
            return z, st
        if st.iters >= maxit:
            return z, st


def cgn(applyD, applyDdag, b, tol, maxit, x0=None):
    """CG on the normal equations D^H D x = D^H b (CGNR: the residual
    r = b - D x is updated alongside and judges convergence, the comparator of
    the paper's Section 4). When the updated residual reaches tol ||b|| the
    true residual is recomputed; if it is still too large, CG starts again
    from the current iterate (counted as a restart)."""
    st = Stats()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    bn = norm(b)
    if bn == 0.0:
        st.converged, st.relres = True, 0.0
        return np.zeros_like(b), st
    while True:
        r = b - applyD(x)
        rn = norm(r)
        st.relres = rn / bn
        if rn <= tol * bn:
            st.converged = True
            return x, st
        if st.iters >= maxit:
            return x, st
        s = applyDdag(r)
        p = s.copy()
        ss = dot(s, s).real
        while st.iters < maxit:
            w = applyD(p)
            alpha = ss / dot(w, w).real
            x = x + alpha * p
            r = r - alpha * w
            st.iters += 1
            if norm(r) <= tol * bn:
                break
            s = applyDdag(r)
            ss_new = dot(s, s).real
            p = s + (ss_new / ss) * p
            ss = ss_new
        st.restarts += 1


# --------------------------------------------------------------------- operator bundle

def parity(dims) -> np.ndarray:
    V = int(np.prod(dims))
    s = np.arange(V)
    x = s % dims[0]
    y = (s // dims[0]) % dims[1]
    zz = (s // (dims[0] * dims[1])) % dims[2]
    t = s // (dims[0] * dims[1] * dims[2])
    return (x + y + zz + t) % 2


class Operator:
    """D = D(U) + m0 with its clover term, on one lattice."""

    def __init__(self, dims, U, m0, csw):
        self.dims = tuple(int(d) for d in dims)
        self.U = np.ascontiguousarray(U, dtype=np.complex128)
        self.A = clover(self.dims, self.U, m0, csw)
        self.m0, self.csw = m0, csw
        self._zeroA = None

    def apply(self, psi, shift=0.0):
        return dirac(self.dims, self.U, self.A, psi, shift)

    def hop(self, psi):
        """Hopping part of D only: D psi - A psi."""
        if self._zeroA is None:
            self._zeroA = np.zeros_like(self.A)
        return dirac(self.dims, self.U, self._zeroA, psi)

    def sap(self, block, b, z0, nsweeps, mr_iters, shift=0.0):
        return sap(self.dims, self.U, self.A, block, b, z0, nsweeps, mr_iters, shift)

    def schwarz(self, block, b, z0, nsweeps, k, block_solver=BLOCK_MR, additive=False, shift=0.0):
        return schwarz(self.dims, self.U, self.A, block, b, z0, nsweeps, k, block_solver, additive, shift)

    def apply_dag(self, psi):
        """D^H psi = gamma_5 D gamma_5 psi (D is gamma_5-Hermitian)."""
        g5 = np.diag(gamma()[1]).real
        x = np.asarray(psi, dtype=np.complex128) * g5[None, :, None]
        return self.apply(x) * g5[None, :, None]

    def block_apply(self, block, blk, psi, shift=0.0):
        return block_apply(self.dims, self.U, self.A, block, blk, psi, shift)


# --------------------------------------------------------------------- two-level method

class TwoLevel:
    """P from test vectors, D_c = P^H D P, and the two-level preconditioner:
    coarse-grid correction with a fixed-step GMRES on D_c, then nu SAP sweeps."""

    def __init__(self, op: Operator, agg, test_vectors, block, mr_iters=4, nu=1, coarse_iters=12,
                 block_solver=BLOCK_MR, additive=False):
        self.op, self.agg, self.block = op, tuple(agg), tuple(block)
        self.mr_iters, self.nu, self.coarse_iters = mr_iters, nu, coarse_iters
        self.block_solver, self.additive = block_solver, additive
        self.set_test_vectors(test_vectors)

    def set_test_vectors(self, tv):
        P, st = build_P(self.op.dims, self.agg, tv)
        if st:
            raise ValueError(f"build_P status {st}")
        self.P = P
        self.N = P.shape[0]
        self.cdims = coarse_dims(self.op.dims, self.agg)
        self.Dc = coarse_build(self.op.dims, self.agg, self.op.U, self.op.A, P)

    def restrict(self, f):
        return restrict(self.op.dims, self.agg, self.P, f)

    def prolong(self, c):
        return prolong(self.op.dims, self.agg, self.P, c)

    def coarse_apply(self, c):
        return coarse_apply(self.cdims, self.Dc, c)

    def coarse_solve(self, c):
        return gmres_fixed(self.coarse_apply, c, self.coarse_iters)

    def precond(self, r):
        """coarse-grid correction, then nu Schwarz sweeps from it (red-black
        with MR blocks unless another variant was chosen)"""
        z0 = self.prolong(self.coarse_solve(self.restrict(r)))
        if self.block_solver == BLOCK_MR and not self.additive:
            return self.op.sap(self.block, r, z0, self.nu, self.mr_iters)
        return self.op.schwarz(self.block, r, z0, self.nu, self.mr_iters, self.block_solver, self.additive)


# --------------------------------------------------------------------- even-odd Schur complement

class EvenOdd:
    """D_hat = A_oo - H_oe A_ee^{-1} H_eo on the odd sites (the even sites are eliminated)."""

    def __init__(self, op: Operator):
        self.op = op
        self.odd = parity(op.dims) == 1
        self.even = ~self.odd
        self.Aee_inv = np.linalg.inv(op.A[self.even])

    def _Ainv_even(self, f):
        out = np.zeros_like(f)
        out[self.even] = np.einsum("nij,nj->ni", self.Aee_inv, f[self.even].reshape(-1, 12)).reshape(-1, 4, 3)
        return out

    def apply_hat(self, fo):
        """fo lives on the odd sites (zero on the even ones)."""
        t = self.op.hop(fo)                    # H_eo fo  (on even sites)
        t[self.odd] = 0
        t = self._Ainv_even(t)
        u = self.op.hop(t)                     # H_oe A_ee^-1 H_eo fo (on odd sites)
        Af = np.einsum("nij,nj->ni", self.op.A[self.odd], fo[self.odd].reshape(-1, 12)).reshape(-1, 4, 3)
        out = np.zeros_like(fo)
        out[self.odd] = Af - u[self.odd]
        return out

    def rhs_hat(self, b):
        t = self._Ainv_even(np.where(self.even[:, None, None], b, 0))
        u = self.op.hop(t)
        out = np.zeros_like(b)
        out[self.odd] = b[self.odd] - u[self.odd]
        return out

    def reconstruct(self, b, zo):
        h = self.op.hop(zo)
        t = np.where(self.even[:, None, None], b - h, 0)
        z = self._Ainv_even(t)
        z[self.odd] = zo[self.odd]
        return z

    def solve(self, b, m, tol, maxit):
        bn = norm(b)
        bh = self.rhs_hat(b)
        check = lambda zo: norm(b - self.op.apply(self.reconstruct(b, zo)))  # noqa: E731
        zo, st = gcr(self.apply_hat, bh, m, tol * bn / max(norm(bh), 1e-300), maxit, check=None)
        # the convergence test is on the full system: tighten until it holds
        inner_tol = tol * bn / max(norm(bh), 1e-300)
        while check(zo) > tol * bn and st.iters < maxit:
            inner_tol *= 0.1
            zo, st2 = gcr(self.apply_hat, bh, m, inner_tol, maxit - st.iters, z0=zo)
            st.iters += st2.iters
        z = self.reconstruct(b, zo)
        st.relres = norm(b - self.op.apply(z)) / bn
        st.converged = st.relres <= tol
        return z, st


# --------------------------------------------------------------------- bootstrap setup

def harmonic_ritz(apply, v0, m, nkeep):
    """Harmonic Ritz pairs for target 0 from m Arnoldi steps: eigenpairs of
    H_m + |h_{m+1,m}|^2 H_m^{-H} e_m e_m^T; the nkeep of smallest modulus
    (ties broken by real part, then imaginary part, so that the choice does
    not depend on the order an eigensolver returns them in). The formula
    assumes an orthonormal Krylov basis (H_m = V_m^H A V_m), so the Arnoldi
    run re-orthogonalises: with one Gram-Schmidt pass the basis of a run as
    long as the space loses its orthogonality and the pairs their meaning.
    Returns (theta[nkeep], vectors list)."""
    V, H, k = arnoldi(apply, v0, m, reorth=True)
    Hm = H[:k, :k]
    T = Hm.copy()
    if H.shape[0] > k:
        hk = H[k, k - 1]
        em = np.zeros(k, dtype=np.complex128)
        em[-1] = 1.0
        f = np.linalg.solve(Hm.conj().T, em)
        T = T + abs(hk) ** 2 * np.outer(f, em)
    theta, Y = np.linalg.eig(T)
    order = sorted(range(k), key=lambda i: (abs(theta[i]), theta[i].real, theta[i].imag))[:nkeep]
    vecs = []
    for i in order:
        y = Y[:, i]
        phi = np.zeros_like(V[0])
        for j in range(k):
            phi = phi + y[j] * V[j]
        vecs.append(phi / norm(phi))
    return theta[order], vecs


def bootstrap(op: Operator, block, agg, N, nu, iota, mr_iters, random_vectors, arnoldi_start, m_arnoldi=None,
              n_part2=1):
    """Bootstrap setup (Section 3). Part 1: nu rounds of one SAP sweep (b = 0)
    on every test vector followed by global MGS, then P and D_c. Part 2 (n_part2
    times): harmonic Ritz pairs of D_c, interpolation, iota shifted SAP sweeps,
    and the 2N -> N reduction by the N smallest eigenpairs of (DV)^H DV with
    V orthonormal. Returns (test vectors, TwoLevel)."""
    zero = np.zeros_like(random_vectors[0])
    V = [np.array(v, dtype=np.complex128) for v in random_vectors]
    for _ in range(nu):
        V = [op.sap(block, zero, v, 1, mr_iters) for v in V]
        V = mgs(V)
    tl = TwoLevel(op, agg, np.stack(V), block, mr_iters=mr_iters)
    nc = tl.Dc.shape[0] * 2 * N
    mA = min(nc, 2 * N + 10) if m_arnoldi is None else m_arnoldi
    for _ in range(n_part2):
        theta, phis = harmonic_ritz(tl.coarse_apply, np.asarray(arnoldi_start).reshape(tl.Dc.shape[0], 2, N), mA, N)
        W = []
        for th, phi in zip(theta, phis):
            w = tl.prolong(phi)
            W.append(op.sap(block, zero, w, iota, mr_iters, shift=complex(th)))
        W = mgs(W + V)
        DW = [op.apply(w) for w in W]
        G = np.array([[dot(a, b) for b in DW] for a in DW])
        sig, Y = np.linalg.eigh(G)
        V = []
        for i in range(N):
            v = np.zeros_like(W[0])
            for j in range(2 * N):
                v = v + Y[j, i] * W[j]
            V.append(v)
        tl.set_test_vectors(np.stack(V))
    return np.stack(V), tl
