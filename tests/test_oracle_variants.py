"""Pins of the oracle's variants of the paper's protocol (Sections 2 and 4):
GMRES(k) block solves (the minimum residual over the block's Krylov space,
exact at full dimension), additive Schwarz (every block solved for the same
residual: dense block inverses), the multiplicative sweep with GMRES blocks
against a dense step-by-step reconstruction, and CGN (the adjoint, the
minimum-residual property of its iterates, convergence to the dense solve)."""
import numpy as np
import pytest

import latgen
import oracle
from helpers import dense, random_op, rel
from oracle.solvers import cgn

DIMS, BLOCK = (4, 4, 4, 4), (2, 2, 2, 2)


@pytest.fixture(scope="module")
def prob():
    op = random_op(DIMS, seed=21, m0=0.1)
    V = int(np.prod(DIMS))
    Dd = dense(op.apply, (V, 4, 3))
    nb = [L // b for L, b in zip(DIMS, BLOCK)]
    blocks = []
    for blk in range(int(np.prod(nb))):
        sites = oracle.block_sites(DIMS, BLOCK, blk)
        t, c = blk, 0
        for m in range(4):
            c += t % nb[m]
            t //= nb[m]
        idx = (sites[:, None] * 12 + np.arange(12)[None, :]).ravel()
        blocks.append((c % 2, idx))
    return op, Dd, blocks


def field(seed):
    return latgen.gaussian_fields(DIMS, 1, seed)[0]


def krylov_basis(A, v, k):
    """an orthonormal basis of span{v, A v, ..., A^(k-1) v}: each new power
    direction A q_last projected out of the previous ones twice (numpy)"""
    Q = (v / np.linalg.norm(v))[:, None]
    for _ in range(k - 1):
        w = A @ Q[:, -1]
        for _ in range(2):
            w = w - Q @ (Q.conj().T @ w)
        Q = np.concatenate([Q, (w / np.linalg.norm(w))[:, None]], 1)
    return Q


def krylov_min(A, r, k):
    """argmin over span{r, A r, ..., A^(k-1) r} of ||r - A e|| (numpy least squares)"""
    K = krylov_basis(A, r, k)
    c = np.linalg.lstsq(A @ K, r, rcond=None)[0]
    return K @ c


@pytest.mark.parametrize("k", [1, 2, 3])
def test_multiplicative_gmres_sweep_equals_dense_reconstruction(prob, k):
    op, Dd, blocks = prob
    b, z0 = field(1), field(2)
    got = op.schwarz(BLOCK, b, z0, 1, k, oracle.BLOCK_GMRES)
    z = z0.ravel().copy()
    for colour in (0, 1):
        r = b.ravel() - Dd @ z
        for c, idx in blocks:
            if c == colour:
                A = Dd[np.ix_(idx, idx)]
                z[idx] += krylov_min(A, r[idx], k)
    assert rel(got.ravel(), z) < 1e-10


def test_gmres_block_at_full_dimension_is_exact():
    op = random_op((2, 2, 2, 2), seed=22, m0=0.2)
    b = latgen.gaussian_fields((2, 2, 2, 2), 1, 3)[0]
    Dd = dense(op.apply, b.shape)
    z = op.schwarz((2, 2, 2, 2), b, np.zeros_like(b), 1, 192, oracle.BLOCK_GMRES)
    assert rel(z.ravel(), np.linalg.solve(Dd, b.ravel())) < 1e-8


def test_mr_through_schwarz_equals_sap(prob):
    op = prob[0]
    b, z0 = field(3), field(4)
    assert np.array_equal(op.schwarz(BLOCK, b, z0, 2, 4), op.sap(BLOCK, b, z0, 2, 4))


@pytest.mark.parametrize("solver,k", [(oracle.BLOCK_GMRES, 192), (oracle.BLOCK_GMRES, 2), (oracle.BLOCK_MR, 3)])
def test_additive_sweep_solves_every_block_for_one_residual(prob, solver, k):
    op, Dd, blocks = prob
    b, z0 = field(5), field(6)
    got = op.schwarz(BLOCK, b, z0, 1, k, solver, additive=True)
    r = b.ravel() - Dd @ z0.ravel()
    z = z0.ravel().copy()
    for _, idx in blocks:
        A = Dd[np.ix_(idx, idx)]
        if solver == oracle.BLOCK_GMRES and k >= len(idx):   # full dimension: the block inverse
            z[idx] += np.linalg.solve(A, r[idx])
        elif solver == oracle.BLOCK_GMRES:
            z[idx] += krylov_min(A, r[idx], k)
        else:   # k MR steps, each the one-dimensional minimum residual along rho
            rho, e = r[idx].copy(), np.zeros(len(idx), dtype=complex)
            for _ in range(k):
                q = A @ rho
                a = np.vdot(q, rho) / np.vdot(q, q).real
                e, rho = e + a * rho, rho - a * q
            z[idx] += e
    assert rel(got.ravel(), z) < 1e-9
    # additive and multiplicative differ (the second colour sees the first's update)
    assert rel(op.schwarz(BLOCK, b, z0, 1, k, solver), got) > 1e-6


def test_adjoint_is_gamma5_sandwich(prob):
    op = prob[0]
    x, y = field(7), field(8)
    assert abs(np.vdot(x, op.apply(y)) - np.vdot(op.apply_dag(x), y)) < 1e-11 * np.linalg.norm(x) * np.linalg.norm(y)


def test_cgn_iterate_minimises_residual_over_normal_krylov_space(prob):
    op, Dd, _ = prob
    b, x0 = field(9), field(10)
    for k in (1, 3, 6):
        x, st = cgn(op.apply, op.apply_dag, b, 1e-30, k, x0)
        assert st.iters == k
        r0 = b.ravel() - Dd @ x0.ravel()
        K = krylov_basis(Dd.conj().T @ Dd, Dd.conj().T @ r0, k)
        c = np.linalg.lstsq(Dd @ K, r0, rcond=None)[0]
        assert rel(x.ravel(), x0.ravel() + K @ c) < 1e-8, k


def test_cgn_converges_to_dense_solution(prob):
    op, Dd, _ = prob
    b = field(11)
    x, st = cgn(op.apply, op.apply_dag, b, 1e-10, 20000)
    assert st.converged
    assert np.linalg.norm(b.ravel() - Dd @ x.ravel()) <= 1e-10 * np.linalg.norm(b)
    assert rel(x.ravel(), np.linalg.solve(Dd, b.ravel())) < 1e-6
