"""Pins of the oracle's Krylov solvers, two-level cycle and setup (Sections 3
and 4): GMRES minimises the residual over the Krylov space and is exact at full
dimension, FGMRES with an exact preconditioner converges in one step and with
the identity reproduces GMRES, the coarse-grid correction is Galerkin
orthogonal, the even-odd Schur solve reproduces the full solve, harmonic Ritz
values at full Krylov dimension are the eigenvalues, and the two-level solver
reaches the dense solution."""
import numpy as np
import pytest

import latgen
import oracle
from helpers import dense, random_op, rel
from oracle import solvers
from oracle.solvers import EvenOdd, TwoLevel


def _small_matrix(n, seed):
    rng = np.random.default_rng(seed)
    return np.eye(n) * 3 + (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n)


def test_gmres_is_minimal_residual():
    n, m = 40, 7
    A = _small_matrix(n, 1)
    b = latgen.gaussian_vector(n, 3)
    x = solvers.gmres_fixed(lambda v: A @ v, b, m)
    K = np.stack([np.linalg.matrix_power(A, j) @ b for j in range(m)], axis=1)
    c = np.linalg.lstsq(A @ K, b, rcond=None)[0]
    assert rel(x, K @ c) < 1e-10
    assert abs(np.linalg.norm(b - A @ x) - np.linalg.norm(b - A @ K @ c)) < 1e-12 * np.linalg.norm(b)


def test_gmres_full_dimension_is_exact():
    n = 24
    A = _small_matrix(n, 2)
    b = latgen.gaussian_vector(n, 4)
    x = solvers.gmres_fixed(lambda v: A @ v, b, n)
    assert rel(x, np.linalg.solve(A, b)) < 1e-12
    assert np.all(solvers.gmres_fixed(lambda v: A @ v, np.zeros(n, complex), 5) == 0)


def test_fgmres_exact_preconditioner_one_step_and_identity_is_gmres():
    n = 30
    A = _small_matrix(n, 5)
    Ai = np.linalg.inv(A)
    b = latgen.gaussian_vector(n, 6)
    x, st = solvers.fgmres(lambda v: A @ v, lambda v: Ai @ v, b, 10, 1e-12, 50)
    assert st.iters == 1 and st.converged
    x1, st1 = solvers.fgmres(lambda v: A @ v, lambda v: v, b, 6, 1e-30, 6)
    assert rel(x1, solvers.gmres_fixed(lambda v: A @ v, b, 6)) < 1e-12


def test_gcr_solves():
    n = 30
    A = _small_matrix(n, 7)
    b = latgen.gaussian_vector(n, 8)
    x, st = solvers.gcr(lambda v: A @ v, b, 8, 1e-11, 200)
    assert st.converged
    assert rel(x, np.linalg.solve(A, b)) < 1e-9


def _two_level(dims, block, agg, N, seed=4, m0=0.3):
    op = random_op(dims, seed=seed, m0=m0)
    tv = latgen.gaussian_fields(dims, N, seed + 7)
    return op, TwoLevel(op, agg, tv, block, mr_iters=4)


def test_coarse_correction_galerkin_orthogonal():
    """With an exact coarse solve, P^H (r - D P D_c^{-1} P^H r) = 0."""
    dims, agg, N = (4, 4, 4, 4), (2, 2, 2, 2), 3
    op, tl = _two_level(dims, (2, 2, 2, 2), agg, N)
    Vc = 16
    Dcd = dense(tl.coarse_apply, (Vc, 2, N))
    r = latgen.gaussian_fields(dims, 1, 1)[0]
    ec = np.linalg.solve(Dcd, tl.restrict(r).ravel()).reshape(Vc, 2, N)
    after = r - op.apply(tl.prolong(ec))
    assert np.linalg.norm(tl.restrict(after)) < 1e-13 * np.linalg.norm(tl.restrict(r))


def test_two_level_fgmres_matches_dense_solution():
    dims, block, agg, N = (4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2), 4
    op, tl = _two_level(dims, block, agg, N, m0=0.1)
    b = latgen.gaussian_fields(dims, 1, 2)[0]
    z, st = solvers.fgmres(op.apply, tl.precond, b, 10, 1e-10, 100)
    assert st.converged
    D = dense(op.apply, b.shape)
    zs = np.linalg.solve(D, b.ravel()).reshape(b.shape)
    assert np.linalg.norm(b - op.apply(z)) <= 1e-10 * np.linalg.norm(b)
    assert rel(z, zs) < 1e-8


def test_even_odd_matches_full():
    dims = (4, 4, 2, 4)
    op = random_op(dims, seed=17, m0=0.2)
    b = latgen.gaussian_fields(dims, 1, 3)[0]
    eo = EvenOdd(op)
    z, st = eo.solve(b, 16, 1e-11, 500)
    assert st.converged
    assert np.linalg.norm(b - op.apply(z)) <= 1e-11 * np.linalg.norm(b)
    # the Schur operator is A_oo - H_oe A_ee^-1 H_eo: check against dense blocks
    V = int(np.prod(dims))
    D = dense(op.apply, (V, 4, 3))
    par = np.repeat(solvers.parity(dims), 12)
    e, o = par == 0, par == 1
    S = D[np.ix_(o, o)] - D[np.ix_(o, e)] @ np.linalg.solve(D[np.ix_(e, e)], D[np.ix_(e, o)])
    fo = np.where(solvers.parity(dims)[:, None, None] == 1, latgen.gaussian_fields(dims, 1, 5)[0], 0)
    got = eo.apply_hat(fo).ravel()[o]
    assert rel(got, S @ fo.ravel()[o]) < 1e-13


def test_harmonic_ritz_petrov_galerkin_and_full_dimension():
    """Harmonic Ritz pairs (target 0) satisfy A phi - theta phi orthogonal to A K_m;
    at full Krylov dimension they are the eigenpairs of smallest modulus."""
    n = 20
    A = _small_matrix(n, 9)
    v0 = latgen.gaussian_vector(n, 1)
    m = 8
    theta, vecs = solvers.harmonic_ritz(lambda v: A @ v, v0, m, 4)
    K = np.stack([np.linalg.matrix_power(A, j) @ v0 for j in range(m)], axis=1)
    Q, _ = np.linalg.qr(K)
    for th, v in zip(theta, vecs):
        # phi lies in K_m and the residual is orthogonal to A K_m
        assert np.linalg.norm(v - Q @ (Q.conj().T @ v)) < 1e-10
        res = A @ v - th * v
        assert np.linalg.norm((A @ Q).conj().T @ res) < 1e-10 * np.linalg.norm(res) * np.linalg.norm(A)
    # modulus ordering
    assert all(abs(theta[i]) <= abs(theta[i + 1]) for i in range(len(theta) - 1))
    theta, vecs = solvers.harmonic_ritz(lambda v: A @ v, v0, n, 5)
    ev = np.linalg.eigvals(A)
    want = ev[np.argsort(np.abs(ev))][:5]
    assert np.max(np.abs(np.sort_complex(theta) - np.sort_complex(want))) < 1e-6


@pytest.mark.slow
def test_bootstrap_invariants():
    """Bootstrap output: orthonormal test vectors whose ||D v_i||^2 are the
    ascending N smallest eigenvalues of the Gram matrix, and an improved
    two-level method compared with random test vectors."""
    dims, block, agg, N = (4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2), 4
    op = random_op(dims, seed=31, m0=0.05)
    rnd = latgen.gaussian_fields(dims, N, 40)
    start = latgen.gaussian_vector(16 * 2 * N, 41)
    tv, tl = solvers.bootstrap(op, block, agg, N, 2, 2, 4, rnd, start)
    G = np.array([[np.vdot(a, b) for b in tv] for a in tv])
    assert np.max(np.abs(G - np.eye(N))) < 1e-12
    nrm = [np.linalg.norm(op.apply(v)) for v in tv]
    assert all(nrm[i] <= nrm[i + 1] + 1e-12 for i in range(N - 1))
    b = latgen.gaussian_fields(dims, 1, 2)[0]
    _, st_boot = solvers.fgmres(op.apply, tl.precond, b, 20, 1e-10, 200)
    _, st_rand = solvers.fgmres(op.apply, TwoLevel(op, agg, rnd, block).precond, b, 20, 1e-10, 200)
    assert st_boot.converged and st_boot.iters <= st_rand.iters
