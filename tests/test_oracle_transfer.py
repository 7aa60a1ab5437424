"""Pins of the oracle's aggregation interpolation P, restriction P^H and coarse
operator D_c = P^H D P (Section 3): P^H P = 1, gamma_5 P = P gamma_5^c, the test
vectors lie in range(P), the thin-QR uniqueness, D_c against the explicit
dense product P^H D P (coarse extents 1, 2 and 4), the gamma_5^c-hermiticity of
D_c, and the special case of single-site aggregates with unit test vectors,
where D_c is D itself."""
import numpy as np
import pytest

import latgen
import oracle
from helpers import dense, gamma5_coarse, gamma5_field, random_op, rel


def _setup(dims, agg, N, seed=3):
    op = random_op(dims, seed=seed)
    tv = latgen.gaussian_fields(dims, N, seed + 100)
    P, st = oracle.build_P(dims, agg, tv)
    assert st == oracle.OK
    return op, tv, P


def test_P_orthonormal_and_chiral():
    dims, agg, N = (4, 4, 4, 4), (2, 2, 2, 2), 5
    op, tv, P = _setup(dims, agg, N)
    Vc = 16
    c = latgen.gaussian_vector(Vc * 2 * N, 9).reshape(Vc, 2, N)
    # P^H P = 1
    assert rel(oracle.restrict(dims, agg, P, oracle.prolong(dims, agg, P, c)), c) < 1e-14
    # gamma_5 P = P gamma_5^c
    assert rel(gamma5_field(oracle.prolong(dims, agg, P, c)), oracle.prolong(dims, agg, P, gamma5_coarse(c))) < 1e-15
    # restriction is the adjoint of prolongation
    f = latgen.gaussian_fields(dims, 1, 4)[0]
    lhs = np.vdot(c, oracle.restrict(dims, agg, P, f))
    rhs = np.vdot(oracle.prolong(dims, agg, P, c), f)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    # every test vector lies in range(P): P P^H v = v
    for k in range(N):
        assert rel(oracle.prolong(dims, agg, P, oracle.restrict(dims, agg, P, tv[k])), tv[k]) < 1e-13


def test_P_is_the_unique_thin_qr():
    """Per (aggregate, chirality) the columns of P are Q of the thin QR of the
    cut-up test vectors with a positive real diagonal of R."""
    dims, agg, N = (4, 4, 2, 2), (2, 2, 2, 2), 6
    op, tv, P = _setup(dims, agg, N, seed=8)
    for a in (0, 3):
        sites = oracle.block_sites(dims, agg, a)
        for chi in (0, 1):
            W = tv[:, sites, 2 * chi:2 * chi + 2, :].reshape(N, -1).T
            Q, R = np.linalg.qr(W)
            ph = np.diag(R) / np.abs(np.diag(R))
            Q = Q * ph[None, :]
            got = P[:, sites, 2 * chi:2 * chi + 2, :].reshape(N, -1).T
            assert np.max(np.abs(got - Q)) < 1e-13


def test_rank_deficiency_reported():
    dims, agg = (4, 4, 4, 4), (2, 2, 2, 2)
    tv = latgen.gaussian_fields(dims, 3, 1)
    tv[2] = tv[0] * (0.5 - 2j)
    _, st = oracle.build_P(dims, agg, tv)
    assert st == oracle.ERANK
    tv = latgen.gaussian_fields((2, 2, 2, 2), 97, 1)   # N > 6 * 16
    _, st = oracle.build_P((2, 2, 2, 2), (2, 2, 2, 2), tv)
    assert st == oracle.ERANK


def _dense_P(dims, agg, P):
    N = P.shape[0]
    Vc = oracle.vol(oracle.coarse_dims(dims, agg))
    return dense(lambda c: oracle.prolong(dims, agg, P, c), (Vc, 2, N), nout=int(np.prod(dims)) * 12)


@pytest.mark.parametrize("dims,agg,N", [((4, 4, 4, 4), (2, 2, 2, 2), 4),     # coarse extent 2
                                        ((4, 4, 2, 2), (2, 2, 2, 2), 3),     # coarse extent 1 in z, t
                                        ((8, 2, 2, 2), (2, 2, 2, 2), 3)])    # coarse extent 4 in x
def test_coarse_operator_equals_dense_PHDP(dims, agg, N):
    op, tv, P = _setup(dims, agg, N, seed=5)
    V = int(np.prod(dims))
    D = dense(op.apply, (V, 4, 3))
    Pd = _dense_P(dims, agg, P)
    want = Pd.conj().T @ D @ Pd
    cdims = oracle.coarse_dims(dims, agg)
    Dc = oracle.coarse_build(dims, agg, op.U, op.A, P)
    Vc = oracle.vol(cdims)
    got = dense(lambda c: oracle.coarse_apply(cdims, Dc, c), (Vc, 2, N))
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def test_coarse_operator_apply_identity_large():
    """D_c e = P^H D P e for random e on 8^4 with 4^4 aggregates, and gamma_5^c-hermiticity."""
    dims, agg, N = (8, 8, 8, 8), (4, 4, 4, 4), 4
    op, tv, P = _setup(dims, agg, N, seed=6)
    cdims = oracle.coarse_dims(dims, agg)
    Dc = oracle.coarse_build(dims, agg, op.U, op.A, P)
    e = latgen.gaussian_vector(16 * 2 * N, 1).reshape(16, 2, N)
    f = latgen.gaussian_vector(16 * 2 * N, 2).reshape(16, 2, N)
    want = oracle.restrict(dims, agg, P, op.apply(oracle.prolong(dims, agg, P, e)))
    got = oracle.coarse_apply(cdims, Dc, e)
    assert rel(got, want) < 1e-13
    lhs = np.vdot(f, gamma5_coarse(oracle.coarse_apply(cdims, Dc, gamma5_coarse(e))))
    rhs = np.vdot(oracle.coarse_apply(cdims, Dc, f), e)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_single_site_aggregates_reproduce_D():
    """1^4 aggregates with the 6 unit test vectors: P is a permutation and D_c = D."""
    dims = (4, 2, 2, 4)
    op = random_op(dims, seed=12)
    V = int(np.prod(dims))
    tv = np.zeros((6, V, 4, 3), dtype=np.complex128)
    for k in range(6):
        for sp in range(4):
            if sp % 2 == k // 3:
                tv[k, :, sp, k % 3] = 1.0
    agg = (1, 1, 1, 1)
    P, st = oracle.build_P(dims, agg, tv)
    assert st == 0
    Dc = oracle.coarse_build(dims, agg, op.U, op.A, P)
    psi = latgen.gaussian_fields(dims, 1, 3)[0]
    c = oracle.restrict(dims, agg, P, psi)
    # coarse dof (s, chi, k) <-> fine dof (s, spin 2 chi + k // 3, colour k % 3)
    assert rel(c.reshape(V, 12), psi.reshape(V, 12)) < 1e-15
    got = oracle.coarse_apply(dims, Dc, c)
    assert rel(got.reshape(V, 12), op.apply(psi).reshape(V, 12)) < 1e-14
