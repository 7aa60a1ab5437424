"""Pins of the oracle's third level (the two-level construction applied to
D_c): P2 orthonormal and exact on its test vectors, restriction the adjoint
of prolongation, D_cc equal to P2^H D_c P2 (as maps and as dense matrices,
with level-3 extents 1, 2 and 4), gamma5 structure, level-2 SAP converging
to the dense solve, and the three-level preconditioned FGMRES reaching the
dense solution."""
import numpy as np
import pytest

import latgen
import oracle
from helpers import dense, random_op, rel
from oracle import multilevel as ml
from oracle.solvers import TwoLevel, fgmres

# fine lattice, SAP block, level-1 aggregate, N1
FINE = ((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 4)


@pytest.fixture(scope="module")
def level2():
    dims, block, agg, N1 = FINE
    op = random_op(dims, seed=11, m0=0.2)
    tv = latgen.gaussian_fields(dims, N1, 12)
    tl = TwoLevel(op, agg, tv, block)
    return op, tl


def coarse_random(shape, seed):
    return latgen.gaussian_vector(int(np.prod(shape)), seed).reshape(shape)


@pytest.mark.parametrize("agg2", [(2, 2, 2, 2), (4, 2, 2, 1), (1, 1, 4, 4)])
def test_P2_orthonormal_exact_adjoint(level2, agg2):
    op, tl = level2
    cd = tl.cdims
    N2 = 3
    tv2 = coarse_random((N2,) + tl.Dc.shape[:1] + (2, tl.N), 20)
    P2 = ml.build_P2(cd, agg2, tv2)
    ccd = tuple(L // g for L, g in zip(cd, agg2))
    Vcc = int(np.prod(ccd))
    cc = coarse_random((Vcc, 2, N2), 21)
    # P2^H P2 = 1
    assert rel(ml.restrict2(cd, agg2, P2, ml.prolong2(cd, agg2, P2, cc)), cc) < 1e-13
    # P2 P2^H v = v for every test vector
    for k in range(N2):
        v = ml.prolong2(cd, agg2, P2, ml.restrict2(cd, agg2, P2, tv2[k]))
        assert rel(v, tv2[k]) < 1e-12
    # adjoint
    c = coarse_random(tl.Dc.shape[:1] + (2, tl.N), 22)
    lhs = np.vdot(ml.restrict2(cd, agg2, P2, c), cc)
    rhs = np.vdot(c, ml.prolong2(cd, agg2, P2, cc))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    # chirality blocks: a level-3 vector of one chirality prolongs to that chirality only
    cc0 = cc.copy()
    cc0[:, 1, :] = 0
    assert np.all(ml.prolong2(cd, agg2, P2, cc0)[:, 1, :] == 0)


@pytest.mark.parametrize("agg2", [(2, 2, 2, 2), (1, 1, 4, 4), (4, 4, 1, 1)])
def test_Dcc_equals_P2H_Dc_P2(level2, agg2):
    op, tl = level2
    cd = tl.cdims
    N2 = 2
    tv2 = coarse_random((N2,) + tl.Dc.shape[:1] + (2, tl.N), 30)
    P2 = ml.build_P2(cd, agg2, tv2)
    Dcc = ml.dcc_build(cd, agg2, tl.Dc, P2)
    ccd = tuple(L // g for L, g in zip(cd, agg2))
    Vcc = int(np.prod(ccd))
    # as maps, on random level-3 vectors
    for seed in (31, 32):
        e = coarse_random((Vcc, 2, N2), seed)
        want = ml.restrict2(cd, agg2, P2, ml.apply_Dc(cd, tl.Dc, ml.prolong2(cd, agg2, P2, e)))
        got = oracle.coarse_apply(ccd, Dcc, e)
        assert rel(got, want) < 1e-12
    # as dense matrices
    M = dense(lambda e: oracle.coarse_apply(ccd, Dcc, e), (Vcc, 2, N2))
    Pd = dense(lambda e: ml.prolong2(cd, agg2, P2, e), (Vcc, 2, N2), nout=tl.Dc.shape[0] * 2 * tl.N)
    Dd = dense(lambda c: ml.apply_Dc(cd, tl.Dc, c), tl.Dc.shape[:1] + (2, tl.N))
    assert rel(M, Pd.conj().T @ Dd @ Pd) < 1e-12


def test_Dcc_gamma5_hermitian(level2):
    op, tl = level2
    cd = tl.cdims
    agg2, N2 = (2, 2, 2, 2), 3
    P2 = ml.build_P2(cd, agg2, coarse_random((N2,) + tl.Dc.shape[:1] + (2, tl.N), 40))
    Dcc = ml.dcc_build(cd, agg2, tl.Dc, P2)
    ccd = tuple(L // g for L, g in zip(cd, agg2))
    Vcc = int(np.prod(ccd))
    M = dense(lambda e: oracle.coarse_apply(ccd, Dcc, e), (Vcc, 2, N2))
    g5 = np.tile(np.concatenate([np.ones(N2), -np.ones(N2)]), Vcc)
    assert rel(g5[:, None] * M * g5[None, :], M.conj().T) < 1e-12


def test_coarse_sap_single_block_converges_to_dense_solve(level2):
    op, tl = level2
    cd = tl.cdims
    shape = tl.Dc.shape[:1] + (2, tl.N)
    b = coarse_random(shape, 50)
    z = ml.coarse_sap(cd, tl.Dc, cd, b, np.zeros_like(b), 1, 60)
    Dd = dense(lambda c: ml.apply_Dc(cd, tl.Dc, c), shape)
    want = np.linalg.solve(Dd, b.ravel()).reshape(shape)
    assert rel(z, want) < 1e-8


def test_coarse_sap_residual_vanishes_on_last_colour(level2):
    """with (nearly) exact block solves the residual after a sweep vanishes on
    the blocks of the colour treated last"""
    op, tl = level2
    cd, block2 = tl.cdims, (2, 2, 2, 2)
    shape = tl.Dc.shape[:1] + (2, tl.N)
    b = coarse_random(shape, 51)
    z = ml.coarse_sap(cd, tl.Dc, block2, b, np.zeros_like(b), 1, 60)
    r = b - ml.apply_Dc(cd, tl.Dc, z)
    last = np.array([ml.block_of(cd, block2, a)[1] == 1 for a in range(shape[0])])
    assert np.abs(r[last]).max() < 1e-9 * np.abs(b).max()
    assert np.abs(r[~last]).max() > 1e-3 * np.abs(b).max()


def test_three_level_fgmres_reaches_dense_solution():
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op = random_op(dims, seed=13, m0=0.2)
    N1, N2 = 6, 4
    tv = latgen.gaussian_fields(dims, N1, 14)
    zero = np.zeros_like(tv[0])
    tv = np.stack([op.sap(block, zero, v, 1, 4) for v in tv])
    tl = TwoLevel(op, (2, 2, 2, 2), tv, block)
    restricted = [tl.restrict(v) for v in tv]
    rnd = [coarse_random(restricted[0].shape, 60 + i) for i in range(N2)]
    tv2 = ml.level2_test_vectors(tl.cdims, tl.Dc, (2, 2, 2, 2), restricted, N2, 1, 4, rnd)
    three = ml.ThreeLevel(tl, (2, 2, 2, 2), (2, 2, 2, 2), tv2, k2=4)
    b = latgen.gaussian_fields(dims, 1, 15)[0]
    z, st = fgmres(op.apply, three.precond, b, 20, 1e-10, 200)
    assert st.converged
    assert np.linalg.norm(b - op.apply(z)) <= 1e-10 * np.linalg.norm(b)


def qr_positive(cols):
    """Q of the thin QR of the matrix with the given columns, diagonal of R made positive."""
    A = np.stack([np.asarray(c).ravel() for c in cols], axis=1)
    Q, R = np.linalg.qr(A)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Q * ph[None, :]


def test_level2_test_vectors_are_qr_of_smoothed_vectors(level2):
    """nu2 = 0: the Q factor (positive diagonal of R) of the restricted vectors
    completed by the random ones; each smoothing round: one level-2 SAP sweep
    with b = 0 from every vector, then the Q factor again (numpy QR instead of
    Gram-Schmidt)"""
    op, tl = level2
    cd, block2 = tl.cdims, (2, 2, 2, 2)
    shape = tl.Dc.shape[:1] + (2, tl.N)
    restricted = [coarse_random(shape, 70 + i) for i in range(tl.N)]
    rnd = [coarse_random(shape, 80 + i) for i in range(3)]
    N2 = tl.N + 2
    v0 = ml.level2_test_vectors(cd, tl.Dc, block2, restricted, N2, 0, 4, rnd)
    Q0 = qr_positive(restricted + rnd[:2])
    assert rel(np.stack([v.ravel() for v in v0], 1), Q0) < 1e-12
    v2 = ml.level2_test_vectors(cd, tl.Dc, block2, restricted, N2, 2, 4, rnd)
    Q = Q0
    for _ in range(2):
        sm = [ml.coarse_sap(cd, tl.Dc, block2, np.zeros(shape), Q[:, k].reshape(shape), 1, 4) for k in range(N2)]
        Q = qr_positive(sm)
    got = np.stack([v.ravel() for v in v2], 1)
    assert rel(got, Q) < 1e-10
    assert np.abs(got.conj().T @ got - np.eye(N2)).max() < 1e-12
    # fewer level-2 vectors than fine ones: only the first restricted vectors are used
    v3 = ml.level2_test_vectors(cd, tl.Dc, block2, restricted, 2, 0, 4, rnd)
    assert rel(np.stack([v.ravel() for v in v3], 1), qr_positive(restricted[:2])) < 1e-12


def test_level2_correction_is_galerkin(level2):
    """with the coarsest equation solved exactly (GMRES at the full dimension
    of D_cc) and no level-2 smoothing, M2 is the coarse-grid correction of
    D_c: P2^H (r - D_c M2 r) = 0"""
    op, tl = level2
    cd, agg2, N2 = tl.cdims, (2, 2, 2, 2), 3
    shape = tl.Dc.shape[:1] + (2, tl.N)
    tv2 = [coarse_random(shape, 90 + i) for i in range(N2)]
    ncc = int(np.prod([L // g for L, g in zip(cd, agg2)])) * 2 * N2
    three = ml.ThreeLevel(tl, agg2, (2, 2, 2, 2), tv2, nu2=0, cit=ncc)
    r = coarse_random(shape, 95)
    e = three.M2(r)
    res = ml.restrict2(cd, agg2, three.P2, r - ml.apply_Dc(cd, tl.Dc, e))
    assert np.abs(res).max() < 1e-9 * np.abs(ml.restrict2(cd, agg2, three.P2, r)).max()
    assert rel(e, np.zeros_like(e)) > 0.1


def test_level2_coarse_solve_exact_with_exact_smoother(level2):
    """one block covering the coarse lattice with converged MR makes M2 = D_c^{-1},
    so one flexible GMRES step solves the coarse equation"""
    op, tl = level2
    cd = tl.cdims
    shape = tl.Dc.shape[:1] + (2, tl.N)
    tv2 = [coarse_random(shape, 100 + i) for i in range(3)]
    three = ml.ThreeLevel(tl, (2, 2, 2, 2), cd, tv2, k2=1, nu2=1, mr2=60, cit=4)
    b = coarse_random(shape, 105)
    Dd = dense(lambda c: ml.apply_Dc(cd, tl.Dc, c), shape)
    want = np.linalg.solve(Dd, b.ravel()).reshape(shape)
    assert rel(three.coarse_solve(b), want) < 1e-7
