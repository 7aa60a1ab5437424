"""Pins of the oracle's red-black Schwarz smoother (Section 2, Algorithm 2.1,
block solvers B_i = I [I^T D I]^{-1} I^T) against dense linear algebra: the
block operator is the submatrix of D, a single block with a converged block
solve is D^{-1}, one minimal-residual step minimises the residual, and a
sweep with converged block solves equals the dense product of the colour-c
error propagators with colour 0 first."""
import numpy as np
import pytest

import latgen
import oracle
from helpers import dense, random_op, rel


def _block_id(dims, block, s):
    x = [s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2],
         s // (dims[0] * dims[1] * dims[2])]
    b, stride, col = 0, 1, 0
    for mu in range(4):
        bm = x[mu] // block[mu]
        b += bm * stride
        stride *= dims[mu] // block[mu]
        col += bm
    return b, col % 2


@pytest.mark.parametrize("dims,block", [((4, 4, 4, 4), (2, 2, 2, 2)), ((4, 2, 2, 4), (2, 2, 2, 2)),
                                        ((8, 4, 2, 2), (4, 2, 2, 2))])
def test_block_operator_is_submatrix(dims, block):
    """I^T D I psi equals D applied to psi zeroed outside the block, read on the block."""
    op = random_op(dims, seed=21)
    V = int(np.prod(dims))
    psi = latgen.gaussian_fields(dims, 1, 2)[0]
    nblk = V // int(np.prod(block))
    for blk in (0, nblk - 1, nblk // 3):
        sites = oracle.block_sites(dims, block, blk)
        pad = np.zeros_like(psi)
        pad[sites] = psi[sites]
        want = op.apply(pad)[sites]
        got = op.block_apply(block, blk, psi)
        assert rel(got[sites], want) < 1e-15
        mask = np.ones(V, bool)
        mask[sites] = False
        assert np.all(got[mask] == 0)
        assert sorted(_block_id(dims, block, s)[0] for s in sites) == [blk] * len(sites)


def test_single_block_converged_is_inverse():
    """One block covering the lattice and a converged block solve: z = D^{-1} b."""
    dims = (2, 2, 2, 4)
    op = random_op(dims, seed=4, m0=0.6)
    b = latgen.gaussian_fields(dims, 1, 3)[0]
    z = op.sap(dims, b, np.zeros_like(b), 1, 400)
    D = dense(op.apply, b.shape)
    want = np.linalg.solve(D, b.ravel()).reshape(b.shape)
    assert rel(z, want) < 1e-12


def test_single_mr_step_is_minimal():
    """MR(1) on one block from e = 0 gives z = alpha b minimising ||b - alpha D b||."""
    dims = (2, 2, 2, 2)
    op = random_op(dims, seed=9, m0=0.2)
    b = latgen.gaussian_fields(dims, 1, 6)[0]
    z = op.sap(dims, b, np.zeros_like(b), 1, 1)
    Db = op.apply(b)
    alpha = np.vdot(b, z) / np.vdot(b, b)
    assert rel(z, alpha * b) < 1e-14                    # z lies in span{b}
    f = lambda a: np.linalg.norm((b - a * Db).ravel())   # noqa: E731
    for d in (1e-4, -1e-4, 1e-4j, -1e-4j):
        assert f(alpha + d) > f(alpha)


@pytest.mark.parametrize("shift", [0.0, 0.25 - 0.1j])
def test_sweep_equals_dense_propagator(shift):
    """One sweep with converged block solves equals
    z1 = z0 + sum_{i black} B_i (b - D z_half), z_half = z0 + sum_{i red} B_i (b - D z0),
    with B_i from dense inverses of the block submatrices of D - shift."""
    dims, block = (4, 4, 2, 2), (2, 2, 2, 2)
    op = random_op(dims, seed=13, m0=0.5)
    V = int(np.prod(dims))
    n = V * 12
    D = dense(lambda p: op.apply(p, shift), (V, 4, 3))
    b = latgen.gaussian_fields(dims, 1, 1)[0].ravel()
    z0 = latgen.gaussian_fields(dims, 1, 2)[0].ravel()
    ids = [_block_id(dims, block, s) for s in range(V)]
    nblk = V // 16
    z = z0.copy()
    for c in (0, 1):
        r = b - D @ z
        for blk in range(nblk):
            sites = [s for s in range(V) if ids[s][0] == blk]
            if ids[sites[0]][1] != c:
                continue
            idx = np.concatenate([np.arange(s * 12, s * 12 + 12) for s in sites])
            z[idx] += np.linalg.solve(D[np.ix_(idx, idx)], r[idx])
    got = op.sap(block, b.reshape(V, 4, 3), z0.reshape(V, 4, 3), 1, 300, shift).ravel()
    assert rel(got, z) < 1e-11
    # after the last colour the residual vanishes on the colour-1 blocks
    res = (b - D @ got).reshape(V, 12)
    col1 = np.array([ids[s][1] == 1 for s in range(V)])
    assert np.linalg.norm(res[col1]) / np.linalg.norm(res) < 1e-10
    assert n == D.shape[0]


def test_zero_rhs_zero_start_stays_zero():
    dims = (4, 4, 4, 4)
    op = random_op(dims, seed=1)
    z = op.sap((2, 2, 2, 2), np.zeros((256, 4, 3), complex), np.zeros((256, 4, 3), complex), 2, 4)
    assert np.all(z == 0)


def test_bad_blocks_rejected():
    assert oracle.sap_check((6, 4, 4, 4), (2, 2, 2, 2)) == oracle.ESHAPE    # 3 blocks in x
    assert oracle.sap_check((4, 4, 4, 4), (3, 2, 2, 2)) == oracle.ESHAPE    # does not divide
    assert oracle.sap_check((4, 4, 4, 4), (4, 2, 2, 2)) == oracle.OK        # 1 block in x
