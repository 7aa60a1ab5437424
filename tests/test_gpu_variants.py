"""GPU parity (through the C ABI) of the paper's protocol variants against
the oracle: Schwarz sweeps with GMRES(k) block solves (the block solver of
Section 4) and additive Schwarz (Section 2), multi-RHS, shifted, on blocks
that span a lattice direction; flexible GMRES preconditioned by the
two-level method with GMRES(3) blocks and restart 25 (the paper's
protocol); CGN, the paper's comparator; error paths."""
import numpy as np
import pytest

import latgen
import oracle
from gpu_common import TOL32, TOL64, lattice, problem, rel, say
from oracle import solvers

pytestmark = pytest.mark.gpu

CASES = [((8, 8, 8, 8), (4, 4, 4, 4)), ((4, 8, 8, 8), (4, 4, 4, 4)), ((8, 8, 8, 16), (4, 4, 4, 2))]


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("solver,k,additive", [(oracle.BLOCK_GMRES, 1, False), (oracle.BLOCK_GMRES, 3, False),
                                               (oracle.BLOCK_GMRES, 2, True), (oracle.BLOCK_MR, 4, True)])
def test_schwarz_variant_parity(dims, block, solver, k, additive):
    from paper_1202_2462_amd.mgdd import F32, F64
    say("schwarz variant parity", dims, block, solver, k, additive)
    op = problem(dims, seed=9, m0=0.2)
    lat = lattice(op, block)
    b = latgen.gaussian_fields(dims, 2, 30)
    z0 = latgen.gaussian_fields(dims, 2, 31)
    z0[1] = 0
    want = np.stack([op.schwarz(block, b[r], z0[r], 2, k, solver, additive) for r in range(2)])
    for prec, tol in ((F64, 1e-11), (F32, 2e-5)):
        z = lat.pack(z0, prec)
        lat.schwarz(lat.pack(b, prec), z, nsweeps=2, k=k, block_solver=solver, additive=additive)
        got = lat.unpack(z)
        for r in range(2):
            assert rel(got[r], want[r]) < tol, (prec, r, rel(got[r], want[r]))


def test_schwarz_gmres_shifted_and_degenerate():
    from paper_1202_2462_amd.mgdd import BLOCK_GMRES, F64
    dims, block = CASES[0]
    say("schwarz gmres shifted / zero rhs")
    op = problem(dims, seed=10, m0=0.2)
    lat = lattice(op, block)
    b = latgen.gaussian_fields(dims, 1, 32)
    z0 = latgen.gaussian_fields(dims, 1, 33)
    shift = 0.3 - 0.2j
    want = op.schwarz(block, b[0], z0[0], 1, 3, oracle.BLOCK_GMRES, False, shift)
    z = lat.pack(z0, F64)
    lat.schwarz(lat.pack(b, F64), z, nsweeps=1, k=3, block_solver=BLOCK_GMRES, shift=shift)
    assert rel(lat.unpack(z)[0], want) < TOL64 * 10
    z = lat.field(F64, 1)   # b = 0, z = 0: beta = 0 on every block, z stays 0
    lat.schwarz(lat.field(F64, 1), z, nsweeps=2, k=3, block_solver=BLOCK_GMRES)
    assert np.all(lat.unpack(z) == 0)


def test_fgmres_with_paper_protocol_matches_oracle():
    """two-level FGMRES(25), GMRES(3) block solves, one sweep, coarse GMRES(12)"""
    from paper_1202_2462_amd.mgdd import BLOCK_GMRES, F64, MIXED, PLAIN_F64
    dims, block, agg, N = (8, 8, 8, 8), (4, 4, 4, 4), (4, 4, 4, 4), 8
    say("fgmres paper protocol", dims)
    op = problem(dims, seed=11, m0=0.05, eps=0.5)
    lat = lattice(op, block)
    tv = latgen.gaussian_fields(dims, N, 34)
    zero = np.zeros_like(tv[0])
    tv = np.stack([op.sap(block, zero, v, 2, 4) for v in tv])
    lat.build_P(agg, lat.pack(tv, F64))
    tl = solvers.TwoLevel(op, agg, tv, block, mr_iters=3, block_solver=oracle.BLOCK_GMRES)
    b = latgen.gaussian_fields(dims, 1, 35)
    z_or, st_or = solvers.fgmres(op.apply, tl.precond, b[0], 25, 1e-10, 400)
    assert st_or.converged
    kw = dict(restart=25, tol=1e-10, maxit=400, mr_iters=3, block_solver=BLOCK_GMRES)
    z, stats = lat.solve(lat.pack(b, F64), precision=PLAIN_F64, **kw)
    got = lat.unpack(z)[0]
    say("gpu iters", stats[0].iters, "oracle iters", st_or.iters)
    assert stats[0].converged and abs(stats[0].iters - st_or.iters) <= 1
    assert rel(got, z_or) < 1e-8
    # additive smoother and mixed precision reach the tolerance too
    z, stats = lat.solve(lat.pack(b, F64), precision=MIXED, additive=True, **kw)
    got = lat.unpack(z)[0]
    say("additive mixed iters", stats[0].iters)
    assert stats[0].converged
    assert np.linalg.norm(b[0] - op.apply(got)) <= 1.5e-10 * np.linalg.norm(b[0])


def test_cgn_matches_oracle():
    from paper_1202_2462_amd.mgdd import F64, SOLVER_CGN
    dims = (8, 8, 8, 8)
    say("cgn", dims)
    op = problem(dims, seed=12, m0=0.1)
    lat = lattice(op, (4, 4, 4, 4))
    b = latgen.gaussian_fields(dims, 2, 36)
    want = [solvers.cgn(op.apply, op.apply_dag, b[r], 1e-10, 20000) for r in range(2)]
    z, stats = lat.solve(lat.pack(b, F64), solver=SOLVER_CGN, tol=1e-10, maxit=20000)
    got = lat.unpack(z)
    for r in range(2):
        x_or, st_or = want[r]
        say("rhs", r, "gpu iters", stats[r].iters, "restarts", stats[r].restarts, "oracle", st_or.iters,
            st_or.restarts)
        assert stats[r].converged and st_or.converged
        assert np.linalg.norm(b[r] - op.apply(got[r])) <= 1e-10 * np.linalg.norm(b[r])
        assert abs(stats[r].iters - st_or.iters) <= max(2, st_or.iters // 100)
        assert rel(got[r], x_or) < 1e-7
    # maxit reached: not converged, the iterate and its residual returned
    z, stats = lat.solve(lat.pack(b[:1], F64), solver=SOLVER_CGN, tol=1e-10, maxit=5, allow_noconv=True)
    x5, st5 = solvers.cgn(op.apply, op.apply_dag, b[0], 1e-10, 5)
    assert stats[0].iters == 5 and not stats[0].converged
    assert rel(lat.unpack(z)[0], x5) < 1e-10


def test_variant_errors():
    from paper_1202_2462_amd.mgdd import BLOCK_GMRES, EINVAL, F64, MgddError
    dims, block = CASES[0]
    say("variant error paths")
    op = problem(dims, seed=13)
    lat = lattice(op, block)
    b, z = lat.field(F64, 1), lat.field(F64, 1)
    for kw in (dict(k=4, block_solver=BLOCK_GMRES), dict(k=0, block_solver=BLOCK_GMRES),
               dict(k=2, block_solver=7), dict(k=2, additive=True, shift=0.1)):
        with pytest.raises(MgddError) as e:
            lat.schwarz(b, z, **kw)
        assert e.value.code == EINVAL, kw
