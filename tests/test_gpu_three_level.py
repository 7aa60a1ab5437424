"""GPU parity of the three-level method (Section 3 applied to the coarse
equation; through the C ABI) against the oracle: the level-2 setup (the
fine test vectors restricted with P^H, completed by random coarse vectors,
smoothed by the Schwarz method on D_c), the three-level preconditioner, and
flexible GMRES preconditioned by it."""
import numpy as np
import pytest

import latgen
from gpu_common import dev_to_np, lattice, np_to_dev, problem, rel, say
from oracle import multilevel as ml
from oracle import solvers

pytestmark = pytest.mark.gpu

DIMS, BLOCK, AGG, N = (8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 4   # coarse lattice 4^4


def two_levels(seed=7, m0=0.05):
    from paper_1202_2462_amd.mgdd import F64
    op = problem(DIMS, seed=seed, m0=m0, eps=0.5)
    tv = latgen.gaussian_fields(DIMS, N, seed + 30)
    lat = lattice(op, BLOCK)
    lat.build_P(AGG, lat.pack(tv, F64))
    tl = solvers.TwoLevel(op, AGG, tv, BLOCK, mr_iters=4, nu=1)
    return op, lat, tl, tv


def level2(lat, tl, tv, agg2, N2, block2, nu2, seed=60):
    """Level-2 setup on the GPU and the oracle's test vectors for it."""
    from paper_1202_2462_amd.mgdd import F64
    V = tl.Dc.shape[0]
    nres = min(N, N2)
    restricted = [tl.restrict(tv[k]) for k in range(nres)]
    rnd2 = latgen.gaussian_vector(max(N2 - nres, 1) * V * 2 * N, seed).reshape(-1, V, 2, N)[:N2 - nres]
    tv2 = ml.level2_test_vectors(tl.cdims, tl.Dc, block2, restricted, N2, nu2, 4, list(rnd2))
    lat.setup_level2(agg2, N2, block2, random2=np_to_dev(rnd2, F64) if N2 > nres else None, nu2=nu2, mr_iters=4)
    return tv2


@pytest.mark.parametrize("agg2,N2,block2,nu2", [((2, 2, 2, 2), 4, (2, 2, 2, 2), 2),
                                                ((2, 2, 2, 2), 6, (4, 2, 2, 1), 1),
                                                ((1, 1, 2, 4), 3, (2, 2, 2, 2), 0)])
def test_level2_setup_parity(agg2, N2, block2, nu2):
    from paper_1202_2462_amd.mgdd import F64
    say("level-2 setup parity", agg2, N2, block2, nu2)
    op, lat, tl, tv = two_levels()
    tv2 = level2(lat, tl, tv, agg2, N2, block2, nu2)
    P2 = ml.build_P2(tl.cdims, agg2, np.stack(tv2))
    c = latgen.gaussian_vector(2 * tl.Dc.shape[0] * 2 * N, 61).reshape(2, -1, 2, N)
    want = np.stack([ml.restrict2(tl.cdims, agg2, P2, c[i]) for i in range(2)])
    got = dev_to_np(lat.restrict2(np_to_dev(c, F64)))
    say("restrict2 rel", rel(got, want))
    assert rel(got, want) < 1e-9


@pytest.mark.parametrize("agg2,N2,block2", [((2, 2, 2, 2), 4, (2, 2, 2, 2)), ((2, 2, 2, 2), 6, (4, 2, 2, 1))])
def test_three_level_preconditioner_parity(agg2, N2, block2):
    from paper_1202_2462_amd.mgdd import F32, F64
    say("three-level preconditioner parity", agg2, N2, block2)
    op, lat, tl, tv = two_levels()
    tv2 = level2(lat, tl, tv, agg2, N2, block2, 1)
    three = ml.ThreeLevel(tl, agg2, block2, tv2, k2=4, nu2=1, mr2=4, cit=8)
    r = latgen.gaussian_fields(DIMS, 1, 11)
    want = three.precond(r[0])
    r64 = lat.pack(r, F64)
    for prec, tol in ((F64, 1e-9), (F32, 1e-3)):
        got = lat.unpack(lat.precondition3(r64, prec=prec, nu=1, mr_iters=4, k2=4, nu2=1, mr2=4,
                                           coarse_iters=8))[0]
        say(prec, "rel", rel(got, want))
        assert rel(got, want) < tol, (prec, rel(got, want))


def test_three_level_fgmres_matches_oracle():
    from paper_1202_2462_amd.mgdd import F64, MIXED, PLAIN_F64
    say("three-level FGMRES")
    op, lat, tl, tv = two_levels()
    agg2, N2, block2 = (2, 2, 2, 2), 6, (2, 2, 2, 2)
    tv2 = level2(lat, tl, tv, agg2, N2, block2, 2)
    three = ml.ThreeLevel(tl, agg2, block2, tv2, k2=4, nu2=1, mr2=4, cit=8)
    b = latgen.gaussian_fields(DIMS, 1, 12)
    z_or, st_or = solvers.fgmres(op.apply, three.precond, b[0], 20, 1e-10, 400)
    assert st_or.converged
    kw = dict(restart=20, tol=1e-10, maxit=400, levels=3, k2=4, nu2=1, mr2=4, coarse_iters=8, nu=1, mr_iters=4)
    z, stats = lat.solve(lat.pack(b, F64), precision=PLAIN_F64, **kw)
    got = lat.unpack(z)[0]
    st = stats[0]
    say("gpu iters", st.iters, "oracle iters", st_or.iters, "relres", st.relres)
    assert st.converged and st.relres <= 1e-10
    assert np.linalg.norm(b[0] - op.apply(got)) <= 1e-10 * np.linalg.norm(b[0])
    assert abs(st.iters - st_or.iters) <= 1
    assert rel(got, z_or) < 1e-8
    # mixed precision (FP32 preconditioner) reaches the same tolerance, two right-hand sides at once
    b2 = latgen.gaussian_fields(DIMS, 2, 13)
    z2, st2 = lat.solve(lat.pack(b2, F64), precision=MIXED, **kw)
    got2 = lat.unpack(z2)
    for i in range(2):
        say("mixed rhs", i, "iters", st2[i].iters, "relres", st2[i].relres)
        assert st2[i].converged
        assert np.linalg.norm(b2[i] - op.apply(got2[i])) <= 1.5e-10 * np.linalg.norm(b2[i])


def test_three_level_errors():
    from paper_1202_2462_amd.mgdd import EINVAL, ENOTREADY, F64, MgddError
    say("three-level error paths")
    op, lat, tl, tv = two_levels(seed=8)
    b = lat.pack(latgen.gaussian_fields(DIMS, 1, 14), F64)
    with pytest.raises(MgddError) as e:
        lat.solve(b, levels=3)
    assert e.value.code == ENOTREADY
    with pytest.raises(MgddError) as e:
        lat.setup_level2((2, 2, 2, 2), 6, (2, 2, 2, 2), random2=None)   # 2 random coarse vectors needed
    assert e.value.code == EINVAL
    level2(lat, tl, tv, (2, 2, 2, 2), 4, (2, 2, 2, 2), 1)
    with pytest.raises(MgddError) as e:
        lat.solve(b, levels=3, k2=0)
    assert e.value.code == EINVAL
    with pytest.raises(MgddError) as e:
        lat.solve(b, levels=4)
    assert e.value.code == EINVAL
