"""GPU parity of the third level (through the C ABI) against the oracle:
P2 (restriction and prolongation), D_cc = P2^H D_c P2, on several level-2
aggregate shapes (level-3 extents 1, 2 and 4), the Schwarz smoother on D_c
(several block shapes, including one block per direction and one-site
blocks), and the error paths."""
import numpy as np
import pytest

import latgen
from gpu_common import TOL32, TOL64, lattice, problem, rel, say
from gpu_common import dev_to_np as to_np
from gpu_common import np_to_dev as to_dev
from oracle import multilevel as ml
from oracle.solvers import TwoLevel

pytestmark = pytest.mark.gpu

FINE = ((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 4)


def two_levels(seed=3, fine=FINE):
    from paper_1202_2462_amd.mgdd import F64
    dims, block, agg, N1 = fine
    op = problem(dims, seed=seed, m0=0.2)
    tv = latgen.gaussian_fields(dims, N1, seed + 40)
    lat = lattice(op, block)
    lat.build_P(agg, lat.pack(tv, F64))
    tl = TwoLevel(op, agg, tv, block)
    return op, lat, tl


def coarse_random(shape, seed):
    return latgen.gaussian_vector(int(np.prod(shape)), seed).reshape(shape)


@pytest.mark.parametrize("agg2,N2", [((2, 2, 2, 2), 3), ((1, 1, 4, 4), 4), ((4, 2, 2, 1), 5)])
def test_P2_and_Dcc_parity(agg2, N2):
    from paper_1202_2462_amd.mgdd import F32, F64
    say("level-2 parity", agg2, N2)
    op, lat, tl = two_levels()
    cd = tl.cdims
    tv2 = coarse_random((N2, tl.Dc.shape[0], 2, tl.N), 70)
    lat.build_P2(agg2, to_dev(tv2, F64))
    P2 = ml.build_P2(cd, agg2, tv2)
    Dcc = ml.dcc_build(cd, agg2, tl.Dc, P2)
    ccd = tuple(L // g for L, g in zip(cd, agg2))
    Vcc = int(np.prod(ccd))
    c = coarse_random((2, tl.Dc.shape[0], 2, tl.N), 71)
    cc = coarse_random((2, Vcc, 2, N2), 72)
    want_r = np.stack([ml.restrict2(cd, agg2, P2, c[i]) for i in range(2)])
    want_p = np.stack([ml.prolong2(cd, agg2, P2, cc[i]) for i in range(2)])
    import oracle
    want_a = np.stack([oracle.coarse_apply(ccd, Dcc, cc[i]) for i in range(2)])
    for prec, tol in ((F64, TOL64), (F32, TOL32)):
        got_r = to_np(lat.restrict2(to_dev(c, prec)))
        assert rel(got_r, want_r) < tol, (prec, rel(got_r, want_r))
        got_p = to_np(lat.prolong2(to_dev(cc, prec)))
        assert rel(got_p, want_p) < tol, (prec, rel(got_p, want_p))
        got_a = to_np(lat.coarse2_apply(to_dev(cc, prec)))
        assert rel(got_a, want_a) < tol, (prec, rel(got_a, want_a))
    # D_cc as a map equals P2^H D_c P2 on the GPU as well
    e = to_dev(cc, F64)
    lhs = to_np(lat.coarse2_apply(e))
    rhs = to_np(lat.restrict2(lat.coarse_apply(lat.prolong2(e))))
    assert rel(lhs, rhs) < TOL64


def test_level2_errors():
    from paper_1202_2462_amd.mgdd import ENOTREADY, ERANK, ESHAPE, F64, MgddError, mgdd_coarse2_apply
    say("level-2 error paths")
    op, lat, tl = two_levels(seed=5)
    x = lat.coarse_field(F64, 1)
    with pytest.raises(MgddError) as e:
        mgdd_coarse2_apply(lat.ctx, F64, 1, x, lat.coarse_field(F64, 1))
    assert e.value.code == ENOTREADY
    tv2 = coarse_random((3, tl.Dc.shape[0], 2, tl.N), 80)
    with pytest.raises(MgddError) as e:
        lat.build_P2((3, 2, 2, 2), to_dev(tv2, F64))
    assert e.value.code == ESHAPE
    tv2[2] = (1 - 2j) * tv2[0]
    with pytest.raises(MgddError) as e:
        lat.build_P2((2, 2, 2, 2), to_dev(tv2, F64))
    assert e.value.code == ERANK


FINE2 = ((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 4)   # coarse lattice 4^4


@pytest.mark.parametrize("fine,block2", [(FINE2, (2, 2, 2, 2)), (FINE2, (4, 2, 2, 1)), (FINE, (1, 1, 1, 1)),
                                         (FINE, (2, 2, 2, 2)), (FINE, (2, 1, 2, 1))])
def test_coarse_sap_parity(fine, block2):
    from paper_1202_2462_amd.mgdd import F32, F64
    say("coarse Schwarz parity", fine[2], block2)
    op, lat, tl = two_levels(seed=4, fine=fine)
    V = tl.Dc.shape[0]
    b = coarse_random((2, V, 2, tl.N), 90)
    z0 = coarse_random((2, V, 2, tl.N), 91)
    z0[0] = 0
    for nsweeps, mr in ((1, 4), (2, 3), (0, 4), (1, 0)):
        want = np.stack([ml.coarse_sap(tl.cdims, tl.Dc, block2, b[i], z0[i], nsweeps, mr) for i in range(2)])
        for prec, tol in ((F64, 1e-11), (F32, 1e-4)):
            z = to_dev(z0, prec)
            lat.coarse_sap(block2, to_dev(b, prec), z, nsweeps=nsweeps, mr_iters=mr)
            got = to_np(z)
            assert rel(got, want) < tol, (nsweeps, mr, prec, rel(got, want))
    # the smoother reduces the residual of D_c z = b
    z = to_dev(np.zeros_like(b), F64)
    lat.coarse_sap(block2, to_dev(b, F64), z, nsweeps=3, mr_iters=4)
    r = to_np(to_dev(b, F64) - lat.coarse_apply(z))
    assert np.linalg.norm(r) < np.linalg.norm(b)


def test_coarse_sap_errors():
    from paper_1202_2462_amd.mgdd import EINVAL, ESHAPE, F64, MgddError
    say("coarse Schwarz error paths")
    op, lat, tl = two_levels(seed=6, fine=FINE2)
    b = lat.coarse_field(F64, 1)
    z = lat.coarse_field(F64, 1)
    for blk in ((3, 2, 2, 2), (4, 4, 4, 4), (0, 2, 2, 2)):   # not dividing; 2N*256 > 1024; empty
        with pytest.raises(MgddError) as e:
            lat.coarse_sap(blk, b, z)
        assert e.value.code == ESHAPE, blk
    with pytest.raises(MgddError) as e:
        lat.coarse_sap((2, 2, 2, 2), b, b)
    assert e.value.code == EINVAL
