"""GPU parity on the largest workload lattice, 48^3 x 96, in the launch
configurations its solve uses: the Wilson-clover apply (FP64 and FP32) and
one FP32 Schwarz sweep with 4 MR steps on 4^4 blocks, element by element over
the whole lattice; and the two- and three-level solves of that size
(bootstrap setup in its memory-lean form, mixed-precision FGMRES(30)), judged
by the oracle's residual of the returned solution.

The gauge field is the 16^3 x 32 workload field repeated three times in every
direction, and each input is a 16^3 x 32 Gaussian field repeated the same way
with the sign (-1)^k on the k-th copy in t. The operator maps such fields to
fields of the same form: the small lattice's antiperiodic sign sits on the
hops across t = 31 -> 0, the large lattice's only on the hops across
t = 95 -> 0, and the copies' alternating signs supply it on the inner copy
boundaries (three copies, so the outermost ones carry the same sign). The
clover term is built from closed loops and repeats with the links. With an
even number of 4^4 blocks per copy and direction, the blocks and their colours
repeat as well, and inside a block the MR iteration is odd in the residual
(its step length is unchanged when the residual changes sign), so the sweep
also commutes with the repetition. The oracle's result on 16^3 x 32,
repeated with the signs, is therefore the exact expected result on 48^3 x 96:
a full-size comparison whose host work is that of the small lattice."""
import gc
import json
import os
import time

import numpy as np
import pytest

import latgen
from gpu_common import TOL32, TOL64, rel, say
from oracle.solvers import Operator

SMALL = (16, 16, 16, 32)
REPS = 3
BIG = tuple(REPS * L for L in SMALL)
M0 = -0.2   # any mass: these are operator applications


def repeat_links(U, small=SMALL):
    U4 = U.reshape(small[3], small[2], small[1], small[0], 4, 3, 3)
    return np.ascontiguousarray(np.tile(U4, (REPS, REPS, REPS, REPS, 1, 1, 1)).reshape(-1, 4, 3, 3))


def repeat_spinor(psi, small=SMALL):
    """(V_small, 4, 3) -> (V_big, 4, 3) with the sign (-1)^k on the k-th copy in t"""
    p4 = psi.reshape(small[3], small[2], small[1], small[0], 4, 3)
    big = np.tile(p4, (REPS, REPS, REPS, REPS, 1, 1))
    sign = np.where((np.arange(REPS * small[3]) // small[3]) % 2 == 1, -1.0, 1.0)
    big *= sign[:, None, None, None, None, None]
    return big.reshape(-1, 4, 3)


def test_repetition_commutes_with_the_oracle():
    """the premise, on the CPU: on 4^3 x 8 repeated to 12^3 x 24 (2^4 blocks,
    an even number per copy and direction) the oracle's apply and Schwarz
    sweep on the repeated inputs equal the repeated results"""
    small = (4, 4, 4, 8)
    big = tuple(REPS * L for L in small)
    U = latgen.gauge_field(small, 0.5, 41)
    op_s = Operator(small, U, M0, 1.0)
    op_b = Operator(big, repeat_links(U, small), M0, 1.0)
    psi = latgen.gaussian_fields(small, 1, 42)[0]
    assert rel(op_b.apply(repeat_spinor(psi, small)), repeat_spinor(op_s.apply(psi), small)) < 1e-13
    blk = (2, 2, 2, 2)
    want = repeat_spinor(op_s.sap(blk, psi, np.zeros_like(psi), 1, 4), small)
    x = repeat_spinor(psi, small)
    got = op_b.sap(blk, x, np.zeros_like(x), 1, 4)
    assert rel(got, want) < 1e-12


@pytest.fixture(scope="module")
def c3():
    from paper_1202_2462_amd.mgdd import Lattice
    w = latgen.WORKLOADS["c1"]
    say("generating the 16^3 x 32 gauge field")
    U = latgen.workload_gauge("c1")
    op = Operator(SMALL, U, M0, w["csw"])
    say("48^3 x 96 lattice from the field repeated three times per direction")
    lat = Lattice(BIG, w["block"])
    lat.set_gauge(repeat_links(U), M0, w["csw"])
    yield op, lat
    lat.close()


def test_c3_repetition_of_the_inputs():
    """the construction itself: the repeated field has the big lattice's
    volume, each t copy is the small field times its sign"""
    psi = latgen.gaussian_fields(SMALL, 1, 31)[0]
    big = repeat_spinor(psi).reshape(BIG[3], BIG[2], BIG[1], BIG[0], 4, 3)
    small = psi.reshape(SMALL[3], SMALL[2], SMALL[1], SMALL[0], 4, 3)
    assert big.shape[0] * big.shape[1] * big.shape[2] * big.shape[3] == int(np.prod(BIG))
    for k in range(REPS):
        blk = big[k * SMALL[3]:(k + 1) * SMALL[3], 16:32, 32:48, 0:16]
        assert np.array_equal(blk, (-1) ** k * small)


@pytest.mark.gpu
def test_c3_dirac_full_lattice(c3):
    from paper_1202_2462_amd.mgdd import F32, F64
    op, lat = c3
    psi = latgen.gaussian_fields(SMALL, 1, 32)[0]
    want = repeat_spinor(op.apply(psi))
    x = repeat_spinor(psi)[None]
    for prec, tol in ((F64, TOL64), (F32, TOL32)):
        say("48^3x96 Wilson-clover apply, precision", prec)
        got = lat.unpack(lat.dirac(lat.pack(x, prec)))[0]
        assert rel(got, want) < tol, (prec, rel(got, want))
        assert np.max(np.abs(got - want)) < 50 * tol * np.max(np.abs(want))


@pytest.mark.gpu
def test_c3_schwarz_sweep_full_lattice(c3):
    from paper_1202_2462_amd.mgdd import F32
    op, lat = c3
    w = latgen.WORKLOADS["c3"]
    b = latgen.gaussian_fields(SMALL, 1, 33)[0]
    say("oracle Schwarz sweep on 16^3x32")
    want = repeat_spinor(op.sap(w["block"], b, np.zeros_like(b), 1, w["mr"]))
    say("48^3x96 FP32 Schwarz sweep, 4^4 blocks,", w["mr"], "MR steps")
    z = lat.field(F32, 1)
    lat.sap(lat.pack(repeat_spinor(b)[None], F32), z, 1, w["mr"])
    got = lat.unpack(z)[0]
    assert rel(got, want) < TOL32, rel(got, want)


def tuned_m0(name):
    with open(os.path.join(os.path.dirname(__file__), "golden", "m0.json")) as f:
        d = json.load(f)
    if name not in d:
        pytest.skip(f"no tuned bare mass for {name} in tests/golden/m0.json")
    return float(d[name]["m0"])


# the third level as in the 16^3 x 32 benchmark's three-level variant:
# level-2 aggregates and Schwarz blocks 2^4 (a 6^3 x 12 level-3 lattice), 28
# level-2 test vectors, 8 level-2 FGMRES steps per coarse solve
LEVEL3 = dict(agg2=(2, 2, 2, 2), ntv2=28, block2=(2, 2, 2, 2), setup_nu2=2, k2=8, nu2=1, mr2=4)


@pytest.mark.gpu
@pytest.mark.timeout(900)
@pytest.mark.parametrize("levels", [2, 3])
def test_c3_multilevel_solve_residual(levels):
    """48^3 x 96 workload parameters (4^4 blocks and aggregates, 20 test
    vectors, 3 + 3 bootstrap sweeps in FP32, FGMRES(30) to 1e-10, mixed
    precision) on the repeated field, with the 16^3 x 32 field's tuned mass
    (the repetition keeps its low modes); one Gaussian right-hand side on the
    whole lattice; two levels, and three. The random vectors of the setup come
    from torch's seeded device generator (20 host-generated fields of this size
    take minutes); the check is the oracle's residual, which needs none of
    them."""
    import torch
    from paper_1202_2462_amd.mgdd import F32, F64, MIXED, Lattice
    w = latgen.WORKLOADS["c3"]
    dims, block, agg, N = BIG, w["block"], w["agg"], w["ntv"]
    m0 = tuned_m0("c1")
    U = repeat_links(latgen.workload_gauge("c1"))
    say("48^3x96 solve,", levels, "levels, m0", m0)
    # device memory held in torch's cache by earlier tests is of no use to
    # the library's own allocations (this test needs most of the 288 GB)
    gc.collect()
    torch.cuda.empty_cache()
    lat = Lattice(dims, block)
    lat.set_gauge(U, m0, w["csw"])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3000 + latgen.TAG_TV)
    rnd = torch.randn(lat.field(F64, N).shape, dtype=torch.float64, device="cuda", generator=gen)
    Vc = int(np.prod(dims)) // int(np.prod(agg))
    st = latgen.gaussian_vector(Vc * 2 * N, 3000 + latgen.TAG_ARNOLDI)
    start = torch.tensor(np.stack([st.real, st.imag], -1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.setup(agg, rnd, start, nu=w["nu"], iota=w["iota"], mr_iters=w["mr"], prec=F32)
    del rnd
    torch.cuda.empty_cache()
    l3 = {}
    if levels == 3:
        q = LEVEL3
        r2 = torch.randn((q["ntv2"] - N, Vc, 2, N, 2), dtype=torch.float64, device="cuda", generator=gen)
        lat.setup_level2(q["agg2"], q["ntv2"], q["block2"], random2=r2, nu2=q["setup_nu2"], mr_iters=q["mr2"])
        l3 = dict(levels=3, k2=q["k2"], nu2=q["nu2"], mr2=q["mr2"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    torch.cuda.empty_cache()
    say("levels", levels, "setup", round(t1 - t0, 2), "s")
    b = latgen.gaussian_fields(dims, 1, 3000 + latgen.TAG_RHS)
    bd = lat.pack(b, F64)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    z, stats = lat.solve(bd, precision=MIXED, restart=w["restart"], tol=w["tol"], maxit=3000, **l3)
    t3 = time.perf_counter()
    say("solve", round(t3 - t2, 2), "s, iterations", stats[0].iters, "restarts", stats[0].restarts,
        "GPU relres", stats[0].relres)
    sol = lat.unpack(z)[0]
    del z, bd
    lat.close()
    op = Operator(dims, U, m0, w["csw"])
    res = np.linalg.norm(b[0] - op.apply(sol)) / np.linalg.norm(b[0])
    say("oracle relres", res)
    assert stats[0].converged
    assert res <= 1.1e-10
