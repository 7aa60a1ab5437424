"""GPU end-to-end: FGMRES with the two-level preconditioner, plain and
even-odd GCR, and the bootstrap setup, against the oracle's solutions."""
import numpy as np
import pytest

import latgen
from gpu_common import lattice, problem, rel, say
from helpers import aligned_difference
from oracle import solvers

pytestmark = pytest.mark.gpu


def small_problem(seed=3, m0=0.05):
    dims, block, agg, N = (8, 8, 8, 8), (4, 4, 4, 4), (4, 4, 4, 4), 8
    op = problem(dims, seed=seed, m0=m0, eps=0.5)
    return dims, block, agg, N, op


def test_fgmres_plain_matches_oracle():
    from paper_1202_2462_amd.mgdd import F64, PLAIN_F64
    dims, block, agg, N, op = small_problem()
    say("fgmres plain fp64", dims)
    lat = lattice(op, block)
    tv = latgen.gaussian_fields(dims, N, 77)
    lat.build_P(agg, lat.pack(tv, F64))
    tl = solvers.TwoLevel(op, agg, tv, block, mr_iters=4)
    b = latgen.gaussian_fields(dims, 1, 3)
    z_or, st_or = solvers.fgmres(op.apply, tl.precond, b[0], 20, 1e-10, 400)
    assert st_or.converged
    z, stats = lat.solve(lat.pack(b, F64), precision=PLAIN_F64, restart=20, tol=1e-10, maxit=400)
    got = lat.unpack(z)[0]
    st = stats[0]
    say("gpu iters", st.iters, "oracle iters", st_or.iters, "relres", st.relres)
    assert st.converged and st.relres <= 1e-10
    assert np.linalg.norm(b[0] - op.apply(got)) <= 1e-10 * np.linalg.norm(b[0])
    assert abs(st.iters - st_or.iters) <= 1
    assert rel(got, z_or) < 1e-8


def test_fgmres_long_cycles_match_oracle():
    """FGMRES(40) with a weak preconditioner (2 test vectors, one coarse GMRES
    step, one MR step per block): the cycles run past 32 basis vectors, where
    the outer Gram-Schmidt passes go over the basis in two launches."""
    from paper_1202_2462_amd.mgdd import F64, PLAIN_F64
    dims, block, agg, _, op = small_problem()
    say("fgmres(40) long cycles", dims)
    lat = lattice(op, block)
    tv = latgen.gaussian_fields(dims, 2, 77)
    lat.build_P(agg, lat.pack(tv, F64))
    tl = solvers.TwoLevel(op, agg, tv, block, mr_iters=1, coarse_iters=1)
    b = latgen.gaussian_fields(dims, 1, 3)
    z_or, st_or = solvers.fgmres(op.apply, tl.precond, b[0], 40, 1e-10, 400)
    assert st_or.converged and st_or.iters > 40
    z, stats = lat.solve(lat.pack(b, F64), precision=PLAIN_F64, restart=40, tol=1e-10, maxit=400,
                         coarse_iters=1, mr_iters=1)
    got = lat.unpack(z)[0]
    st = stats[0]
    say("gpu iters", st.iters, "oracle iters", st_or.iters, "relres", st.relres)
    assert st.converged and st.relres <= 1e-10
    assert np.linalg.norm(b[0] - op.apply(got)) <= 1e-10 * np.linalg.norm(b[0])
    assert abs(st.iters - st_or.iters) <= 1
    assert rel(got, z_or) < 1e-8


def test_fgmres_mixed_reaches_tolerance():
    from paper_1202_2462_amd.mgdd import F64, MIXED
    dims, block, agg, N, op = small_problem(seed=5)
    say("fgmres mixed", dims)
    lat = lattice(op, block)
    tv = latgen.gaussian_fields(dims, N, 78)
    lat.build_P(agg, lat.pack(tv, F64))
    b = latgen.gaussian_fields(dims, 2, 4)
    z, stats = lat.solve(lat.pack(b, F64), precision=MIXED, restart=20, tol=1e-10, maxit=400)
    got = lat.unpack(z)
    for r in range(2):
        assert stats[r].converged
        assert np.linalg.norm(b[r] - op.apply(got[r])) <= 1e-10 * np.linalg.norm(b[r])


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_fgmres_equals_single_solves(precision):
    """Several right-hand sides in one batched FGMRES: each has its own
    Krylov space and stopping test, so every solution and iteration count
    equals that of solving it alone (the per-segment reductions use the same
    grid and order). The batch mixes a zero right-hand side, a point source
    and Gaussian ones, so they converge after different iteration counts."""
    from paper_1202_2462_amd.mgdd import F64
    dims, block, agg, N, op = small_problem(seed=6)
    say("batched fgmres precision", precision, dims)
    lat = lattice(op, block)
    lat.build_P(agg, lat.pack(latgen.gaussian_fields(dims, N, 79), F64))
    g = latgen.gaussian_fields(dims, 2, 8)
    pt = latgen.point_sources(dims, 9)[4:5]
    b = np.concatenate([g[:1], np.zeros_like(g[:1]), pt, 1e-3 * g[1:]], 0)
    zb, sb = lat.solve(lat.pack(b, F64), precision=precision, restart=8, tol=1e-10, maxit=400)
    got = lat.unpack(zb)
    for r in range(b.shape[0]):
        z1, s1 = lat.solve(lat.pack(b[r:r + 1], F64), precision=precision, restart=8, tol=1e-10, maxit=400)
        one = lat.unpack(z1)[0]
        say("rhs", r, "batched iters", sb[r].iters, "restarts", sb[r].restarts, "single", s1[0].iters)
        assert sb[r].converged and s1[0].converged
        assert sb[r].iters == s1[0].iters and sb[r].restarts == s1[0].restarts
        nb = np.linalg.norm(b[r])
        if nb == 0:
            assert np.all(got[r] == 0)
            continue
        assert np.linalg.norm(b[r] - op.apply(got[r])) <= 1e-10 * nb
        assert np.abs(got[r] - one).max() <= 1e-12 * np.abs(one).max()


def test_batched_coarse_solve_and_preconditioner_equal_single():
    from paper_1202_2462_amd.mgdd import F32, F64
    dims, block, agg, N, op = small_problem(seed=7)
    say("batched coarse solve / preconditioner", dims)
    lat = lattice(op, block)
    lat.build_P(agg, lat.pack(latgen.gaussian_fields(dims, N, 80), F64))
    for prec in (F64, F32):
        cb = lat.coarse_field(prec, 3)
        cb.normal_()
        xb = lat.coarse_solve(cb, 12)
        for r in range(3):
            x1 = lat.coarse_solve(cb[r:r + 1].clone(), 12)
            assert (xb[r] - x1[0]).abs().max().item() <= 1e-12 * x1.abs().max().item()
        r64 = lat.pack(latgen.gaussian_fields(dims, 3, 11), F64)
        zb = lat.precondition(r64, prec=prec)
        for r in range(3):
            z1 = lat.precondition(r64[r:r + 1].clone(), prec=prec)
            assert (zb[r] - z1[0]).abs().max().item() <= 1e-12 * z1.abs().max().item()


@pytest.mark.parametrize("solver", [1, 2])
def test_gcr_and_even_odd_gcr(solver):
    from paper_1202_2462_amd.mgdd import F64
    dims = (8, 8, 4, 8)
    say("gcr solver", solver, dims)
    op = problem(dims, seed=9, m0=0.3)
    lat = lattice(op, (4, 4, 4, 4))
    b = latgen.gaussian_fields(dims, 1, 5)
    z, stats = lat.solve(lat.pack(b, F64), solver=solver, restart=16, tol=1e-10, maxit=3000)
    got = lat.unpack(z)[0]
    assert stats[0].converged
    assert np.linalg.norm(b[0] - op.apply(got)) <= 1e-10 * np.linalg.norm(b[0])
    z_or, st_or = solvers.gcr(op.apply, b[0], 16, 1e-12, 5000)
    assert rel(got, z_or) < 1e-7


def test_even_odd_gcr_with_an_indefinite_clover_term():
    """m0 = -9 makes every clover block negative definite: the clover inverse
    of the even-odd operator then comes from the Gauss-Jordan fallback
    instead of the Cholesky factorisation (D itself stays well conditioned)."""
    from paper_1202_2462_amd.mgdd import F64, SOLVER_GCR_EO
    dims = (8, 8, 4, 8)
    say("even-odd gcr, clover term not positive definite", dims)
    op = problem(dims, seed=9, m0=-9.0)
    lat = lattice(op, (4, 4, 4, 4))
    b = latgen.gaussian_fields(dims, 1, 5)
    z, stats = lat.solve(lat.pack(b, F64), solver=SOLVER_GCR_EO, restart=16, tol=1e-10, maxit=3000)
    got = lat.unpack(z)[0]
    assert stats[0].converged
    assert np.linalg.norm(b[0] - op.apply(got)) <= 1e-10 * np.linalg.norm(b[0])
    z_or, st_or = solvers.gcr(op.apply, b[0], 16, 1e-12, 5000)
    assert rel(got, z_or) < 1e-7


def test_solver_degenerate_cases():
    from paper_1202_2462_amd.mgdd import ENAN, ENOCONV, F64, MgddError
    dims, block, agg, N, op = small_problem()
    say("solver degenerate cases")
    lat = lattice(op, block)
    lat.build_P(agg, lat.pack(latgen.gaussian_fields(dims, N, 1), F64))
    # zero right-hand side: immediate success with z = 0
    z, stats = lat.solve(lat.field(F64, 1))
    assert stats[0].converged and stats[0].iters == 0 and np.all(lat.unpack(z) == 0)
    # maxit too small: ENOCONV with the stats filled in
    b = lat.pack(latgen.gaussian_fields(dims, 1, 2), F64)
    with pytest.raises(MgddError) as e:
        lat.solve(b, maxit=1)
    assert e.value.code == ENOCONV
    z, stats = lat.solve(b, maxit=1, allow_noconv=True)
    assert stats[0].iters == 1 and not stats[0].converged and 0 < stats[0].relres < 1
    # NaN in the right-hand side
    bad = b.clone()
    bad[0, 0, 0, 0] = float("nan")
    with pytest.raises(MgddError) as e:
        lat.solve(bad)
    assert e.value.code == ENAN


def _boot_inputs(dims, N):
    import torch
    rnd = latgen.gaussian_fields(dims, N, 90)
    Vc = 16
    start = latgen.gaussian_vector(Vc * 2 * N, 91)
    st = torch.tensor(np.stack([start.real, start.imag], -1), dtype=torch.float64, device="cuda")
    return rnd, start, st


# chunk 0: the full form of the setup at this size; chunk 3: the memory-lean
# form of large lattices (sweeps over chunks of vectors, the second part's
# Gram matrix as <w_i, D^H D w_j> over column chunks), forced here, with
# ragged chunks (8 vectors; 16 columns cut at the end of the 8 new ones)
@pytest.mark.parametrize("chunk", [0, 3])
def test_bootstrap_part1_matches_oracle(chunk):
    """First setup part only (nu rounds of one Schwarz sweep with b = 0 and a
    global Gram-Schmidt): a well-conditioned map, compared element-wise."""
    from paper_1202_2462_amd.mgdd import F32, F64
    dims, block, agg, N, op = small_problem(seed=11, m0=0.02)
    say("bootstrap part 1", dims, "chunk", chunk)
    lat = lattice(op, block)
    rnd, start, st = _boot_inputs(dims, N)
    tv_or, _ = solvers.bootstrap(op, block, agg, N, 3, 3, 4, rnd, start, n_part2=0)
    lat.setup(agg, lat.pack(rnd, F64), st, nu=3, iota=3, mr_iters=4, n_part2=0, prec=F64, chunk=chunk)
    tv_gpu = lat.unpack(lat.test_vectors())
    assert rel(tv_gpu, tv_or) < 1e-10
    lat.setup(agg, lat.pack(rnd, F64), st, nu=3, iota=3, mr_iters=4, n_part2=0, prec=F32, chunk=chunk)
    assert rel(lat.unpack(lat.test_vectors()), tv_or) < 1e-4


def test_bootstrap_chunk_error():
    """a negative chunk is refused before anything changes"""
    from paper_1202_2462_amd.mgdd import EINVAL, F64, MgddError
    dims, block, agg, N, op = small_problem(seed=11, m0=0.02)
    lat = lattice(op, block)
    rnd, start, st = _boot_inputs(dims, N)
    with pytest.raises(MgddError) as e:
        lat.setup(agg, lat.pack(rnd, F64), st, nu=1, iota=1, mr_iters=4, n_part2=0, prec=F64, chunk=-1)
    assert e.value.code == EINVAL


@pytest.mark.parametrize("chunk", [0, 3])
def test_bootstrap_full_invariants(chunk):
    """Both setup parts. The second part starts from unconverged harmonic Ritz
    pairs of a short Arnoldi run, which amplify rounding: perturbing the input
    of the oracle's own setup by 1e-13 moves its Ritz values by up to 3e-4,
    ||D v_i||^2 by up to 1.3e-4 and the projector P P^H by 1e-3. The GPU result
    is compared within bounds derived from that: ||D v_i||^2 to 5e-3, the
    projector to 2e-2; what is exact is checked exactly (orthonormal test
    vectors, ||D v_i|| ascending), and the two-level solves built on either
    setup need the same number of outer iterations within 2."""
    from paper_1202_2462_amd.mgdd import F64, PLAIN_F64
    dims, block, agg, N, op = small_problem(seed=11, m0=0.02)
    say("bootstrap full", dims, "chunk", chunk)
    lat = lattice(op, block)
    rnd, start, st = _boot_inputs(dims, N)
    tv_or, tl = solvers.bootstrap(op, block, agg, N, 3, 3, 4, rnd, start)
    lat.setup(agg, lat.pack(rnd, F64), st, nu=3, iota=3, mr_iters=4, prec=F64, chunk=chunk)
    tv_gpu = lat.unpack(lat.test_vectors())
    G = np.array([[np.vdot(a, b) for b in tv_gpu] for a in tv_gpu])
    assert np.max(np.abs(G - np.eye(N))) < 1e-10
    s_gpu = np.array([np.linalg.norm(op.apply(v)) ** 2 for v in tv_gpu])
    s_or = np.array([np.linalg.norm(op.apply(v)) ** 2 for v in tv_or])
    assert np.all(np.diff(s_gpu) >= -1e-12)
    say("||D v||^2 gpu", s_gpu, "oracle", s_or)
    assert np.max(np.abs(s_gpu - s_or) / s_or) < 5e-3
    x = latgen.gaussian_fields(dims, 2, 92)
    for i in range(2):
        proj_or = tl.prolong(tl.restrict(x[i]))
        proj_gpu = lat.unpack(lat.prolong(lat.restrict(lat.pack(x[i:i + 1], F64))))[0]
        say("projector difference", rel(proj_gpu, proj_or))
        assert rel(proj_gpu, proj_or) < 2e-2
    b = latgen.gaussian_fields(dims, 1, 93)
    _, st_or = solvers.fgmres(op.apply, tl.precond, b[0], 20, 1e-10, 400)
    z, stats = lat.solve(lat.pack(b, F64), precision=PLAIN_F64, restart=20, tol=1e-10, maxit=400)
    say("bootstrap solve iters gpu", stats[0].iters, "oracle", st_or.iters)
    assert stats[0].converged and abs(stats[0].iters - st_or.iters) <= 2


def test_bootstrap_full_dimension_matches_oracle():
    """Both setup parts element by element (Section 3, "Bootstrap Setup"): with
    as many Arnoldi steps as D_c has rows (4^3 x 8, 4^4 blocks and aggregates,
    N = 8: 32 rows) the harmonic Ritz pairs are the exact eigenpairs of D_c,
    so the second part is a well-conditioned map and the GPU's test vectors
    (unique up to one phase each) must equal the oracle's, which are pinned by
    a step-by-step dense reconstruction in test_oracle_bootstrap.py."""
    import torch
    from paper_1202_2462_amd.mgdd import F64
    dims, block, N = (4, 4, 4, 8), (4, 4, 4, 4), 8
    op = problem(dims, seed=17, eps=0.5, m0=0.05, csw=1.0)
    say("bootstrap full dimension", dims)
    rnd = latgen.gaussian_fields(dims, N, 50)
    nc = 2 * 2 * N
    start = latgen.gaussian_vector(nc, 51)
    st = torch.tensor(np.stack([start.real, start.imag], -1), dtype=torch.float64, device="cuda")
    tv_or, tl = solvers.bootstrap(op, block, block, N, 3, 3, 4, rnd, start, m_arnoldi=nc)
    lat = lattice(op, block)
    lat.setup(block, lat.pack(rnd, F64), st, nu=3, iota=3, mr_iters=4, arnoldi_m=nc, prec=F64)
    tv_gpu = lat.unpack(lat.test_vectors())
    diff = aligned_difference(tv_gpu, tv_or)
    say("test vectors (phase aligned)", diff)
    assert diff < 1e-8
    x = latgen.gaussian_fields(dims, 1, 52)
    proj_or = tl.prolong(tl.restrict(x[0]))
    proj_gpu = lat.unpack(lat.prolong(lat.restrict(lat.pack(x, F64))))[0]
    say("projector", rel(proj_gpu, proj_or))
    assert rel(proj_gpu, proj_or) < 1e-8


def test_c0_recipe_two_level_solve():
    """The 8^4 workload exactly as its recipe states it: links exp(0.35 i H),
    c_sw = 1.0, the bare mass from tests/golden/m0.json (leftmost eigenvalue
    of D at real part 0.05), SAP blocks and aggregates 4^4, N = 8, nu = iota =
    3, MR(4), FGMRES(20), plain FP64, tolerance 1e-10, one Gaussian right-hand
    side (seeds of the workload). The GPU's residual is recomputed by the
    oracle; its solution is compared with an oracle solution converged to
    1e-12 (the bound ||z - z*|| / ||z*|| <= kappa(D) ||r|| / ||b|| is reported
    beside the measured difference, kappa from power and inverse iterations of
    the oracle)."""
    import json
    import os

    import torch
    from paper_1202_2462_amd.mgdd import F64, PLAIN_F64
    w = latgen.WORKLOADS["c0"]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "m0.json")
    m0 = json.load(open(path))["c0"]["m0"]
    dims, block, agg, N = tuple(w["dims"]), tuple(w["block"]), tuple(w["agg"]), w["ntv"]
    say("c0 recipe", dims, "m0", m0)
    op = solvers.Operator(dims, latgen.workload_gauge("c0"), m0, w["csw"])
    rnd = latgen.gaussian_fields(dims, N, latgen.TAG_TV)
    Vc = int(np.prod(dims) // np.prod(agg))
    start = latgen.gaussian_vector(Vc * 2 * N, latgen.TAG_ARNOLDI)
    b = latgen.gaussian_fields(dims, 1, latgen.TAG_RHS)
    _, tl = solvers.bootstrap(op, block, agg, N, w["nu"], w["iota"], w["mr"], rnd, start)
    z_ref, st_ref = solvers.fgmres(op.apply, tl.precond, b[0], w["restart"], 1e-12, 2000)
    _, st_or = solvers.fgmres(op.apply, tl.precond, b[0], w["restart"], w["tol"], 2000)
    assert st_ref.converged
    lat = lattice(op, block)
    st = torch.tensor(np.stack([start.real, start.imag], -1), dtype=torch.float64, device="cuda")
    lat.setup(agg, lat.pack(rnd, F64), st, nu=w["nu"], iota=w["iota"], mr_iters=w["mr"], prec=F64)
    z, stats = lat.solve(lat.pack(b, F64), precision=PLAIN_F64, restart=w["restart"], tol=w["tol"], maxit=2000)
    zg = lat.unpack(z)[0]
    res = np.linalg.norm(b[0] - op.apply(zg)) / np.linalg.norm(b[0])
    diff = rel(zg, z_ref)
    # kappa(D) = sigma_max / sigma_min: power iteration on D^H D, inverse
    # iteration through oracle solves of D and D^H = gamma_5 D gamma_5
    g5 = np.array([1, 1, -1, -1], dtype=float)[None, :, None]
    x = latgen.gaussian_fields(dims, 1, 77)[0]
    for _ in range(30):
        x = op.apply_dag(op.apply(x))
        smax2 = np.linalg.norm(x)
        x /= smax2
    y = latgen.gaussian_fields(dims, 1, 78)[0]
    y /= np.linalg.norm(y)
    for _ in range(4):
        u, _ = solvers.fgmres(op.apply, tl.precond, g5 * y, w["restart"], 1e-12, 2000)
        u, _ = solvers.fgmres(op.apply, tl.precond, g5 * u, w["restart"], 1e-12, 2000)
        smin2 = 1.0 / np.linalg.norm(u)
        y = u / np.linalg.norm(u)
    kappa = np.sqrt(smax2 / smin2)
    say(f"c0: GPU {stats[0].iters} iterations (oracle {st_or.iters}), residual {res:.3e}, "
        f"|z - z*| / |z*| = {diff:.3e}, kappa ~ {kappa:.1f}, bound kappa * res = {kappa * res:.3e}")
    assert stats[0].converged and res <= 1e-10
    assert abs(stats[0].iters - st_or.iters) <= 2
    assert diff <= 1e-8


@pytest.mark.parametrize("seed", [12345, 2 ** 63 + 977])
def test_setup_draws_its_random_vectors(seed):
    """random_vectors = NULL: the library draws the setup's random fields from
    stream `seed` of its counter-based generator (SplitMix64 + Box-Muller).
    With no smoothing round and no second part the test vectors are those
    fields, equal to latgen.gaussian_fields of the same stream (the same
    published generator written in numpy; the transcendental functions may
    differ in the last bit); a first setup part from them equals the one from
    the host-drawn fields."""
    import torch
    from paper_1202_2462_amd.mgdd import F64
    dims, block, agg, N, op = small_problem(seed=11, m0=0.02)
    say("library-drawn random vectors, seed", seed)
    lat = lattice(op, block)
    rnd = latgen.gaussian_fields(dims, N, seed)
    start = latgen.gaussian_vector(16 * 2 * N, 91)
    st = torch.tensor(np.stack([start.real, start.imag], -1), dtype=torch.float64, device="cuda")
    lat.setup(agg, None, st, nu=0, iota=0, mr_iters=4, n_part2=0, prec=F64, ntv=N, seed=seed)
    tv = lat.unpack(lat.test_vectors())
    say("drawn vs latgen", rel(tv, rnd), np.max(np.abs(tv - rnd)))
    assert rel(tv, rnd) < 1e-14
    lat.setup(agg, None, st, nu=3, iota=3, mr_iters=4, n_part2=0, prec=F64, ntv=N, seed=seed)
    a = lat.unpack(lat.test_vectors())
    lat.setup(agg, lat.pack(rnd, F64), st, nu=3, iota=3, mr_iters=4, n_part2=0, prec=F64)
    b = lat.unpack(lat.test_vectors())
    assert rel(a, b) < 1e-12
