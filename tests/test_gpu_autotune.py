"""GPU: the Schwarz block-shape autotuner times setup + solve for every
admissible shape and picks the fastest converged one; the oracle is then
rerun with the chosen shape (one Schwarz sweep, element by element)."""
import numpy as np
import pytest

import latgen
from gpu_common import TOL32, lattice, problem, rel, say

pytestmark = pytest.mark.gpu


def test_candidate_blocks_admissible():
    from paper_1202_2462_amd.autotune import candidate_blocks
    c = candidate_blocks((8, 8, 8, 8))
    assert (4, 4, 4, 4) in c and (2, 4, 4, 4) in c
    for blk in c:
        vb = int(np.prod(blk))
        assert 64 <= vb <= 256
        for L, b in zip((8, 8, 8, 8), blk):
            assert L % b == 0 and (L // b == 1 or (L // b) % 2 == 0)
    assert (8, 8, 8, 8) not in c          # 4096 sites: too large for the kernel
    assert all(np.prod(b) <= 256 for b in candidate_blocks((16, 16, 16, 32)))


def test_autotune_picks_a_converged_shape_and_oracle_agrees():
    import torch
    from paper_1202_2462_amd.autotune import tune_sap_block
    from paper_1202_2462_amd.mgdd import F32
    dims, agg, N = (8, 8, 8, 8), (4, 4, 4, 4), 8
    op = problem(dims, seed=4, m0=0.05, eps=0.5)
    say("autotune on", dims)
    rv = latgen.gaussian_fields(dims, N, 31)
    Vc = int(np.prod(dims)) // int(np.prod(agg))
    st = latgen.gaussian_vector(Vc * 2 * N, 32)
    start = torch.tensor(np.stack([st.real, st.imag], -1), dtype=torch.float64, device="cuda")
    b = latgen.gaussian_fields(dims, 1, 33)
    cands = [(4, 4, 4, 4), (2, 4, 4, 4), (4, 4, 4, 2), (4, 4, 2, 2)]
    res = tune_sap_block(dims, op.U, op.m0, op.csw, agg, rv, start, b, restart=20, tol=1e-10, candidates=cands,
                         log=say)
    assert len(res["results"]) == len(cands)
    assert res["best"] in cands
    assert all(r["converged"] for r in res["results"])
    best = min(res["results"], key=lambda r: r["seconds"])
    assert tuple(best["block"]) == tuple(res["best"])
    # the smoother with the chosen shape against the oracle
    blk = res["best"]
    lat = lattice(op, blk)
    bb = latgen.gaussian_fields(dims, 1, 34)
    want = op.sap(blk, bb[0], np.zeros_like(bb[0]), 1, 4)
    z = lat.field(F32, 1)
    lat.sap(lat.pack(bb, F32), z, 1, 4)
    assert rel(lat.unpack(z)[0], want) < TOL32


def test_kernel_options_match_oracle():
    """Every thread tile the tuner can pick computes the same sweep: the FP32
    Schwarz sweep on 1, 2 and 4 lanes per site and the Wilson-clover apply
    with and without the LDS staging all match the oracle; values outside
    the sets are refused, and two lanes per site without special unitary
    links fail at launch with ESHAPE."""
    from paper_1202_2462_amd.mgdd import EINVAL, ESHAPE, F32, F64, MgddError, mgdd_set_kernel_options
    from oracle import solvers
    from gpu_common import TOL64
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    say("kernel options")
    op = problem(dims, seed=9, m0=0.1)
    lat = lattice(op, block)
    b = latgen.gaussian_fields(dims, 2, 35)
    want = np.stack([op.sap(block, b[i], np.zeros_like(b[i]), 1, 4) for i in range(2)])
    for lanes in (1, 2, 4):
        mgdd_set_kernel_options(lat.ctx, sap_lanes=lanes)
        z = lat.field(F32, 2)
        lat.sap(lat.pack(b, F32), z, 1, 4)
        assert rel(lat.unpack(z), want) < TOL32, lanes
    want_d = np.stack([op.apply(b[i]) for i in range(2)])
    for stage in (-1, 1):
        mgdd_set_kernel_options(lat.ctx, dirac_stage=stage)
        for prec, tol in ((F64, TOL64), (F32, TOL32)):
            assert rel(lat.unpack(lat.dirac(lat.pack(b, prec))), want_d) < tol, (stage, prec)
    for bad in ((3, 0), (0, 2)):
        with pytest.raises(MgddError) as e:
            mgdd_set_kernel_options(lat.ctx, *bad)
        assert e.value.code == EINVAL
    lat.close()
    # links outside SU(3): no two-lanes kernel
    op2 = solvers.Operator(dims, op.U * np.exp(0.3j), 0.1, 1.0)
    lat2 = lattice(op2, block)
    mgdd_set_kernel_options(lat2.ctx, sap_lanes=2)
    with pytest.raises(MgddError) as e:
        lat2.sap(lat2.pack(b, F32), lat2.field(F32, 2), 1, 4)
    assert e.value.code == ESHAPE
    mgdd_set_kernel_options(lat2.ctx, sap_lanes=4)
    z = lat2.field(F32, 2)
    lat2.sap(lat2.pack(b, F32), z, 1, 4)
    want2 = np.stack([op2.sap(block, b[i], np.zeros_like(b[i]), 1, 4) for i in range(2)])
    assert rel(lat2.unpack(z), want2) < TOL32
    lat2.close()


def test_autotune_32x32x32x64_then_oracle_sweep():
    """The tuner at 32^3 x 64 (the 16^3 x 32 workload field repeated twice per
    direction, with that field's tuned bare mass) on a batched solve of two
    point sources, over two block shapes and two lanes-per-site tiles; then
    one Schwarz sweep with the chosen shape and tile against the oracle's
    sweep at that size."""
    import json
    import os

    import torch
    from paper_1202_2462_amd.autotune import tune_sap_block
    from paper_1202_2462_amd.mgdd import F32, mgdd_set_kernel_options
    from oracle import solvers
    w = latgen.WORKLOADS["c1"]
    m0 = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "m0.json")))["c1"]["m0"]
    small = tuple(w["dims"])
    dims = tuple(2 * L for L in small)
    U = latgen.workload_gauge("c1").reshape(small[3], small[2], small[1], small[0], 4, 3, 3)
    U = np.tile(U, (2, 2, 2, 2, 1, 1, 1)).reshape(-1, 4, 3, 3)
    say("autotune at", dims)
    agg, N = (4, 4, 4, 4), 8
    Vc = int(np.prod(dims)) // int(np.prod(agg))
    st = latgen.gaussian_vector(Vc * 2 * N, 36)
    start = torch.tensor(np.stack([st.real, st.imag], -1), dtype=torch.float64, device="cuda")
    b = np.zeros((2, int(np.prod(dims)), 4, 3), dtype=np.complex128)   # two point sources at one site
    b[0, 123457, 0, 0] = 1.0
    b[1, 123457, 2, 1] = 1.0
    cands = [(4, 4, 4, 4), (2, 4, 4, 4)]
    res = tune_sap_block(dims, U, m0, w["csw"], agg, None, start, b, nu=2, iota=2, restart=20, tol=1e-10,
                         candidates=cands, lanes=(2, 4), setup_kwargs=dict(ntv=N, seed=38), log=say)
    assert len(res["results"]) == 4 and all(r["converged"] for r in res["results"])
    blk, lanes = res["best"], res["best_lanes"]
    say("chosen", blk, "lanes", lanes)
    op = solvers.Operator(dims, U, m0, w["csw"])
    from paper_1202_2462_amd.mgdd import Lattice
    lat = Lattice(dims, blk)
    lat.set_gauge(U, m0, w["csw"])
    mgdd_set_kernel_options(lat.ctx, sap_lanes=lanes)
    bb = latgen.gaussian_fields(dims, 1, 39)
    z = lat.field(F32, 1)
    lat.sap(lat.pack(bb, F32), z, 1, 4)
    want = op.sap(blk, bb[0], np.zeros_like(bb[0]), 1, 4)
    err = rel(lat.unpack(z)[0], want)
    say("  sweep vs oracle", err)
    assert err < TOL32
    lat.close()
