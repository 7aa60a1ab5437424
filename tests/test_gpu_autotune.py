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
