"""mgdd_coarse_solve_noalloc (the coarse solve with its workspace in the
library's fixed device array, for callers that cannot allocate) against
mgdd_coarse_solve and the oracle, on two calls in a row, the second with a
smaller input; sizes beyond the array are refused."""
import numpy as np
import pytest

import latgen
from gpu_common import lattice, problem, rel, say
from oracle import solvers

pytestmark = pytest.mark.gpu


def _coarse(lat, c, prec):
    import torch
    from paper_1202_2462_amd.mgdd import F64
    return torch.tensor(np.stack([c.real, c.imag], -1), dtype=torch.float64 if prec == F64 else torch.float32,
                        device="cuda")


def _np(t):
    a = t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def test_noalloc_coarse_solve_matches_coarse_solve():
    from paper_1202_2462_amd.mgdd import (EINVAL, F32, F64, MgddError, mgdd_coarse_solve,
                                           mgdd_coarse_solve_noalloc)
    dims, block, agg, N = (8, 8, 8, 8), (4, 4, 4, 4), (4, 4, 4, 4), 8
    op = problem(dims, seed=3, m0=0.1)
    lat = lattice(op, block)
    tv = latgen.gaussian_fields(dims, N, 43)
    lat.build_P(agg, lat.pack(tv, F64))
    tl = solvers.TwoLevel(op, agg, tv, block)
    Vc = lat.Vc
    # two calls in a row, the second with fewer right-hand sides and steps
    for call, (nrhs, iters) in enumerate(((5, 12), (2, 7))):
        c = latgen.gaussian_vector(nrhs * Vc * 2 * N, 60 + call).reshape(nrhs, Vc, 2, N)
        want = np.stack([solvers.gmres_fixed(tl.coarse_apply, c[i], iters) for i in range(nrhs)])
        for prec, tol_same, tol_or in ((F64, 1e-13, 1e-10), (F32, 1e-6, 1e-4)):
            say("noalloc coarse solve, call", call, "nrhs", nrhs, "iters", iters, "prec", prec)
            b = _coarse(lat, c, prec)
            x_ref = lat.torch.zeros_like(b)
            x = lat.torch.full_like(b, 7.0)
            mgdd_coarse_solve(lat.ctx, prec, nrhs, iters, b, x_ref)
            mgdd_coarse_solve_noalloc(lat.ctx, prec, nrhs, iters, b, x)
            got, ref = _np(x), _np(x_ref)
            d_same = max(rel(got[i], ref[i]) for i in range(nrhs))
            d_or = max(rel(got[i], want[i]) for i in range(nrhs))
            say("  vs mgdd_coarse_solve", d_same, "vs oracle", d_or)
            assert d_same <= tol_same and d_or <= tol_or
    # beyond the limits: refused before anything is launched
    b = _coarse(lat, np.zeros((1, Vc, 2, N), dtype=np.complex128), F64)
    x = lat.torch.zeros_like(b)
    with pytest.raises(MgddError) as e:
        mgdd_coarse_solve_noalloc(lat.ctx, F64, 1, 16, b, x)
    assert e.value.code == EINVAL
    with pytest.raises(MgddError) as e:
        mgdd_coarse_solve_noalloc(lat.ctx, F64, 5000, 12, b, x)
    assert e.value.code == EINVAL and "scratch" in str(e.value)
    lat.close()
