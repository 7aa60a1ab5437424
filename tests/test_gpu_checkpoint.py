"""Setup checkpoint (mgdd_save_setup / mgdd_load_setup) and run-to-run
determinism, through the C ABI: a setup written to a file and read back
into a new context (also with another Schwarz block shape) gives the same
interpolation and the same solve; damaged, truncated or foreign files are
refused before anything changes; two solves on one context are bitwise
equal (every reduction runs in a fixed order)."""
import os

import numpy as np
import pytest

import latgen
from gpu_common import lattice, problem, rel, say

pytestmark = pytest.mark.gpu

DIMS, BLOCK, AGG, N = (8, 8, 8, 8), (4, 4, 4, 4), (4, 4, 4, 4), 6


def setup_lattice(op, block=BLOCK):
    import torch
    from paper_1202_2462_amd.mgdd import F64
    lat = lattice(op, block)
    rnd = lat.pack(latgen.gaussian_fields(DIMS, N, 50), F64)
    Vc = int(np.prod(DIMS)) // int(np.prod(AGG))
    st = latgen.gaussian_vector(Vc * 2 * N, 51)
    start = torch.tensor(np.stack([st.real, st.imag], -1), dtype=torch.float64, device="cuda")
    lat.setup(AGG, rnd, start, nu=2, iota=2, mr_iters=4)
    return lat


def test_save_load_roundtrip(tmp_path):
    from paper_1202_2462_amd.mgdd import F64, MIXED
    say("setup checkpoint round trip")
    op = problem(DIMS, seed=52, m0=0.05)
    lat = setup_lattice(op)
    path = str(tmp_path / "setup.bin")
    lat.save_setup(path)
    x = latgen.gaussian_fields(DIMS, 1, 53)
    b = lat.pack(latgen.gaussian_fields(DIMS, 1, 54), F64)
    want_pp = lat.unpack(lat.prolong(lat.restrict(lat.pack(x, F64))))
    z0, st0 = lat.solve(b, precision=MIXED, tol=1e-10, maxit=500)
    for block in (BLOCK, (4, 4, 4, 2)):
        lat2 = lattice(op, block)
        lat2.load_setup(path)
        got_pp = lat2.unpack(lat2.prolong(lat2.restrict(lat2.pack(x, F64))))
        assert rel(got_pp, want_pp) < 1e-12, block
        z, st = lat2.solve(lat2.pack(lat.unpack(b), F64), precision=MIXED, tol=1e-10, maxit=500)
        say(block, "iters", st[0].iters, "original", st0[0].iters)
        assert st[0].converged
        if block == BLOCK:
            assert st[0].iters == st0[0].iters
            assert np.array_equal(lat2.unpack(z), lat.unpack(z0))


def test_bad_setup_files_are_refused(tmp_path):
    from paper_1202_2462_amd.mgdd import EINVAL, ESHAPE, MgddError
    say("setup checkpoint errors")
    op = problem(DIMS, seed=55, m0=0.05)
    lat = setup_lattice(op)
    path = str(tmp_path / "setup.bin")
    lat.save_setup(path)
    raw = open(path, "rb").read()
    cases = {"corrupt": raw[:200] + bytes([raw[200] ^ 1]) + raw[201:], "truncated": raw[:-16], "foreign": b"x" * 100}
    for name, data in cases.items():
        p = str(tmp_path / f"{name}.bin")
        open(p, "wb").write(data)
        with pytest.raises(MgddError) as e:
            lat.load_setup(p)
        assert e.value.code == EINVAL, name
    with pytest.raises(MgddError) as e:
        lat.load_setup(str(tmp_path / "missing.bin"))
    assert e.value.code == EINVAL
    other = lattice(problem((8, 8, 8, 16), seed=56), (4, 4, 4, 4))
    with pytest.raises(MgddError) as e:
        other.load_setup(path)
    assert e.value.code == ESHAPE
    # the refused loads left the setup of the first context untouched
    x = latgen.gaussian_fields(DIMS, 1, 57)
    from paper_1202_2462_amd.mgdd import F64
    assert np.isfinite(lat.unpack(lat.prolong(lat.restrict(lat.pack(x, F64))))).all()


def test_solves_are_bitwise_reproducible():
    from paper_1202_2462_amd.mgdd import F64, MIXED, PLAIN_F64
    say("run-to-run determinism")
    op = problem(DIMS, seed=58, m0=0.05)
    lat = setup_lattice(op)
    b = lat.pack(latgen.gaussian_fields(DIMS, 2, 59), F64)
    for prec in (MIXED, PLAIN_F64):
        z1, s1 = lat.solve(b, precision=prec, tol=1e-10, maxit=500)
        z2, s2 = lat.solve(b, precision=prec, tol=1e-10, maxit=500)
        assert [s.iters for s in s1] == [s.iters for s in s2]
        assert np.array_equal(z1.cpu().numpy(), z2.cpu().numpy()), prec
