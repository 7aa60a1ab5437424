"""Half-precision spinor storage (through the C ABI): layout conversion
rounds each component once to the nearest binary16 value (equal to numpy's
float64 -> float16 conversion), and the Wilson-clover apply on half-stored
fields equals the oracle's FP64 operator applied to the half-rounded input,
up to the final rounding to half (FP32 arithmetic inside)."""
import numpy as np
import pytest

import latgen
from gpu_common import lattice, problem, say

pytestmark = pytest.mark.gpu

CASES = [((8, 8, 8, 8), (4, 4, 4, 4)), ((8, 8, 8, 16), (4, 4, 4, 2))]


def round16(c):
    out = np.empty_like(c)
    out.real = c.real.astype(np.float16)
    out.imag = c.imag.astype(np.float16)
    return out


@pytest.mark.parametrize("dims,block", CASES)
def test_pack_unpack_half_is_one_rounding(dims, block):
    from paper_1202_2462_amd.mgdd import F16
    say("half pack/unpack", dims)
    op = problem(dims, seed=14)
    lat = lattice(op, block)
    x = latgen.gaussian_fields(dims, 2, 40)
    x[0, 5, 1, 2] = 1e-6 + 70000.0j      # a subnormal-range and an overflowing (to inf) component
    got = lat.unpack(lat.pack(x, F16))
    with np.errstate(over="ignore"):
        want = round16(x)
    assert np.array_equal(got.real, want.real) and np.array_equal(got.imag, want.imag)


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("nrhs", [1, 3])
def test_dirac_half_storage(dims, block, nrhs):
    from paper_1202_2462_amd.mgdd import F16
    say("half dirac", dims, nrhs)
    op = problem(dims, seed=15, m0=0.1)
    lat = lattice(op, block)
    x = latgen.gaussian_fields(dims, nrhs, 41)
    xh = round16(x)
    want = np.stack([op.apply(v) for v in xh])
    got = lat.unpack(lat.dirac(lat.pack(x, F16)))
    # each stored component is the FP32 result rounded to half: within half an
    # ulp of binary16 (2^-11 relative) plus the FP32 arithmetic error
    scale = np.abs(want).max()
    for part in (np.real, np.imag):
        err = np.abs(part(got) - part(want))
        assert np.all(err <= 2.0 ** -11 * np.abs(part(want)) * 1.001 + 1e-6 * scale), err.max()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 4e-4


def test_half_timing_and_errors():
    from paper_1202_2462_amd.mgdd import EINVAL, F16, KERNEL_DIRAC, MgddError, mgdd_timing_enable, mgdd_timing_read
    dims, block = CASES[0]
    say("half timing / errors")
    op = problem(dims, seed=16)
    lat = lattice(op, block)
    x = lat.pack(latgen.gaussian_fields(dims, 1, 42), F16)
    mgdd_timing_read(lat.ctx, KERNEL_DIRAC, F16, reset=True)
    mgdd_timing_enable(lat.ctx, True)
    lat.dirac(x)
    lat.dirac(x)
    ms, units, n, nbytes = mgdd_timing_read(lat.ctx, KERNEL_DIRAC, F16)
    mgdd_timing_enable(lat.ctx, False)
    # algorithmic bytes: FP32 links (two rows each: special unitary links) and
    # clover term once, half spinor in and out
    assert n == 2 and units == 2 * lat.V and ms > 0 and nbytes == 2 * lat.V * (192 + 288 + 96)
    with pytest.raises(MgddError) as e:   # half precision is a storage format of fine fields only
        lat.sap(x, lat.field(F16, 1), 1, 4)
    assert e.value.code == EINVAL
