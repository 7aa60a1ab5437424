"""Shared helpers of the test-suite (dense matrices built column by column,
small random problems). Imported by tests only."""
from __future__ import annotations

import numpy as np

import latgen
import oracle
from oracle.solvers import Operator


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return float(d / n) if n > 0 else float(d)


def random_op(dims, seed=7, eps=0.6, m0=0.3, csw=1.0, ape=0):
    U = latgen.gauge_field(dims, eps, seed, ape_steps=ape)
    return Operator(dims, U, m0, csw)


def dense(apply, shape, dtype=np.complex128, nout=None):
    """Dense matrix of a linear map on arrays of the given shape (nout rows,
    default square)."""
    n = int(np.prod(shape))
    M = np.zeros((n if nout is None else nout, n), dtype=dtype)
    e = np.zeros(n, dtype=dtype)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = np.asarray(apply(e.reshape(shape))).ravel()
        e[j] = 0.0
    return M


def gamma5_field(psi):
    out = psi.copy()
    out[..., 2:, :] *= -1
    return out


def gamma5_coarse(c):
    out = c.copy()
    out[:, 1, :] *= -1
    return out


def sort_spectrum(ev):
    """Eigenvalues sorted by (rounded real part, imaginary part), so that
    multisets equal up to rounding line up element by element."""
    ev = np.asarray(ev)
    key = np.lexsort((np.round(ev.imag, 8), np.round(ev.real, 8)))
    return ev[key]


def aligned_difference(a, ref) -> float:
    """Relative difference of two sets of vectors that are unique up to one
    phase per vector: each vector of a is rotated onto its partner in ref
    before the difference is taken."""
    num = den = 0.0
    for x, r in zip(a, ref):
        x, r = np.ravel(x), np.ravel(r)
        ph = np.vdot(x, r)
        x = x * (ph / abs(ph))
        num += np.linalg.norm(x - r) ** 2
        den += np.linalg.norm(r) ** 2
    return float(np.sqrt(num / den))
