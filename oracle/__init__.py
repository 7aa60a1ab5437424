"""Plain FP64 CPU oracle of the SAP + aggregation multilevel solver.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU timing leg of the benchmark. The GPU library does not import it and shares
no code with it.

The site-loop operators (Wilson-clover apply, clover term, SAP, P, restriction,
prolongation, D_c) are plain C in `oracle.c`; the Krylov methods and the
bootstrap setup, which only combine those operators with small dense linear
algebra, are numpy in `solvers.py`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OK, ESHAPE, ERANK = 0, -2, -3


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (OpenMP, IEEE arithmetic, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = ctypes.CDLL(_SO)
    return _lib


def _i4(v):
    return (ctypes.c_int * 4)(*[int(t) for t in v])


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def vol(dims) -> int:
    return int(np.prod(dims))


def num_threads() -> int:
    return int(lib().or_num_threads())


def gamma() -> tuple[np.ndarray, np.ndarray]:
    """(gamma_mu[4,4,4], gamma_5[4,4]) in the chiral basis."""
    out = np.zeros((5, 4, 4), dtype=np.complex128)
    lib().or_gamma(_p(out))
    return out[:4].copy(), out[4].copy()


def clover(dims, U, m0: float, csw: float) -> np.ndarray:
    """A[V,12,12] = (4+m0) + csw (i/4) sum sigma F."""
    U = _c(U)
    A = np.zeros((vol(dims), 12, 12), dtype=np.complex128)
    lib().or_clover(_i4(dims), _p(U), ctypes.c_double(m0), ctypes.c_double(csw), _p(A))
    return A


def dirac(dims, U, A, psi, shift: complex = 0.0) -> np.ndarray:
    """(D - shift) psi for one field psi[V,4,3]."""
    U, A, psi = _c(U), _c(A), _c(psi)
    out = np.zeros_like(psi)
    lib().or_dirac(_i4(dims), _p(U), _p(A), ctypes.c_double(complex(shift).real),
                   ctypes.c_double(complex(shift).imag), _p(psi), _p(out))
    return out


def sap(dims, U, A, block, b, z0, nsweeps: int, mr_iters: int, shift: complex = 0.0) -> np.ndarray:
    """nsweeps red-black Schwarz sweeps on (D - shift) z = b from z0."""
    U, A, b = _c(U), _c(A), _c(b)
    z = _c(z0).copy()
    rc = lib().or_sap(_i4(dims), _p(U), _p(A), _i4(block), int(nsweeps), int(mr_iters),
                      ctypes.c_double(complex(shift).real), ctypes.c_double(complex(shift).imag), _p(b), _p(z))
    if rc:
        raise ValueError(f"or_sap: status {rc}")
    return z


BLOCK_MR, BLOCK_GMRES = 0, 1


def schwarz(dims, U, A, block, b, z0, nsweeps: int, k: int, block_solver: int = BLOCK_MR, additive: bool = False,
            shift: complex = 0.0) -> np.ndarray:
    """nsweeps Schwarz sweeps on (D - shift) z = b from z0: red-black
    multiplicative (Algorithm 2.1) or additive, block systems by k MR or GMRES
    steps."""
    U, A, b = _c(U), _c(A), _c(b)
    z = _c(z0).copy()
    rc = lib().or_schwarz(_i4(dims), _p(U), _p(A), _i4(block), int(nsweeps), int(k), int(block_solver),
                          int(bool(additive)), ctypes.c_double(complex(shift).real),
                          ctypes.c_double(complex(shift).imag), _p(b), _p(z))
    if rc:
        raise ValueError(f"or_schwarz: status {rc}")
    return z


def block_apply(dims, U, A, block, blk: int, psi, shift: complex = 0.0) -> np.ndarray:
    """I^T (D - shift) I psi on block blk; zero elsewhere."""
    U, A, psi = _c(U), _c(A), _c(psi)
    out = np.zeros_like(psi)
    rc = lib().or_block_apply(_i4(dims), _p(U), _p(A), _i4(block), int(blk), ctypes.c_double(complex(shift).real),
                              ctypes.c_double(complex(shift).imag), _p(psi), _p(out))
    if rc:
        raise ValueError(f"or_block_apply: status {rc}")
    return out


def block_sites(dims, block, blk: int) -> np.ndarray:
    n = vol(block)
    out = np.zeros(n, dtype=np.int32)
    lib().or_block_sites(_i4(dims), _i4(block), int(blk), out.ctypes.data_as(ctypes.c_void_p))
    return out


def sap_check(dims, block) -> int:
    return int(lib().or_sap_check(_i4(dims), _i4(block)))


def build_P(dims, agg, V_tv) -> tuple[np.ndarray, int]:
    """Locally orthonormalised test vectors: (P[N,V,4,3], status)."""
    V_tv = _c(V_tv)
    N = V_tv.shape[0]
    P = np.zeros_like(V_tv)
    rc = lib().or_build_P(_i4(dims), _i4(agg), int(N), _p(V_tv), _p(P))
    return P, int(rc)


def coarse_dims(dims, agg):
    return tuple(int(d) // int(a) for d, a in zip(dims, agg))


def restrict(dims, agg, P, f) -> np.ndarray:
    P, f = _c(P), _c(f)
    N = P.shape[0]
    c = np.zeros((vol(coarse_dims(dims, agg)), 2, N), dtype=np.complex128)
    lib().or_restrict(_i4(dims), _i4(agg), int(N), _p(P), _p(f), _p(c))
    return c


def prolong(dims, agg, P, c) -> np.ndarray:
    P, c = _c(P), _c(c)
    N = P.shape[0]
    f = np.zeros((vol(dims), 4, 3), dtype=np.complex128)
    lib().or_prolong(_i4(dims), _i4(agg), int(N), _p(P), _p(c), _p(f))
    return f


def coarse_build(dims, agg, U, A, P) -> np.ndarray:
    U, A, P = _c(U), _c(A), _c(P)
    N = P.shape[0]
    Vc = vol(coarse_dims(dims, agg))
    Dc = np.zeros((Vc, 9, 2 * N, 2 * N), dtype=np.complex128)
    rc = lib().or_coarse_build(_i4(dims), _i4(agg), int(N), _p(U), _p(A), _p(P), _p(Dc))
    if rc:
        raise ValueError(f"or_coarse_build: status {rc}")
    return Dc


def coarse_apply(cdims, Dc, x) -> np.ndarray:
    Dc, x = _c(Dc), _c(x)
    N = Dc.shape[-1] // 2
    y = np.zeros_like(x)
    lib().or_coarse_apply(_i4(cdims), int(N), _p(Dc), _p(x), _p(y))
    return y
