"""Thin ctypes binding of libmgdd.so (argument marshalling only).

Every function here has the name of the C entry point it calls, and does no
arithmetic of its own: PyTorch supplies device memory and the stream. The
library must have been built (python -m paper_1202_2462_amd.build); importing
this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgdd.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mgdd.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1202_2462_amd.build`")

# PyTorch ships its own HIP runtime (same soname as the system one). It is
# loaded first, so that libmgdd.so binds to that copy and the process holds a
# single HIP runtime, whose device memory and streams both sides share.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ESHAPE, ERANK, ENOTREADY, ENOCONV, EBREAKDOWN, ENAN, EHIP, ENOMEM = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
F64, F32, F16 = 0, 1, 2
KERNEL_DIRAC, KERNEL_SAP, KERNEL_COARSE = 0, 1, 2
_NAMES = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ERANK", -4: "ENOTREADY", -5: "ENOCONV", -6: "EBREAKDOWN",
          -7: "ENAN", -8: "EHIP", -9: "ENOMEM"}


class MgddError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_i4 = ctypes.c_int * 4


def _sig(name, restype, *args):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(args)
    return f


_sig("mgdd_create", ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.c_int, _vp,
     ctypes.POINTER(_vp))
ALLOC_FN = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp)
FREE_FN = ctypes.CFUNCTYPE(None, _vp, _vp)
_sig("mgdd_set_allocator", ctypes.c_int, _vp, ALLOC_FN, FREE_FN, _vp)
_sig("mgdd_destroy", ctypes.c_int, _vp)
_sig("mgdd_last_error", ctypes.c_char_p, _vp)
_sig("mgdd_field_bytes", ctypes.c_size_t, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int)
_sig("mgdd_set_gauge", ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_double)
_sig("mgdd_pack", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp)
_sig("mgdd_unpack", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int)
_sig("mgdd_dirac_apply", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_sap", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
     ctypes.c_int, ctypes.c_double, ctypes.c_double, _vp, _vp)


class SetupParams(ctypes.Structure):
    _fields_ = [("agg", ctypes.c_int * 4), ("ntv", ctypes.c_int), ("nu", ctypes.c_int), ("iota", ctypes.c_int),
                ("mr_iters", ctypes.c_int), ("arnoldi_m", ctypes.c_int), ("n_part2", ctypes.c_int),
                ("prec", ctypes.c_int), ("chunk", ctypes.c_int), ("seed", ctypes.c_ulonglong)]


class SolveParams(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("precision", ctypes.c_int), ("restart", ctypes.c_int),
                ("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("coarse_iters", ctypes.c_int),
                ("nu", ctypes.c_int), ("mr_iters", ctypes.c_int), ("levels", ctypes.c_int), ("k2", ctypes.c_int),
                ("nu2", ctypes.c_int), ("mr2", ctypes.c_int), ("block_solver", ctypes.c_int),
                ("additive", ctypes.c_int)]


class SchwarzParams(ctypes.Structure):
    _fields_ = [("nsweeps", ctypes.c_int), ("block_iters", ctypes.c_int), ("block_solver", ctypes.c_int),
                ("additive", ctypes.c_int), ("shift_re", ctypes.c_double), ("shift_im", ctypes.c_double)]


class KernelOptions(ctypes.Structure):
    _fields_ = [("sap_lanes", ctypes.c_int), ("dirac_stage", ctypes.c_int)]


class Level2Params(ctypes.Structure):
    _fields_ = [("agg2", ctypes.c_int * 4), ("ntv2", ctypes.c_int), ("block2", ctypes.c_int * 4),
                ("nu2", ctypes.c_int), ("mr_iters", ctypes.c_int)]


class NetShape(ctypes.Structure):
    _fields_ = [("nlayers", ctypes.c_int), ("widths", ctypes.c_int * 9)]


def net_shape(widths):
    w = list(widths) + [0] * (9 - len(widths))
    return NetShape(len(widths) - 1, (ctypes.c_int * 9)(*w))


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("relres", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SOLVER_FGMRES_MG, SOLVER_GCR, SOLVER_GCR_EO, SOLVER_CGN = 0, 1, 2, 3
BLOCK_MR, BLOCK_GMRES = 0, 1
PLAIN_F64, MIXED, MIXED_F16 = 0, 1, 2

_sig("mgdd_set_kernel_options", ctypes.c_int, _vp, _vp)
_sig("mgdd_setup_fallback", ctypes.c_int, _vp)
_sig("mgdd_release_workspace", ctypes.c_int, _vp)
_sig("mgdd_save_setup", ctypes.c_int, _vp, ctypes.c_char_p)
_sig("mgdd_load_setup", ctypes.c_int, _vp, ctypes.c_char_p)
_sig("mgdd_net_weight_count", ctypes.c_size_t, ctypes.POINTER(NetShape))
_sig("mgdd_net_apply", ctypes.c_int, _vp, ctypes.POINTER(NetShape), _vp, ctypes.c_int, _vp, _vp)
_sig("mgdd_net_grad", ctypes.c_int, _vp, ctypes.POINTER(NetShape), _vp, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double),
     _vp)
_sig("mgdd_net_adam", ctypes.c_int, _vp, ctypes.POINTER(NetShape), _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_double)
_sig("mgdd_setup_learned", ctypes.c_int, _vp, ctypes.POINTER(NetShape), _vp, ctypes.POINTER(SetupParams), _vp, _vp)
_sig("mgdd_schwarz", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
     ctypes.POINTER(SchwarzParams), _vp, _vp)
_sig("mgdd_build_P", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, _vp)
_sig("mgdd_get_test_vectors", ctypes.c_int, _vp, _vp)
_sig("mgdd_restrict", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_prolong", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_coarse_apply", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_coarse_solve", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_coarse_solve_noalloc", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_precondition", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     _vp, _vp)
_sig("mgdd_setup_bootstrap", ctypes.c_int, _vp, ctypes.POINTER(SetupParams), _vp, _vp)
_sig("mgdd_solve", ctypes.c_int, _vp, ctypes.POINTER(SolveParams), ctypes.c_int, _vp, _vp, ctypes.POINTER(SolveStats))
_sig("mgdd_build_P2", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, _vp)
_sig("mgdd_restrict2", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_prolong2", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_coarse2_apply", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_precondition3", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp)
_sig("mgdd_setup_level2", ctypes.c_int, _vp, ctypes.POINTER(Level2Params), _vp)
_sig("mgdd_coarse_sap", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
     _vp, _vp)
_sig("mgdd_timing_enable", ctypes.c_int, _vp, ctypes.c_int)
_sig("mgdd_timing_read", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double))


def declared_symbols() -> list[str]:
    """Names of the entry points declared in include/mgdd.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mgdd_[A-Za-z0-9_]+)\s*\(", txt)))


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"]
        return x.ctypes.data
    raise TypeError(type(x))


def _check(ctx, rc):
    if rc != OK:
        msg = _lib.mgdd_last_error(ctx).decode() if ctx else ""
        raise MgddError(rc, msg)
    return rc


# --------------------------------------------------------------------- entry points

def mgdd_create(dims, block, stream=None, t_antiperiodic=True):
    """Returns the context handle. stream: a torch.cuda.Stream, a raw
    hipStream_t int, or None for torch's current stream."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    out = _vp()
    rc = _lib.mgdd_create(_i4(*dims), _i4(*block), 1 if t_antiperiodic else 0, stream, ctypes.byref(out))
    if rc != OK:
        raise MgddError(rc, "mgdd_create failed (dims/block do not fit)")
    return out.value


def mgdd_destroy(ctx):
    return _lib.mgdd_destroy(ctx)


def mgdd_last_error(ctx) -> str:
    return _lib.mgdd_last_error(ctx).decode()


def mgdd_field_bytes(ctx, prec, nrhs, level=0) -> int:
    return int(_lib.mgdd_field_bytes(ctx, prec, nrhs, level))


def mgdd_set_gauge(ctx, U, m0: float, csw: float):
    """U: canonical complex128 [V,4,3,3] (numpy on the host) or the same bytes
    as a float64 torch tensor on the device."""
    on_dev = 0 if isinstance(U, np.ndarray) else 1
    if on_dev == 0:
        U = np.ascontiguousarray(U, dtype=np.complex128)
    return _check(ctx, _lib.mgdd_set_gauge(ctx, _ptr(U), on_dev, m0, csw))


def mgdd_pack(ctx, prec, nrhs, src, dst):
    """src: canonical complex128 fields (numpy on the host, or a torch tensor on the device)."""
    on_dev = 0 if isinstance(src, np.ndarray) else 1
    if on_dev == 0:
        src = np.ascontiguousarray(src, dtype=np.complex128)
    return _check(ctx, _lib.mgdd_pack(ctx, prec, nrhs, _ptr(src), on_dev, _ptr(dst)))


def mgdd_unpack(ctx, prec, nrhs, src, dst):
    on_dev = 0 if isinstance(dst, np.ndarray) else 1
    return _check(ctx, _lib.mgdd_unpack(ctx, prec, nrhs, _ptr(src), _ptr(dst), on_dev))


def mgdd_dirac_apply(ctx, prec, nrhs, x, y):
    return _check(ctx, _lib.mgdd_dirac_apply(ctx, prec, nrhs, _ptr(x), _ptr(y)))


def mgdd_set_allocator(ctx, alloc, free, user=None):
    """alloc, free: ALLOC_FN / FREE_FN instances (kept alive by the caller),
    or None for both."""
    return _check(ctx, _lib.mgdd_set_allocator(ctx, alloc or ALLOC_FN(), free or FREE_FN(), user))


def mgdd_set_kernel_options(ctx, sap_lanes=0, dirac_stage=0):
    """lanes per site of the FP32 Schwarz kernel (0 automatic, 1, 2, 4) and
    the LDS staging of the Wilson-clover apply (0 automatic, 1, -1)."""
    return _check(ctx, _lib.mgdd_set_kernel_options(ctx, ctypes.byref(KernelOptions(sap_lanes, dirac_stage))))


def mgdd_sap(ctx, prec, nrhs, block, nsweeps, mr_iters, shift, b, z):
    shift = complex(shift)
    blk = None if block is None else _i4(*block)
    return _check(ctx, _lib.mgdd_sap(ctx, prec, nrhs, blk, nsweeps, mr_iters, shift.real, shift.imag, _ptr(b),
                                     _ptr(z)))


def mgdd_build_P(ctx, agg, ntv, test_vectors):
    return _check(ctx, _lib.mgdd_build_P(ctx, _i4(*agg), ntv, _ptr(test_vectors)))


def mgdd_get_test_vectors(ctx, dst):
    return _check(ctx, _lib.mgdd_get_test_vectors(ctx, _ptr(dst)))


def mgdd_restrict(ctx, prec, nrhs, fine, coarse):
    return _check(ctx, _lib.mgdd_restrict(ctx, prec, nrhs, _ptr(fine), _ptr(coarse)))


def mgdd_prolong(ctx, prec, nrhs, coarse, fine):
    return _check(ctx, _lib.mgdd_prolong(ctx, prec, nrhs, _ptr(coarse), _ptr(fine)))


def mgdd_coarse_apply(ctx, prec, nrhs, x, y):
    return _check(ctx, _lib.mgdd_coarse_apply(ctx, prec, nrhs, _ptr(x), _ptr(y)))


def mgdd_coarse_solve(ctx, prec, nrhs, iters, b, x):
    return _check(ctx, _lib.mgdd_coarse_solve(ctx, prec, nrhs, iters, _ptr(b), _ptr(x)))


def mgdd_coarse_solve_noalloc(ctx, prec, nrhs, iters, b, x):
    return _check(ctx, _lib.mgdd_coarse_solve_noalloc(ctx, prec, nrhs, iters, _ptr(b), _ptr(x)))


def mgdd_precondition(ctx, prec, nrhs, nu, mr_iters, coarse_iters, r, z):
    return _check(ctx, _lib.mgdd_precondition(ctx, prec, nrhs, nu, mr_iters, coarse_iters, _ptr(r), _ptr(z)))


def mgdd_net_weight_count(widths):
    sh = net_shape(widths)
    return _lib.mgdd_net_weight_count(ctypes.byref(sh))


def mgdd_net_apply(ctx, widths, weights, nsamples, x, y):
    sh = net_shape(widths)
    return _check(ctx, _lib.mgdd_net_apply(ctx, ctypes.byref(sh), _ptr(weights), nsamples, _ptr(x), _ptr(y)))


def mgdd_net_grad(ctx, widths, weights, nsamples, x, grad):
    sh = net_shape(widths)
    loss = ctypes.c_double()
    _check(ctx, _lib.mgdd_net_grad(ctx, ctypes.byref(sh), _ptr(weights), nsamples, _ptr(x), ctypes.byref(loss),
                                   _ptr(grad)))
    return loss.value


def mgdd_net_adam(ctx, widths, weights, grad, m, v, step, lr):
    sh = net_shape(widths)
    return _check(ctx, _lib.mgdd_net_adam(ctx, ctypes.byref(sh), _ptr(weights), _ptr(grad), _ptr(m), _ptr(v), step, lr))


def mgdd_setup_learned(ctx, widths, weights, params, random_vectors, arnoldi_start):
    sh = net_shape(widths)
    return _check(ctx, _lib.mgdd_setup_learned(ctx, ctypes.byref(sh), _ptr(weights), ctypes.byref(params),
                                               _ptr(random_vectors),
                                               None if arnoldi_start is None else _ptr(arnoldi_start)))


def mgdd_schwarz(ctx, prec, nrhs, block, params: SchwarzParams, b, z):
    blk = None if block is None else _i4(*block)
    return _check(ctx, _lib.mgdd_schwarz(ctx, prec, nrhs, blk, ctypes.byref(params), _ptr(b), _ptr(z)))


def mgdd_precondition3(ctx, prec, nrhs, nu, mr_iters, k2, nu2, mr2, coarse_iters, r, z):
    return _check(ctx, _lib.mgdd_precondition3(ctx, prec, nrhs, nu, mr_iters, k2, nu2, mr2, coarse_iters, _ptr(r),
                                               _ptr(z)))


def mgdd_setup_level2(ctx, params: Level2Params, random2):
    return _check(ctx, _lib.mgdd_setup_level2(ctx, ctypes.byref(params), None if random2 is None else _ptr(random2)))


def mgdd_setup_bootstrap(ctx, params: SetupParams, random_vectors, arnoldi_start):
    return _check(ctx, _lib.mgdd_setup_bootstrap(ctx, ctypes.byref(params), _ptr(random_vectors), _ptr(arnoldi_start)))


def mgdd_solve(ctx, params: SolveParams, nrhs, b, z, allow_noconv=False):
    """Returns a list of SolveStats (one per right-hand side)."""
    stats = (SolveStats * nrhs)()
    rc = _lib.mgdd_solve(ctx, ctypes.byref(params), nrhs, _ptr(b), _ptr(z), stats)
    if not (rc == ENOCONV and allow_noconv):
        _check(ctx, rc)
    return [stats[i] for i in range(nrhs)]


def mgdd_build_P2(ctx, agg2, ntv2, test_vectors2):
    return _check(ctx, _lib.mgdd_build_P2(ctx, _i4(*agg2), ntv2, _ptr(test_vectors2)))


def mgdd_restrict2(ctx, prec, nrhs, coarse, coarse2):
    return _check(ctx, _lib.mgdd_restrict2(ctx, prec, nrhs, _ptr(coarse), _ptr(coarse2)))


def mgdd_prolong2(ctx, prec, nrhs, coarse2, coarse):
    return _check(ctx, _lib.mgdd_prolong2(ctx, prec, nrhs, _ptr(coarse2), _ptr(coarse)))


def mgdd_coarse2_apply(ctx, prec, nrhs, x, y):
    return _check(ctx, _lib.mgdd_coarse2_apply(ctx, prec, nrhs, _ptr(x), _ptr(y)))


def mgdd_coarse_sap(ctx, prec, nrhs, block2, nsweeps, mr_iters, b, z):
    return _check(ctx, _lib.mgdd_coarse_sap(ctx, prec, nrhs, _i4(*block2), nsweeps, mr_iters, _ptr(b), _ptr(z)))


def mgdd_timing_enable(ctx, on=True):
    return _check(ctx, _lib.mgdd_timing_enable(ctx, 1 if on else 0))


def mgdd_timing_read(ctx, kernel, prec, reset=False):
    """Returns (total_ms, site_updates, launches) for one kernel family."""
    ms, units, n, nbytes = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
    _check(ctx, _lib.mgdd_timing_read(ctx, kernel, prec, 1 if reset else 0, ctypes.byref(ms), ctypes.byref(units),
                                      ctypes.byref(n), ctypes.byref(nbytes)))
    return ms.value, units.value, n.value, nbytes.value


# --------------------------------------------------------------------- convenience wrapper

class Lattice:
    """Owns one context; fields are torch tensors shaped (nrhs, 12, V, 2) of
    float64 (F64) or float32 (F32) in the device layout."""

    def __init__(self, dims, block, stream=None, t_antiperiodic=True):
        import torch
        self.torch = torch
        self.dims = tuple(int(d) for d in dims)
        self.block = tuple(int(b) for b in block)
        self.V = int(np.prod(self.dims))
        self.ctx = mgdd_create(self.dims, block, stream, t_antiperiodic)

    def close(self):
        if self.ctx:
            mgdd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, prec=F64, nrhs=1):
        t = self.torch
        dt = {F64: t.float64, F32: t.float32, F16: t.float16}[prec]
        return t.zeros((nrhs, 12, self.V, 2), dtype=dt, device="cuda")

    def set_gauge(self, U, m0, csw):
        mgdd_set_gauge(self.ctx, U, m0, csw)

    def pack(self, canon: np.ndarray, prec=F64):
        canon = np.asarray(canon, dtype=np.complex128)
        if canon.ndim == 3:
            canon = canon[None]
        f = self.field(prec, canon.shape[0])
        mgdd_pack(self.ctx, prec, canon.shape[0], canon, f)
        return f

    def unpack(self, f, prec=None) -> np.ndarray:
        prec = self.prec_of(f) if prec is None else prec
        nrhs = f.shape[0]
        out = np.zeros((nrhs, self.V, 4, 3), dtype=np.complex128)
        mgdd_unpack(self.ctx, prec, nrhs, f, out)
        return out

    @staticmethod
    def prec_of(f):
        import torch
        return {torch.float64: F64, torch.float32: F32, torch.float16: F16}[f.dtype]

    def dirac(self, x, y=None):
        y = self.torch.empty_like(x) if y is None else y
        mgdd_dirac_apply(self.ctx, self.prec_of(x), x.shape[0], x, y)
        return y

    def sap(self, b, z, nsweeps, mr_iters, shift=0.0):
        mgdd_sap(self.ctx, self.prec_of(b), b.shape[0], self.block, nsweeps, mr_iters, shift, b, z)
        return z

    def schwarz(self, b, z, nsweeps=1, k=3, block_solver=BLOCK_GMRES, additive=False, shift=0.0):
        """Schwarz sweeps on (D - shift) z = b (z updated in place): red-black or
        additive, MR(k) or GMRES(k) block solves."""
        q = SchwarzParams(nsweeps, k, block_solver, 1 if additive else 0, complex(shift).real, complex(shift).imag)
        mgdd_schwarz(self.ctx, self.prec_of(b), b.shape[0], self.block, q, b, z)
        return z

    # coarse level -------------------------------------------------------
    def build_P(self, agg, test_vectors):
        """test_vectors: (N, 12, V, 2) float64 device tensor."""
        mgdd_build_P(self.ctx, agg, test_vectors.shape[0], test_vectors)
        self.agg = tuple(agg)
        self.N = test_vectors.shape[0]
        self.cdims = tuple(d // a for d, a in zip(self.dims, self.agg))
        self.Vc = int(np.prod(self.cdims))

    # third level -------------------------------------------------------
    def build_P2(self, agg2, test_vectors2):
        """test_vectors2: (N2, Vc, 2, N, 2) float64 device tensor of coarse fields."""
        mgdd_build_P2(self.ctx, agg2, test_vectors2.shape[0], test_vectors2)
        self.agg2 = tuple(agg2)
        self.N2 = test_vectors2.shape[0]
        self.ccdims = tuple(d // a for d, a in zip(self.cdims, self.agg2))
        self.Vcc = int(np.prod(self.ccdims))

    def coarse2_field(self, prec=F64, nrhs=1):
        t = self.torch
        dt = t.float64 if prec == F64 else t.float32
        return t.zeros((nrhs, self.Vcc, 2, self.N2, 2), dtype=dt, device="cuda")

    def restrict2(self, c, cc=None):
        cc = self.coarse2_field(self.prec_of(c), c.shape[0]) if cc is None else cc
        mgdd_restrict2(self.ctx, self.prec_of(c), c.shape[0], c, cc)
        return cc

    def prolong2(self, cc, c=None):
        c = self.coarse_field(self.prec_of(cc), cc.shape[0]) if c is None else c
        mgdd_prolong2(self.ctx, self.prec_of(cc), cc.shape[0], cc, c)
        return c

    def coarse_sap(self, block2, b, z, nsweeps=1, mr_iters=4):
        """nsweeps red-black Schwarz sweeps on D_c z = b (z updated in place)."""
        mgdd_coarse_sap(self.ctx, self.prec_of(b), b.shape[0], block2, nsweeps, mr_iters, b, z)
        return z

    def coarse2_apply(self, x, y=None):
        y = self.torch.empty_like(x) if y is None else y
        mgdd_coarse2_apply(self.ctx, self.prec_of(x), x.shape[0], x, y)
        return y

    def coarse_field(self, prec=F64, nrhs=1):
        t = self.torch
        dt = t.float64 if prec == F64 else t.float32
        return t.zeros((nrhs, self.Vc, 2, self.N, 2), dtype=dt, device="cuda")

    def restrict(self, f, c=None):
        """coarse = P^H f; a half-precision f gives an FP32 coarse field."""
        p = self.prec_of(f)
        c = self.coarse_field(F32 if p == F16 else p, f.shape[0]) if c is None else c
        mgdd_restrict(self.ctx, p, f.shape[0], f, c)
        return c

    def prolong(self, c, f=None):
        """f = P c; f in the precision of c, or of the given f (half precision
        from an FP32 c)."""
        f = self.field(self.prec_of(c), c.shape[0]) if f is None else f
        mgdd_prolong(self.ctx, self.prec_of(f), c.shape[0], c, f)
        return f

    def coarse_apply(self, x, y=None):
        y = self.torch.empty_like(x) if y is None else y
        mgdd_coarse_apply(self.ctx, self.prec_of(x), x.shape[0], x, y)
        return y

    def coarse_solve(self, b, iters=12, x=None):
        x = self.torch.empty_like(b) if x is None else x
        mgdd_coarse_solve(self.ctx, self.prec_of(b), b.shape[0], iters, b, x)
        return x

    def precondition(self, r, prec=F64, nu=1, mr_iters=4, coarse_iters=12):
        z = self.field(prec, r.shape[0])
        mgdd_precondition(self.ctx, prec, r.shape[0], nu, mr_iters, coarse_iters, r, z)
        return z

    def precondition3(self, r, prec=F64, nu=1, mr_iters=4, k2=8, nu2=1, mr2=4, coarse_iters=12):
        z = self.field(prec, r.shape[0])
        mgdd_precondition3(self.ctx, prec, r.shape[0], nu, mr_iters, k2, nu2, mr2, coarse_iters, r, z)
        return z

    def setup_level2(self, agg2, ntv2, block2, random2=None, nu2=2, mr_iters=4):
        """random2: (ntv2 - N, Vc, 2, N, 2) float64 device tensor (needed when ntv2 > N)."""
        lp = Level2Params((ctypes.c_int * 4)(*agg2), ntv2, (ctypes.c_int * 4)(*block2), nu2, mr_iters)
        mgdd_setup_level2(self.ctx, lp, random2)
        self.agg2 = tuple(agg2)
        self.N2 = ntv2
        self.ccdims = tuple(d // a for d, a in zip(self.cdims, self.agg2))
        self.Vcc = int(np.prod(self.ccdims))

    def save_setup(self, path):
        _check(self.ctx, _lib.mgdd_save_setup(self.ctx, os.fsencode(path)))

    def load_setup(self, path):
        """rebuilds P and D_c from a setup file written by save_setup"""
        import struct
        _check(self.ctx, _lib.mgdd_load_setup(self.ctx, os.fsencode(path)))
        with open(path, "rb") as f:
            head = struct.unpack("<8s4i4i2i2d2Q", f.read(80))
        agg, ntv = head[5:9], head[9]
        self.agg = tuple(agg)
        self.N = ntv
        self.cdims = tuple(d // a for d, a in zip(self.dims, self.agg))
        self.Vc = int(np.prod(self.cdims))

    def release_workspace(self):
        _check(self.ctx, _lib.mgdd_release_workspace(self.ctx))

    # learned setup ----------------------------------------------------
    def weights_to_dev(self, Ws):
        """list of complex arrays [c_out, c_in, 9] -> device FP64 weights"""
        flat = np.concatenate([np.asarray(W, dtype=np.complex128).ravel() for W in Ws])
        return self.torch.tensor(np.stack([flat.real, flat.imag], -1), dtype=self.torch.float64, device="cuda")

    @staticmethod
    def weights_from_dev(t, widths):
        a = t.detach().cpu().numpy()
        flat = a[:, 0] + 1j * a[:, 1]
        out, o = [], 0
        for cin, cout in zip(widths[:-1], widths[1:]):
            out.append(flat[o:o + cout * cin * 9].reshape(cout, cin, 9))
            o += cout * cin * 9
        return out

    def net_apply(self, widths, weights, x):
        y = self.torch.empty_like(x)
        mgdd_net_apply(self.ctx, widths, weights, x.shape[0], x, y)
        return y

    def net_grad(self, widths, weights, x):
        grad = self.torch.empty_like(weights)
        loss = mgdd_net_grad(self.ctx, widths, weights, x.shape[0], x, grad)
        return loss, grad

    def net_adam(self, widths, weights, grad, m, v, step, lr):
        mgdd_net_adam(self.ctx, widths, weights, grad, m, v, step, lr)

    def setup_learned(self, widths, weights, agg, random_vectors, arnoldi_start=None, nu=0, iota=3, mr_iters=4,
                      n_part2=0, prec=F32, ntv=None, seed=0):
        """random_vectors: N FP64 fields, or None to have the library draw ntv
        of them from stream `seed`"""
        N = random_vectors.shape[0] if random_vectors is not None else int(ntv)
        sp = SetupParams((ctypes.c_int * 4)(*agg), N, nu, iota, mr_iters, 0, n_part2, prec, 0, seed)
        mgdd_setup_learned(self.ctx, widths, weights, sp, random_vectors, arnoldi_start)
        self.agg = tuple(agg)
        self.N = N
        self.cdims = tuple(d // a for d, a in zip(self.dims, self.agg))
        self.Vc = int(np.prod(self.cdims))

    def setup_fell_back(self):
        """True when the last setup_learned fell back to the plain bootstrap"""
        return bool(_lib.mgdd_setup_fallback(self.ctx))

    def setup(self, agg, random_vectors, arnoldi_start, nu=3, iota=3, mr_iters=4, arnoldi_m=0, n_part2=1, prec=F64,
              chunk=0, ntv=None, seed=0):
        """random_vectors: N FP64 fields, or None to have the library draw
        ntv of them from stream `seed`"""
        N = random_vectors.shape[0] if random_vectors is not None else int(ntv)
        sp = SetupParams((ctypes.c_int * 4)(*agg), N, nu, iota, mr_iters, arnoldi_m, n_part2, prec, chunk, seed)
        mgdd_setup_bootstrap(self.ctx, sp, random_vectors, arnoldi_start)
        self.agg = tuple(agg)
        self.N = N
        self.cdims = tuple(d // a for d, a in zip(self.dims, self.agg))
        self.Vc = int(np.prod(self.cdims))

    def test_vectors(self):
        out = self.field(F64, self.N)
        mgdd_get_test_vectors(self.ctx, out)
        return out

    def solve(self, b, z=None, solver=SOLVER_FGMRES_MG, precision=PLAIN_F64, restart=20, tol=1e-10, maxit=1000,
              coarse_iters=12, nu=1, mr_iters=4, allow_noconv=False, levels=2, k2=8, nu2=1, mr2=4,
              block_solver=BLOCK_MR, additive=False):
        z = self.torch.zeros_like(b) if z is None else z
        sp = SolveParams(solver, precision, restart, tol, maxit, coarse_iters, nu, mr_iters, levels, k2, nu2, mr2,
                         block_solver, 1 if additive else 0)
        stats = mgdd_solve(self.ctx, sp, b.shape[0], b, z, allow_noconv=allow_noconv)
        return z, stats
