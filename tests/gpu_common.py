"""Helpers of the GPU parity tests: small seeded problems and the comparison
bar. The oracle supplies every expected value."""
from __future__ import annotations

import sys

import numpy as np

import latgen
from oracle.solvers import Operator

TOL64 = 1e-12     # relative, FP64 operator applies
TOL32 = 1e-5      # relative, FP32 operator applies


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b) -> float:
    d = np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
    n = np.linalg.norm(np.asarray(b).ravel())
    return float(d / n) if n > 0 else float(d)


def problem(dims, seed=3, eps=0.6, m0=0.1, csw=1.2, ape=0):
    U = latgen.gauge_field(dims, eps, seed, ape_steps=ape)
    return Operator(dims, U, m0, csw)


def lattice(op, block):
    from paper_1202_2462_amd.mgdd import Lattice
    lat = Lattice(op.dims, block)
    lat.set_gauge(op.U, op.m0, op.csw)
    return lat


def dev_to_np(t):
    """Complex numpy array of a device tensor with a trailing (re, im) axis."""
    a = t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def np_to_dev(c, prec):
    """Device tensor (trailing (re, im) axis) of a complex array, in FP64 or FP32."""
    import torch
    from paper_1202_2462_amd.mgdd import F64
    return torch.tensor(np.stack([np.real(c), np.imag(c)], -1), dtype=torch.float64 if prec == F64 else torch.float32,
                        device="cuda")
