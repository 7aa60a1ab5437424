"""Pins of the oracle's learned-setup network (oracle/learned.py): the hops
against plane waves of the free field and against the Wilson operator's own
hopping term, adjointness of the hops and of a layer, gauge covariance of the
network, and the hand-derived gradients against finite differences of the
loss."""
import numpy as np
import pytest

import latgen
import oracle
from helpers import random_op, rel
from oracle import learned as nl
from oracle.solvers import TwoLevel

DIMS = (4, 4, 2, 6)


def gauge_transformed(dims, U, Om):
    """U^Om_mu(x) = Om(x) U_mu(x) Om(x + mu)^H"""
    Lx, Ly, Lz, Lt = dims
    V = U.shape[0]
    s = np.arange(V)
    x = np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], 1)
    out = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % dims[mu]
        sn = y[:, 0] + Lx * (y[:, 1] + Ly * (y[:, 2] + Lz * y[:, 3]))
        out[:, mu] = np.einsum("sab,sbc,sdc->sad", Om, U[:, mu], np.conj(Om[sn]))
    return out


def test_hops_on_free_plane_waves():
    """U = 1: T_{1+2mu} e^{ipx} chi = e^{i p_mu} e^{ipx} chi and T_{2+2mu} gives
    e^{-i p_mu}, with p_t = (2k+1) pi / L_t (antiperiodic) and p_k = 2 pi n / L_k"""
    V = int(np.prod(DIMS))
    U = np.tile(np.eye(3, dtype=complex), (V, 4, 1, 1))
    Lx, Ly, Lz, Lt = DIMS
    s = np.arange(V)
    x = np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], 1)
    p = np.array([2 * np.pi * 1 / Lx, 2 * np.pi * 3 / Ly, 0.0, (2 * 2 + 1) * np.pi / Lt])
    chi = latgen.gaussian_vector(12, 3).reshape(4, 3)
    psi = np.exp(1j * (x @ p))[:, None, None] * chi[None]
    for mu in range(4):
        assert rel(nl.hop(DIMS, U, 1 + 2 * mu, psi), np.exp(1j * p[mu]) * psi) < 1e-13
        assert rel(nl.hop(DIMS, U, 2 + 2 * mu, psi), np.exp(-1j * p[mu]) * psi) < 1e-13


def test_hops_rebuild_the_wilson_operator():
    """D = A - 1/2 sum_mu [(1 - gamma_mu) T_{1+2mu} + (1 + gamma_mu) T_{2+2mu}]
    with the spin matrices applied to the colour hops of the network"""
    op = random_op(DIMS, seed=31, m0=0.2)
    psi = latgen.gaussian_fields(DIMS, 1, 4)[0]
    G, _ = oracle.gamma()
    out = np.einsum("sij,sj->si", op.A, psi.reshape(-1, 12)).reshape(psi.shape)
    for mu in range(4):
        f = nl.hop(DIMS, op.U, 1 + 2 * mu, psi)
        b = nl.hop(DIMS, op.U, 2 + 2 * mu, psi)
        out = out - 0.5 * (np.einsum("ij,sjc->sic", np.eye(4) - G[mu], f) + np.einsum("ij,sjc->sic", np.eye(4) + G[mu], b))
    assert rel(out, op.apply(psi)) < 1e-13


def test_hop_and_layer_adjoints():
    op = random_op(DIMS, seed=32)
    x, y = latgen.gaussian_fields(DIMS, 2, 5)
    for h in range(9):
        hb = 0 if h == 0 else (h + 1 if h % 2 else h - 1)
        lhs = np.vdot(nl.hop(DIMS, op.U, h, x), y)
        rhs = np.vdot(x, nl.hop(DIMS, op.U, hb, y))
        assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)
    W = latgen.network_weights([3, 2], 6)[0]
    X = latgen.gaussian_fields(DIMS, 3, 7)
    Y = latgen.gaussian_fields(DIMS, 2, 8)
    lhs = np.vdot(nl.layer(DIMS, op.U, W, X), Y)
    rhs = np.vdot(X, nl.layer_adjoint(DIMS, op.U, W, Y))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(X) * np.linalg.norm(Y)


def test_network_is_gauge_covariant_and_linear():
    op = random_op(DIMS, seed=33)
    V = op.U.shape[0]
    Ws = latgen.network_weights([1, 3, 3, 1], 9)
    Om = latgen.gauge_transform(10, V)
    Ug = gauge_transformed(DIMS, op.U, Om)
    psi, chi = latgen.gaussian_fields(DIMS, 2, 11)
    f = nl.forward(DIMS, op.U, Ws, psi)[-1][0]
    fg = nl.forward(DIMS, Ug, Ws, np.einsum("sab,spb->spa", Om, psi))[-1][0]
    assert rel(fg, np.einsum("sab,spb->spa", Om, f)) < 1e-13
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    lin = nl.forward(DIMS, op.U, Ws, a * psi + b * chi)[-1][0]
    fc = nl.forward(DIMS, op.U, Ws, chi)[-1][0]
    assert rel(lin, a * f + b * fc) < 1e-13


def test_gradients_match_finite_differences():
    dims, block, agg = (4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)
    op = random_op(dims, seed=34, m0=0.2)
    tv = latgen.gaussian_fields(dims, 3, 12)
    tl = TwoLevel(op, agg, tv, block)
    project = lambda v: tl.prolong(tl.restrict(v))
    Ws = latgen.network_weights([1, 2, 2, 1], 13)
    psi = latgen.gaussian_fields(dims, 1, 14)[0]
    L, grads = nl.loss_and_grad(dims, op.U, Ws, psi, project)
    assert 0 < L < 1
    rng = np.random.default_rng(0)
    eps = 1e-6
    for _ in range(8):
        l = int(rng.integers(len(Ws)))
        idx = tuple(int(rng.integers(n)) for n in Ws[l].shape)
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            Wp = [W.copy() for W in Ws]
            Wm = [W.copy() for W in Ws]
            Wp[l][idx] += eps * unit
            Wm[l][idx] -= eps * unit
            Lp = nl.loss_and_grad(dims, op.U, Wp, psi, project)[0]
            Lm = nl.loss_and_grad(dims, op.U, Wm, psi, project)[0]
            fd = (Lp - Lm) / (2 * eps)
            assert abs(fd - 2 * part(grads[l][idx])) < 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][idx])
