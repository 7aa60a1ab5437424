"""Pins of the oracle's Wilson-clover operator (Section 1, D = D(U) + m) against
closed forms and exact invariants: the gamma algebra, the free-field
plane-wave spectrum, gamma_5-hermiticity, gauge covariance, and a constant
abelian field whose clover term is known in closed form."""
import numpy as np
import pytest

import latgen
import oracle
from helpers import gamma5_field, random_op, rel, sort_spectrum
from oracle.solvers import Operator


def test_gamma_algebra():
    g, g5 = oracle.gamma()
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T, atol=0)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2.0 * np.eye(4) * (m == n), atol=1e-15)
    # chiral basis: gamma_5 diagonal, spins 0,1 chirality +, spins 2,3 chirality -
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=0)
    assert np.allclose(g5, g[3] @ g[0] @ g[1] @ g[2], atol=0)


def _free_symbol(dims, p, m0):
    """12x12 matrix M with D (e^{ipx} u) = e^{ipx} M u, read off the oracle."""
    V = int(np.prod(dims))
    s = np.arange(V)
    x = np.stack([s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2],
                  s // (dims[0] * dims[1] * dims[2])], axis=1)
    phase = np.exp(1j * (x @ np.asarray(p)))
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    op = Operator(dims, U, m0, 1.0)
    M = np.zeros((12, 12), dtype=np.complex128)
    for i in range(12):
        u = np.zeros(12, dtype=np.complex128)
        u[i] = 1
        psi = (phase[:, None] * u[None, :]).reshape(V, 4, 3)
        out = op.apply(psi).reshape(V, 12)
        col = out / phase[:, None]
        # the plane wave is mapped to a plane wave: the same column at every site
        assert np.max(np.abs(col - col[0])) < 1e-13
        M[:, i] = col[0]
    return M


@pytest.mark.parametrize("dims", [(4, 2, 2, 2), (2, 4, 3, 4)])
def test_free_field_plane_wave_spectrum(dims):
    """U = 1: D e^{ipx} u has eigenvalues m0 + sum(1-cos p) +- i sqrt(sum sin^2 p),
    each six-fold, with p_k = 2 pi n_k / L_k and p_t = (2 n_t + 1) pi / L_t."""
    m0 = 0.1
    rng = np.random.default_rng(0)
    for _ in range(6):
        n = [rng.integers(0, L) for L in dims]
        p = [2 * np.pi * n[k] / dims[k] for k in range(3)] + [(2 * n[3] + 1) * np.pi / dims[3]]
        M = _free_symbol(dims, p, m0)
        ev = sort_spectrum(np.linalg.eigvals(M))
        re = m0 + sum(1 - np.cos(q) for q in p)
        im = np.sqrt(sum(np.sin(q) ** 2 for q in p))
        want = sort_spectrum(np.array([re + 1j * im] * 6 + [re - 1j * im] * 6))
        assert np.max(np.abs(ev - want)) < 1e-12


def test_free_field_full_spectrum_dense():
    """All 192 eigenvalues of the dense free D on a 2^3 x 2 lattice match the
    closed form over every allowed momentum."""
    dims = (2, 2, 2, 2)
    m0 = 0.1
    V = 16
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    op = Operator(dims, U, m0, 1.0)
    from helpers import dense
    D = dense(op.apply, (V, 4, 3))
    ev = sort_spectrum(np.linalg.eigvals(D))
    want = []
    for nx in range(2):
        for ny in range(2):
            for nz in range(2):
                for nt in range(2):
                    p = [np.pi * nx, np.pi * ny, np.pi * nz, (2 * nt + 1) * np.pi / 2]
                    re = m0 + sum(1 - np.cos(q) for q in p)
                    im = np.sqrt(sum(np.sin(q) ** 2 for q in p))
                    want += [re + 1j * im] * 6 + [re - 1j * im] * 6
    want = sort_spectrum(np.array(want))
    assert np.max(np.abs(ev - want)) < 1e-12


def test_gamma5_hermiticity():
    dims = (4, 4, 4, 4)
    op = random_op(dims, seed=11, eps=0.8, m0=-0.2, csw=1.3)
    x = latgen.gaussian_fields(dims, 2, 5)
    lhs = np.vdot(x[0], gamma5_field(op.apply(gamma5_field(x[1]))))
    rhs = np.vdot(op.apply(x[0]), x[1])
    assert abs(lhs - rhs) / abs(rhs) < 1e-14


def test_clover_hermitian_and_chiral():
    dims = (4, 4, 2, 4)
    op = random_op(dims, seed=3, eps=0.9, csw=1.7)
    A = op.A
    assert np.max(np.abs(A - np.conj(np.swapaxes(A, 1, 2)))) < 1e-15
    # commutes with gamma_5: no coupling between spins {0,1} and {2,3}
    assert np.max(np.abs(A[:, :6, 6:])) == 0.0 or np.max(np.abs(A[:, :6, 6:])) < 1e-15
    assert np.max(np.abs(A[:, 6:, :6])) < 1e-15
    # m0 shifts the diagonal rigidly
    op2 = Operator(dims, op.U, op.m0 + 0.37, op.csw)
    assert np.max(np.abs(op2.A - op.A - 0.37 * np.eye(12))) < 1e-14


def _transform(dims, U, Om):
    V = int(np.prod(dims))
    Ug = np.empty_like(U)
    s = np.arange(V)
    for mu in range(4):
        x = [s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2],
             s // (dims[0] * dims[1] * dims[2])]
        x[mu] = (x[mu] + 1) % dims[mu]
        nb = x[0] + dims[0] * (x[1] + dims[1] * (x[2] + dims[2] * x[3]))
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[nb], 1, 2))
    return Ug


def test_gauge_covariance():
    """D[U^Om] (Om psi) = Om D[U] psi with U^Om_mu(x) = Om(x) U_mu(x) Om(x+mu)^H."""
    dims = (4, 2, 4, 6)
    op = random_op(dims, seed=5, eps=0.7, m0=0.1, csw=1.1)
    V = op.U.shape[0]
    Om = latgen.gauge_transform(99, V)
    opg = Operator(dims, _transform(dims, op.U, Om), op.m0, op.csw)
    psi = latgen.gaussian_fields(dims, 1, 8)[0]
    Om_psi = np.einsum("sab,spb->spa", Om, psi)
    lhs = opg.apply(Om_psi)
    rhs = np.einsum("sab,spb->spa", Om, op.apply(psi))
    assert rel(lhs, rhs) < 1e-14
    # the clover term is covariant on its own
    Ag = opg.A.reshape(V, 4, 3, 4, 3)
    Ar = np.einsum("sab,sibjc,sdc->siajd", Om, op.A.reshape(V, 4, 3, 4, 3), np.conj(Om))
    assert np.max(np.abs(Ag - Ar)) < 1e-14


def test_clover_constant_abelian_field():
    """U_y(x) = diag(exp(i theta_a x)), other links 1: every (x,y) leaf is
    diag(exp(i theta_a)), so F_xy = i diag(sin theta_a) and
    A = (4+m0) + (c_sw/2) (i sigma_xy)(i diag(sin theta)) ... = (4+m0) - (c_sw/2) sigma_xy (x) diag(sin theta)."""
    dims = (6, 4, 2, 2)
    V = int(np.prod(dims))
    th = np.array([2 * np.pi / 6, 2 * 2 * np.pi / 6])
    th = np.append(th, -th.sum())
    s = np.arange(V)
    x = s % dims[0]
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        U[:, mu] = np.eye(3)
    for a in range(3):
        U[:, 1, a, a] = np.exp(1j * th[a] * x)
    m0, csw = 0.2, 1.4
    g, _ = oracle.gamma()
    sigma_xy = 0.5j * (g[0] @ g[1] - g[1] @ g[0])
    want = (4 + m0) * np.eye(12) - 0.5 * csw * np.kron(sigma_xy, np.diag(np.sin(th)))
    for Uc in (U, _transform(dims, U, latgen.gauge_transform(4, V))):
        A = oracle.clover(dims, Uc, m0, csw)
        if Uc is U:
            assert np.max(np.abs(A - want[None])) < 1e-14
        else:
            # covariance: colour-rotated closed form, same spectrum at every site
            ev = np.linalg.eigvalsh(A)
            assert np.max(np.abs(ev - np.linalg.eigvalsh(want)[None])) < 1e-13
    # sigma_xy is diagonal in this basis: the closed form is diagonal
    assert np.allclose(sigma_xy, np.diag([-1, 1, -1, 1]))


def test_shifted_apply():
    dims = (2, 2, 4, 2)
    op = random_op(dims, seed=2)
    psi = latgen.gaussian_fields(dims, 1, 1)[0]
    sh = 0.3 - 0.7j
    assert rel(op.apply(psi, sh), op.apply(psi) - sh * psi) < 1e-15
