"""Seeded synthetic inputs for the Wilson-clover multilevel solver.

This module is the only code shared by the GPU library's callers and the CPU
oracle. It holds no arithmetic of the solver itself: it draws random numbers,
builds SU(3) gauge links from them, smooths those links, and lays out
right-hand sides and random start vectors. Everything the solver computes from
these inputs (clover term, Dirac operator, smoother, interpolation, coarse
operator, Krylov solvers) lives elsewhere.

Conventions shared by every caller (canonical host layout, complex128):
  * site index  s = x + Lx*(y + Ly*(z + Lz*t)),  dims = (Lx, Ly, Lz, Lt)
  * gauge field U[s, mu, a, b]     mu = 0..3 for x, y, z, t
  * spinor field psi[s, spin, colour]  (4 spins x 3 colours = 12 dof/site)
  * a batch of fields is stacked on a leading axis.

Random numbers: SplitMix64 (Steele, Lea, Flood 2014) used as a counter-based
generator, value i of stream `seed` = mix64(seed*GOLDEN + (i+1)*GOLDEN);
uniforms take the top 53 bits; normals come from the Box-Muller transform.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# seed tags: seed = 1000*config + tag
TAG_GAUGE, TAG_EPS, TAG_RHS, TAG_TV, TAG_POINT, TAG_ARNOLDI, TAG_TV2 = 1, 2, 3, 4, 5, 6, 7


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n uniforms in [0,1) from counter positions offset..offset+n-1."""
    with np.errstate(over="ignore"):
        base = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * _GOLDEN
        ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = _mix64(base + ctr * _GOLDEN)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed: int, n: int) -> np.ndarray:
    """n standard normals (Box-Muller on pairs of uniforms)."""
    m = (n + 1) // 2
    u = uniform(seed, 2 * m)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log1p(-u1))
    th = 2.0 * np.pi * u2
    out = np.empty(2 * m)
    out[0::2] = r * np.cos(th)
    out[1::2] = r * np.sin(th)
    return out[:n]


def volume(dims) -> int:
    return int(dims[0]) * int(dims[1]) * int(dims[2]) * int(dims[3])


# ---------------------------------------------------------------- gauge links

def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def reunitarize(U: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 1, 2; row 3 = conj(row1 x row2): exact SU(3)."""
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def random_links(dims, eps: float, seed: int) -> np.ndarray:
    """U = exp(i*eps*H) per link, H = sum_a w_a lambda_a / 2, w_a ~ N(0,1)."""
    V = volume(dims)
    w = normal(seed, V * 4 * 8).reshape(V * 4, 8)
    H = np.einsum("na,aij->nij", w, _gell_mann() / 2.0)
    h, Q = np.linalg.eigh(H)
    U = np.einsum("nij,nj,nkj->nik", Q, np.exp(1j * eps * h), np.conj(Q))
    return reunitarize(U).reshape(V, 4, 3, 3)


def _shift(U4: np.ndarray, mu: int, step: int) -> np.ndarray:
    """Field at x + step*mu_hat (periodic), for fields shaped (Lt,Lz,Ly,Lx,...)."""
    axis = 3 - mu
    return np.roll(U4, -step, axis=axis)


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def project_su3(X: np.ndarray) -> np.ndarray:
    """Polar projection X (X^H X)^(-1/2), then divide by the principal cube root of det."""
    h, Q = np.linalg.eigh(_dag(X) @ X)
    inv_sqrt = np.einsum("...ij,...j,...kj->...ik", Q, 1.0 / np.sqrt(h), np.conj(Q))
    W = X @ inv_sqrt
    d = np.linalg.det(W)
    W = W / (d ** (1.0 / 3.0))[..., None, None]
    return reunitarize(W)


def ape_smear(U: np.ndarray, dims, alpha: float, steps: int) -> np.ndarray:
    """APE smearing of periodic links, all links updated together per step."""
    Lx, Ly, Lz, Lt = dims
    U4 = U.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)
    for _ in range(steps):
        new = np.empty_like(U4)
        for mu in range(4):
            Umu = U4[..., mu, :, :]
            stap = np.zeros_like(Umu)
            for nu in range(4):
                if nu == mu:
                    continue
                Unu = U4[..., nu, :, :]
                # upper: U_nu(x) U_mu(x+nu) U_nu(x+mu)^H
                stap += Unu @ _shift(Umu, nu, 1) @ _dag(_shift(Unu, mu, 1))
                # lower: U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu)
                Unu_m = _shift(Unu, nu, -1)
                stap += _dag(Unu_m) @ _shift(Umu, nu, -1) @ _shift(_shift(Unu, nu, -1), mu, 1)
            new[..., mu, :, :] = project_su3((1.0 - alpha) * Umu + (alpha / 6.0) * stap)
        U4 = new
    return U4.reshape(-1, 4, 3, 3)


def gauge_field(dims, eps: float, seed: int, ape_steps: int = 0, ape_alpha: float = 0.5) -> np.ndarray:
    U = random_links(dims, eps, seed)
    if ape_steps:
        U = ape_smear(U, dims, ape_alpha, ape_steps)
    return np.ascontiguousarray(U)


def eps_from_seed(seed: int, lo: float = 0.4, hi: float = 0.6) -> float:
    return float(lo + (hi - lo) * uniform(seed, 1)[0])


def gauge_transform(seed: int, V: int) -> np.ndarray:
    """Random SU(3) matrix per site (for covariance tests)."""
    return random_links((V, 1, 1, 1), 1.0, seed)[:, 0]


# ---------------------------------------------------------------- fields

def gaussian_fields(dims, n: int, seed: int) -> np.ndarray:
    """n complex Gaussian spinor fields, re and im ~ N(0,1): shape (n, V, 4, 3)."""
    V = volume(dims)
    g = normal(seed, 2 * n * V * 12)
    return (g[0::2] + 1j * g[1::2]).reshape(n, V, 4, 3)


def point_sources(dims, seed: int) -> np.ndarray:
    """12 point sources (spin, colour) at one seeded site: shape (12, V, 4, 3)."""
    V = volume(dims)
    x0 = int(uniform(seed, 1)[0] * V)
    out = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for i in range(12):
        out[i, x0, i // 3, i % 3] = 1.0
    return out


def gaussian_vector(n: int, seed: int) -> np.ndarray:
    g = normal(seed, 2 * n)
    return g[0::2] + 1j * g[1::2]


# ---------------------------------------------------------------- workloads

WORKLOADS = {
    # 8^4, plain FP64 two-level solve
    "c0": dict(dims=(8, 8, 8, 8), eps=0.35, ape=0, csw=1.0, target=0.05, block=(4, 4, 4, 4),
               agg=(4, 4, 4, 4), ntv=8, nu=3, iota=3, mr=4, restart=20, tol=1e-10, nrhs=1),
    # 16^3x32, FP32 SAP inside FP64 FGMRES
    "c1": dict(dims=(16, 16, 16, 32), eps=0.5, ape=2, csw=1.0, target=0.01, block=(4, 4, 4, 4),
               agg=(4, 4, 4, 4), ntv=20, nu=3, iota=3, mr=4, restart=20, tol=1e-10, nrhs=1),
    # 32^3x64, 12 point sources batched
    "c2": dict(dims=(32, 32, 32, 64), eps=None, ape=2, csw=1.0, target=0.01, block=(4, 4, 4, 4),
               agg=(4, 4, 4, 4), ntv=24, nu=3, iota=3, mr=4, restart=20, tol=1e-10, nrhs=12),
    # 48^3x96
    "c3": dict(dims=(48, 48, 48, 96), eps=None, ape=2, csw=1.0, target=0.005, block=(4, 4, 4, 4),
               agg=(4, 4, 4, 4), ntv=20, nu=3, iota=3, mr=4, restart=30, tol=1e-10, nrhs=1),
}


def workload_gauge(name: str, dims=None) -> np.ndarray:
    """Gauge field of a named workload (optionally on other dims, same recipe)."""
    k = int(name[1:])
    w = WORKLOADS[name]
    dims = tuple(dims or w["dims"])
    eps = w["eps"] if w["eps"] is not None else eps_from_seed(1000 * k + TAG_EPS)
    return gauge_field(dims, eps, 1000 * k + TAG_GAUGE, ape_steps=w["ape"])


def network_weights(widths, seed):
    """Seeded complex weights of a gauge-covariant network with the given
    channel widths (layer l: [widths[l+1], widths[l], 9]): Gaussian entries of
    scale 0.1 / sqrt(fan-in), plus 1 / fan-in on the identity hop, so that the
    initial network is close to a multiple of the identity."""
    rng = np.random.default_rng(seed)
    Ws = []
    for cin, cout in zip(widths[:-1], widths[1:]):
        W = (rng.standard_normal((cout, cin, 9)) + 1j * rng.standard_normal((cout, cin, 9))) * (0.1 / np.sqrt(cin))
        W[:, :, 0] += 1.0 / cin
        Ws.append(W)
    return Ws
