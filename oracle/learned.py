"""Learned setup, for the oracle: a gauge-covariant network that maps random
vectors to test vectors, its training loss and gradients.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py). Plain numpy in FP64 on
canonical fields psi[site][spin][colour] (site = x + Lx (y + Ly (z + Lz t))).

The network is not part of the paper; it replaces the test-vector
iterations of its bootstrap setup (Section 3). Each layer maps C_in channels
to C_out channels:

    y[c] = sum_{c', h} W[c, c', h] T_h x[c'],   h = 0 .. 8,

with complex scalar weights and the colour hops of the Wilson stencil
(no spin projection): T_0 = 1, (T_{1+2mu} x)(s) = eta U_mu(s) x(s + mu),
(T_{2+2mu} x)(s) = eta U_mu(s - mu)^H x(s - mu), eta = -1 on hops across
the time boundary (the antiperiodic condition of D). T_{2+2mu} is the
adjoint of T_{1+2mu}, and a gauge transformation G acts as G T_h G^H, so
every layer, and the network, commutes with gauge transformations.

Training loss for one input psi and the interpolation P of a bootstrap
setup on the same gauge field: L = ||(1 - P P^H) f||^2 / ||f||^2 with
f = net(psi): the part of the output outside the bootstrap's coarse space.
Gradients are the Wirtinger derivatives dL/dconj(.) (for a real loss the
direction of steepest ascent), by the chain rule through the layers:
g_f = ((1 - P P^H) f - L f) / ||f||^2; for a layer, grad W[c, c', h] =
<T_h x[c'], g_y[c]> and g_x[c'] = sum_{c, h} conj(W[c, c', h]) T_h^H g_y[c].
"""
from __future__ import annotations

import numpy as np

NHOP = 9


def _grid(dims, a):
    """(V, ...) -> (Lt, Lz, Ly, Lx, ...)"""
    Lx, Ly, Lz, Lt = dims
    return a.reshape((Lt, Lz, Ly, Lx) + a.shape[1:])


def _axis(mu):
    return 3 - mu   # x, y, z, t -> axes 3, 2, 1, 0 of the grid


def _tsign(dims, forward):
    """-1 on the sites whose t hop crosses the boundary"""
    Lt = dims[3]
    s = np.ones(Lt)
    s[Lt - 1 if forward else 0] = -1.0
    return s[:, None, None, None, None, None]


def hop(dims, U, h, x):
    """T_h x for one field x[V, 4, 3]"""
    if h == 0:
        return np.array(x, dtype=np.complex128, copy=True)
    mu, back = (h - 1) // 2, (h - 1) % 2
    Ug = _grid(dims, np.asarray(U))[..., mu, :, :]        # (Lt, Lz, Ly, Lx, 3, 3)
    xg = _grid(dims, np.asarray(x, dtype=np.complex128))   # (..., 4, 3)
    ax = _axis(mu)
    if not back:
        y = np.einsum('...ab,...sb->...sa', Ug, np.roll(xg, -1, axis=ax))
    else:
        y = np.roll(np.einsum('...ba,...sb->...sa', Ug.conj(), xg), 1, axis=ax)
    if mu == 3:
        y = y * _tsign(dims, not back)
    return y.reshape(np.shape(x))


def layer(dims, U, W, x):
    """y[c] = sum_{c', h} W[c, c', h] T_h x[c']; W[C_out, C_in, 9], x[C_in, V, 4, 3]"""
    cout, cin, _ = W.shape
    y = np.zeros((cout,) + x.shape[1:], dtype=np.complex128)
    for cp in range(cin):
        for h in range(NHOP):
            t = hop(dims, U, h, x[cp])
            for c in range(cout):
                y[c] += W[c, cp, h] * t
    return y


def layer_adjoint(dims, U, W, g):
    """x-gradient of a layer: g_x[c'] = sum_{c, h} conj(W[c, c', h]) T_h^H g[c]"""
    cout, cin, _ = W.shape
    out = np.zeros((cin,) + g.shape[1:], dtype=np.complex128)
    for c in range(cout):
        for h in range(NHOP):
            hb = 0 if h == 0 else (h + 1 if h % 2 else h - 1)   # T_h^H = T_{h-bar}
            t = hop(dims, U, hb, g[c])
            for cp in range(cin):
                out[cp] += np.conj(W[c, cp, h]) * t
    return out


def layer_weight_grad(dims, U, x, g):
    """grad W[c, c', h] = <T_h x[c'], g[c]>"""
    cin, cout = x.shape[0], g.shape[0]
    G = np.zeros((cout, cin, NHOP), dtype=np.complex128)
    for cp in range(cin):
        for h in range(NHOP):
            t = hop(dims, U, h, x[cp]).ravel()
            for c in range(cout):
                G[c, cp, h] = np.vdot(t, g[c].ravel())
    return G


def forward(dims, U, Ws, psi):
    """activations [x_0 = psi[None], x_1, ..., x_L]; the output is x_L[0]"""
    xs = [np.asarray(psi, dtype=np.complex128)[None]]
    for W in Ws:
        xs.append(layer(dims, U, W, xs[-1]))
    return xs


def loss_and_grad(dims, U, Ws, psi, project):
    """L = ||(1 - Pi) f||^2 / ||f||^2 for f = net(psi), Pi = project (the
    map v -> P P^H v), and dL/dconj(W_l) for every layer"""
    xs = forward(dims, U, Ws, psi)
    f = xs[-1][0]
    ff = np.vdot(f, f).real
    qf = f - project(f)
    L = np.vdot(qf, qf).real / ff
    g = ((qf - L * f) / ff)[None]
    grads = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        grads[l] = layer_weight_grad(dims, U, xs[l], g)
        if l > 0:
            g = layer_adjoint(dims, U, Ws[l], g)
    return L, grads
