"""A second, independent formulation of one step, for pinning the oracle on
tiny grids.

It differs from the oracle on purpose:
  * streaming is an explicit permutation matrix acting on the flattened state;
  * the D2Q9 BGK relaxation is done in raw-moment space, with equilibrium
    moments written in closed form (derived by hand from the second-order
    equilibrium of eq. feq with c_s^2 = 1/3), then mapped back with the
    inverse moment matrix;
  * the conservation projection is I - U U^T with U an orthonormal basis of
    span{1, c_x, c_y} obtained by QR, not the kappa formulas;
  * every routine accepts complex arrays, so exact Jacobian-vector products
    follow from the complex-step derivative Im f(x + i h v) / h.
"""
from __future__ import annotations

import numpy as np

# D2Q9 velocities in the order read from the paper's D3Q19 convention.
C9 = np.array([[0, 0], [-1, 0], [0, -1], [0, 1], [1, 0],
               [-1, -1], [-1, 1], [1, -1], [1, 1]], dtype=np.int64)
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def raw_moment_matrix():
    """Rows: monomials 1, cx, cy, cx^2, cy^2, cx cy, cx^2 cy, cx cy^2, cx^2 cy^2."""
    cx = C9[:, 0].astype(float)
    cy = C9[:, 1].astype(float)
    return np.stack([np.ones(9), cx, cy, cx * cx, cy * cy, cx * cy,
                     cx * cx * cy, cx * cy * cy, cx * cx * cy * cy])


def eq_moments(rho, jx, jy):
    """Raw moments of the second-order equilibrium, closed form:
    [rho, jx, jy, rho/3 + rho ux^2, rho/3 + rho uy^2, rho ux uy,
     rho uy / 3, rho ux / 3, rho (1/9 + |u|^2 / 3)]."""
    ux = jx / rho
    uy = jy / rho
    return np.stack([rho, jx, jy, rho / 3 + rho * ux * ux, rho / 3 + rho * uy * uy,
                     rho * ux * uy, rho * uy / 3, rho * ux / 3,
                     rho * (1.0 / 9.0 + (ux * ux + uy * uy) / 3.0)])


def projector():
    """I - U U^T, U orthonormal basis of span{1, c_x, c_y} (QR)."""
    B = np.stack([np.ones(9), C9[:, 0].astype(float), C9[:, 1].astype(float)], axis=1)
    U, _ = np.linalg.qr(B)
    return np.eye(9) - U @ U.T


def streaming_matrix(nx, ny):
    """S with (S v)[q, y', x'] = v[q, y, x] for (x', y') = (x + c_qx, y + c_qy) mod n."""
    N = nx * ny
    S = np.zeros((9 * N, 9 * N))
    for q in range(9):
        for y in range(ny):
            for x in range(nx):
                xd = (x + C9[q, 0]) % nx
                yd = (y + C9[q, 1]) % ny
                S[q * N + yd * nx + xd, q * N + y * nx + x] = 1.0
    return S


def mlp(theta, x, H):
    """y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3 for x of shape (9, N)."""
    Q = 9
    o = 0
    W1 = theta[o:o + H * Q].reshape(H, Q); o += H * Q
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    W3 = theta[o:o + Q * H].reshape(Q, H); o += Q * H
    b3 = theta[o:o + Q]
    h1 = np.tanh(W1 @ x + b1[:, None])
    h2 = np.tanh(W2 @ h1 + b2[:, None])
    return W3 @ h2 + b3[:, None]


def leaky(z, slope=0.01):
    """LeakyReLU on real or complex arrays; the branch is chosen by the real
    part, so complex-step derivatives are exact away from the kink."""
    return np.where(np.real(z) > 0, z, slope * z)


def mlp_paper(theta, x, widths=(300, 300, 100)):
    """The SI's network for x of shape (Q, N): three LeakyReLU layers of the
    given widths, then a linear layer back to Q; parameters packed per layer
    as W (out x in, row-major) then b."""
    Q = x.shape[0]
    dims = (Q,) + tuple(widths) + (Q,)
    o = 0
    h = x
    for l in range(len(dims) - 1):
        nin, nout = dims[l], dims[l + 1]
        W = theta[o:o + nout * nin].reshape(nout, nin); o += nout * nin
        b = theta[o:o + nout]; o += nout
        h = W @ h + b[:, None]
        if l + 2 < len(dims):
            h = leaky(h)
    assert o == theta.size
    return h


def step(g, nx, ny, tau, rho0=1.0, theta=None, H=0, out_scale=1.0, force=None, net="tanh"):
    """One step on a flattened canonical state g of length 9 nx ny (deviations).
    force: (Fx, Fy) arrays of shape (N,) or None.  net "paper" uses the SI's
    LeakyReLU network (H is then ignored, theta selects it)."""
    N = nx * ny
    M = raw_moment_matrix()
    Minv = np.linalg.inv(M)
    gq = g.reshape(9, N)
    f = gq + W9[:, None] * rho0
    m = M @ f
    rho, jx, jy = m[0], m[1], m[2]
    meq = eq_moments(rho, jx, jy)
    upd = Minv @ ((meq - m) / tau)
    if theta is not None and net == "paper":
        upd = upd + (out_scale / tau) * mlp_paper(theta, gq)
    elif theta is not None and H > 0:
        upd = upd + (out_scale / tau) * mlp(theta, gq, H)
    upd = projector() @ upd
    post = gq + upd
    if force is not None:
        Fx, Fy = force
        post = post + Minv @ (eq_moments(rho, jx + Fx, jy + Fy) - eq_moments(rho, jx, jy))
    return streaming_matrix(nx, ny) @ post.reshape(-1)


def kolmogorov_force(nx, ny, amp, k):
    y = np.repeat(np.arange(ny, dtype=float), nx)
    return amp * np.sin(2 * np.pi * k * y / ny), np.zeros(nx * ny)
