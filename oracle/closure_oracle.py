"""Plain FP64 CPU reference of the learned-closure network (test infrastructure).

This module is the oracle of the closure kernels: it is imported only by the
tests.  It shares nothing with the HIP path.  Everything here is a direct,
unblocked transcription of the definitions below, in float64 numpy with
explicit loops over the nine stencil taps.

Grid and padding.  Cells (r, c) of an n_theta x n_phi latitude-longitude grid,
theta_r = (r + 1/2) pi / n_theta, phi_c = (c + 1/2) 2 pi / n_phi (Sec. III.D,
eq. (discrete_coord_sphere), 0-based).  A 3x3 stencil tap (dy, dx) of cell (r, c)
reads cell (r + dy, c + dx) with phi periodic (eq. (bcs_phi)).  A row index
beyond a pole continues across it as the ghost rows of the populations do
(Sec. III.E, eq. (bcs_theta)): row -1 is row 0 and row n_theta is row
n_theta - 1, both at phi + pi (column + n_phi / 2).  A scalar keeps its value
across the pole; the orthonormal components (u_theta, u_phi) of a vector both
change sign, because the unit vectors e_theta and e_phi at (theta, phi + pi)
are minus those reached by continuing theta through the pole.

Network.  Three 3x3 convolutions with ReLU between them,
    a1 = relu(conv(x; W1, b1)), a2 = relu(conv(a1; W2, b2)), z = conv(a2; W3, b3),
    conv(x; W, b)[p, co] = b[co] + sum_{tap, ci} W[co, tap, ci] s(p, tap, ci) x[nbr(p, tap), ci],
with s = -1 for a vector channel read across a pole, else 1.  Loss: the
sin(theta)-weighted mean square error over cells and output channels.  Adam
(Kingma and Ba, 2015) with bias correction updates the parameters.

Coarse graining: box averages of f x f fine cells with the area weight
sin(theta), density by area, velocity by momentum (rho u).
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# grid and pole-crossing neighbourhood
def taps():
    """The nine taps (dy, dx) in the order tap = 3 (dy + 1) + (dx + 1)."""
    return [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def neighbours(n_theta: int, n_phi: int):
    """nbr[r, c, tap] = flat index r' n_phi + c' of the cell a tap reads;
    cross[r, c, tap] = True where the tap continues across a pole."""
    if n_theta < 2 or n_phi < 2 or n_phi % 2:
        raise ValueError("need n_theta >= 2 and an even n_phi >= 2")
    nbr = np.zeros((n_theta, n_phi, 9), dtype=np.int64)
    cross = np.zeros((n_theta, n_phi, 9), dtype=bool)
    for r in range(n_theta):
        for c in range(n_phi):
            for t, (dy, dx) in enumerate(taps()):
                rr, cc, x = r + dy, c + dx, False
                if rr < 0:
                    rr, cc, x = -rr - 1, cc + n_phi // 2, True
                elif rr >= n_theta:
                    rr, cc, x = 2 * n_theta - rr - 1, cc + n_phi // 2, True
                nbr[r, c, t] = rr * n_phi + cc % n_phi
                cross[r, c, t] = x
    return nbr, cross


def gather(x, nbr, cross, vector_channels=()):
    """Stencil view g[b, r, c, tap, ch] = s x[b, nbr, ch] of x[b, r, c, ch]."""
    B, H, W, C = x.shape
    flat = x.reshape(B, H * W, C)
    g = flat[:, nbr.reshape(-1), :].reshape(B, H, W, 9, C).copy()
    for ch in vector_channels:
        g[..., ch] = np.where(cross[None], -g[..., ch], g[..., ch])
    return g


# ---------------------------------------------------------------------------
# convolution and its gradients
def conv_forward(x, w, b, nbr, cross, vector_channels=()):
    """x [B,H,W,Cin], w [Cout,9,Cin], b [Cout] -> z [B,H,W,Cout]."""
    g = gather(x, nbr, cross, vector_channels)
    z = np.zeros(x.shape[:3] + (w.shape[0],))
    for t in range(9):
        z += g[:, :, :, t, :] @ w[:, t, :].T
    return z + b


def conv_backward(x, w, dz, nbr, cross, vector_channels=()):
    """Gradients (dx, dw, db) of sum(dz * conv_forward(x, w, b))."""
    B, H, W, Cin = x.shape
    g = gather(x, nbr, cross, vector_channels)
    dw = np.zeros_like(w)
    for t in range(9):
        dw[:, t, :] = np.einsum("bhwo,bhwi->oi", dz, g[:, :, :, t, :])
    db = dz.sum(axis=(0, 1, 2))
    # dx: every tap scatters its contribution back to the cell it read
    dx = np.zeros((B, H * W, Cin))
    flat_nbr = nbr.reshape(H * W, 9)
    flat_cross = cross.reshape(H * W, 9)
    for t in range(9):
        contrib = (dz @ w[:, t, :]).reshape(B, H * W, Cin)
        for ch in vector_channels:
            contrib[:, flat_cross[:, t], ch] *= -1.0
        for bb in range(B):
            np.add.at(dx[bb], flat_nbr[:, t], contrib[bb])
    return dx.reshape(B, H, W, Cin), dw, db


def relu(z):
    return np.maximum(z, 0.0)


# ---------------------------------------------------------------------------
# the three-layer network
def init_params(rng, cin=3, hidden=32, cout=3, scale=1.0):
    """He-style normal initialisation, zero biases (layers: cin->h->h->cout)."""
    shapes = [(hidden, 9, cin), (hidden, 9, hidden), (cout, 9, hidden)]
    ps = []
    for i, s in enumerate(shapes):
        fan_in = 9 * s[2]
        std = np.sqrt(2.0 / fan_in) * (scale if i < 2 else 0.1 * scale)
        ps.append(rng.normal(0.0, std, size=s))
        ps.append(np.zeros(s[0]))
    return ps


def net_forward(params, x, nbr, cross, vector_channels=(1, 2)):
    w1, b1, w2, b2, w3, b3 = params
    z1 = conv_forward(x, w1, b1, nbr, cross, vector_channels)
    a1 = relu(z1)
    z2 = conv_forward(a1, w2, b2, nbr, cross)
    a2 = relu(z2)
    z3 = conv_forward(a2, w3, b3, nbr, cross)
    return z3, (x, z1, a1, z2, a2)


def row_weights(n_theta):
    th = (np.arange(n_theta) + 0.5) * np.pi / n_theta
    return np.sin(th)


def loss_and_grad(z, target, n_theta):
    """Weighted MSE L = sum w (z - t)^2 / (sum w * C) over all cells, channels
    and samples, and dL/dz."""
    w = row_weights(n_theta)[None, :, None, None]
    B, H, W, C = z.shape
    norm = w.sum() * W * B * C
    d = z - target
    return float((w * d * d).sum() / norm), 2.0 * w * d / norm


def net_backward(params, cache, dz3, nbr, cross, vector_channels=(1, 2)):
    w1, b1, w2, b2, w3, b3 = params
    x, z1, a1, z2, a2 = cache
    da2, dw3, db3 = conv_backward(a2, w3, dz3, nbr, cross)
    dz2 = da2 * (z2 > 0)
    da1, dw2, db2 = conv_backward(a1, w2, dz2, nbr, cross)
    dz1 = da1 * (z1 > 0)
    _, dw1, db1 = conv_backward(x, w1, dz1, nbr, cross, vector_channels)
    return [dw1, db1, dw2, db2, dw3, db3]


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# coarse graining
def box_filter(rho, ut, up, factor):
    """Fields [H, W] on the fine grid -> [H/f, W/f]: rho by area average,
    u by momentum average (sum w rho u / sum w rho), weight w = sin(theta)."""
    H, W = rho.shape
    f = factor
    w = row_weights(H)[:, None] * np.ones((1, W))
    blk = lambda a: a.reshape(H // f, f, W // f, f).sum(axis=(1, 3))
    ws, m = blk(w), blk(w * rho)
    return m / ws, blk(w * rho * ut) / m, blk(w * rho * up) / m
