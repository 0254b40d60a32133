"""Independent references used to pin the oracle: dense matrices built from
their definitions with plain loops, brute-force scalar minimisation, and the
augmented Lagrangian of the split problem (eqs. admm1 / admm2) written term by
term.  Nothing here calls the oracle's FFT or DCT routines."""
from __future__ import annotations

import math

import numpy as np


def dense_conv_matrix(psf_band, dtype=np.float64):
    """Dense H_l for one band: 2-D circular convolution with a PSF whose peak
    sits at 0-based pixel (ny/2, nx/2).  (H x)[p] = sum_q psf[p - q + c] x[q]."""
    ny, nx = psf_band.shape
    cy, cx = ny // 2, nx // 2
    n = ny * nx
    H = np.zeros((n, n), dtype=dtype)
    for py in range(ny):
        for px in range(nx):
            for qy in range(ny):
                for qx in range(nx):
                    H[py * nx + px, qy * nx + qx] = psf_band[(py - qy + cy) % ny,
                                                             (px - qx + cx) % nx]
    return H


def dct_matrix(L):
    """W_nu with entries W[l, k] = a_k cos(pi (2l + 1) k / (2L)), so that the
    spectrum of a pixel is x @ W (orthonormal DCT-II)."""
    W = np.zeros((L, L))
    for l in range(L):
        for k in range(L):
            a = math.sqrt(1.0 / L) if k == 0 else math.sqrt(2.0 / L)
            W[l, k] = a * math.cos(math.pi * (2 * l + 1) * k / (2 * L))
    return W


def spec(A, W):
    """A W_nu for a cube A[L][ny][nx]: per pixel, the row vector of its bands times W."""
    L = A.shape[0]
    return np.einsum("lk,l...->k...", W, A)


def spec_t(C, W):
    """C W_nu^T."""
    return np.einsum("lk,k...->l...", W, C)


def brute_min(f, center, halfwidth, n_grid=4001, n_golden=200):
    """Vectorised scalar minimisation of a convex f over [center-hw, center+hw]:
    grid search, then golden-section refinement around the best grid point."""
    center = np.asarray(center, np.float64)
    hw = np.broadcast_to(np.asarray(halfwidth, np.float64), center.shape)
    t = np.linspace(-1.0, 1.0, n_grid)
    grid = center[..., None] + hw[..., None] * t
    vals = f(grid)
    i = np.argmin(vals, axis=-1)
    step = 2.0 * hw / (n_grid - 1)
    best = np.take_along_axis(grid, i[..., None], axis=-1)[..., 0]
    a, b = best - step, best + step
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c[..., None])[..., 0], f(d[..., None])[..., 0]
    for _ in range(n_golden):
        left = fc < fd
        b = np.where(left, d, b)
        a = np.where(left, a, c)
        c2 = b - g * (b - a)
        d2 = a + g * (b - a)
        c, d = c2, d2
        fc, fd = f(c[..., None])[..., 0], f(d[..., None])[..., 0]
    return 0.5 * (a + b)


def dense_dwt_matrix(h, ny, nx, levels):
    """Dense matrix of the periodised multi-level 2-D DWT (Mallat layout), row
    per coefficient, built from the one-level definition with plain loops:
    level j maps the top-left (ny >> j) x (nx >> j) block through
      c[i, m] = sum_{a, b} f_y[a] f_x[b] x[(2 i + a) mod sy, (2 m + b) mod sx]
    with (f_y, f_x) in {h, g}^2, g[k] = (-1)^k h[K-1-k], and leaves the rest."""
    K = len(h)
    g = [(-1) ** k * h[K - 1 - k] for k in range(K)]
    n = ny * nx
    M = np.eye(n)
    for j in range(levels):
        sy, sx = ny >> j, nx >> j
        Lj = np.eye(n)
        for q in range(sy * sx):                   # clear the transformed block
            qy, qx = divmod(q, sx)
            Lj[qy * nx + qx, qy * nx + qx] = 0.0
        for by, fy in ((0, h), (1, g)):
            for bx, fx in ((0, h), (1, g)):
                for i in range(sy // 2):
                    for m in range(sx // 2):
                        row = (by * (sy // 2) + i) * nx + bx * (sx // 2) + m
                        for a in range(K):
                            for b in range(K):
                                col = ((2 * i + a) % sy) * nx + (2 * m + b) % sx
                                Lj[row, col] += fy[a] * fx[b]
        M = Lj @ M
    return M
