"""Visibility-domain data model of the oracle: Algorithm 1 with the sampled
visibilities in place of the dirty images and H_l the operator from the sky
to the visibilities of band l (Section 2, the remark after eq. wbmodel), so
that step I is no longer a Fourier-domain filter and is solved by conjugate
gradients (Algorithm 1's step I; Q_l of eq. Qlsimp; Hestenes and Stiefel
1952).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper names the model and the solver, not these details):
* H_l: visibility j of band l sits at (u_j, v_j), in cycles per image width
  (cells of the nx x ny Fourier grid at that band's frequency), with the
  phase centre at pixel (ny/2, nx/2) as the PSF peak of the dirty-image
  model:  (H_l x)_j = sum_{m, n} x[m, n] exp(-2 pi i (u_j (n - nx/2) / nx
  + v_j (m - ny/2) / ny)).
* The sky is real and the data complex: the fidelity is 1/2 sum_j
  |y_j - (H x)_j|^2, H^T is the adjoint of H as a map into C^M viewed as
  R^(2M), i.e. Re(H^H .), so Q_l = Re(H_l^H H_l) + rho I and the data term of
  eq. matB is Re(H_l^H y_l).
* Re(H^H H) is two-level Toeplitz: (Re(H^H H) x)[p] = sum_q c(p - q) x[q] with
  c(d) = sum_j cos(2 pi (u_j d_x / nx + v_j d_y / ny)) for |d_x| < nx,
  |d_y| < ny.
* Step I runs a fixed number n_cg of CG iterations per band (Hestenes-
  Stiefel: r = b - Q x, p = r; alpha = r.r / p.Qp, x += alpha p,
  r -= alpha Qp, beta = r'.r' / r.r, p = r' + beta p), started from the
  previous pass's X (zero at the first pass).  alpha = 0 when p.Qp = 0 and
  beta = 0 when r.r = 0 (an exact solution stays put).
"""
from __future__ import annotations

import numpy as np

from .muffin_oracle import Params, State
from .spectral import DCT, SpectralDictionary
from .wavelets import DIRAC, Dictionary


def _phase(uv, ny: int, nx: int):
    """exp(-2 pi i (u (n - nx/2) / nx + v (m - ny/2) / ny)) as two factors:
    e_u [M, nx] over n and e_v [M, ny] over m."""
    u = np.asarray(uv, np.float64)[:, 0][:, None]
    v = np.asarray(uv, np.float64)[:, 1][:, None]
    n = np.arange(nx)[None, :] - nx // 2
    m = np.arange(ny)[None, :] - ny // 2
    return np.exp(-2j * np.pi * u * n / nx), np.exp(-2j * np.pi * v * m / ny)


def vis_forward(x, uv):
    """H x for one band: x [ny][nx] real, uv [M][2] -> M complex visibilities
    (the sum over pixels of the definition, done as two matrix products over
    the separable phase)."""
    ny, nx = x.shape
    eu, ev = _phase(uv, ny, nx)
    # sum_n x[m, n] e_u[j, n] -> [ny, M]; then sum_m e_v[j, m] (.)[m, j]
    a = np.asarray(x, np.complex128) @ eu.T
    return np.einsum("jm,mj->j", ev, a)


def vis_adjoint(y, uv, ny: int, nx: int):
    """Re(H^H y) for one band: the real adjoint of vis_forward."""
    eu, ev = _phase(uv, ny, nx)
    # sum_j conj(e_v[j, m]) conj(e_u[j, n]) y_j
    return np.real(np.conj(ev).T @ (np.asarray(y, np.complex128)[:, None] * np.conj(eu)))


def toeplitz_kernel(uv, ny: int, nx: int):
    """c(d) = sum_j cos(2 pi (u_j d_x / nx + v_j d_y / ny)) on the lags
    d_y in (-ny, ny), d_x in (-nx, nx): array [2 ny - 1][2 nx - 1], lag
    (0, 0) at [ny - 1, nx - 1]."""
    u = np.asarray(uv, np.float64)[:, 0]
    v = np.asarray(uv, np.float64)[:, 1]
    dx = np.arange(-(nx - 1), nx)
    dy = np.arange(-(ny - 1), ny)
    ax = 2 * np.pi * u[:, None] * dx[None, :] / nx          # [M, 2nx-1]
    ay = 2 * np.pi * v[:, None] * dy[None, :] / ny          # [M, 2ny-1]
    # cos(a + b) = cos a cos b - sin a sin b, summed over j
    return np.cos(ay).T @ np.cos(ax) - np.sin(ay).T @ np.sin(ax)


def toeplitz_apply(c, x):
    """sum_q c(p - q) x[q] for one band, by zero padding to a 2ny x 2nx
    circular convolution (exact: every lag p - q lies in the kernel's range)."""
    ny, nx = x.shape
    cc = np.zeros((2 * ny, 2 * nx))
    # lag (d_y, d_x) at index (d_y mod 2ny, d_x mod 2nx)
    for dy in range(-(ny - 1), ny):
        cc[dy % (2 * ny), [d % (2 * nx) for d in range(-(nx - 1), nx)]] = c[dy + ny - 1, :]
    xp = np.zeros((2 * ny, 2 * nx))
    xp[:ny, :nx] = x
    out = np.fft.ifft2(np.fft.fft2(cc) * np.fft.fft2(xp)).real
    return out[:ny, :nx]


def cg(apply_Q, b, x0, n_iter: int):
    """n_iter Hestenes-Stiefel CG iterations on Q x = b from x0 (arrays of
    one band; dot products summed over the band)."""
    x = x0.copy()
    r = b - apply_Q(x)
    p = r.copy()
    rr = float(np.sum(r * r))
    for _ in range(n_iter):
        q = apply_Q(p)
        pq = float(np.sum(p * q))
        alpha = rr / pq if pq > 0 else 0.0
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.sum(r * r))
        beta = rr_new / rr if rr > 0 else 0.0
        rr = rr_new
        p = r + beta * p
    return x


class VisProblem:
    """One cube in the visibility domain: per band l the visibility
    coordinates uv[l] ([M_l][2], cells at that band) and the visibilities
    vis[l] (M_l complex), the image shape (L, ny, nx), the parameters and
    n_cg.  Provides what the steps of Algorithm 1 use (``HtY``, ``step_one``,
    ``H``, ``Ws``, ``Wnu``, ...), so ``admm_iteration``, ``run``,
    ``residuals``, ``energy`` and ``objective`` run on it unchanged."""

    def __init__(self, uv, vis, shape, params, n_cg: int, spectral=(DCT,)):
        self.L, self.ny, self.nx = shape
        assert len(uv) == len(vis) == self.L
        self.uv = [np.asarray(a, np.float64) for a in uv]
        self.vis = [np.asarray(a, np.complex128) for a in vis]
        self.p = Params.from_any(params)
        self.n_cg = int(n_cg)
        self.W = Dictionary((DIRAC,))
        self.Wnu = SpectralDictionary(spectral)
        self.HtY = np.stack([vis_adjoint(self.vis[l], self.uv[l], self.ny, self.nx) for l in range(self.L)])
        self.kernels = [toeplitz_kernel(self.uv[l], self.ny, self.nx) for l in range(self.L)]

    def with_params(self, params):
        q = object.__new__(VisProblem)
        q.__dict__.update(self.__dict__)
        q.p = Params.from_any(params)
        return q

    @property
    def shape(self):
        return (self.L, self.ny, self.nx)

    n_s = 1
    m_nu = property(lambda self: self.Wnu.m)
    dirac_only = True

    @property
    def rho_Q(self) -> float:
        return self.p.rho_Q_for(1)

    def Ws(self, x):
        return x

    def WsT(self, c):
        return c

    def zero_state(self):
        return State.zeros(self.shape, 1, self.m_nu)

    def HtH(self, x):
        """Re(H^H H) x, band by band."""
        return np.stack([toeplitz_apply(self.kernels[l], x[l]) for l in range(self.L)])

    def apply_Q(self, x):
        return self.HtH(x) + self.rho_Q * x

    def step_one(self, b, x0):
        """Step I: n_cg CG iterations on Q_l x_l = b_l per band from x0."""
        rho = self.rho_Q
        return np.stack([cg(lambda z, l=l: toeplitz_apply(self.kernels[l], z) + rho * z, b[l], x0[l], self.n_cg)
                         for l in range(self.L)])

    def H(self, x):
        """The visibilities of the cube x (a list of per-band arrays)."""
        return [vis_forward(x[l], self.uv[l]) for l in range(self.L)]

    def misfit(self, x) -> float:
        """1/2 sum over bands and visibilities of |y - H x|^2."""
        return float(0.5 * sum(np.sum(np.abs(self.vis[l] - h) ** 2) for l, h in enumerate(self.H(x))))
