"""FP64 CPU oracle of the spatio-spectral ADMM reconstruction (Ferrari et al.,
"Multi-frequency image reconstruction for radio interferometry. A regularized
inverse problem approach", arXiv 1504.06847).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  It shares no code with the GPU
library.

What it computes, and where the paper defines it
------------------------------------------------
* Data model (Section 2, eqs. nbmodel / wbmodel): band l of the dirty cube is
  the band-l sky convolved with the band-l PSF.  H_l is read as a 2-D circular
  convolution on the N x N grid, the PSF peak sitting at 0-based pixel
  (ny/2, nx/2); the transfer function is h_hat = FFT2(ifftshift(psf)) and the
  adjoint H_l^T is circular correlation (multiplication by conj(h_hat)).
* Criterion (eqs. costreg, RegAll): 1/2 ||Y - HX||^2 + 1_{R+}(X)
  + mu_eps/2 ||X||_F^2 + mu_s ||W_s X||_1 + mu_nu ||X W_nu||_1, with W_s the
  Dirac basis (identity, n_s = 1) or a union of n_s orthonormal bases (the
  Dirac basis and Daubechies wavelets, Section 4; ``oracle/wavelets.py``) and
  W_nu the orthonormal DCT-II along the band axis.
* Algorithm 1 (Section 3, steps I-VI): all nine arrays X, P, T, V, S,
  Gamma_P, Gamma_T, Gamma_V, Gamma_S are stored explicitly and start at zero.
  Step I solves Q_l x_l = b_l with Q_l = H_l^T H_l + rho I,
  rho = mu_eps + rho_S + rho_P + n_s rho_T (eq. Qlsimp), exactly, through the
  Fourier-domain filter 1 / (|h_hat|^2 + rho) (end of Section 3); with the
  visibility-domain model (``oracle/visibility.py``) by conjugate gradients.  Step V uses
  the closed form for one orthonormal W_nu (m_nu = 1).
* Stopping quantities: primal / dual residuals of the two-block splitting
  (block 1 = {X, V}, block 2 = {P, T, S}) in the standard form of Boyd et al.
  (2011, Section 3.3), and E^k = ||w^k - w^{k+1}||_H, the quantity He & Yuan
  (2015) prove non-increasing for ADMM.
* Gradient oracle: forward-mode tangents through K iterations, for the
  derivative of ||X^K - sky||^2 with respect to (mu_s, mu_nu, rho) with the
  four rho's tied.  Kink convention: d soft(z, t)/dz = 1[|z| > t],
  d max(0, z)/dz = 1[z > 0].

Layout: every cube is a float64 array [L][ny][nx]; the paper's matrix X
(pixels x bands) is its transpose-reshape, so "X W_nu" is a DCT along axis 0.

Precision: float64 by default.  ``Problem(..., dtype=np.longdouble)`` runs
the same steps in the host's extended precision (64-bit significand,
eps = 1.1e-19; scipy.fft transforms long doubles natively).  Step I divides
by |h_hat|^2 + rho, so rounding in the right-hand side reaches X amplified
by up to max |h_hat|^2 / rho (about 1e6 on the 1024^2 workloads): there the
float64 oracle's own error is of the order of a float64 GPU pass's, and the
extended-precision run is the reference that the FP64 GPU path is held to.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, fields

import numpy as np
import scipy.fft as sfft

from .spectral import DCT, SpectralDictionary
from .wavelets import DIRAC, Dictionary

_WORKERS = int(os.environ.get("MUFFIN_ORACLE_WORKERS", "1"))


def set_workers(n: int) -> None:
    """Threads used by scipy.fft inside the oracle."""
    global _WORKERS
    _WORKERS = max(1, int(n))


def _fft2(a):
    return sfft.fft2(a, axes=(-2, -1), workers=_WORKERS)


def _ifft2(a):
    return sfft.ifft2(a, axes=(-2, -1), workers=_WORKERS)


def dct_nu(A):
    """A W_nu: orthonormal DCT-II along the band axis (axis 0)."""
    return sfft.dct(A, type=2, norm="ortho", axis=0, workers=_WORKERS)


def idct_nu(C):
    """C W_nu^T: the inverse (transpose) of ``dct_nu``."""
    return sfft.idct(C, type=2, norm="ortho", axis=0, workers=_WORKERS)


def soft(z, t):
    """Element-wise soft threshold S_t(z) = sign(z) max(|z| - t, 0) (steps III, IV)."""
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


@dataclass
class Params:
    mu_eps: float
    mu_s: float
    mu_nu: float
    rho_P: float
    rho_T: float
    rho_V: float
    rho_S: float

    @classmethod
    def from_any(cls, p):
        if isinstance(p, cls):
            return p
        if isinstance(p, dict):
            return cls(**{f.name: float(p[f.name]) for f in fields(cls)})
        return cls(**{f.name: float(getattr(p, f.name)) for f in fields(cls)})

    def with_(self, **kw):
        from dataclasses import replace
        return replace(self, **kw)

    @property
    def rho_Q(self):
        # eq. Qlsimp with the Dirac basis: n_s = 1
        return self.mu_eps + self.rho_S + self.rho_P + 1.0 * self.rho_T

    def rho_Q_for(self, n_s: int):
        # eq. Qlsimp for a union of n_s orthonormal bases
        return self.mu_eps + self.rho_S + self.rho_P + float(n_s) * self.rho_T


class Problem:
    """One cube: PSFs, dirty images and parameters, in float64 (or in the
    floating type ``dtype``: np.longdouble for the extended-precision
    reference).  ``bases``: the spatial dictionary W_s (codes of
    ``oracle/wavelets.py``; the Dirac basis alone by default)."""

    def __init__(self, psf, dirty, params, bases=(DIRAC,), dtype=np.float64, spectral=(DCT,)):
        self.psf = np.asarray(psf, dtype=dtype)
        self.Y = np.asarray(dirty, dtype=dtype)
        self.Wnu = SpectralDictionary(spectral)
        assert self.psf.shape == self.Y.shape and self.psf.ndim == 3
        self.p = Params.from_any(params)
        self.W = Dictionary(bases)
        # transfer function of H_l: PSF peak moved to lag (0, 0)
        self.hhat = _fft2(np.fft.ifftshift(self.psf, axes=(-2, -1)))
        self.HtY = self.HT(self.Y)
        self._set_filter()

    def _set_filter(self):
        self.filt = 1.0 / (np.abs(self.hhat) ** 2 + self.rho_Q)

    def with_params(self, params):
        q = object.__new__(Problem)
        q.psf, q.Y, q.hhat, q.HtY, q.W = self.psf, self.Y, self.hhat, self.HtY, self.W
        q.Wnu = self.Wnu
        q.p = Params.from_any(params)
        q._set_filter()
        return q

    @property
    def shape(self):
        return self.Y.shape

    @property
    def n_s(self) -> int:
        return self.W.n_s

    @property
    def rho_Q(self) -> float:
        return self.p.rho_Q_for(self.n_s)

    @property
    def dirac_only(self) -> bool:
        return self.W.bases == (DIRAC,)

    @property
    def m_nu(self) -> int:
        return self.Wnu.m

    def Ws(self, x):
        """W_s x: x itself for the Dirac basis alone, else the stacked
        coefficient cubes [n_s][L][ny][nx]."""
        return x if self.dirac_only else self.W.forward(x)

    def WsT(self, c):
        """W_s^T c (the adjoint of ``Ws``)."""
        return c if self.dirac_only else self.W.adjoint(c)

    def zero_state(self):
        return State.zeros(self.shape, 1 if self.dirac_only else self.n_s, self.m_nu)

    def H(self, x):
        """Band-wise circular convolution with the PSF (eq. nbmodel)."""
        return _ifft2(self.hhat * _fft2(x)).real

    def HT(self, y):
        """Adjoint of H: band-wise circular correlation."""
        return _ifft2(np.conj(self.hhat) * _fft2(y)).real

    def solve_Q(self, b):
        """Q_l^{-1} b_l for every band: filter with (|h_hat|^2 + rho)^{-1}."""
        return _ifft2(self.filt * _fft2(b)).real

    def step_one(self, b, x0):
        """Step I: the exact solve (x0, the previous X, is not needed)."""
        return self.solve_Q(b)

    def misfit(self, x):
        """1/2 ||Y - H x||^2."""
        r = self.Y - self.H(x)
        return 0.5 * np.sum(r * r)


@dataclass
class State:
    X: np.ndarray
    P: np.ndarray
    T: np.ndarray
    V: np.ndarray
    S: np.ndarray
    GP: np.ndarray
    GT: np.ndarray
    GV: np.ndarray
    GS: np.ndarray

    @classmethod
    def zeros(cls, shape, n_s: int = 1, m_nu: int = 1):
        """All nine arrays zero; with n_s > 1 spatial bases T and Gamma_T hold
        one coefficient cube per basis ([n_s][L][ny][nx]), with m_nu > 1
        spectral bases V and Gamma_V likewise ([m_nu][L][ny][nx])."""
        tshape = tuple(shape) if n_s == 1 else (n_s,) + tuple(shape)
        vshape = tuple(shape) if m_nu == 1 else (m_nu,) + tuple(shape)
        a = [np.zeros(tshape) if f in ("T", "GT") else (np.zeros(vshape) if f in ("V", "GV") else np.zeros(shape))
             for f in ("X", "P", "T", "V", "S", "GP", "GT", "GV", "GS")]
        return cls(*a)

    def copy(self):
        return State(*(getattr(self, f.name).copy() for f in fields(self)))


def admm_iteration(prob: Problem, st: State) -> State:
    """One pass of Algorithm 1: steps I-VI in the paper's order."""
    p = prob.p
    # Step I: b_l from eq. matB, then Q_l x_l = b_l
    B = (prob.HtY + prob.WsT(st.GT + p.rho_T * st.T) + st.GP + p.rho_P * st.P
         + st.GS + p.rho_S * st.S)
    X = prob.step_one(B, st.X)
    # Step II: positivity
    P = np.maximum(0.0, X - st.GP / p.rho_P)
    # Step III: spatial soft threshold, per coefficient of every basis
    WX = prob.Ws(X)
    T = soft(WX - st.GT / p.rho_T, p.mu_s / p.rho_T)
    # Step IV: spectral soft threshold, on the S of the previous pass, per
    # coefficient of every spectral basis
    V = soft(prob.Wnu.forward(st.S) - st.GV / p.rho_V, p.mu_nu / p.rho_V)
    # Step V: closed form for a union of m_nu orthonormal W_nu
    S = (prob.Wnu.adjoint(st.GV + p.rho_V * V) - st.GS + p.rho_S * X) / (prob.m_nu * p.rho_V + p.rho_S)
    # Step VI: multipliers, with the new P, T, V, S
    GP = st.GP + p.rho_P * (P - X)
    GT = st.GT + p.rho_T * (T - WX)
    GV = st.GV + p.rho_V * (V - prob.Wnu.forward(S))
    GS = st.GS + p.rho_S * (S - X)
    return State(X, P, T, V, S, GP, GT, GV, GS)


def run(prob: Problem, K: int, state: State | None = None, callback=None) -> State:
    """K passes of Algorithm 1 from the all-zero state (or from ``state``).

    ``callback(k, prev, cur)`` is called after pass k (1-based)."""
    st = prob.zero_state() if state is None else state
    for k in range(1, K + 1):
        nxt = admm_iteration(prob, st)
        if callback is not None:
            callback(k, st, nxt)
        st = nxt
    return st


def objective(prob: Problem, P: np.ndarray) -> float:
    """Criterion (costreg) + (RegAll) at P; finite because P >= 0."""
    p = prob.p
    return float(prob.misfit(P) + 0.5 * p.mu_eps * np.sum(P * P)
                 + p.mu_s * np.sum(np.abs(prob.Ws(P))) + p.mu_nu * np.sum(np.abs(prob.Wnu.forward(P))))


def residuals(prob: Problem, prev: State, cur: State, eps_abs=1e-5, eps_rel=1e-4):
    """Primal / dual residual norms and tolerances (Boyd et al. 2011, Sec. 3.3).

    Constraints P - X, T - W_s X, V - S W_nu, S - X; block 1 = (X, V),
    block 2 = (P, T, S).  The constraint space has (2 + n_s + m_nu) nvox
    entries, block 1 (1 + m_nu) nvox."""
    p = prob.p
    WX = prob.Ws(cur.X)
    SW = prob.Wnu.forward(cur.S)
    r2 = (np.sum((cur.P - cur.X) ** 2) + np.sum((cur.T - WX) ** 2)
          + np.sum((cur.V - SW) ** 2) + np.sum((cur.S - cur.X) ** 2))
    dP, dT, dS = cur.P - prev.P, cur.T - prev.T, cur.S - prev.S
    sX = p.rho_P * dP + p.rho_T * prob.WsT(dT) + p.rho_S * dS
    sV = p.rho_V * prob.Wnu.forward(dS)
    s2 = np.sum(sX ** 2) + np.sum(sV ** 2)
    nvox = cur.X.size
    Ax = np.sqrt(2.0 * np.sum(cur.X ** 2) + np.sum(WX ** 2) + np.sum(cur.V ** 2))
    Bz = np.sqrt(np.sum(cur.P ** 2) + np.sum(cur.T ** 2) + np.sum(SW ** 2) + np.sum(cur.S ** 2))
    Aty = np.sqrt(np.sum((cur.GP + prob.WsT(cur.GT) + cur.GS) ** 2) + np.sum(cur.GV ** 2))
    eps_pri = np.sqrt((2.0 + prob.n_s + prob.m_nu) * nvox) * eps_abs + eps_rel * max(Ax, Bz)
    eps_dual = np.sqrt((1.0 + prob.m_nu) * nvox) * eps_abs + eps_rel * Aty
    return dict(r=float(np.sqrt(r2)), s=float(np.sqrt(s2)),
                eps_pri=float(eps_pri), eps_dual=float(eps_dual))


def energy(prob: Problem, prev: State, cur: State) -> float:
    """E^k = ||w^k - w^{k+1}||_H^2 with w = (B z, Gamma) (He & Yuan 2015)."""
    p = prob.p
    dS = cur.S - prev.S
    return float(p.rho_P * np.sum((cur.P - prev.P) ** 2)
                 + p.rho_T * np.sum((cur.T - prev.T) ** 2)
                 + p.rho_S * np.sum(dS ** 2)
                 + p.rho_V * np.sum(prob.Wnu.forward(dS) ** 2)
                 + np.sum((cur.GP - prev.GP) ** 2) / p.rho_P
                 + np.sum((cur.GT - prev.GT) ** 2) / p.rho_T
                 + np.sum((cur.GV - prev.GV) ** 2) / p.rho_V
                 + np.sum((cur.GS - prev.GS) ** 2) / p.rho_S)


def solve_adaptive(prob: Problem, max_iter: int, check_every: int, mu: float, tau: float,
                   eps_abs=1e-5, eps_rel=1e-4):
    """Algorithm 1 with the stopping rule and residual balancing of Boyd et
    al. (2011, Sec. 3.3.1 and 3.4.1), checked every ``check_every`` passes
    and after the last one: stop when r <= eps_pri and s <= eps_dual; else
    multiply the four rho's by tau when r > mu s, divide them by tau when
    s > mu r, keeping every array (the multipliers Gamma are not rescaled).
    Returns (state, problem with the final rho's, [(k, rho_P, r, s), ...])."""
    st = prob.zero_state()
    k = 0
    history = []
    while k < max_iter:
        plain = min(check_every - 1, max_iter - k - 1)
        for _ in range(plain):
            st = admm_iteration(prob, st)
        k += plain
        prev = st
        st = admm_iteration(prob, st)
        k += 1
        res = residuals(prob, prev, st, eps_abs, eps_rel)
        history.append((k, prob.p.rho_P, res["r"], res["s"]))
        if (res["r"] <= res["eps_pri"] and res["s"] <= res["eps_dual"]) or k >= max_iter:
            break
        f = tau if res["r"] > mu * res["s"] else (1.0 / tau if res["s"] > mu * res["r"] else 1.0)
        if f != 1.0:
            p = prob.p
            prob = prob.with_params(p.with_(rho_P=p.rho_P * f, rho_T=p.rho_T * f,
                                            rho_V=p.rho_V * f, rho_S=p.rho_S * f))
    return st, prob, history


def mse_loss(XK, sky) -> float:
    """||X^K - sky||_2^2 (a sum, not a mean)."""
    d = np.asarray(XK, np.float64) - np.asarray(sky, np.float64)
    return float(np.sum(d * d))


def _jvp_iteration(prob: Problem, st: State, dst: State, dp: Params, dHtY=None):
    """Primal pass of Algorithm 1 with its forward-mode tangent (W_s the
    Dirac basis or a union of orthonormal bases, one orthonormal spectral
    basis W_nu); dHtY: the tangent of H^T Y (a change of the dirty images),
    or None.  W_s is linear, so it carries tangents as it carries values."""
    assert prob.m_nu == 1, "the tangent pass is written for one spectral basis"
    fw, bw = prob.Wnu.forward, prob.Wnu.adjoint
    Ws, WsT = prob.Ws, prob.WsT
    p = prob.p
    # rho of eq. Qlsimp: mu_eps + rho_S + rho_P + n_s rho_T
    drhoQ = dp.mu_eps + dp.rho_S + dp.rho_P + prob.n_s * dp.rho_T
    B = (prob.HtY + WsT(st.GT + p.rho_T * st.T) + st.GP + p.rho_P * st.P
         + st.GS + p.rho_S * st.S)
    dB = (WsT(dst.GT + dp.rho_T * st.T + p.rho_T * dst.T) + dst.GP + dp.rho_P * st.P
          + p.rho_P * dst.P + dst.GS + dp.rho_S * st.S + p.rho_S * dst.S)
    if dHtY is not None:
        dB = dB + dHtY
    X = prob.solve_Q(B)
    dX = prob.solve_Q(dB - drhoQ * X)          # d(Q^{-1}) = -Q^{-1} dQ Q^{-1}
    zP = X - st.GP / p.rho_P
    dzP = dX - dst.GP / p.rho_P + st.GP * dp.rho_P / p.rho_P ** 2
    P = np.maximum(0.0, zP)
    dP = np.where(zP > 0.0, dzP, 0.0)
    WX, dWX = Ws(X), Ws(dX)
    zT = WX - st.GT / p.rho_T
    dzT = dWX - dst.GT / p.rho_T + st.GT * dp.rho_T / p.rho_T ** 2
    tT = p.mu_s / p.rho_T
    dtT = dp.mu_s / p.rho_T - p.mu_s * dp.rho_T / p.rho_T ** 2
    T = soft(zT, tT)
    dT = np.where(np.abs(zT) > tT, dzT - np.sign(zT) * dtT, 0.0)
    zV = fw(st.S) - st.GV / p.rho_V
    dzV = fw(dst.S) - dst.GV / p.rho_V + st.GV * dp.rho_V / p.rho_V ** 2
    tV = p.mu_nu / p.rho_V
    dtV = dp.mu_nu / p.rho_V - p.mu_nu * dp.rho_V / p.rho_V ** 2
    V = soft(zV, tV)
    dV = np.where(np.abs(zV) > tV, dzV - np.sign(zV) * dtV, 0.0)
    den = p.rho_V + p.rho_S
    dden = dp.rho_V + dp.rho_S
    num = bw(st.GV + p.rho_V * V) - st.GS + p.rho_S * X
    dnum = (bw(dst.GV + dp.rho_V * V + p.rho_V * dV) - dst.GS
            + dp.rho_S * X + p.rho_S * dX)
    S = num / den
    dS = (dnum - S * dden) / den
    cS, dcS = fw(S), fw(dS)
    GP = st.GP + p.rho_P * (P - X)
    dGP = dst.GP + dp.rho_P * (P - X) + p.rho_P * (dP - dX)
    GT = st.GT + p.rho_T * (T - WX)
    dGT = dst.GT + dp.rho_T * (T - WX) + p.rho_T * (dT - dWX)
    GV = st.GV + p.rho_V * (V - cS)
    dGV = dst.GV + dp.rho_V * (V - cS) + p.rho_V * (dV - dcS)
    GS = st.GS + p.rho_S * (S - X)
    dGS = dst.GS + dp.rho_S * (S - X) + p.rho_S * (dS - dX)
    return (State(X, P, T, V, S, GP, GT, GV, GS),
            State(dX, dP, dT, dV, dS, dGP, dGT, dGV, dGS))


def jvp_run(prob: Problem, K: int, direction, dY=None):
    """X^K and its directional derivative along ``direction``.

    ``direction`` = (d mu_s, d mu_nu, d rho) with rho_P = rho_T = rho_V = rho_S
    = rho tied, or a full ``Params`` of tangents; ``dY``: a tangent of the
    dirty images (entering through H^T Y of eq. matB) added to it."""
    if isinstance(direction, Params):
        dp = direction
    else:
        a, b, c = (float(v) for v in direction)
        dp = Params(0.0, a, b, c, c, c, c)
    st = prob.zero_state()
    dst = prob.zero_state()
    dHtY = None if dY is None else prob.HT(np.asarray(dY, np.float64))
    for _ in range(K):
        st, dst = _jvp_iteration(prob, st, dst, dp, dHtY)
    return st.X, dst.X


def mse_grad(prob: Problem, K: int, sky):
    """d ||X^K - sky||^2 / d(mu_s, mu_nu, rho) by three forward-mode passes."""
    g = np.zeros(3)
    loss = None
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        XK, dXK = jvp_run(prob, K, e)
        r = XK - np.asarray(sky, np.float64)
        g[i] = 2.0 * np.sum(r * dXK)
        loss = float(np.sum(r * r))
    return loss, g
