"""Spatial dictionary of the oracle: the Dirac basis and the orthonormal
Daubechies wavelet bases Db1-Db8 (Section 4: W_s is the concatenation of
these bases), as plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What it computes
----------------
* ``daubechies_filter(p)``: the length-2p scaling filter with p vanishing
  moments, by Daubechies' spectral factorisation: |m0(w)|^2 =
  cos(w/2)^(2p) Q(sin(w/2)^2) with Q(y) = sum_{k<p} C(p-1+k, k) y^k.  Each
  root y_i of Q gives the root pair of z^2 - (2 - 4 y_i) z + 1; the filter
  polynomial is (1 + z)^p prod_i (z - z_i) over the roots outside the unit
  circle, h_k its z^k coefficient, scaled to sum sqrt(2).  (The tabulated
  Db2, (1 + sqrt3, 3 + sqrt3, 3 - sqrt3, 1 - sqrt3) / (4 sqrt2), is this
  orientation.)
* Periodised analysis of a length-n signal (n even):
      a[m] = sum_k h[k] x[(2m + k) mod n],  d[m] = sum_k g[k] x[(2m + k) mod n],
  g[k] = (-1)^k h[2p-1-k]; synthesis is its transpose.
* One 2-D level on an ny x nx image: analysis along x (rows) then along y;
  Mallat layout [[LL, x-high], [y-high, HH]] (LL top-left, n/2 x n/2 each).
  ``levels`` levels recurse on LL (reading: ``dwt_levels`` below).
* ``Dictionary``: W_s X stacks the coefficient cubes of every basis (the
  Dirac basis gives X itself); W_s^T sums the per-basis adjoints.  With n_s
  orthonormal bases W_s^T W_s = n_s I, the identity behind eq. Qlsimp.
"""
from __future__ import annotations

from math import comb

import numpy as np

DIRAC = 0          # spatial basis codes: 0 = Dirac, p = Daubechies Db_p (1..8)


def dwt_levels(nx: int, ny: int) -> int:
    """Decomposition depth (reading): 4 levels, fewer on images too small to
    keep a 2 x 2 coarsest band."""
    return max(1, min(4, int(np.log2(min(nx, ny))) - 1))


def daubechies_filter(p: int) -> np.ndarray:
    """Scaling filter h (length 2p, sum sqrt 2) of the Daubechies wavelet Db_p."""
    if not 1 <= p <= 8:
        raise ValueError("p must be in 1..8")
    # Q(y) = sum_k C(p-1+k, k) y^k, highest degree first for np.roots
    q = [comb(p - 1 + k, k) for k in range(p)][::-1]
    poly = np.array([1.0 + 0j])
    for _ in range(p):
        poly = np.convolve(poly, [1.0, 1.0])                     # (1 + z)^p
    for y in (np.roots(q) if p > 1 else []):
        b = 2.0 - 4.0 * y
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0              # z1 z2 = 1
        z = z1 if abs(z1) > 1.0 else z2
        poly = np.convolve(poly, [-z, 1.0])                      # (z - z_i), ascending powers
    h = poly.real
    return h * (np.sqrt(2.0) / h.sum())


def wavelet_filter(h: np.ndarray) -> np.ndarray:
    """g[k] = (-1)^k h[K-1-k]."""
    K = len(h)
    return np.array([(-1) ** k * h[K - 1 - k] for k in range(K)])


def _real(x):
    """x as an array of its floating type (float64, or the extended type of an
    extended-precision run)."""
    x = np.asarray(x)
    return x.astype(np.result_type(x.dtype, np.float64), copy=False)


def analysis_1d(x: np.ndarray, h: np.ndarray, axis: int):
    """Periodised one-level analysis along ``axis``: (a, d), each half length."""
    g = wavelet_filter(h)
    x = np.moveaxis(_real(x), axis, -1)
    n = x.shape[-1]
    idx = (2 * np.arange(n // 2)[:, None] + np.arange(len(h))[None, :]) % n   # [m, k]
    a = np.einsum("...mk,k->...m", x[..., idx], h)
    d = np.einsum("...mk,k->...m", x[..., idx], g)
    return np.moveaxis(a, -1, axis), np.moveaxis(d, -1, axis)


def synthesis_1d(a: np.ndarray, d: np.ndarray, h: np.ndarray, axis: int):
    """Transpose of ``analysis_1d``: x[(2m + k) mod n] += h[k] a[m] + g[k] d[m]."""
    g = wavelet_filter(h)
    a = np.moveaxis(_real(a), axis, -1)
    d = np.moveaxis(_real(d), axis, -1)
    half = a.shape[-1]
    n = 2 * half
    x = np.zeros(a.shape[:-1] + (n,), dtype=np.result_type(a.dtype, d.dtype))
    for m in range(half):
        for k in range(len(h)):
            x[..., (2 * m + k) % n] += h[k] * a[..., m] + g[k] * d[..., m]
    return np.moveaxis(x, -1, axis)


def dwt2(img: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Multi-level periodised 2-D DWT of [..., ny, nx] arrays, Mallat layout."""
    out = np.array(_real(img), copy=True)
    ny, nx = out.shape[-2:]
    for j in range(levels):
        sy, sx = ny >> j, nx >> j
        blk = out[..., :sy, :sx]
        lo, hi = analysis_1d(blk, h, axis=-1)             # along x
        ll, lh = analysis_1d(lo, h, axis=-2)              # along y of x-low
        hl, hh = analysis_1d(hi, h, axis=-2)              # along y of x-high
        out[..., :sy // 2, :sx // 2] = ll
        out[..., :sy // 2, sx // 2:sx] = hl               # x high, y low
        out[..., sy // 2:sy, :sx // 2] = lh               # x low, y high
        out[..., sy // 2:sy, sx // 2:sx] = hh
    return out


def idwt2(coef: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Inverse (= transpose) of ``dwt2``."""
    out = np.array(_real(coef), copy=True)
    ny, nx = out.shape[-2:]
    for j in reversed(range(levels)):
        sy, sx = ny >> j, nx >> j
        ll = out[..., :sy // 2, :sx // 2]
        hl = out[..., :sy // 2, sx // 2:sx]
        lh = out[..., sy // 2:sy, :sx // 2]
        hh = out[..., sy // 2:sy, sx // 2:sx]
        lo = synthesis_1d(ll, lh, h, axis=-2)
        hi = synthesis_1d(hl, hh, h, axis=-2)
        out[..., :sy, :sx] = synthesis_1d(lo, hi, h, axis=-1)
    return out


class Dictionary:
    """W_s as a union of orthonormal bases, codes DIRAC or p (Db_p)."""

    def __init__(self, bases=(DIRAC,), shape=None):
        self.bases = tuple(int(b) for b in bases)
        if not self.bases:
            raise ValueError("empty dictionary")
        self.filters = {b: daubechies_filter(b) for b in self.bases if b != DIRAC}
        self.shape = shape

    @property
    def n_s(self) -> int:
        return len(self.bases)

    def _levels(self, x):
        ny, nx = x.shape[-2:]
        return dwt_levels(nx, ny)

    def forward(self, X: np.ndarray) -> np.ndarray:
        """W_s X: [n_s][L][ny][nx] coefficient cubes."""
        J = self._levels(X)
        return np.stack([X if b == DIRAC else dwt2(X, self.filters[b], J) for b in self.bases])

    def adjoint(self, C: np.ndarray) -> np.ndarray:
        """W_s^T C for stacked coefficient cubes C [n_s][L][ny][nx]."""
        J = self._levels(C[0])
        out = np.zeros(C.shape[1:], dtype=_real(C).dtype)
        for i, b in enumerate(self.bases):
            out += C[i] if b == DIRAC else idwt2(C[i], self.filters[b], J)
        return out


PAPER_DICTIONARY = (DIRAC, 1, 2, 3, 4, 5, 6, 7, 8)   # Section 4: Dirac + Db1..Db8
