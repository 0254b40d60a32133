"""Spectral dictionary of the oracle: W_nu as one orthonormal transform along
the bands or a union of m_nu of them (Section 3, the closed form of step V
for a union of orthonormal transforms; Section 4: a DCT, with Chebyshev
polynomial basis functions named as an alternative).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Bases (codes as the library's):
* DCT (0): the orthonormal DCT-II, W[l, k] = a_k cos(pi (2l + 1) k / 2L).
* CHEBYSHEV (1): the Chebyshev polynomials T_0 .. T_{L-1} at the band
  positions x_l = -1 + 2l / (L - 1) (the bands equally spaced in frequency,
  mapped onto [-1, 1]), orthonormalised in order of degree (reading: the
  paper names the family, not its normalisation).  Column k spans the
  polynomials of degree <= k that are orthogonal to those of lower degree;
  its sign makes the degree-k coefficient positive.  Built here by
  Gram-Schmidt in exact rational arithmetic (T_k at rational points is
  rational; only the final normalisation is floating point), so it carries
  no rounding from the ill conditioning of polynomials at equispaced
  points.
* DIRAC (2): the identity (sparsity of the spectrum values themselves).

A union stacks the coefficients of its bases: X W_nu is [m][L][ny][nx] (one
coefficient cube per basis), W_nu^T sums the per-basis inverses, and
W_nu W_nu^T = m I, the identity behind the m_nu rho_V of step V.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import numpy as np
import scipy.fft as sfft

DCT, CHEBYSHEV, SPECTRAL_DIRAC = 0, 1, 2


def chebyshev_values(L: int):
    """T_k(x_l), k, l < L, at x_l = -1 + 2l / (L - 1), as exact Fractions
    (rows l, columns k), by T_0 = 1, T_1 = x, T_{k+1} = 2 x T_k - T_{k-1}."""
    xs = [Fraction(0)] if L == 1 else [Fraction(-1) + Fraction(2 * l, L - 1) for l in range(L)]
    rows = []
    for x in xs:
        t = [Fraction(1), x]
        while len(t) < L:
            t.append(2 * x * t[-1] - t[-2])
        rows.append(t[:L])
    return rows


@lru_cache(maxsize=None)
def _chebyshev_orthogonal(L: int):
    """Gram-Schmidt of the Chebyshev columns in exact arithmetic: the
    orthogonal (not yet normalised) columns as lists of Fractions."""
    T = chebyshev_values(L)
    ortho = []
    for k in range(L):
        v = [T[l][k] for l in range(L)]
        for u in ortho:
            uu = sum(a * a for a in u)
            c = sum(a * b for a, b in zip(u, v)) / uu
            v = [a - c * b for a, b in zip(v, u)]
        ortho.append(v)
    # orthogonalising T_k against lower degrees keeps T_k's leading
    # coefficient (2^(k-1) > 0), so the sign is already the stated one
    return ortho


@lru_cache(maxsize=None)
def chebyshev_basis(L: int, dtype=np.float64) -> np.ndarray:
    """The orthonormalised Chebyshev basis (L x L columns), each entry the
    exact value a / sqrt(sum a^2) rounded once to ``dtype`` (float64 or the
    extended np.longdouble)."""
    from decimal import Decimal, localcontext
    W = np.empty((L, L), dtype=dtype)
    with localcontext() as ctx:
        ctx.prec = 50
        for k, v in enumerate(_chebyshev_orthogonal(L)):
            s2 = sum(a * a for a in v)
            inv = 1 / (Decimal(s2.numerator) / Decimal(s2.denominator)).sqrt()
            for l, a in enumerate(v):
                W[l, k] = dtype(str(Decimal(a.numerator) / Decimal(a.denominator) * inv))
    return W


def basis_matrix(code: int, L: int, dtype=np.float64) -> np.ndarray:
    """W of one basis, spectrum of a pixel = x @ W."""
    if code == DCT:
        return sfft.dct(np.eye(L, dtype=dtype), type=2, norm="ortho", axis=1)
    if code == CHEBYSHEV:
        return chebyshev_basis(L, dtype)
    if code == SPECTRAL_DIRAC:
        return np.eye(L, dtype=dtype)
    raise ValueError(f"unknown spectral basis {code}")


class SpectralDictionary:
    """W_nu: one orthonormal basis or a union of them (codes above)."""

    def __init__(self, bases=(DCT,)):
        self.bases = tuple(int(b) for b in bases)
        if not self.bases:
            raise ValueError("empty spectral dictionary")
        for b in self.bases:
            if b not in (DCT, CHEBYSHEV, SPECTRAL_DIRAC):
                raise ValueError(f"unknown spectral basis {b}")

    @property
    def m(self) -> int:
        return len(self.bases)

    def _apply(self, code, A, inverse):
        # A: [L][...] cube (bands first); x @ W per pixel, or c @ W^T
        if code == DCT:
            f = sfft.idct if inverse else sfft.dct
            return f(A, type=2, norm="ortho", axis=0)
        if code == SPECTRAL_DIRAC:
            return A.copy()
        W = basis_matrix(code, A.shape[0], A.dtype.type)
        return np.tensordot(W if inverse else W.T, A, axes=(1, 0))

    def forward(self, S):
        """S W_nu: a cube for one basis, [m][L][ny][nx] for a union."""
        if self.m == 1:
            return self._apply(self.bases[0], S, False)
        return np.stack([self._apply(b, S, False) for b in self.bases])

    def adjoint(self, C):
        """C W_nu^T (the inverse for one basis, the sum of the inverses for a union)."""
        if self.m == 1:
            return self._apply(self.bases[0], C, True)
        out = self._apply(self.bases[0], C[0], True)
        for j in range(1, self.m):
            out = out + self._apply(self.bases[j], C[j], True)
        return out
