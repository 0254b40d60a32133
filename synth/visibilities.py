"""Seeded synthetic visibilities: the sky cube of ``make_instance`` observed
at the uv points of its antenna tracks, without gridding.

Per band l the uv points of ``make_instance`` (same seed: same antennas, same
6 h track) are scaled by nu_l / nu_0 to cells of the nx x ny Fourier grid,
the longest baseline at the top band reaching ``nu_max_cells`` N, and kept
at their exact positions (``integer_uv`` rounds them to the nearest cell,
as the gridded PSF of the dirty-image instances does).  Each baseline is
listed once.  The visibilities are the band's sky sampled there,

    y_j = sum_{m,n} sky[m, n] exp(-2 pi i (u_j (n - nx/2) / nx + v_j (m - ny/2) / ny)),

plus complex Gaussian noise of standard deviation ``noise_sigma`` per real
and imaginary part (drawn after everything ``make_instance`` draws, from
the stream seeded with ``seed + 1``).  uv points and visibilities are
float64 (both the GPU path and the oracle read these values); the sky is
the float32 cube of ``make_instance``.  ``n_time`` sets the samples per
track (120 in the dirty-image instances).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .generator import _antennas, _uv_tracks, band_frequencies, make_instance


@dataclass
class VisInstance:
    uv: list          # per band [M][2] float64: (u, v) in cells
    vis: list         # per band [M] complex128
    sky: np.ndarray   # [L][ny][nx] float32
    freqs_ghz: np.ndarray
    shape: tuple      # (L, ny, nx)


def _sample(sky, uv):
    ny, nx = sky.shape
    u, v = uv[:, 0][:, None], uv[:, 1][:, None]
    eu = np.exp(-2j * np.pi * u * (np.arange(nx)[None, :] - nx // 2) / nx)
    ev = np.exp(-2j * np.pi * v * (np.arange(ny)[None, :] - ny // 2) / ny)
    rows = np.asarray(sky, np.float64) @ eu.T                  # [ny][M]
    return np.sum(ev * rows.T, axis=1)


def make_vis_instance(ny: int, nx: int, L: int, *, n_points: int, n_gauss: int, n_ant: int,
                      noise_sigma: float, seed: int, n_time: int = 120, nu_max_cells: float = 0.45,
                      integer_uv: bool = False) -> VisInstance:
    inst = make_instance(ny, nx, L, n_points=n_points, n_gauss=n_gauss, n_ant=n_ant,
                         noise_sigma=0.0, seed=seed, nu_max_cells=nu_max_cells, n_time=n_time)
    freqs = band_frequencies(L)
    rng = np.random.default_rng(seed)
    east, north = _antennas(rng, n_ant)
    u, v = _uv_tracks(east, north, n_time=n_time)
    uvmax = max(np.abs(u).max(), np.abs(v).max())
    base = nu_max_cells * min(ny, nx) / (uvmax * freqs.max())
    noise = np.random.default_rng(seed + 1)
    uvs, viss = [], []
    for l in range(L):
        uv = np.stack([u, v], axis=1) * (base * freqs[l])
        if integer_uv:
            uv = np.rint(uv)
        y = _sample(inst.sky[l], uv)
        y = y + noise_sigma * (noise.normal(size=y.shape) + 1j * noise.normal(size=y.shape))
        uvs.append(uv)
        viss.append(y)
    return VisInstance(uv=uvs, vis=viss, sky=inst.sky, freqs_ghz=freqs, shape=(L, ny, nx))
