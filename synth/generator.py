"""Seeded synthetic wide-band instances shaped like the paper's simulations.

The paper (Section 4) reconstructs 256x256 images over 15 bands from MeerKAT
PSFs computed with MeqTrees, and skies made of Gaussian profiles with
power-law spectra.  Neither the PSFs nor the M31 image are available, so this
module draws stand-ins with the same structure:

* uv coverage: ``n_ant`` antennas uniform in the unit disc, all baselines
  i < j, a 6 h Earth-rotation track (hour angle -3 h .. +3 h, 120 samples) at
  latitude -30.7 deg and declination -30 deg;
* per band, the uv points scale with nu_l / nu_0; they are gridded to the
  nearest cell (mod N) with their Hermitian mirror, and the PSF is
  ``fftshift(|IFFT2(mask)|)`` normalised to a peak of 1 (peak at
  0-based pixel (N/2, N/2));
* sky: point sources at integer pixels and elliptical Gaussians (sigma
  2..6 px), amplitude log-uniform in [0.1, 10], spectrum
  A (nu/nu_0)^(alpha + beta ln(nu/nu_0)) with alpha ~ U(-1.5, 0.5) and,
  for curved spectra, beta ~ N(0, 0.2);
* dirty image: circular convolution of each band's sky with its PSF plus
  white Gaussian noise.

The random stream is ``numpy.random.default_rng(seed)`` with the fixed draw
order antennas -> sources -> noise.  Everything is drawn in float64 and the
returned cubes are rounded to float32: both the GPU path and the oracle read
those float32 values.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Instance:
    """One synthetic cube: float32 arrays of shape [L][ny][nx]."""
    psf: np.ndarray
    dirty: np.ndarray
    sky: np.ndarray
    freqs_ghz: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.psf.shape


def band_frequencies(L: int, lo_ghz: float = 1.0, hi_ghz: float = 2.0,
                     spacing_ghz: float | None = None) -> np.ndarray:
    """Band centre frequencies in GHz.

    Default: linear from ``lo_ghz`` to ``hi_ghz``.  With ``spacing_ghz`` the
    bands start at ``lo_ghz`` and step by that spacing (the paper's layout is
    15 bands from 1.025 GHz, 50 MHz apart).
    """
    if spacing_ghz is not None:
        return lo_ghz + spacing_ghz * np.arange(L, dtype=np.float64)
    if L == 1:
        return np.array([lo_ghz], dtype=np.float64)
    return np.linspace(lo_ghz, hi_ghz, L, dtype=np.float64)


def _antennas(rng, n_ant):
    r = np.sqrt(rng.uniform(size=n_ant))
    th = rng.uniform(0.0, 2.0 * np.pi, size=n_ant)
    return r * np.cos(th), r * np.sin(th)   # east, north


def _uv_tracks(east, north, n_time=120, ha_hours=3.0, lat_deg=-30.7,
               dec_deg=-30.0):
    i, j = np.triu_indices(east.size, 1)
    eb = east[j] - east[i]
    nb = north[j] - north[i]
    phi = np.deg2rad(lat_deg)
    dec = np.deg2rad(dec_deg)
    # local east-north baseline -> equatorial XYZ
    X = -nb * np.sin(phi)
    Y = eb
    Z = nb * np.cos(phi)
    H = np.deg2rad(15.0 * np.linspace(-ha_hours, ha_hours, n_time))
    sH, cH = np.sin(H)[None, :], np.cos(H)[None, :]
    u = sH * X[:, None] + cH * Y[:, None]
    v = (-np.sin(dec) * cH * X[:, None] + np.sin(dec) * sH * Y[:, None]
         + np.cos(dec) * Z[:, None])
    return u.ravel(), v.ravel()


def _psf_band(u, v, scale, ny, nx):
    iu = np.rint(u * scale).astype(np.int64)
    iv = np.rint(v * scale).astype(np.int64)
    mask = np.zeros((ny, nx), dtype=np.float64)
    mask[iv % ny, iu % nx] = 1.0
    mask[(-iv) % ny, (-iu) % nx] = 1.0
    beam = np.abs(np.fft.ifft2(mask))
    beam = np.fft.fftshift(beam)
    return beam / beam.max()


def _gaussian_window(ny, nx, cy, cx, sa, sb, ang):
    half = int(np.ceil(6.0 * max(sa, sb)))
    dy = np.arange(-half, half + 1, dtype=np.float64)
    DY, DX = np.meshgrid(dy, dy, indexing="ij")
    c, s = np.cos(ang), np.sin(ang)
    a = c * DX + s * DY
    b = -s * DX + c * DY
    prof = np.exp(-0.5 * ((a / sa) ** 2 + (b / sb) ** 2))
    rows = (cy + dy.astype(np.int64)) % ny
    cols = (cx + dy.astype(np.int64)) % nx
    return rows, cols, prof


def make_instance(ny: int, nx: int, L: int, *, n_points: int, n_gauss: int,
                  n_ant: int, noise_sigma: float, seed: int,
                  curvature_sigma: float = 0.0, freqs_ghz=None,
                  sigma_range=(2.0, 6.0), nu_max_cells: float = 0.45,
                  n_time: int = 120) -> Instance:
    """Draw one instance (see the module docstring for the recipe)."""
    rng = np.random.default_rng(seed)
    freqs = band_frequencies(L) if freqs_ghz is None else np.asarray(freqs_ghz, np.float64)
    assert freqs.shape == (L,)
    nu0 = 1.0                       # reference frequency of the spectra (GHz)
    # 1. antennas and uv tracks
    east, north = _antennas(rng, n_ant)
    u, v = _uv_tracks(east, north, n_time=n_time)
    uvmax = max(np.abs(u).max(), np.abs(v).max())
    base = nu_max_cells * min(ny, nx) / (uvmax * freqs.max() / nu0)
    # 2. sources
    lo_y, hi_y = ny // 8, (7 * ny) // 8
    lo_x, hi_x = nx // 8, (7 * nx) // 8
    pts_y = rng.integers(lo_y, hi_y, size=n_points)
    pts_x = rng.integers(lo_x, hi_x, size=n_points)
    pts_amp = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=n_points))
    pts_alpha = rng.uniform(-1.5, 0.5, size=n_points)
    pts_beta = (rng.normal(0.0, curvature_sigma, size=n_points)
                if curvature_sigma > 0 else np.zeros(n_points))
    g_y = rng.integers(lo_y, hi_y, size=n_gauss)
    g_x = rng.integers(lo_x, hi_x, size=n_gauss)
    g_sa = rng.uniform(*sigma_range, size=n_gauss)
    g_sb = rng.uniform(*sigma_range, size=n_gauss)
    g_ang = rng.uniform(0.0, np.pi, size=n_gauss)
    g_amp = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=n_gauss))
    g_alpha = rng.uniform(-1.5, 0.5, size=n_gauss)
    g_beta = (rng.normal(0.0, curvature_sigma, size=n_gauss)
              if curvature_sigma > 0 else np.zeros(n_gauss))

    lnr = np.log(freqs / nu0)
    def spectrum(amp, alpha, beta):
        return amp[:, None] * np.exp((alpha[:, None] + beta[:, None] * lnr[None, :])
                                     * lnr[None, :])
    pts_spec = spectrum(pts_amp, pts_alpha, pts_beta)      # [n_points][L]
    g_spec = spectrum(g_amp, g_alpha, g_beta)              # [n_gauss][L]
    windows = [_gaussian_window(ny, nx, g_y[j], g_x[j], g_sa[j], g_sb[j], g_ang[j])
               for j in range(n_gauss)]

    psf = np.empty((L, ny, nx), dtype=np.float32)
    sky = np.empty((L, ny, nx), dtype=np.float32)
    dirty = np.empty((L, ny, nx), dtype=np.float32)

    def band(l, noise):
        beam = _psf_band(u, v, base * freqs[l] / nu0, ny, nx)
        s = np.zeros((ny, nx), dtype=np.float64)
        np.add.at(s, (pts_y, pts_x), pts_spec[:, l])
        for j, (rows, cols, prof) in enumerate(windows):
            np.add.at(s, np.ix_(rows, cols), g_spec[j, l] * prof)
        # circular convolution with the band's PSF (peak moved to lag 0)
        conv = np.fft.irfft2(np.fft.rfft2(np.fft.ifftshift(beam)) * np.fft.rfft2(s),
                             s=(ny, nx))
        conv += noise
        psf[l] = beam
        sky[l] = s
        dirty[l] = conv

    # 3. noise: drawn band by band, after every source draw, in this thread;
    # the bands themselves are independent and large ones run in a thread
    # pool (the FFTs release the GIL), with the same results
    workers = min(16, os.cpu_count() or 1) if ny * nx >= 1 << 18 and L > 1 else 1
    if workers == 1:
        for l in range(L):
            band(l, rng.normal(0.0, noise_sigma, size=(ny, nx)))
    else:
        from collections import deque
        from concurrent.futures import ThreadPoolExecutor
        pending = deque()
        with ThreadPoolExecutor(workers) as ex:
            for l in range(L):
                pending.append(ex.submit(band, l, rng.normal(0.0, noise_sigma, size=(ny, nx))))
                if len(pending) > 2 * workers:
                    pending.popleft().result()
            while pending:
                pending.popleft().result()
    meta = dict(seed=seed, n_points=n_points, n_gauss=n_gauss, n_ant=n_ant,
                noise_sigma=noise_sigma, curvature_sigma=curvature_sigma)
    return Instance(psf=psf, dirty=dirty, sky=sky, freqs_ghz=freqs, meta=meta)
