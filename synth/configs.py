"""Named workloads: cube shape, generator settings and solver parameters.

Parameter sets:

* ``PAPER``: the values of the paper's simulations (Section 4):
  mu_eps = 0.001, mu_s = 0.5, mu_nu = 1.0, rho_P = 1, rho_T = 5, rho_V = 2,
  rho_S = 1.
* ``TIED``: one common augmented-Lagrangian value rho = 1 for all four
  constraints, mu_s = mu_nu = 0.02, mu_eps = 0.001 (the Tikhonov weight of
  the paper's runs, which keeps the problem strongly convex).
"""
from __future__ import annotations

from dataclasses import dataclass, replace, asdict

from .generator import band_frequencies, make_instance


@dataclass(frozen=True)
class SolverParams:
    mu_eps: float
    mu_s: float
    mu_nu: float
    rho_P: float
    rho_T: float
    rho_V: float
    rho_S: float

    @staticmethod
    def tied(rho: float, mu_s: float, mu_nu: float, mu_eps: float = 1e-3):
        return SolverParams(mu_eps, mu_s, mu_nu, rho, rho, rho, rho)

    def with_(self, **kw):
        return replace(self, **kw)

    def asdict(self):
        return asdict(self)


PAPER = SolverParams(mu_eps=1e-3, mu_s=0.5, mu_nu=1.0,
                     rho_P=1.0, rho_T=5.0, rho_V=2.0, rho_S=1.0)
TIED = SolverParams.tied(1.0, 0.02, 0.02, 1e-3)


@dataclass(frozen=True)
class Config:
    name: str
    ny: int
    nx: int
    L: int
    n_points: int
    n_gauss: int
    n_ant: int
    noise_sigma: float
    seed: int
    params: SolverParams
    iters: int
    curvature_sigma: float = 0.0
    freqs: str = "linear"       # "linear": 1..2 GHz; "paper": 1.025 GHz + 50 MHz steps

    @property
    def voxels(self):
        return self.ny * self.nx * self.L

    def frequencies(self):
        if self.freqs == "paper":
            return band_frequencies(self.L, lo_ghz=1.025, spacing_ghz=0.05)
        return band_frequencies(self.L)

    def make(self, seed=None):
        return make_instance(self.ny, self.nx, self.L, n_points=self.n_points,
                             n_gauss=self.n_gauss, n_ant=self.n_ant,
                             noise_sigma=self.noise_sigma,
                             seed=self.seed if seed is None else seed,
                             curvature_sigma=self.curvature_sigma,
                             freqs_ghz=self.frequencies())

    def scaled(self, **kw):
        return replace(self, **kw)


CONFIGS = {
    # 64x64x8, paper parameters, 100 iterations
    "plain64": Config("plain64", 64, 64, 8, 5, 2, 20, 0.01, 1, PAPER, 100),
    # 256x256x32, tied rho = 1, 300 iterations (FP32 vs FP64 error study)
    "fp32_256": Config("fp32_256", 256, 256, 32, 40, 10, 40, 0.005, 2, TIED, 300),
    # 1024x1024x64: the throughput / roofline / differentiation workload
    "cube1024": Config("cube1024", 1024, 1024, 64, 40, 10, 40, 0.005, 4, TIED, 20),
    # 64x64x8 instance drawn with the 1024-cube generator settings (seed 4)
    "grad64": Config("grad64", 64, 64, 8, 40, 10, 40, 0.005, 4, TIED, 20),
    # 2048x2048x256 with curved spectra
    "large2048": Config("large2048", 2048, 2048, 256, 500, 100, 200, 0.005, 5, TIED,
                        200, curvature_sigma=0.2),
    # the paper's run shape: 256x256, 15 bands from 1.025 GHz, 350 iterations
    "paper256": Config("paper256", 256, 256, 15, 5, 2, 20, 0.01, 6, PAPER, 350,
                       freqs="paper"),
}


def batched_shapes(seed: int = 3, n_cubes: int = 16):
    """Shapes of the uneven batch: N^2 in {128^2, 256^2, 512^2}, L in {16..128}."""
    import numpy as np
    rng = np.random.default_rng(seed)
    ns = rng.choice([128, 256, 512], size=n_cubes)
    ls = rng.choice([16, 32, 64, 128], size=n_cubes)
    return [(int(n), int(n), int(l)) for n, l in zip(ns, ls)]


def get_config(name: str) -> Config:
    return CONFIGS[name]


def batch_instances(seed: int = 3, n_cubes: int = 16):
    """The uneven batch: ``n_cubes`` cubes with the shapes of
    ``batched_shapes`` (N^2 in {128^2, 256^2, 512^2} x L in {16, 32, 64,
    128}), cube i drawn with the 256^2 x 32 generator settings (40 points,
    10 Gaussians, 40 antennas, sigma 0.005) and seed 300 + i.  Returns
    ([(psf, dirty), ...], parameters)."""
    c = get_config("fp32_256")
    out = []
    for i, (ny, nx, L) in enumerate(batched_shapes(seed, n_cubes)):
        inst = make_instance(ny, nx, L, n_points=c.n_points, n_gauss=c.n_gauss, n_ant=c.n_ant,
                             noise_sigma=c.noise_sigma, seed=300 + i)
        out.append((inst.psf, inst.dirty))
    return out, c.params
