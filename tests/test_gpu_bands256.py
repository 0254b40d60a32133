"""256 bands (the large workload's band count; Section 3, step IV's DCT
along the bands at L = 256): the spectral pass splits each pixel's band
vector over two waves (a butterfly, a DCT-II and a DCT-IV of length 128).
Against the oracle per iterate on small images (FP32 against float64 1e-5,
FP64 against the extended-precision run 1e-12), the FP64 convergence
reductions of a reporting pass, graph replay and state round trips; at the
full 2048 x 2048 x 256 size, the first pass band by band against the oracle
(step I from the zero state separates into bands) and the He-Yuan
monotonicity of E^k over the following passes."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth import get_config, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TIED = dict(mu_eps=1e-3, mu_s=0.02, mu_nu=0.02, rho_P=1.0, rho_T=1.0, rho_V=1.0, rho_S=1.0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


def _instance(ny, nx, seed, L=256):
    c = get_config("large2048")
    return make_instance(ny, nx, L, n_points=20, n_gauss=5, n_ant=30, noise_sigma=c.noise_sigma, seed=seed,
                         curvature_sigma=c.curvature_sigma)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("shape", [(8, 8), (16, 32), (64, 32)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_256_bands_match_oracle_per_iterate(gpu_lib, shape, dtype):
    from paper_1504_06847_amd import Solver
    ny, nx = shape
    _say("256 bands", shape, dtype)
    inst = _instance(ny, nx, seed=90 + ny)
    s = Solver(inst.psf, inst.dirty, dtype=dtype, **TIED)
    prob = O.Problem(inst.psf, inst.dirty, O.Params(**TIED),
                     dtype=np.longdouble if dtype == torch.float64 else np.float64)
    st = O.State.zeros(prob.shape)
    errs = []
    for _ in range(8):
        s.iterate(1)
        st = O.admm_iteration(prob, st)
        errs.append(rel(s.x.cpu().double().numpy(), st.X.astype(np.float64)))
    _say("  per-iterate rel err", ["%.2e" % e for e in errs])
    assert max(errs) < (1e-5 if dtype == torch.float32 else 1e-12), errs


def test_256_bands_report_matches_oracle(gpu_lib):
    """Residuals, E^k and the objective (its spectral l1 term a DCT of 256
    bands per pixel) of one reporting pass, FP64, against the oracle."""
    from paper_1504_06847_amd import Solver
    inst = _instance(32, 32, seed=7)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **TIED)
    prob = O.Problem(inst.psf, inst.dirty, O.Params(**TIED))
    s.iterate(4)
    prev = O.run(prob, 4)
    rep = s.step_report()
    cur = O.admm_iteration(prob, prev)
    res = O.residuals(prob, prev, cur, eps_abs=1e-5, eps_rel=1e-4)
    _say("report", rep, res)
    assert rep["iters"] == 5
    assert rep["r_pri"] == pytest.approx(res["r"], rel=1e-9)
    assert rep["r_dual"] == pytest.approx(res["s"], rel=1e-9)
    assert rep["eps_pri"] == pytest.approx(res["eps_pri"], rel=1e-9)
    assert rep["eps_dual"] == pytest.approx(res["eps_dual"], rel=1e-9)
    assert rep["E"] == pytest.approx(O.energy(prob, prev, cur), rel=1e-9)
    assert rep["objective"] == pytest.approx(O.objective(prob, cur.P), rel=1e-9)


def test_256_bands_graph_and_state_are_bitwise(gpu_lib):
    from paper_1504_06847_amd import Solver
    inst = _instance(32, 64, seed=8)
    a = Solver(inst.psf, inst.dirty, **TIED)
    b = Solver(inst.psf, inst.dirty, graph=True, **TIED)
    a.iterate(3)
    b.iterate(3)
    st = a.get_state().clone()
    a.iterate(4)
    b.iterate(4)
    torch.cuda.synchronize()
    assert torch.equal(a.x, b.x)
    c = Solver(inst.psf, inst.dirty, **TIED)
    c.set_state(st)
    c.iterate(4)
    torch.cuda.synchronize()
    assert torch.equal(c.x, a.x) and c.iterations == 7


def test_256_bands_reject_batches_and_the_gradient(gpu_lib):
    from paper_1504_06847_amd import Batch, Solver
    from paper_1504_06847_amd import lib as L
    inst = _instance(16, 16, seed=9)
    s = Solver(inst.psf, inst.dirty, **TIED)
    with pytest.raises(L.MuffinError, match="128"):
        s.grad(3, sky=inst.sky, ckpt_every=3)
    with pytest.raises(L.MuffinError):
        Batch([(inst.psf, inst.dirty)], params=TIED)


@pytest.mark.timeout(900)
def test_large2048_first_pass_and_energy(gpu_lib):
    """2048 x 2048 x 256 FP32 (the large workload): X^1 of sampled bands
    against the oracle's step I on those bands alone, then E^k of 8
    reporting passes non-increasing and every reduction finite."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("large2048")
    _say("generating", cfg.name)
    inst = cfg.make()
    p = cfg.params
    _say("setup")
    s = Solver(inst.psf, inst.dirty, mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    s.iterate(1)
    x = s.x
    for l in (0, 101, 128, 255):
        prob = O.Problem(inst.psf[l:l + 1], inst.dirty[l:l + 1], p)
        xo = O.admm_iteration(prob, O.State.zeros(prob.shape)).X[0]
        e = rel(x[l].cpu().double().numpy(), xo)
        _say("  band", l, "X^1 rel err", e)
        assert e < 1e-5
    del x
    E = []
    for k in range(8):
        rep = s.step_report()
        assert all(np.isfinite(v) for v in rep.values())
        E.append(rep["E"])
    _say("  E^k", ["%.4e" % v for v in E])
    E = np.array(E)
    assert np.all(E[1:] <= E[:-1] * (1 + 1e-4) + 1e-6 * E[0])
    s.close()
