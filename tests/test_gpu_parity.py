"""Parity of the HIP path (through the C ABI) with the oracle.

Error metric: relative L2 over the whole cube, ||X_gpu^k - X_or^k|| / ||X_or^k||,
for every iterate k.  Bars: FP32 1e-5 per iterate and 1e-4 on the final cube
against the float64 oracle (the stated FP32-vs-FP64 tolerance); the FP64
instantiation 1e-12 against the oracle run in extended precision (step I
amplifies the rounding of either float64 evaluation by up to
max |h_hat|^2 / rho, so float64 against float64 would measure the
oracle's error as much as the kernel's).
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth import get_config, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _params(p):
    return dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho_P=p.rho_P, rho_T=p.rho_T,
                rho_V=p.rho_V, rho_S=p.rho_S)


def _per_iterate(inst, params, K, dtype, every=1):
    from paper_1504_06847_amd import Solver
    s = Solver(inst.psf, inst.dirty, dtype=dtype, **_params(params))
    prob = O.Problem(inst.psf, inst.dirty, params,
                     dtype=np.longdouble if dtype == torch.float64 else np.float64)
    st = O.State.zeros(prob.shape)
    errs = []
    for k in range(1, K + 1):
        s.iterate(1)
        st = O.admm_iteration(prob, st)
        if k % every == 0 or k == K:
            errs.append(rel(s.x.cpu().double().numpy(), st.X.astype(np.float64)))
    return errs, s, prob, st


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


SHAPES = [
    (1, 8, 8), (3, 16, 32), (2, 32, 16), (8, 64, 64), (15, 32, 32), (4, 128, 64),
    (64, 16, 16), (5, 8, 256), (2, 256, 8),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_step_I_fp64_matches_oracle(gpu_lib, shape):
    """First passes from the zero state (X^1 = Q^{-1} H^T Y), FP64 instantiation."""
    L, ny, nx = shape
    _say("step I fp64", shape)
    inst = make_instance(ny, nx, L, n_points=4, n_gauss=2, n_ant=12, noise_sigma=0.01,
                         seed=100 + L + ny + nx, sigma_range=(1.0, 3.0))
    p = O.Params(1e-3, 0.5, 1.0, 1.0, 5.0, 2.0, 1.0)
    errs, s, prob, st = _per_iterate(inst, p, 3, torch.float64)
    _say("errs", errs)
    assert max(errs) < 1e-12, errs


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_step_I_fp32_matches_oracle(gpu_lib, shape):
    L, ny, nx = shape
    _say("step I fp32", shape)
    inst = make_instance(ny, nx, L, n_points=4, n_gauss=2, n_ant=12, noise_sigma=0.01,
                         seed=100 + L + ny + nx, sigma_range=(1.0, 3.0))
    errs, *_ = _per_iterate(inst, O.Params(1e-3, 0.5, 1.0, 1.0, 5.0, 2.0, 1.0), 3, torch.float32)
    assert max(errs) < 1e-5, errs


def test_plain64_fp64_every_iterate(gpu_lib):
    """64x64x8, paper parameters, 100 passes: FP64 instantiation vs oracle."""
    cfg = get_config("plain64")
    _say("plain64 fp64")
    errs, *_ = _per_iterate(cfg.make(), cfg.params, cfg.iters, torch.float64)
    _say("max rel err", max(errs))
    assert max(errs) < 1e-12


def test_plain64_fp32_every_iterate(gpu_lib):
    cfg = get_config("plain64")
    _say("plain64 fp32")
    errs, *_ = _per_iterate(cfg.make(), cfg.params, cfg.iters, torch.float32)
    _say("max rel err", max(errs), "final", errs[-1])
    assert max(errs) < 1e-5 and errs[-1] < 1e-4


def test_paper_shape_fp32_dense_dct(gpu_lib):
    """256x256x15 (the paper's run shape, 15 bands -> dense DCT path), 40 passes."""
    cfg = get_config("paper256")
    _say("paper256 fp32 40 passes")
    errs, *_ = _per_iterate(cfg.make(), cfg.params, 40, torch.float32, every=5)
    _say("errs", errs)
    assert max(errs) < 1e-5


def test_fp32_256x256x32_300_iterations(gpu_lib):
    """256x256x32, rho = 1, mu_s = mu_nu = 0.02: per-iterate error over 300 passes
    (compared every 10th iterate)."""
    cfg = get_config("fp32_256")
    _say("fp32_256 fp32 300 passes")
    errs, *_ = _per_iterate(cfg.make(), cfg.params, cfg.iters, torch.float32, every=10)
    _say("errs", errs[:3], "...", errs[-3:])
    assert max(errs) < 1e-5 and errs[-1] < 1e-4


def test_state_roundtrip_is_bitwise(gpu_lib):
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    s = Solver(inst.psf, inst.dirty, **_params(cfg.params))
    s.iterate(7)
    saved = s.get_state().clone()
    s.iterate(9)
    x_direct = s.x.clone()
    assert s.iterations == 16
    s.set_state(saved)
    assert s.iterations == 7
    s.iterate(9)
    assert torch.equal(s.x, x_direct)
    s.reset()
    assert s.iterations == 0
    s.iterate(16)
    assert torch.equal(s.x, x_direct)


def test_set_params_new_rhos_continue_algorithm_1(gpu_lib):
    """New rho's (and mu_nu) mid-run: the multipliers are held, so the run is
    the oracle's nine-array iteration continued with the new values."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    p1 = cfg.params
    p2 = p1.with_(rho_P=2.5, rho_T=2.0, rho_V=1.5, rho_S=0.7, mu_nu=0.6)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **_params(p1))
    s.iterate(10)
    s.set_params(**_params(p2))
    s.iterate(10)
    prob1 = O.Problem(inst.psf, inst.dirty, p1)
    st = O.run(prob1, 10)
    st = O.run(prob1.with_params(p2), 10, state=st)
    assert rel(s.x.cpu().numpy(), st.X) < 1e-12


def test_set_params_new_mu_s_converges_to_new_problem(gpu_lib):
    """A new mu_s restarts from the stored prox inputs: the run converges to the
    minimiser of the new problem (oracle run to convergence)."""
    from paper_1504_06847_amd import Solver
    inst = make_instance(32, 32, 4, n_points=3, n_gauss=1, n_ant=12, noise_sigma=0.01, seed=9)
    p1 = O.Params(1e-2, 0.05, 0.05, 1.0, 1.0, 1.0, 1.0)
    p2 = p1.with_(mu_s=1.0, rho_T=1.5)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **_params(p1))
    s.iterate(30)
    s.set_params(**_params(p2))
    s.iterate(4000)
    ref = O.run(O.Problem(inst.psf, inst.dirty, p2), 4000).X
    old_sol = O.run(O.Problem(inst.psf, inst.dirty, p1), 4000).X
    x = s.x.cpu().numpy()
    assert rel(old_sol, ref) > 1e-3          # the two problems differ (6e-3)
    assert rel(x, ref) < 1e-8                # a CPU model of this run reaches 7e-12


def test_report_matches_oracle(gpu_lib):
    """Residuals, E^k and the objective of one pass against the oracle."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **_params(cfg.params))
    prob = O.Problem(inst.psf, inst.dirty, cfg.params)
    s.iterate(5)
    prev = O.run(prob, 5)
    rep = s.step_report()
    cur = O.admm_iteration(prob, prev)
    res = O.residuals(prob, prev, cur, eps_abs=1e-5, eps_rel=1e-4)
    assert rep["iters"] == 6
    assert rep["r_pri"] == pytest.approx(res["r"], rel=1e-9)
    assert rep["r_dual"] == pytest.approx(res["s"], rel=1e-9)
    assert rep["eps_pri"] == pytest.approx(res["eps_pri"], rel=1e-9)
    assert rep["eps_dual"] == pytest.approx(res["eps_dual"], rel=1e-9)
    assert rep["E"] == pytest.approx(O.energy(prob, prev, cur), rel=1e-9)
    assert rep["objective"] == pytest.approx(O.objective(prob, cur.P), rel=1e-9)
    assert rel(s.p.cpu().numpy(), cur.P) < 1e-12


def test_energy_non_increasing_fp32(gpu_lib):
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    s = Solver(inst.psf, inst.dirty, **_params(cfg.params))
    E = [s.step_report()["E"] for _ in range(40)]
    E = np.array(E)
    # FP32 state: allow rounding-level increases once E is tiny
    assert np.all(E[1:] <= E[:-1] * (1 + 1e-4) + 1e-6 * E[0])


def test_solve_stops_on_residuals(gpu_lib):
    from paper_1504_06847_amd import Solver
    inst = make_instance(32, 32, 4, n_points=3, n_gauss=1, n_ant=12, noise_sigma=0.01, seed=9)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, rho=1.0, mu_s=0.05, mu_nu=0.05,
               check_every=5, eps_abs=1e-6, eps_rel=1e-5)
    rep = s.solve(5000)
    assert rep["status"] == 0 and rep["converged"] == 1
    assert rep["r_pri"] <= rep["eps_pri"] and rep["r_dual"] <= rep["eps_dual"]
    assert rep["iters"] % 5 == 0
    s2 = Solver(inst.psf, inst.dirty, dtype=torch.float64, rho=1.0, mu_s=0.05, mu_nu=0.05,
                check_every=5, eps_abs=1e-12, eps_rel=1e-12)
    rep2 = s2.solve(20)
    assert rep2["status"] == 1 and rep2["iters"] == 20


def test_nonfinite_input_is_rejected(gpu_lib):
    from paper_1504_06847_amd import Solver, lib
    inst = make_instance(16, 16, 2, n_points=2, n_gauss=1, n_ant=8, noise_sigma=0.01, seed=3)
    d = inst.dirty.copy()
    d[1, 3, 4] = np.nan
    with pytest.raises(lib.MuffinError) as e:
        Solver(inst.psf, d)
    assert e.value.code == lib.MUFFIN_ENONFINITE


def test_full_size_first_passes_fp32(gpu_lib):
    """1024x1024x64 (the throughput workload, same kernels and launch shapes as
    the benchmark): the first two iterates against the oracle."""
    cfg = get_config("cube1024")
    _say("cube1024: generating")
    inst = cfg.make()
    _say("cube1024: 2 passes")
    errs, s, prob, st = _per_iterate(inst, cfg.params, 2, torch.float32)
    _say("cube1024 errs", errs)
    assert max(errs) < 1e-5
