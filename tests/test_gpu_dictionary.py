"""Parity of the HIP path with the FP64 oracle when W_s is the paper's
spatial dictionary (Section 4: the Dirac basis and the Daubechies bases
Db1-Db8, n_s = 9; eq. Qlsimp with n_s rho_T), through the C ABI.

Error metric as in test_gpu_parity.py: relative L2 of X per iterate.  Bars:
FP32 1e-5 per iterate and 1e-4 on the final cube against the float64 oracle;
FP64 1e-12 against the oracle in extended precision.  The oracle's
dictionary is pinned in test_wavelet_pins.py.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth import get_config, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAPER = (0, 1, 2, 3, 4, 5, 6, 7, 8)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _kw(p):
    return dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho_P=p.rho_P, rho_T=p.rho_T,
                rho_V=p.rho_V, rho_S=p.rho_S)


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


def _per_iterate(inst, params, bases, K, dtype):
    from paper_1504_06847_amd import Solver
    s = Solver(inst.psf, inst.dirty, dtype=dtype, spatial=bases, **_kw(params))
    prob = O.Problem(inst.psf, inst.dirty, params, bases=bases,
                     dtype=np.longdouble if dtype == torch.float64 else np.float64)
    st = prob.zero_state()
    errs = []
    for _ in range(K):
        s.iterate(1)
        st = O.admm_iteration(prob, st)
        errs.append(rel(s.x.cpu().double().numpy(), st.X.astype(np.float64)))
    return errs, s, prob, st


CASES = [
    # (L, ny, nx, bases, K): the paper's dictionary; non-square images; images
    # smaller than the longest filter (periodic wrap at every level)
    (8, 64, 64, PAPER, 12),
    (4, 32, 64, (0, 1, 2, 8), 10),
    (2, 64, 16, (0, 3, 5), 10),
    (3, 16, 16, (0, 8), 10),
    (2, 8, 8, PAPER, 10),
    # short and wide: 8 coefficient rows per sub-band (half a tile's rows)
    # across two tiles of columns at the finest level
    (2, 16, 128, (0, 2, 8), 8),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("L,ny,nx,bases,K", CASES)
def test_dictionary_matches_oracle_per_iterate(gpu_lib, L, ny, nx, bases, K, dtype):
    cfg = get_config("plain64")
    inst = make_instance(ny, nx, L, n_points=5, n_gauss=2, n_ant=20, noise_sigma=0.01, seed=21 + L)
    p = cfg.params
    _say("dictionary", L, ny, nx, bases, dtype)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    errs, s, _, _ = _per_iterate(inst, p, bases, K, tdt)
    _say("  errs", ["%.2e" % e for e in errs])
    if dtype == "f32":
        assert max(errs) <= 1e-5 and errs[-1] <= 1e-4
    else:
        assert max(errs) <= 1e-12
    assert s.schedule[2] == 0 and not s.fused_available


def test_paper_shape_with_the_paper_dictionary(gpu_lib):
    """256 x 256 x 15 (Section 4's run shape) with Dirac + Db1..Db8, FP32."""
    cfg = get_config("paper256")
    inst = cfg.make()
    _say("paper256 dictionary")
    errs, _, _, _ = _per_iterate(inst, cfg.params, PAPER, 3, torch.float32)
    _say("  errs", ["%.2e" % e for e in errs])
    assert max(errs) <= 1e-5


def test_dictionary_graph_state_and_params(gpu_lib):
    """Graph replay equals the launched pass bit for bit; a saved state
    resumes the run bit for bit; a change of the rho's mid-run (multipliers
    held, the prox inputs re-encoded) continues as the oracle does."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = make_instance(32, 32, 4, n_points=5, n_gauss=2, n_ant=20, noise_sigma=0.01, seed=5)
    p = cfg.params
    bases = (0, 2, 4, 6)
    eager = Solver(inst.psf, inst.dirty, spatial=bases, dtype=torch.float64, **_kw(p))
    graph = Solver(inst.psf, inst.dirty, spatial=bases, dtype=torch.float64, graph=True, **_kw(p))
    for k in range(6):
        eager.iterate(1)
        graph.iterate(1)
        assert torch.equal(eager.x, graph.x), k
    saved = eager.get_state().clone()
    eager.iterate(4)
    x_ref = eager.x.clone()
    eager.set_state(saved)
    eager.iterate(4)
    assert torch.equal(eager.x, x_ref)
    # parameter change after 6 + 4 passes, then 5 more, against the oracle
    prob = O.Problem(inst.psf, inst.dirty, p, bases=bases)
    st = O.run(prob, 10)
    p2 = O.Params.from_any(p).with_(rho_T=2.5, rho_P=0.7, rho_V=1.5)
    st = O.run(prob.with_params(p2), 5, state=st)
    eager.set_params(rho_T=2.5, rho_P=0.7, rho_V=1.5)
    eager.iterate(5)
    err = rel(eager.x.cpu().numpy(), st.X)
    _say("after set_params", err)
    assert err <= 1e-10


def test_dictionary_rejects_new_bases(gpu_lib):
    from paper_1504_06847_amd import Solver
    from paper_1504_06847_amd.lib import MuffinError
    inst = make_instance(16, 16, 2, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.01, seed=2)
    s = Solver(inst.psf, inst.dirty, spatial=PAPER)
    s.iterate(2)
    with pytest.raises(MuffinError):
        s.set_params(spatial=(0, 1))
    s.iterate(1)           # the context still works


GRAD_CASES = [
    # (L, ny, nx, bases): a subset on a non-square image; the paper's
    # dictionary on images smaller than the longest filter
    (4, 32, 64, (0, 1, 4, 8)),
    (3, 16, 16, PAPER),
]


@pytest.mark.parametrize("L,ny,nx,bases", GRAD_CASES)
def test_dictionary_gradient_matches_oracle_jvp(gpu_lib, L, ny, nx, bases):
    """The reverse sweep with wavelet bases (their z_b stored with the
    state, the adjoint of their updates and of their B_rest terms):
    (J^T gx) along each of the seven parameters equals <gx, J e_i> from the
    oracle's tangents (FP64, 1e-8 as for the Dirac basis), bit for bit the
    same for two checkpoint spacings; dL/dY against the tangent along a
    change of the dirty images; the context ends in the state after K
    passes."""
    from paper_1504_06847_amd import Solver
    inst = make_instance(ny, nx, L, n_points=4, n_gauss=2, n_ant=16, noise_sigma=0.01, seed=60 + L)
    p = get_config("grad64").params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    rng = np.random.default_rng(13)
    gx = rng.standard_normal(inst.dirty.shape)
    K = 7
    _say("dictionary gradient", L, ny, nx, bases)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, spatial=bases, **kw)
    # the scratch the header documents: m = 4 + n_w cubes per stored state
    cube = -(-(L * ny * nx * 8) // 256) * 256
    m, nw = 4 + len(bases) - 1, len(bases) - 1
    for C, n_cubes in ((3, m * 3 + 2 * (m + 1) * 3 + 6 + nw), (K, m + (m + 1) * K + 6 + nw)):
        # plus the FP64 block sums: two sets of max(ny nx / 64, 8192) blocks
        # of eight slots, and the eight accumulators
        sums = 2 * max(ny * nx // 64, 8192) * 8 * 8 + 8 * 8
        assert s.grad_workspace_bytes(K, C) == n_cubes * cube + sums, C
    _, g = s.grad_params(K, gx=gx, ckpt_every=3)
    _, g1 = s.grad_params(K, gx=gx, ckpt_every=K)
    assert g == g1
    prob = O.Problem(inst.psf, inst.dirty, p, bases=bases)
    scale = max(abs(v) for v in g.values())
    for name in Solver.GRAD_PARAMS:
        dp = O.Params(**{f: (1.0 if f == name else 0.0) for f in Solver.GRAD_PARAMS})
        _, dX = O.jvp_run(prob, K, dp)
        ref = float(np.sum(gx * dX))
        _say("  ", name, g[name], ref)
        assert abs(g[name] - ref) <= 1e-8 * max(abs(ref), scale), name
    loss, gy = s.grad_dirty(K, gx=gx, ckpt_every=3)
    gy = gy.cpu().double().numpy()
    dY = rng.standard_normal(inst.dirty.shape)
    _, dX = O.jvp_run(prob, K, (0.0, 0.0, 0.0), dY=dY)
    lhs, rhs = float(np.sum(gy * dY)), float(np.sum(gx * dX))
    _say("   dL/dY", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-9 * max(abs(rhs), float(np.sqrt(np.sum(gy ** 2) * np.sum(dY ** 2))))
    ref = Solver(inst.psf, inst.dirty, dtype=torch.float64, spatial=bases, **kw)
    ref.iterate(K)
    assert torch.equal(s.x, ref.x)
    # and the run goes on from there as the iterated one does
    s.iterate(2)
    ref.iterate(2)
    assert torch.equal(s.x, ref.x)


def test_dictionary_mse_gradient_fp32(gpu_lib):
    """FP32 reverse sweep with the paper's dictionary: the MSE gradient
    against the oracle's (float64), 1e-4 as for the Dirac basis."""
    from paper_1504_06847_amd import Solver
    inst = make_instance(32, 32, 4, n_points=4, n_gauss=2, n_ant=16, noise_sigma=0.01, seed=71)
    p = get_config("grad64").params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float32, spatial=PAPER, **kw)
    loss, g = s.grad(8, sky=inst.sky, ckpt_every=3)
    loss_o, g_o = O.mse_grad(O.Problem(inst.psf, inst.dirty, p, bases=PAPER), 8, inst.sky)
    err = np.abs(g - g_o) / np.abs(g_o).max()
    _say("dictionary fp32 grad", g, g_o, err)
    assert abs(loss - loss_o) <= 1e-5 * loss_o
    assert err.max() <= 1e-4


REPORT_CASES = [
    # (L, ny, nx, bases, dtype): the paper's dictionary; a subset on a
    # non-square image; images smaller than the longest filter
    (8, 64, 64, PAPER, "f64"),
    (4, 32, 64, (0, 1, 2, 8), "f64"),
    (2, 8, 8, PAPER, "f64"),
    (8, 64, 64, PAPER, "f32"),
]


@pytest.mark.parametrize("L,ny,nx,bases,dtype", REPORT_CASES)
def test_dictionary_report_matches_oracle(gpu_lib, L, ny, nx, bases, dtype):
    """The residuals (with ||T - W_s X||, W_s^T dT and W_s^T Gamma_T over
    every basis), E^k and the objective (mu_s sum_b ||W_b P||_1) of one
    reporting pass against the oracle; then the run goes on from the state
    the reporting pass left as the oracle's does.  Bars: FP64 1e-9 (the
    Dirac report's), FP32 against the float64 oracle 1e-3 on the residuals
    and E (differences of nearby iterates), 1e-5 on the tolerances and the
    objective."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = make_instance(ny, nx, L, n_points=5, n_gauss=2, n_ant=20, noise_sigma=0.01, seed=31 + L)
    p = cfg.params
    f64 = dtype == "f64"
    _say("dictionary report", L, ny, nx, bases, dtype)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64 if f64 else torch.float32, spatial=bases, **_kw(p))
    prob = O.Problem(inst.psf, inst.dirty, p, bases=bases, dtype=np.longdouble if f64 else np.float64)
    s.iterate(5)
    prev = O.run(prob, 5)
    rep = s.step_report()
    cur = O.admm_iteration(prob, prev)
    res = O.residuals(prob, prev, cur, eps_abs=1e-5, eps_rel=1e-4)
    E = O.energy(prob, prev, cur)
    F = O.objective(prob, cur.P)
    _say("  gpu", {k: rep[k] for k in ("r_pri", "r_dual", "eps_pri", "eps_dual", "E", "objective")})
    _say("  oracle", res, "E", E, "F", F)
    b1, b2 = (1e-9, 1e-9) if f64 else (1e-3, 1e-5)
    assert rep["iters"] == 6
    assert rep["r_pri"] == pytest.approx(res["r"], rel=b1)
    assert rep["r_dual"] == pytest.approx(res["s"], rel=b1)
    assert rep["E"] == pytest.approx(E, rel=b1)
    assert rep["eps_pri"] == pytest.approx(res["eps_pri"], rel=b2)
    assert rep["eps_dual"] == pytest.approx(res["eps_dual"], rel=b2)
    assert rep["objective"] == pytest.approx(F, rel=b2)
    s.iterate(3)
    st = O.run(prob, 3, state=cur)
    err = rel(s.x.cpu().double().numpy(), st.X.astype(np.float64))
    _say("  X after 3 more", err)
    assert err <= (1e-12 if f64 else 1e-4)


def test_dictionary_report_at_the_paper_shape(gpu_lib):
    """256 x 256 x 15 (Section 4's run shape) with Dirac + Db1..Db8, FP32: the
    report of the fourth pass against the float64 oracle's (bars as for the
    FP32 case above)."""
    cfg = get_config("paper256")
    inst = cfg.make()
    p = cfg.params
    from paper_1504_06847_amd import Solver
    s = Solver(inst.psf, inst.dirty, dtype=torch.float32, spatial=PAPER, **_kw(p))
    prob = O.Problem(inst.psf, inst.dirty, p, bases=PAPER)
    s.iterate(3)
    prev = O.run(prob, 3)
    rep = s.step_report()
    cur = O.admm_iteration(prob, prev)
    res = O.residuals(prob, prev, cur, eps_abs=1e-5, eps_rel=1e-4)
    _say("paper shape report", {k: rep[k] for k in ("r_pri", "r_dual", "E", "objective")}, res)
    assert rep["r_pri"] == pytest.approx(res["r"], rel=1e-3)
    assert rep["r_dual"] == pytest.approx(res["s"], rel=1e-3)
    assert rep["E"] == pytest.approx(O.energy(prob, prev, cur), rel=1e-3)
    assert rep["eps_pri"] == pytest.approx(res["eps_pri"], rel=1e-5)
    assert rep["eps_dual"] == pytest.approx(res["eps_dual"], rel=1e-5)
    assert rep["objective"] == pytest.approx(O.objective(prob, cur.P), rel=1e-5)


def test_dictionary_adaptive_solve_matches_oracle(gpu_lib):
    """muffin_solve_adaptive with wavelet bases: the same rho decisions at
    the same checks, the same stopping iteration and the same X as the
    oracle's solve_adaptive (FP64, 1e-12)."""
    from paper_1504_06847_amd import Solver
    inst = make_instance(32, 32, 4, n_points=4, n_gauss=1, n_ant=14, noise_sigma=0.01, seed=13)
    bases = (0, 1, 4)
    p = O.Params(1e-3, 0.02, 0.02, 0.05, 0.05, 0.05, 0.05)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, spatial=bases, mu_eps=p.mu_eps, mu_s=p.mu_s,
               mu_nu=p.mu_nu, rho=0.05, check_every=10, eps_abs=1e-6, eps_rel=1e-5)
    rep = s.solve(150, adaptive=(10.0, 2.0))
    prob = O.Problem(inst.psf, inst.dirty, p, bases=bases, dtype=np.longdouble)
    st, pr, hist = O.solve_adaptive(prob, 150, 10, 10.0, 2.0, eps_abs=1e-6, eps_rel=1e-5)
    _say("gpu rho", s.params["rho_P"], "iters", rep["iters"], "oracle rho", pr.p.rho_P, "iters", hist[-1][0],
         "history", [(k, r) for k, r, _, _ in hist])
    assert s.params["rho_P"] == pr.p.rho_P
    assert pr.p.rho_P != 0.05                       # the rule fired
    assert rep["iters"] == hist[-1][0]
    err = rel(s.x.cpu().numpy(), st.X.astype(np.float64))
    _say("  X rel err", err)
    assert err <= 1e-12


def test_dictionary_solve_stops_on_residuals(gpu_lib):
    """muffin_solve with the paper's dictionary stops at a check whose
    residuals are under their tolerances."""
    from paper_1504_06847_amd import Solver
    inst = make_instance(16, 16, 4, n_points=3, n_gauss=1, n_ant=12, noise_sigma=0.01, seed=9)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, spatial=PAPER, rho=1.0, mu_s=0.05, mu_nu=0.05,
               check_every=5, eps_abs=1e-6, eps_rel=1e-5)
    rep = s.solve(5000)
    _say("dictionary solve", rep)
    assert rep["status"] == 0 and rep["converged"] == 1
    assert rep["r_pri"] <= rep["eps_pri"] and rep["r_dual"] <= rep["eps_dual"]
    assert rep["iters"] % 5 == 0
