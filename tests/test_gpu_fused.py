"""The fused launch (inverse row pass, steps II-VI, forward row pass of the
next step I) against the FP64 oracle and against the three-launch pass, and
the driver's bookkeeping around it (the row spectra of B_rest kept in place
of B_rest between passes)."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth import get_config, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PARAMS = dict(mu_eps=1e-3, mu_s=0.05, mu_nu=0.05, rho_P=1.0, rho_T=1.0, rho_V=1.0, rho_S=1.0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


# (L, ny, nx): every built row length and band count, a non-square image,
# more rows than pixels per row and the reverse
SHAPES = [(4, 16, 64), (8, 32, 128), (16, 64, 256), (32, 32, 512), (32, 16, 512), (64, 8, 1024),
          (64, 128, 64), (16, 256, 128), (8, 8, 1024)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_fused_pass_matches_oracle(gpu_lib, shape):
    from paper_1504_06847_amd import Solver
    L, ny, nx = shape
    inst = make_instance(ny, nx, L, n_points=4, n_gauss=2, n_ant=12, noise_sigma=0.01, seed=31)
    s = Solver(inst.psf, inst.dirty, **PARAMS)
    u = Solver(inst.psf, inst.dirty, **PARAMS)
    u.set_schedule((1, 1, 0))
    assert s.fused_available and s.schedule[2] == 1
    prob = O.Problem(inst.psf, inst.dirty, O.Params(**PARAMS))
    st = O.State.zeros(prob.shape)
    worst = worst_u = 0.0
    for k in range(12):
        s.iterate(1)
        u.iterate(1)
        st = O.admm_iteration(prob, st)
        worst = max(worst, rel(s.x.cpu().double().numpy(), st.X))
        worst_u = max(worst_u, rel(u.x.cpu().double().numpy(), st.X))
    _say("fused", shape, "worst per-iterate rel err", worst, "three launches", worst_u)
    assert worst < 1e-5 and worst_u < 1e-5


@pytest.mark.parametrize("shape", [(64, 8, 1024), (64, 16, 512), (64, 32, 256), (32, 8, 1024), (32, 16, 512), (64, 128, 64)],
                         ids=lambda s: "x".join(map(str, s)))
def test_two_pixel_form_matches_oracle_and_one_pixel_form(gpu_lib, shape):
    """Fused form 2 (two pixels per thread, half-size work-groups) against
    the oracle per iterate, and against form 1 to rounding (the same
    formulas; the compiler fuses products and sums into FMAs differently in
    the two kernels, as between tile schedules).  Where the two-pixel kernel
    is not built (fewer bands, short rows) form 2 runs as form 1, bit for
    bit.  Graph replay of form 2 repeats its launched passes bit for bit."""
    from paper_1504_06847_amd import Solver
    L, ny, nx = shape
    inst = make_instance(ny, nx, L, n_points=4, n_gauss=2, n_ant=12, noise_sigma=0.01, seed=33)
    a = Solver(inst.psf, inst.dirty, **PARAMS)
    b = Solver(inst.psf, inst.dirty, **PARAMS)
    g = Solver(inst.psf, inst.dirty, graph=True, **PARAMS)
    b.set_schedule((1, 1, 2))
    g.set_schedule((1, 1, 2))
    assert b.schedule == (1, 1, 2)
    built = (L == 64 and nx >= 256) or (L == 32 and nx == 1024)
    prob = O.Problem(inst.psf, inst.dirty, O.Params(**PARAMS))
    st = O.State.zeros(prob.shape)
    worst = 0.0
    for k in range(8):
        a.iterate(1)
        b.iterate(1)
        g.iterate(1)
        st = O.admm_iteration(prob, st)
        worst = max(worst, rel(b.x.cpu().double().numpy(), st.X))
        torch.cuda.synchronize()
        d = float((a.x.double() - b.x.double()).abs().max() / a.x.double().abs().max())
        assert d <= 1e-6, (k, d)
        if not built:
            assert torch.equal(a.x, b.x)
        assert torch.equal(b.x, g.x)
    _say("two-pixel form", shape, "worst per-iterate rel err", worst, "vs form 1", d)
    assert worst < 1e-5


def test_fused_and_three_launch_agree_over_a_long_run(gpu_lib):
    from paper_1504_06847_amd import Solver
    cfg = get_config("fp32_256")
    inst = cfg.make()
    p = cfg.params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    a = Solver(inst.psf, inst.dirty, **kw)
    b = Solver(inst.psf, inst.dirty, **kw)
    b.set_schedule((1, 1, 0))
    a.iterate(100)
    b.iterate(100)
    torch.cuda.synchronize()
    d = rel(a.x.double().cpu().numpy(), b.x.double().cpu().numpy())
    _say("fused vs three launches after 100 passes", d)
    assert d < 1e-5


def test_driver_calls_between_fused_passes(gpu_lib):
    """Reports, parameter changes, schedule switches, state round trips and
    graph replay interleaved with fused passes give the three-launch results
    (to rounding)."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    p = cfg.params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho_P=p.rho_P, rho_T=p.rho_T,
              rho_V=p.rho_V, rho_S=p.rho_S)
    a = Solver(inst.psf, inst.dirty, **kw)            # fused (the default)
    b = Solver(inst.psf, inst.dirty, **kw)
    b.set_schedule((1, 1, 0))

    def same(tag, bar=1e-6):
        torch.cuda.synchronize()
        d = rel(a.x.double().cpu().numpy(), b.x.double().cpu().numpy())
        _say(tag, d)
        assert d < bar, tag

    for s in (a, b):
        s.iterate(5)
    same("5 passes")
    ra, rb = a.step_report(), b.step_report()
    assert abs(ra["E"] - rb["E"]) <= 1e-5 * abs(rb["E"]) and ra["iters"] == rb["iters"]
    for s in (a, b):
        s.iterate(3)
    same("after a report")
    for s in (a, b):
        s.set_params(rho_P=1.5, rho_T=4.0)
        s.iterate(4)
    same("after set_params")
    st = a.get_state().clone()
    for s in (a, b):
        s.set_graph(True)
        s.iterate(6)
    same("graph replay")
    a.set_schedule((1, 1, 0))
    a.set_schedule((1, 1, 1))
    for s in (a, b):
        s.iterate(2)
    same("schedule switches")
    a.set_state(st)
    a.iterate(8)
    c = Solver(inst.psf, inst.dirty, **kw)
    c.set_schedule((1, 1, 0))
    c.set_params(rho_P=1.5, rho_T=4.0)
    c.set_state(st)
    c.iterate(8)
    torch.cuda.synchronize()
    assert rel(a.x.double().cpu().numpy(), c.x.double().cpu().numpy()) < 1e-6


@pytest.mark.parametrize("graph", [False, True], ids=["launch", "graph"])
def test_a_run_stores_x_on_its_last_pass(gpu_lib, graph):
    """A fused run of n passes stores X in its last pass only: X, the state
    snapshot and the passes after it are bit for bit those of n runs of one
    pass (every pass storing X)."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    p = cfg.params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho_P=p.rho_P, rho_T=p.rho_T,
              rho_V=p.rho_V, rho_S=p.rho_S)
    a = Solver(inst.psf, inst.dirty, graph=graph, **kw)
    b = Solver(inst.psf, inst.dirty, graph=graph, **kw)
    assert a.schedule[2] != 0                      # the fused pass
    a.iterate(7)
    for _ in range(7):
        b.iterate(1)
    torch.cuda.synchronize()
    assert torch.equal(a.x, b.x)
    assert torch.equal(a.get_state(), b.get_state())
    a.iterate(3)
    b.iterate(2)
    b.iterate(1)
    torch.cuda.synchronize()
    assert torch.equal(a.x, b.x)


def test_batch_after_fused_single_cube_passes(gpu_lib):
    """A batched pass after fused single-cube passes on the same cube starts
    from B_rest rebuilt from the state."""
    from paper_1504_06847_amd import Batch, Solver
    shapes = [(8, 32, 64), (16, 64, 64)]
    cubes = []
    for i, (L, ny, nx) in enumerate(shapes):
        inst = make_instance(ny, nx, L, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.005, seed=40 + i)
        cubes.append((inst.psf, inst.dirty))
    b = Batch(cubes, params=PARAMS)
    ref = [Solver(p, d, **PARAMS) for p, d in cubes]
    for s in ref:
        s.set_schedule((1, 1, 0))
    b.cube(0).iterate(4)            # fused single-cube passes
    ref[0].iterate(4)
    b.iterate(5)
    for s in ref:
        s.iterate(5)
    torch.cuda.synchronize()
    d0 = rel(b.cube(0).x.double().cpu().numpy(), ref[0].x.double().cpu().numpy())
    _say("batch after fused passes", d0)
    assert d0 < 1e-6
    assert b.cube(0).iterations == 9 and b.cube(1).iterations == 5


def test_full_size_fused_first_passes(gpu_lib):
    from paper_1504_06847_amd import Solver
    cfg = get_config("cube1024")
    inst = cfg.make()
    p = cfg.params
    s = Solver(inst.psf, inst.dirty, mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    assert s.schedule[2] == 1 and s.fused_available
    t = Solver(inst.psf, inst.dirty, mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    t.set_schedule((1, 1, 2))                 # two pixels per thread
    prob = O.Problem(inst.psf, inst.dirty, p)
    st = O.State.zeros(prob.shape)
    for k in range(3):
        s.iterate(1)
        t.iterate(1)
        st = O.admm_iteration(prob, st)
        e = rel(s.x.cpu().double().numpy(), st.X)
        e2 = rel(t.x.cpu().double().numpy(), st.X)
        _say("full size fused pass", k + 1, e, "two pixels per thread", e2)
        assert e < 1e-5 and e2 < 1e-5
