"""The driver around the kernels: graph replay of a pass, the widest band
count, and the calls that change the solver between passes.  Every GPU result
is compared with the eager launch form (bitwise) or with the FP64 oracle."""
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


def _kw(p):
    return dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho_P=p.rho_P, rho_T=p.rho_T,
                rho_V=p.rho_V, rho_S=p.rho_S)


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_graph_replay_is_bitwise_the_launched_pass(gpu_lib, dtype):
    """Replays of the recorded pass, interleaved with eager torch work, host
    synchronisations, reporting passes (which switch the state set) and a
    parameter change (which records a new graph), match the launched form
    bit for bit after every replay."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    _say("graph replay", dtype)
    eager = Solver(inst.psf, inst.dirty, dtype=dtype, **_kw(cfg.params))
    graph = Solver(inst.psf, inst.dirty, dtype=dtype, graph=True, **_kw(cfg.params))
    junk = torch.rand(1 << 20, device="cuda")
    for k in range(12):
        eager.iterate(1)
        graph.iterate(1)
        junk.mul_(0.5).add_(1.0)          # unrelated work between replays
        torch.cuda.synchronize()
        assert torch.equal(eager.x, graph.x), f"replay {k}"
        if k == 4:
            ra, rb = eager.step_report(), graph.step_report()
            assert ra == rb
        if k == 7:
            eager.set_params(rho=1.5)
            graph.set_params(rho=1.5)
    eager.iterate(25)
    graph.iterate(25)
    torch.cuda.synchronize()
    assert torch.equal(eager.x, graph.x)
    assert torch.equal(eager.get_state(), graph.get_state())
    assert eager.iterations == graph.iterations == 12 + 1 + 25
    rep = graph.solve(40)
    ref = eager.solve(40)
    assert rep == ref


def test_graph_replay_on_a_side_stream(gpu_lib):
    """The recorded pass replays on the stream the solver was set up with."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    side = torch.cuda.Stream()
    eager = Solver(inst.psf, inst.dirty, **_kw(cfg.params))
    with torch.cuda.stream(side):
        graph = Solver(inst.psf, inst.dirty, stream=side, graph=True, **_kw(cfg.params))
        graph.iterate(30)
        side.synchronize()
    eager.iterate(30)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        gx = graph.x
        side.synchronize()
    assert torch.equal(eager.x, gx)


def test_128_bands_fp32_matches_oracle(gpu_lib):
    """The widest band count (power-of-two register DCT of length 128)."""
    from paper_1504_06847_amd import Solver
    L, ny, nx = 128, 16, 32
    _say("128 bands", (L, ny, nx))
    inst = make_instance(ny, nx, L, n_points=4, n_gauss=2, n_ant=12, noise_sigma=0.01, seed=11)
    p = O.Params(1e-3, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0)
    s = Solver(inst.psf, inst.dirty, **_kw(p))
    prob = O.Problem(inst.psf, inst.dirty, p)
    st = O.State.zeros(prob.shape)
    worst = 0.0
    for k in range(20):
        s.iterate(1)
        st = O.admm_iteration(prob, st)
        worst = max(worst, rel(s.x.cpu().double().numpy(), st.X))
    _say("128 bands worst", worst)
    assert worst < 1e-5


def test_128_bands_fp64_matches_oracle(gpu_lib):
    from paper_1504_06847_amd import Solver
    L, ny, nx = 128, 8, 16
    inst = make_instance(ny, nx, L, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.01, seed=12)
    p = O.Params(1e-3, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **_kw(p))
    prob = O.Problem(inst.psf, inst.dirty, p)
    st = O.State.zeros(prob.shape)
    worst = 0.0
    for k in range(10):
        s.iterate(1)
        st = O.admm_iteration(prob, st)
        worst = max(worst, rel(s.x.cpu().double().numpy(), st.X))
    _say("128 bands fp64 worst", worst)
    assert worst < 1e-11
