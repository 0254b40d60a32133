"""The reverse sweep (muffin_grad) against the oracle's forward-mode
derivatives, finite differences and its own invariants."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth import get_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


def _grad64():
    """64 x 64 x 8 instance drawn with the 1024-cube generator settings, tied
    rho = 1, mu_s = mu_nu = 0.02, its sky as the reference."""
    cfg = get_config("grad64")
    inst = cfg.make()
    p = cfg.params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    return inst, p, kw


@pytest.fixture(scope="module")
def oracle_grad():
    inst, p, _ = _grad64()
    prob = O.Problem(inst.psf, inst.dirty, p)
    return O.mse_grad(prob, 20, inst.sky)


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-8), (torch.float32, 1e-4)], ids=["f64", "f32"])
def test_mse_gradient_matches_oracle(gpu_lib, oracle_grad, dtype, bar):
    from paper_1504_06847_amd import Solver
    inst, p, kw = _grad64()
    loss_o, g_o = oracle_grad
    s = Solver(inst.psf, inst.dirty, dtype=dtype, **kw)
    loss, g = s.grad(20, sky=inst.sky, ckpt_every=5)
    err = np.abs(g - g_o) / np.abs(g_o).max()
    _say(dtype, "loss", loss, loss_o, "grad", g, g_o, "rel err", err)
    assert abs(loss - loss_o) <= max(bar, 1e-6 if dtype == torch.float32 else 0) * loss_o
    assert err.max() <= bar


def test_checkpoint_spacing_does_not_change_the_gradient(gpu_lib):
    from paper_1504_06847_amd import Solver
    inst, p, kw = _grad64()
    s = Solver(inst.psf, inst.dirty, **kw)
    ref = s.grad(20, sky=inst.sky, ckpt_every=5)
    for C in (1, 3, 7, 20, 50):
        r = s.grad(20, sky=inst.sky, ckpt_every=C)
        assert r[0] == ref[0] and np.array_equal(r[1], ref[1]), C


def test_default_checkpoint_spacing_from_free_memory(gpu_lib):
    """The default spacing recomputes the fewest passes within the memory
    budget: K for a small cube, smaller for a small budget, and the gradient
    at the default equals the one at that spacing."""
    from paper_1504_06847_amd import Solver
    inst, p, kw = _grad64()
    s = Solver(inst.psf, inst.dirty, **kw)
    assert s.sweep_ckpt_every(20) == 20
    # the workspace of spacing 5 (4 x 4 + 10 x 5 + 6 cubes): every spacing
    # that recomputes fewer passes (7, 10, 20) needs more
    b5 = s.grad_workspace_bytes(20, 5)
    assert s.grad_workspace_bytes(20, 20) == s.grad_workspace_bytes(20, 50) > b5
    assert s.sweep_ckpt_every(20, budget=b5) == 5
    smallest = min(s.grad_workspace_bytes(20, C) for C in range(1, 21))
    assert s.sweep_ckpt_every(20, budget=smallest - 1) == 1      # nothing fits
    r0 = s.grad(20, sky=inst.sky)
    r1 = s.grad(20, sky=inst.sky, ckpt_every=20)
    assert r0[0] == r1[0] and np.array_equal(r0[1], r1[1])


def test_vjp_matches_oracle_jvp(gpu_lib):
    """<gx, J e_i> from the oracle's tangents equals the GPU's (J^T gx)_i."""
    from paper_1504_06847_amd import Solver
    inst, p, kw = _grad64()
    rng = np.random.default_rng(7)
    gx = rng.standard_normal(inst.sky.shape)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    loss, g = s.grad(12, gx=gx, ckpt_every=4)
    assert loss == 0.0
    prob = O.Problem(inst.psf, inst.dirty, p)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        _, dX = O.jvp_run(prob, 12, e)
        ref = float(np.sum(gx * dX))
        _say("vjp", i, g[i], ref)
        assert abs(g[i] - ref) <= 1e-8 * max(abs(ref), np.abs(g).max())


@pytest.mark.parametrize("L", [6, 15])
def test_vjp_at_band_counts_off_the_power_of_two_path(gpu_lib, L):
    """L = 6 and 15 take the dense band transform; K = 8 with checkpoints
    every 3 puts the step-I adjoint of a segment's first pass into the next
    segment's first launch.  <gx, J e_i> as in the test above."""
    from synth import make_instance
    from paper_1504_06847_amd import Solver
    inst = make_instance(32, 32, L, n_points=4, n_gauss=2, n_ant=16, noise_sigma=0.01, seed=40 + L)
    p = get_config("grad64").params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    gx = np.random.default_rng(11).standard_normal(inst.dirty.shape)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    _, g = s.grad(8, gx=gx, ckpt_every=3)
    _, g1 = s.grad(8, gx=gx, ckpt_every=8)
    assert np.array_equal(g, g1)
    prob = O.Problem(inst.psf, inst.dirty, p)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        _, dX = O.jvp_run(prob, 8, e)
        ref = float(np.sum(gx * dX))
        _say("vjp L", L, i, g[i], ref)
        assert abs(g[i] - ref) <= 1e-8 * max(abs(ref), np.abs(g).max())


@pytest.mark.parametrize("L,ny,nx", [(32, 16, 8), (64, 8, 16), (128, 8, 8)], ids=["L32", "L64", "L128"])
def test_vjp_at_the_register_band_widths(gpu_lib, L, ny, nx):
    """The register-resident adjoint at 32, 64 and 128 bands (FP64) on small
    images: <gx, J e_i> from the oracle's tangents, with checkpoints every
    4 of 6 passes (two segments, the second short: the step-I adjoint of
    pass 5 runs inside pass 4's launch, across the segment boundary) and
    bitwise the same with every pass stored."""
    from synth import make_instance
    from paper_1504_06847_amd import Solver
    inst = make_instance(ny, nx, L, n_points=3, n_gauss=1, n_ant=12, noise_sigma=0.01, seed=50 + L)
    p = get_config("grad64").params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    gx = np.random.default_rng(12).standard_normal(inst.dirty.shape)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    _, g = s.grad(6, gx=gx, ckpt_every=4)
    _, g1 = s.grad(6, gx=gx, ckpt_every=6)
    assert np.array_equal(g, g1)
    prob = O.Problem(inst.psf, inst.dirty, p)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        _, dX = O.jvp_run(prob, 6, e)
        ref = float(np.sum(gx * dX))
        _say("vjp L", L, i, g[i], ref)
        assert abs(g[i] - ref) <= 1e-8 * max(abs(ref), np.abs(g).max())


def test_per_parameter_gradient_matches_oracle_jvp(gpu_lib):
    """muffin_grad_params: (J^T gx) along each of mu_eps, mu_s, mu_nu and the
    four rho's equals <gx, J e_i> from the oracle's tangents; the four rho
    components sum to the tied-rho derivative of muffin_grad."""
    from paper_1504_06847_amd import Solver
    inst, p, kw = _grad64()
    rng = np.random.default_rng(8)
    gx = rng.standard_normal(inst.sky.shape)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    _, g = s.grad_params(10, gx=gx, ckpt_every=3)
    prob = O.Problem(inst.psf, inst.dirty, p)
    scale = max(abs(v) for v in g.values())
    for name in Solver.GRAD_PARAMS:
        dp = O.Params(**{f: (1.0 if f == name else 0.0) for f in Solver.GRAD_PARAMS})
        _, dX = O.jvp_run(prob, 10, dp)
        ref = float(np.sum(gx * dX))
        _say("per-parameter", name, g[name], ref)
        assert abs(g[name] - ref) <= 1e-8 * max(abs(ref), scale)
    s2 = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    _, g3 = s2.grad(10, gx=gx, ckpt_every=3)
    assert abs(g3[2] - (g["rho_P"] + g["rho_T"] + g["rho_V"] + g["rho_S"])) <= 1e-12 * scale
    assert g3[0] == g["mu_s"] and g3[1] == g["mu_nu"]


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-9), (torch.float32, 1e-4)], ids=["f64", "f32"])
def test_dirty_image_gradient_matches_oracle_jvp(gpu_lib, dtype, bar):
    """muffin_grad_dirty: <dL/dY, dY> equals <gx, dX> for the oracle's tangent
    along random changes dY of the dirty images (H applied to the summed
    B-bar in the Fourier domain, the packed kx = 0 and nx/2 columns
    included); the context ends in the state after K passes."""
    from paper_1504_06847_amd import Solver
    inst, p, kw = _grad64()
    rng = np.random.default_rng(9)
    gx = rng.standard_normal(inst.sky.shape)
    s = Solver(inst.psf, inst.dirty, dtype=dtype, **kw)
    loss, gy = s.grad_dirty(10, gx=gx, ckpt_every=4)
    assert loss == 0.0
    gy = gy.cpu().double().numpy()
    prob = O.Problem(inst.psf, inst.dirty, p)
    for trial in range(2):
        dY = rng.standard_normal(inst.sky.shape)
        _, dX = O.jvp_run(prob, 10, (0.0, 0.0, 0.0), dY=dY)
        lhs, rhs = float(np.sum(gy * dY)), float(np.sum(gx * dX))
        _say("dL/dY", dtype, lhs, rhs)
        assert abs(lhs - rhs) <= bar * max(abs(rhs), float(np.sqrt(np.sum(gy ** 2) * np.sum(dY ** 2))))
    ref = Solver(inst.psf, inst.dirty, dtype=dtype, **kw)
    ref.iterate(10)
    assert torch.equal(s.x, ref.x)


@pytest.mark.parametrize("ckpt_every", [4, 9, 20])
@pytest.mark.parametrize("report_first", [False, True], ids=["iterate", "report"])
def test_context_holds_the_K_pass_state_afterwards(gpu_lib, ckpt_every, report_first):
    """The last forward pass of the sweep writes the context's own state
    arrays, and recomputed segments (checkpoints every 4) never touch them;
    with one segment (every 9 or 20) nothing is recomputed.  A reporting
    pass before the sweep (which switches the context's state set) changes
    nothing."""
    from paper_1504_06847_amd import Solver
    inst, p, kw = _grad64()
    a = Solver(inst.psf, inst.dirty, **kw)
    b = Solver(inst.psf, inst.dirty, **kw)
    a.iterate(3)
    if report_first:
        a.step_report()
    a.grad(9, sky=inst.sky, ckpt_every=ckpt_every)
    b.iterate(9)
    torch.cuda.synchronize()
    assert a.iterations == 9
    assert torch.equal(a.x, b.x)
    a.iterate(2)
    b.iterate(2)
    torch.cuda.synchronize()
    assert torch.equal(a.x, b.x)


def test_fp32_gradient_against_central_differences(gpu_lib):
    """Central differences of the FP32 GPU loss (h = 1e-3, the loss summed in
    FP64) against the adjoint: agreement to 1e-2 (kinks of the prox maps
    limit it)."""
    from paper_1504_06847_amd import Solver
    inst, p, kw = _grad64()
    sky = torch.as_tensor(inst.sky, dtype=torch.float64)
    s = Solver(inst.psf, inst.dirty, **kw)
    _, g = s.grad(20, sky=inst.sky)
    base = dict(mu_s=kw["mu_s"], mu_nu=kw["mu_nu"], rho=kw["rho"])
    h = 1e-3
    for i, name in enumerate(("mu_s", "mu_nu", "rho")):
        vals = []
        for sgn in (1, -1):
            q = dict(base)
            q[name] = base[name] + sgn * h
            t = Solver(inst.psf, inst.dirty, mu_eps=kw["mu_eps"], **q)
            t.iterate(20)
            vals.append(float(((t.x.double().cpu() - sky) ** 2).sum()))
            t.close()
        fd = (vals[0] - vals[1]) / (2 * h)
        _say("fd", name, fd, "adjoint", g[i])
        assert abs(fd - g[i]) <= 1e-2 * max(abs(fd), np.abs(g).max())


def test_autograd_function(gpu_lib):
    from paper_1504_06847_amd import MuffinUnroll, Solver
    inst, p, kw = _grad64()
    dev = torch.device("cuda")
    psf = torch.as_tensor(inst.psf, dtype=torch.float64, device=dev)
    dirty = torch.as_tensor(inst.dirty, dtype=torch.float64, device=dev)
    sky = torch.as_tensor(inst.sky, dtype=torch.float64, device=dev)
    mu_s = torch.tensor(kw["mu_s"], dtype=torch.float64, requires_grad=True)
    mu_nu = torch.tensor(kw["mu_nu"], dtype=torch.float64, requires_grad=True)
    rho = torch.tensor(kw["rho"], dtype=torch.float64, requires_grad=True)
    mu_eps = torch.tensor(kw["mu_eps"], dtype=torch.float64, requires_grad=True)
    dirty.requires_grad_(True)
    x = MuffinUnroll.apply(psf, dirty, mu_s, mu_nu, rho, 15, 5, mu_eps)
    loss = ((x - sky) ** 2).sum()
    loss.backward()
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    l2, g = s.grad(15, sky=inst.sky)
    got = np.array([mu_s.grad.item(), mu_nu.grad.item(), rho.grad.item()])
    _say("autograd", got, g)
    assert abs(loss.item() - l2) <= 1e-12 * l2
    assert np.abs(got - g).max() <= 1e-10 * np.abs(g).max()
    # the same sweep as muffin_grad_params / muffin_grad_dirty at this spacing
    s2 = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    _, gp = s2.grad_params(15, sky=inst.sky, ckpt_every=5)
    assert mu_eps.grad.item() == gp["mu_eps"]
    _, gy = s2.grad_dirty(15, sky=inst.sky, ckpt_every=5)
    assert torch.equal(dirty.grad, gy)


def test_recorded_sweep_matches_one_call(gpu_lib):
    """muffin_grad_record + muffin_grad_replay: X^K after the record equals
    K iterated passes, and the replay gives what one muffin_grad_params and
    one muffin_grad_dirty call give, bit for bit, with each forward pass run
    once; a replay without a record, or after another pass, is refused."""
    from paper_1504_06847_amd import Solver
    from paper_1504_06847_amd.lib import MuffinError
    from synth import make_instance
    inst = make_instance(32, 32, 8, n_points=4, n_gauss=2, n_ant=16, noise_sigma=0.01, seed=77)
    p = get_config("grad64").params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    gx = np.random.default_rng(14).standard_normal(inst.dirty.shape)
    K, C = 9, 4
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    s.grad_record(K, ckpt_every=C, dirty=True)
    ref = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw)
    ref.iterate(K)
    assert torch.equal(s.x, ref.x)
    _, g, gy = s.grad_replay(gx=gx)
    _, gp = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw).grad_params(K, gx=gx, ckpt_every=C)
    _, gd = Solver(inst.psf, inst.dirty, dtype=torch.float64, **kw).grad_dirty(K, gx=gx, ckpt_every=C)
    assert g == gp
    assert torch.equal(gy, gd)
    assert torch.equal(s.x, ref.x)
    with pytest.raises(MuffinError):
        s.grad_replay(gx=gx)
    s.grad_record(K, ckpt_every=C)
    s.iterate(1)
    with pytest.raises(MuffinError) as ei:
        s.grad_replay(gx=gx)
    assert ei.value.code == -1


def test_full_size_gradient_fp32(gpu_lib):
    """The 1024 x 1024 x 64 FP32 cube, K = 20, checkpoints every 5 passes:
    the adjoint against central differences (h = 1e-3, FP64 loss sums)."""
    from paper_1504_06847_amd import Solver
    cfg = get_config("cube1024")
    inst = cfg.make()
    p = cfg.params
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    _say("full-size gradient")
    sky = torch.as_tensor(inst.sky, device="cuda").double()
    s = Solver(inst.psf, inst.dirty, **kw)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    loss, g = s.grad(20, sky=inst.sky, ckpt_every=5)
    e1.record()
    torch.cuda.synchronize()
    _say("full-size loss", loss, "grad", g, "ms", e0.elapsed_time(e1))
    assert np.all(np.isfinite(g))
    base = dict(mu_s=kw["mu_s"], mu_nu=kw["mu_nu"], rho=kw["rho"])
    h = 1e-3
    for i, name in enumerate(("mu_s", "mu_nu", "rho")):
        vals = []
        for sgn in (1, -1):
            q = dict(base)
            q[name] = base[name] + sgn * h
            s.set_params(mu_eps=kw["mu_eps"], **q)
            s.reset()
            s.iterate(20)
            vals.append(float(((s.x.double() - sky) ** 2).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        _say("full-size fd", name, fd, "adjoint", g[i])
        assert abs(fd - g[i]) <= 1e-2 * max(abs(fd), np.abs(g).max())
