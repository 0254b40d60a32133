"""The visibility-domain model on the GPU (Section 2: the data are the
sampled visibilities; step I of Algorithm 1 by conjugate gradients on Q_l of
eq. Qlsimp) against the oracle's VisProblem, per iterate: the setup sums
(the Toeplitz kernel and Re(H^H y)) in FP64, n_cg CG iterations per band on
the zero-padded convolution, then the ordinary steps II-VI.  Also graph
replay, state round trips, parameter changes, a band without visibilities
and the calls the model does not have."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth.visibilities import make_vis_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PARAMS = dict(mu_eps=1e-3, mu_s=0.05, mu_nu=0.05, rho_P=1.0, rho_T=1.5, rho_V=1.2, rho_S=0.8)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


def _inst(L, ny, nx, seed, n_ant=10, n_time=12, noise=0.05):
    return make_vis_instance(ny, nx, L, n_points=4, n_gauss=2, n_ant=n_ant, noise_sigma=noise, seed=seed,
                             n_time=n_time)


def _per_iterate(inst, dtype, n_cg, K, params=PARAMS):
    from paper_1504_06847_amd import VisSolver
    s = VisSolver(inst.uv, inst.vis, inst.shape, n_cg=n_cg, dtype=dtype, **params)
    prob = O.VisProblem(inst.uv, inst.vis, inst.shape, O.Params(**params), n_cg=n_cg)
    st = prob.zero_state()
    errs = []
    for _ in range(K):
        s.iterate(1)
        st = O.admm_iteration(prob, st)
        errs.append(rel(s.x.cpu().double().numpy(), st.X))
    return errs, s, prob, st


CASES = [((4, 16, 16), 5), ((3, 32, 16), 12), ((2, 8, 32), 20), ((5, 16, 16), 1), ((8, 32, 32), 8)]


def _sensitivity(inst, n_cg, K, u, params=PARAMS):
    """How far the oracle's own iterates move when its CG inputs (the
    Toeplitz kernels and Re(H^H y)) are perturbed by relative u (the unit
    roundoff of the GPU's precision): the largest per-iterate relative
    difference over K passes.  A fixed number of CG iterations in finite
    precision amplifies rounding (loss of orthogonality) by a factor that
    grows with n_cg and the conditioning of Q_l, so this is the scale on
    which two correct implementations can differ."""
    p = O.VisProblem(inst.uv, inst.vis, inst.shape, O.Params(**params), n_cg=n_cg)
    q = O.VisProblem(inst.uv, inst.vis, inst.shape, O.Params(**params), n_cg=n_cg)
    rng = np.random.default_rng(7)
    q.kernels = [k * (1 + u * rng.standard_normal(k.shape)) for k in q.kernels]
    q.HtY = q.HtY * (1 + u * rng.standard_normal(q.HtY.shape))
    a, b, worst = p.zero_state(), q.zero_state(), 0.0
    for _ in range(K):
        a, b = O.admm_iteration(p, a), O.admm_iteration(q, b)
        worst = max(worst, rel(b.X, a.X))
    return worst


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape,n_cg", CASES, ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else str(v))
def test_vis_model_matches_oracle_per_iterate(gpu_lib, shape, n_cg, dtype):
    """Per iterate within 30 x the oracle's own spread under unit-roundoff
    perturbations of its CG inputs (at least 1e-11 in FP64, 1e-5 in FP32);
    with one CG iteration, where nothing is amplified, within 1e-12 (FP64)
    and 1e-5 (FP32) outright."""
    L, ny, nx = shape
    _say("visibility model", shape, "n_cg", n_cg, dtype)
    inst = _inst(L, ny, nx, seed=60 + L + ny)
    errs, s, _, _ = _per_iterate(inst, dtype, n_cg, 8)
    u = 2.0 ** -53 if dtype == torch.float64 else 2.0 ** -24
    sens = _sensitivity(inst, n_cg, 8, u)
    bar = max(1e-11 if dtype == torch.float64 else 1e-5, 30 * sens)
    _say("  per-iterate rel err", ["%.2e" % e for e in errs], "oracle spread %.2e" % sens, "bar %.2e" % bar)
    assert s.n_cg == n_cg and s.iterations == 8
    assert max(errs) < bar, errs
    if n_cg == 1:
        assert max(errs) < (1e-12 if dtype == torch.float64 else 1e-5)


def test_vis_graph_state_and_params(gpu_lib):
    """Graph replay and restored states repeat the launched passes bit for
    bit; new rho's continue Algorithm 1 as the oracle does."""
    from paper_1504_06847_amd import VisSolver
    inst = _inst(3, 16, 16, seed=70)
    kw = dict(n_cg=6, dtype=torch.float64, **PARAMS)
    a = VisSolver(inst.uv, inst.vis, inst.shape, **kw)
    b = VisSolver(inst.uv, inst.vis, inst.shape, graph=True, **kw)
    a.iterate(3)
    b.iterate(3)
    st = a.get_state().clone()
    a.iterate(4)
    b.iterate(4)
    torch.cuda.synchronize()
    assert torch.equal(a.x, b.x)
    # the state holds X too, where the CG of the next pass starts
    c = VisSolver(inst.uv, inst.vis, inst.shape, **kw)
    c.set_state(st)
    c.iterate(4)
    torch.cuda.synchronize()
    assert torch.equal(c.x, a.x) and c.iterations == 7
    new = dict(PARAMS, rho_P=1.7, rho_T=0.9, rho_V=2.1, rho_S=1.3)
    a.set_params(**new)
    a.iterate(5)
    prob = O.VisProblem(inst.uv, inst.vis, inst.shape, O.Params(**PARAMS), n_cg=6)
    ref = O.run(prob.with_params(O.Params(**new)), 5, O.run(prob, 7))
    e = rel(a.x.cpu().numpy(), ref.X)
    _say("after set_params", e)
    assert e < 1e-10


def test_vis_band_without_visibilities_and_refusals(gpu_lib):
    from paper_1504_06847_amd import VisSolver
    from paper_1504_06847_amd import lib as L
    inst = _inst(3, 16, 16, seed=71)
    uv = [inst.uv[0], np.zeros((0, 2)), inst.uv[2]]
    vis = [inst.vis[0], np.zeros(0, np.complex128), inst.vis[2]]
    s = VisSolver(uv, vis, inst.shape, n_cg=4, dtype=torch.float64, **PARAMS)
    prob = O.VisProblem(uv, vis, inst.shape, O.Params(**PARAMS), n_cg=4)
    s.iterate(5)
    st = O.run(prob, 5)
    e = rel(s.x.cpu().numpy(), st.X)
    _say("band without visibilities", e)
    assert e < 1e-10
    for call in (lambda: s.step_report(), lambda: s.autotune(reps=1), lambda: s.grad(2, sky=inst.sky)):
        with pytest.raises(L.MuffinError, match="visibility"):
            call()
    with pytest.raises(L.MuffinError):
        VisSolver(inst.uv, inst.vis, inst.shape, n_cg=0, **PARAMS)
