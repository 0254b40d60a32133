"""W_nu other than the DCT alone (Section 3, step V's closed form for a union
of m_nu orthonormal transforms; Section 4, the Chebyshev polynomials as an
alternative to the DCT) against the oracle through the C ABI: one Chebyshev
or identity basis (the reduced four-array state with a dense band
transform), and unions (state z_P, z_T, S, Gamma_S and a coefficient cube
per basis), per iterate (FP32 against float64 1e-5, FP64 against the
extended-precision oracle 1e-12), the reporting pass, the Boyd stop,
parameter changes, state round trips, graph replay, residual balancing and
the gradient with one Chebyshev basis."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth import make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PARAMS = dict(mu_eps=1e-3, mu_s=0.05, mu_nu=0.08, rho_P=1.0, rho_T=1.5, rho_V=1.2, rho_S=0.8)
CHEB, DIRAC_NU, DCT = O.CHEBYSHEV, O.SPECTRAL_DIRAC, O.DCT


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


def _inst(L, ny, nx, seed):
    return make_instance(ny, nx, L, n_points=6, n_gauss=2, n_ant=14, noise_sigma=0.01, seed=seed)


def _per_iterate(inst, spectral, dtype, K, params=PARAMS):
    from paper_1504_06847_amd import Solver
    s = Solver(inst.psf, inst.dirty, dtype=dtype, spectral=spectral, **params)
    prob = O.Problem(inst.psf, inst.dirty, O.Params(**params), spectral=spectral,
                     dtype=np.longdouble if dtype == torch.float64 else np.float64)
    st = prob.zero_state()
    errs = []
    for _ in range(K):
        s.iterate(1)
        st = O.admm_iteration(prob, st)
        errs.append(rel(s.x.cpu().double().numpy(), st.X.astype(np.float64)))
    return errs, s


CASES = [
    ((CHEB,), (8, 32, 32)), ((CHEB,), (15, 32, 16)), ((CHEB,), (64, 16, 16)), ((DIRAC_NU,), (8, 32, 32)),
    ((DCT, CHEB), (8, 32, 32)), ((DCT, DIRAC_NU), (16, 16, 32)), ((CHEB, DCT, DIRAC_NU), (32, 16, 16)),
    ((DCT, CHEB), (64, 8, 16)), ((DIRAC_NU, CHEB), (5, 8, 8)),
]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("spectral,shape", CASES, ids=lambda v: "-".join(map(str, v)))
def test_spectral_bases_match_oracle_per_iterate(gpu_lib, spectral, shape, dtype):
    L, ny, nx = shape
    _say("spectral", spectral, shape, dtype)
    errs, s = _per_iterate(_inst(L, ny, nx, seed=40 + L), spectral, dtype, 10)
    _say("  per-iterate rel err", ["%.2e" % e for e in errs])
    assert max(errs) < (1e-5 if dtype == torch.float32 else 1e-12), errs
    assert not s.fused_available


@pytest.mark.parametrize("spectral", [(CHEB,), (DCT, CHEB), (DCT, CHEB, DIRAC_NU)], ids=lambda v: "-".join(map(str, v)))
def test_spectral_bases_report_matches_oracle(gpu_lib, spectral):
    """Residuals, tolerances, E^k and the objective (its spectral term a sum
    over the bases) of one reporting pass, FP64."""
    from paper_1504_06847_amd import Solver
    inst = _inst(8, 32, 32, seed=5)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64, spectral=spectral, **PARAMS)
    prob = O.Problem(inst.psf, inst.dirty, O.Params(**PARAMS), spectral=spectral)
    s.iterate(4)
    prev = O.run(prob, 4)
    rep = s.step_report()
    cur = O.admm_iteration(prob, prev)
    res = O.residuals(prob, prev, cur, eps_abs=1e-5, eps_rel=1e-4)
    _say(spectral, rep, res)
    assert rep["iters"] == 5
    for k, o in (("r_pri", "r"), ("r_dual", "s"), ("eps_pri", "eps_pri"), ("eps_dual", "eps_dual")):
        assert rep[k] == pytest.approx(res[o], rel=1e-9), k
    assert rep["E"] == pytest.approx(O.energy(prob, prev, cur), rel=1e-9)
    assert rep["objective"] == pytest.approx(O.objective(prob, cur.P), rel=1e-9)
    # the report wrote the new state into the other set: the next pass goes on from it
    s.iterate(2)
    st = O.run(prob, 2, cur)
    assert rel(s.x.cpu().numpy(), st.X) < 1e-12


def test_union_state_graph_and_params(gpu_lib):
    """A union: graph replay and restored states repeat the launched run bit
    for bit; new rho's (rho_V included) continue Algorithm 1 with the
    multipliers held, as the oracle does with the same arrays."""
    from paper_1504_06847_amd import Solver
    spectral = (DCT, CHEB)
    inst = _inst(16, 32, 32, seed=6)
    a = Solver(inst.psf, inst.dirty, spectral=spectral, dtype=torch.float64, **PARAMS)
    b = Solver(inst.psf, inst.dirty, spectral=spectral, dtype=torch.float64, graph=True, **PARAMS)
    a.iterate(3)
    b.iterate(3)
    st = a.get_state().clone()
    a.iterate(4)
    b.iterate(4)
    torch.cuda.synchronize()
    assert torch.equal(a.x, b.x)
    c = Solver(inst.psf, inst.dirty, spectral=spectral, dtype=torch.float64, **PARAMS)
    c.set_state(st)
    c.iterate(4)
    torch.cuda.synchronize()
    assert torch.equal(c.x, a.x) and c.iterations == 7
    # rho's change after 7 passes, then 6 more
    new = dict(PARAMS, rho_P=1.7, rho_T=0.9, rho_V=2.1, rho_S=1.3)
    a.set_params(**new)
    a.iterate(6)
    prob = O.Problem(inst.psf, inst.dirty, O.Params(**PARAMS), spectral=spectral)
    ref = O.run(prob.with_params(O.Params(**new)), 6, O.run(prob, 7))
    e = rel(a.x.cpu().numpy(), ref.X)
    _say("after set_params", e)
    assert e < 1e-11


def test_union_solve_and_adaptive(gpu_lib):
    """The Boyd stop with a union, and residual balancing taking the
    oracle's decisions."""
    from paper_1504_06847_amd import Solver
    spectral = (DCT, CHEB)
    inst = _inst(8, 16, 16, seed=7)
    kw = dict(PARAMS, check_every=5, eps_abs=1e-6, eps_rel=1e-5)
    s = Solver(inst.psf, inst.dirty, spectral=spectral, dtype=torch.float64, **kw)
    rep = s.solve(4000)
    assert rep["status"] == 0 and rep["converged"] == 1
    p = O.Params(1e-3, 0.05, 0.08, 0.05, 0.05, 0.05, 0.05)
    kw2 = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=0.05, check_every=10, eps_abs=1e-6, eps_rel=1e-5)
    g = Solver(inst.psf, inst.dirty, spectral=spectral, dtype=torch.float64, **kw2)
    rep = g.solve(120, adaptive=(10.0, 2.0))
    prob = O.Problem(inst.psf, inst.dirty, p, spectral=spectral, dtype=np.longdouble)
    st, pr, hist = O.solve_adaptive(prob, 120, 10, 10.0, 2.0, eps_abs=1e-6, eps_rel=1e-5)
    _say("adaptive: gpu rho", g.params["rho_P"], rep["iters"], "oracle", pr.p.rho_P, hist[-1][0])
    assert g.params["rho_P"] == pr.p.rho_P and rep["iters"] == hist[-1][0]
    assert rel(g.x.cpu().numpy(), st.X.astype(np.float64)) < 1e-12


@pytest.mark.parametrize("basis,shape", [(CHEB, (8, 32, 32)), (DIRAC_NU, (16, 16, 16)), (CHEB, (12, 16, 16))],
                         ids=["cheb8", "dirac16", "cheb12"])
def test_gradient_with_one_other_basis_matches_oracle(gpu_lib, basis, shape):
    """The reverse sweep with a dense band transform against the oracle's
    forward-mode tangents (FP64)."""
    from paper_1504_06847_amd import Solver
    L, ny, nx = shape
    inst = _inst(L, ny, nx, seed=8)
    kw = dict(mu_eps=1e-3, mu_s=0.05, mu_nu=0.05, rho=1.0)
    s = Solver(inst.psf, inst.dirty, spectral=(basis,), dtype=torch.float64, **kw)
    K = 8
    loss, g = s.grad(K, sky=inst.sky, ckpt_every=3)
    prob = O.Problem(inst.psf, inst.dirty, O.Params(1e-3, 0.05, 0.05, 1.0, 1.0, 1.0, 1.0), spectral=(basis,))
    lo, go = O.mse_grad(prob, K, inst.sky)
    _say("grad", basis, shape, g, go)
    assert loss == pytest.approx(lo, rel=1e-10)
    assert np.abs(g - go).max() <= 1e-8 * np.abs(go).max()


def test_unsupported_combinations_are_refused(gpu_lib):
    from paper_1504_06847_amd import Batch, Solver
    from paper_1504_06847_amd import lib as L
    inst = _inst(8, 16, 16, seed=9)
    s = Solver(inst.psf, inst.dirty, spectral=(DCT, CHEB), **PARAMS)
    with pytest.raises(L.MuffinError, match="one spectral basis"):
        s.grad(3, sky=inst.sky, ckpt_every=3)
    with pytest.raises(L.MuffinError, match="spectral dictionary"):
        s.set_params(spectral=(DCT,))
    with pytest.raises(L.MuffinError):
        Batch([(inst.psf, inst.dirty)], params=dict(PARAMS, spectral=(CHEB,)))
