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


def test_dictionary_rejects_reports_gradient_and_new_bases(gpu_lib):
    from paper_1504_06847_amd import Solver
    from paper_1504_06847_amd.lib import MuffinError
    inst = make_instance(16, 16, 2, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.01, seed=2)
    s = Solver(inst.psf, inst.dirty, spatial=PAPER)
    s.iterate(2)
    for call in (lambda: s.step_report(), lambda: s.solve(5), lambda: s.grad(2, sky=inst.dirty)):
        with pytest.raises(MuffinError) as ei:
            call()
        assert ei.value.code == -2
    with pytest.raises(MuffinError):
        s.set_params(spatial=(0, 1))
    s.iterate(1)           # the context still works
