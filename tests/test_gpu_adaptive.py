"""Residual balancing (Boyd et al. 2011, Sec. 3.4.1) through the C ABI
(muffin_solve_adaptive) against the oracle's solve_adaptive: the same rho
decisions at the same checks, the same stopping iteration and the same X.
Bars: FP64 1e-12 relative L2 on X; FP32 1e-4 on the final cube."""
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


@pytest.mark.parametrize("dtype,rho,bar", [("f64", 0.02, 1e-12), ("f64", 50.0, 1e-12), ("f32", 0.02, 1e-4)])
def test_adaptive_solve_matches_oracle(gpu_lib, dtype, rho, bar):
    from paper_1504_06847_amd import Solver
    cfg = get_config("plain64")
    inst = cfg.make()
    p = O.Params(1e-3, 0.02, 0.02, rho, rho, rho, rho)
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=rho, check_every=10,
              eps_abs=1e-6, eps_rel=1e-5)
    s = Solver(inst.psf, inst.dirty, dtype=torch.float64 if dtype == "f64" else torch.float32, **kw)
    rep = s.solve(120, adaptive=(10.0, 2.0))
    # FP64 against the oracle in extended precision, FP32 against float64
    prob = O.Problem(inst.psf, inst.dirty, p, dtype=np.longdouble if dtype == "f64" else np.float64)
    st, pr, hist = O.solve_adaptive(prob, 120, 10, 10.0, 2.0, eps_abs=1e-6, eps_rel=1e-5)
    _say(dtype, rho, "gpu rho", s.params["rho_P"], "iters", rep["iters"], "oracle rho", pr.p.rho_P,
         "iters", hist[-1][0], "history", [(k, r) for k, r, _, _ in hist])
    assert s.params["rho_P"] == pr.p.rho_P and s.params["rho_S"] == pr.p.rho_S
    assert pr.p.rho_P != rho                       # the rule fired
    assert rep["iters"] == hist[-1][0]
    x = s.x.cpu().double().numpy()
    xr = st.X.astype(np.float64)
    err = float(np.linalg.norm(x - xr) / np.linalg.norm(xr))
    _say("  X rel err", err)
    assert err <= bar
