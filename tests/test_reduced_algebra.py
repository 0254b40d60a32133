"""The GPU path stores a reduced state (z_P, z_T, S, Gamma_S, Gamma_V) instead
of Algorithm 1's nine arrays.  This pins that algebra against the explicit
oracle in FP64.

Reduced form (derived from steps II, III and VI with W_s = identity):
  P = max(0, z_P), Gamma_P = rho_P max(0, -z_P), z_P <- X - max(0, -z_P)
  T = soft(z_T, tau_T), Gamma_T = -rho_T clip(z_T, tau_T), z_T <- X + clip(z_T, tau_T)
  b = H^T Y + rho_T (2 soft(z_T) - z_T) + rho_P |z_P| + Gamma_S + rho_S S
and the spectral pass keeps one band vector per pixel live:
  a = DCT(S_old); V = soft(a - Gamma_V / rho_V); a = Gamma_V + rho_V V;
  a = IDCT(a); S = (a - Gamma_S + rho_S X) / (rho_V + rho_S);
  Gamma_S += rho_S (S - X); a -= rho_V S; Gamma_V = DCT(a).
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.cpu


def _reduced_run(prob, K):
    p = prob.p
    shape = prob.shape
    zP, zT, S, GS, GV = (np.zeros(shape) for _ in range(5))
    tT, tV = p.mu_s / p.rho_T, p.mu_nu / p.rho_V
    Xs = []
    for _ in range(K):
        B = (prob.HtY + p.rho_T * (2 * O.soft(zT, tT) - zT) + p.rho_P * np.abs(zP)
             + GS + p.rho_S * S)
        X = prob.solve_Q(B)
        a = O.dct_nu(S)
        V = O.soft(a - GV / p.rho_V, tV)
        a = GV + p.rho_V * V
        a = O.idct_nu(a)
        Sn = (a - GS + p.rho_S * X) / (p.rho_V + p.rho_S)
        GS = GS + p.rho_S * (Sn - X)
        a = a - p.rho_V * Sn
        GV = O.dct_nu(a)
        zP = X - np.maximum(0.0, -zP)
        zT = X + np.clip(zT, -tT, tT)
        S = Sn
        Xs.append(X)
    return Xs, dict(zP=zP, zT=zT, S=S, GS=GS, GV=GV)


@pytest.mark.parametrize("params", [
    O.Params(1e-3, 0.5, 1.0, 1.0, 5.0, 2.0, 1.0),
    O.Params(1e-3, 0.02, 0.02, 1.0, 1.0, 1.0, 1.0),
])
def test_reduced_state_equals_explicit(params):
    from synth import get_config
    inst = get_config("plain64").make()
    prob = O.Problem(inst.psf, inst.dirty, params)
    Xs, red = _reduced_run(prob, 50)
    st = O.State.zeros(prob.shape)
    worst = 0.0
    for k in range(50):
        st = O.admm_iteration(prob, st)
        worst = max(worst, np.linalg.norm(Xs[k] - st.X) / np.linalg.norm(st.X))
    assert worst < 1e-12
    scale = np.abs(st.X).max()
    np.testing.assert_allclose(np.maximum(0, red["zP"]), st.P, atol=1e-11 * scale)
    np.testing.assert_allclose(params.rho_P * np.maximum(0, -red["zP"]), st.GP, atol=1e-11 * scale)
    np.testing.assert_allclose(O.soft(red["zT"], params.mu_s / params.rho_T), st.T, atol=1e-11 * scale)
    np.testing.assert_allclose(red["S"], st.S, atol=1e-11 * scale)
    np.testing.assert_allclose(red["GS"], st.GS, atol=1e-11 * scale)
    np.testing.assert_allclose(red["GV"], st.GV, atol=1e-11 * scale)
