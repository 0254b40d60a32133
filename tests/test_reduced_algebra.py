"""The GPU path stores a reduced state (z_P, z_T, z_V, Gamma_S) instead of
Algorithm 1's nine arrays.  This pins that algebra against the explicit oracle
in FP64.

Reduced form (from steps II, III and VI with W_s = identity):
  P = max(0, z_P), Gamma_P = rho_P max(0, -z_P), z_P <- X - max(0, -z_P)
  T = soft(z_T, tau_T), Gamma_T = -rho_T clip(z_T, tau_T), z_T <- X + clip(z_T, tau_T)
  b = H^T Y + rho_T (2 soft(z_T) - z_T) + rho_P |z_P| + Gamma_S + rho_S S
Spectral pair: step V minimises the augmented Lagrangian in S exactly, so its
optimality condition Gamma_S^+ = Gamma_V^+ W_nu^T holds after every pass;
with Gamma_V = Gamma_S W_nu,
  V = soft(DCT(S - Gamma_S / rho_V), mu_nu / rho_V),  q = IDCT(V),
  S^+ = (rho_V q + rho_S X) / (rho_V + rho_S),  Gamma_S^+ = Gamma_S + rho_V (q - S^+).
The state holds z_V = S - Gamma_S / rho_V (the DCT input of step IV) in place
of S, and S = z_V + Gamma_S / rho_V where S enters b.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.cpu


def _reduced_run(prob, K):
    p = prob.p
    shape = prob.shape
    zP, zT, zV, GS = (np.zeros(shape) for _ in range(4))
    tT, tV = p.mu_s / p.rho_T, p.mu_nu / p.rho_V
    Xs = []
    for _ in range(K):
        B = (prob.HtY + p.rho_T * (2 * O.soft(zT, tT) - zT) + p.rho_P * np.abs(zP)
             + GS + p.rho_S * (zV + GS / p.rho_V))
        X = prob.solve_Q(B)
        q = O.idct_nu(O.soft(O.dct_nu(zV), tV))
        Sn = (p.rho_V * q + p.rho_S * X) / (p.rho_V + p.rho_S)
        GS = GS + p.rho_V * (q - Sn)
        zV = Sn - GS / p.rho_V
        zP = X - np.maximum(0.0, -zP)
        zT = X + np.clip(zT, -tT, tT)
        Xs.append(X)
    return Xs, dict(zP=zP, zT=zT, S=zV + GS / p.rho_V, GS=GS)


def test_gamma_S_equals_gamma_V_transformed_after_every_pass():
    """Optimality of step V: Gamma_S^k = Gamma_V^k W_nu^T for every k (explicit oracle)."""
    from synth import get_config
    inst = get_config("plain64").make()
    prob = O.Problem(inst.psf, inst.dirty, O.Params(1e-3, 0.5, 1.0, 1.0, 5.0, 2.0, 1.0))
    worst = []
    O.run(prob, 60, callback=lambda k, a, b: worst.append(
        np.abs(b.GS - O.idct_nu(b.GV)).max() / max(np.abs(b.GS).max(), 1e-300)))
    assert max(worst) < 1e-12


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
    np.testing.assert_allclose(O.dct_nu(red["GS"]), st.GV, atol=1e-11 * scale)
