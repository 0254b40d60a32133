"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each step of Algorithm 1 (Section 3, steps I-VI) is the exact minimiser of the
augmented Lagrangian of eqs. (admm1)-(admm2) over one block of variables.  The
tests below check that property for the oracle's steps with dense matrices
built from the definitions and with brute-force scalar minimisation, then pin
the whole iteration by closed-form fixed points, a library NNLS solve, a KKT
certificate and the He-Yuan monotonicity of E^k.
"""
import numpy as np
import pytest
import scipy.optimize

import oracle as O
from tests.independent import (brute_min, dct_matrix, dense_conv_matrix, spec,
                               spec_t)

pytestmark = pytest.mark.cpu


def _psf(rng, L, n, symmetric=False):
    psf = rng.uniform(0.0, 0.3, size=(L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    if symmetric:
        psf = 0.5 * (psf + np.roll(np.flip(psf, axis=(1, 2)), (1, 1), axis=(1, 2)))
    return psf


def _random_state(rng, shape, scale=1.0):
    return O.State(*(scale * rng.standard_normal(shape) for _ in range(9)))


@pytest.fixture(scope="module")
def tiny():
    rng = np.random.default_rng(11)
    L, n = 4, 8
    psf = _psf(rng, L, n)
    Y = rng.standard_normal((L, n, n)) + 1.0
    p = O.Params(mu_eps=1e-3, mu_s=0.5, mu_nu=1.0, rho_P=1.0, rho_T=5.0,
                 rho_V=2.0, rho_S=1.0)
    prob = O.Problem(psf, Y, p)
    Hd = [dense_conv_matrix(psf[l]) for l in range(L)]
    return prob, Hd, rng


def _apply_dense(Hd, x):
    L, ny, nx = x.shape
    return np.stack([(Hd[l] @ x[l].ravel()).reshape(ny, nx) for l in range(L)])


def _apply_dense_T(Hd, x):
    L, ny, nx = x.shape
    return np.stack([(Hd[l].T @ x[l].ravel()).reshape(ny, nx) for l in range(L)])


# ---------------------------------------------------------------- P1: H, H^T
def test_H_is_circular_convolution_with_centred_psf(tiny):
    prob, Hd, rng = tiny
    x = rng.standard_normal(prob.shape)
    np.testing.assert_allclose(prob.H(x), _apply_dense(Hd, x), rtol=0, atol=1e-13)


def test_HT_is_transpose_of_H(tiny):
    prob, Hd, rng = tiny
    y = rng.standard_normal(prob.shape)
    np.testing.assert_allclose(prob.HT(y), _apply_dense_T(Hd, y), rtol=0, atol=1e-13)


def test_point_source_maps_to_psf_at_its_position(tiny):
    prob, _, _ = tiny
    L, ny, nx = prob.shape
    x = np.zeros(prob.shape)
    x[:, 2, 5] = 1.0
    out = prob.H(x)
    for l in range(L):
        np.testing.assert_allclose(out[l], np.roll(prob.psf[l], (2 - ny // 2, 5 - nx // 2),
                                                    axis=(0, 1)), atol=1e-14)


# ------------------------------------------------ Step I (eqs. linsystemX..Qlsimp)
def test_step_I_zeroes_lagrangian_gradient_in_X(tiny):
    """grad_X of the augmented Lagrangian vanishes at the new X (dense H)."""
    prob, Hd, rng = tiny
    p = prob.p
    st = _random_state(rng, prob.shape)
    X = O.admm_iteration(prob, st).X
    g = (_apply_dense_T(Hd, _apply_dense(Hd, X) - prob.Y) + p.mu_eps * X
         - st.GP - p.rho_P * (st.P - X)
         - st.GT - p.rho_T * (st.T - X)
         - st.GS - p.rho_S * (st.S - X))
    assert np.abs(g).max() < 1e-11 * max(1.0, np.abs(X).max())


def test_fourier_solve_equals_dense_solve(tiny):
    """The Fourier-diagonal inverse equals a dense solve of H^T H + rho I."""
    prob, Hd, rng = tiny
    b = rng.standard_normal(prob.shape)
    rho = 0.37
    q = prob.with_params(O.Params(rho - 3.0, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0))
    L, ny, nx = prob.shape
    for l in range(L):
        Q = Hd[l].T @ Hd[l] + rho * np.eye(ny * nx)
        ref = np.linalg.solve(Q, b[l].ravel()).reshape(ny, nx)
        np.testing.assert_allclose(q.solve_Q(b)[l], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_fourier_solve_nonsymmetric_psf():
    """A PSF with a complex transfer function: conj(h_hat) must be used."""
    rng = np.random.default_rng(3)
    psf = _psf(rng, 2, 8)
    psf[:, 4, 5] = 0.9
    prob = O.Problem(psf, rng.standard_normal((2, 8, 8)),
                     O.Params(1e-3, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0))
    assert np.abs(prob.hhat.imag).max() > 0.1
    Hd = [dense_conv_matrix(psf[l]) for l in range(2)]
    b = rng.standard_normal((2, 8, 8))
    for l in range(2):
        Q = Hd[l].T @ Hd[l] + (1e-3 + 3.0) * np.eye(64)
        ref = np.linalg.solve(Q, b[l].ravel()).reshape(8, 8)
        np.testing.assert_allclose(prob.solve_Q(b)[l], ref, atol=1e-12)


def _ill_conditioned(dtype):
    """An 8 x 8 problem whose filter gain spans about 1e5 (a PSF with a large
    DC response, a small rho)."""
    rng = np.random.default_rng(21)
    psf = rng.uniform(0.5, 1.0, size=(2, 8, 8))
    psf[:, 4, 4] = 1.0
    Y = rng.standard_normal((2, 8, 8))
    prob = O.Problem(psf, Y, O.Params(1e-3, 0.1, 0.1, 0.01, 0.01, 0.01, 0.01), dtype=dtype)
    return prob, psf, rng


@pytest.mark.parametrize("dtype,bar", [(np.float64, 1e-15), (np.longdouble, 1e-18)],
                         ids=["float64", "extended"])
def test_fourier_solve_residual_at_working_precision(dtype, bar):
    """Step I in float64 and in extended precision: the residual of
    (H^T H + rho I) x = b against the dense matrices (built from the PSF and
    multiplied in extended precision) is at the working precision's rounding
    level, relative to ||Q|| ||x||, on a system with condition number ~1e5."""
    prob, psf, rng = _ill_conditioned(dtype)
    ld = np.longdouble
    b = rng.standard_normal(prob.shape)
    x = prob.solve_Q(b.astype(dtype))
    assert x.dtype == dtype
    gain = float((np.abs(prob.hhat) ** 2).max() / prob.rho_Q)
    assert gain > 1e4
    for l in range(2):
        H = dense_conv_matrix(psf[l], dtype=ld)
        Q = H.T @ H + ld(prob.rho_Q) * np.eye(64, dtype=ld)
        xv = x[l].ravel().astype(ld)
        r = Q @ xv - b[l].ravel().astype(ld)
        qn = float(np.abs(Q).sum(axis=1).max())            # ||Q||_inf
        res = float(np.abs(r).max()) / (qn * float(np.abs(xv).max()))
        assert res < bar, (l, res)


def test_extended_precision_oracle_agrees_with_float64(tiny):
    """The same iteration in the two precisions: 20 passes on a well
    conditioned cube agree to float64 rounding."""
    prob, Hd, rng = tiny
    a = O.run(prob, 20)
    b = O.run(O.Problem(prob.psf, prob.Y, prob.p, dtype=np.longdouble), 20)
    assert b.X.dtype == np.longdouble and b.GV.dtype == np.longdouble
    d = float(np.linalg.norm((a.X - b.X).astype(np.float64)) / np.linalg.norm(b.X.astype(np.float64)))
    assert d < 1e-13, d


# ------------------------------------------------ Steps II-IV: proximity operators
def test_steps_II_III_IV_are_block_minimisers(tiny):
    """Comparison-based minimisation resolves an argmin to about sqrt(eps) of
    the function scale, hence the 1e-7 tolerance."""
    prob, _, rng = tiny
    p = prob.p
    st = _random_state(rng, prob.shape)
    new = O.admm_iteration(prob, st)
    X = new.X
    W = dct_matrix(prob.shape[0])
    big = 1e30
    # Step II: min_P 1_{R+}(P) + <Gamma_P, P - X> + rho_P/2 (P - X)^2
    fP = lambda t: (np.where(t < 0, big, 0.0) + st.GP[..., None] * (t - X[..., None])
                    + 0.5 * p.rho_P * (t - X[..., None]) ** 2)
    P_ref = brute_min(fP, X, 3.0 + np.abs(st.GP) / p.rho_P)
    np.testing.assert_allclose(new.P, P_ref, rtol=0, atol=1e-7)
    # Step III: min_T mu_s |T| + <Gamma_T, T - X> + rho_T/2 (T - X)^2
    fT = lambda t: (p.mu_s * np.abs(t) + st.GT[..., None] * (t - X[..., None])
                    + 0.5 * p.rho_T * (t - X[..., None]) ** 2)
    T_ref = brute_min(fT, X, 3.0 + np.abs(st.GT) / p.rho_T)
    np.testing.assert_allclose(new.T, T_ref, rtol=0, atol=1e-7)
    # Step IV: min_V mu_nu |V| + <Gamma_V, V - S W> + rho_V/2 (V - S W)^2, old S
    SW = spec(st.S, W)
    fV = lambda t: (p.mu_nu * np.abs(t) + st.GV[..., None] * (t - SW[..., None])
                    + 0.5 * p.rho_V * (t - SW[..., None]) ** 2)
    V_ref = brute_min(fV, SW, 3.0 + np.abs(st.GV) / p.rho_V)
    np.testing.assert_allclose(new.V, V_ref, rtol=0, atol=1e-7)


def test_soft_threshold_edge_values():
    z = np.array([-2.0, -0.5, 0.0, 0.5, 2.0, 1.0, -1.0])
    np.testing.assert_array_equal(O.soft(z, 1.0), [-1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0])


# ------------------------------------------------ Step V (S update)
def test_step_V_zeroes_lagrangian_gradient_in_S(tiny):
    """grad_S of <Gamma_V, V - S W> + rho_V/2 ||V - S W||^2 + <Gamma_S, S - X>
    + rho_S/2 ||S - X||^2 vanishes at the new S (dense W from its definition)."""
    prob, _, rng = tiny
    p = prob.p
    st = _random_state(rng, prob.shape)
    new = O.admm_iteration(prob, st)
    W = dct_matrix(prob.shape[0])
    g = (-spec_t(st.GV, W) - p.rho_V * spec_t(new.V - spec(new.S, W), W)
         + st.GS + p.rho_S * (new.S - new.X))
    assert np.abs(g).max() < 1e-12 * max(1.0, np.abs(new.S).max())


def test_step_V_dense_solve(tiny):
    """S R = C with R = rho_V W W^T + rho_S I solved densely (step V)."""
    prob, _, rng = tiny
    p = prob.p
    st = _random_state(rng, prob.shape)
    new = O.admm_iteration(prob, st)
    L = prob.shape[0]
    W = dct_matrix(L)
    R = p.rho_V * W @ W.T + p.rho_S * np.eye(L)
    C = spec_t(st.GV + p.rho_V * new.V, W) - st.GS + p.rho_S * new.X
    Cm = C.reshape(L, -1).T                      # pixels x bands
    Sm = np.linalg.solve(R.T, Cm.T).T            # S R = C
    np.testing.assert_allclose(new.S, Sm.T.reshape(prob.shape), atol=1e-13)


# ------------------------------------------------ Step VI (multipliers)
def test_multiplier_updates_follow_constraint_residuals(tiny):
    prob, _, rng = tiny
    p = prob.p
    st = _random_state(rng, prob.shape)
    new = O.admm_iteration(prob, st)
    W = dct_matrix(prob.shape[0])
    np.testing.assert_allclose((new.GP - st.GP) / p.rho_P, new.P - new.X, atol=1e-12)
    np.testing.assert_allclose((new.GT - st.GT) / p.rho_T, new.T - new.X, atol=1e-12)
    np.testing.assert_allclose((new.GV - st.GV) / p.rho_V, new.V - spec(new.S, W), atol=1e-12)
    np.testing.assert_allclose((new.GS - st.GS) / p.rho_S, new.S - new.X, atol=1e-12)


# ------------------------------------------------ P5: W_nu
@pytest.mark.parametrize("L", [1, 2, 3, 8, 15, 64])
def test_dct_is_the_orthonormal_cosine_transform(L):
    W = dct_matrix(L)
    np.testing.assert_allclose(W.T @ W, np.eye(L), atol=1e-13)
    np.testing.assert_allclose(W @ W.T, np.eye(L), atol=1e-13)
    rng = np.random.default_rng(L)
    A = rng.standard_normal((L, 3, 2))
    np.testing.assert_allclose(O.dct_nu(A), spec(A, W), atol=1e-13)
    np.testing.assert_allclose(O.idct_nu(A), spec_t(A, W), atol=1e-13)


# ------------------------------------------------ whole iteration
def _small_instance():
    from synth import make_instance
    inst = make_instance(16, 16, 4, n_points=3, n_gauss=1, n_ant=10,
                         noise_sigma=0.01, seed=21, sigma_range=(1.0, 2.0))
    return inst


def test_energy_is_non_increasing():
    """He & Yuan (2015): ||w^k - w^{k+1}||_H is non-increasing for ADMM."""
    from synth import get_config
    cfg = get_config("plain64")
    inst = cfg.make()
    prob = O.Problem(inst.psf, inst.dirty, cfg.params)
    E = []
    O.run(prob, 60, callback=lambda k, a, b: E.append(O.energy(prob, a, b)))
    E = np.array(E)
    assert np.all(E[1:] <= E[:-1] * (1 + 1e-12)), np.diff(E).max()
    assert E[-1] < 1e-2 * E[0]


def test_multiplier_invariants_every_iterate():
    """Gamma_P >= 0, Gamma_P * P = 0, |Gamma_T| <= mu_s after every pass
    (sub-gradient conditions of steps II and III)."""
    inst = _small_instance()
    p = O.Params(1e-3, 0.5, 1.0, 1.0, 5.0, 2.0, 1.0)
    prob = O.Problem(inst.psf, inst.dirty, p)
    bad = []

    def cb(k, a, b):
        sc = 1e-12 * max(1.0, np.abs(b.X).max())
        if (b.GP.min() < -sc or np.abs(b.GP * b.P).max() > sc
                or np.abs(b.GT).max() > p.mu_s + 1e-12):
            bad.append(k)
    O.run(prob, 80, callback=cb)
    assert not bad


def _converge(prob, K):
    return O.run(prob, K)


def test_fixed_point_identity_psf_spatial_only():
    """H = I, mu_nu = 0: X* = max(0, Y - mu_s) / (1 + mu_eps)."""
    rng = np.random.default_rng(5)
    L, n = 4, 16
    psf = np.zeros((L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = rng.uniform(-0.5, 2.0, (L, n, n))
    p = O.Params(1e-3, 0.5, 0.0, 1.0, 5.0, 2.0, 1.0)
    st = _converge(O.Problem(psf, Y, p), 600)
    np.testing.assert_allclose(st.X, np.maximum(0.0, Y - p.mu_s) / (1 + p.mu_eps), atol=1e-11)


def test_fixed_point_identity_psf_spectral_only():
    """H = I, mu_s = 0, positive solution: X* = IDCT(soft(DCT(Y), mu_nu)) / (1 + mu_eps)."""
    rng = np.random.default_rng(6)
    L, n = 8, 8
    psf = np.zeros((L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = 5.0 + rng.uniform(-0.5, 0.5, (L, n, n))
    p = O.Params(1e-3, 0.0, 0.3, 1.0, 1.0, 1.0, 1.0)
    W = dct_matrix(L)
    c = spec(Y, W)
    ref = spec_t(np.sign(c) * np.maximum(np.abs(c) - p.mu_nu, 0.0), W) / (1 + p.mu_eps)
    assert ref.min() > 0
    st = _converge(O.Problem(psf, Y, p), 800)
    np.testing.assert_allclose(st.X, ref, atol=1e-10)


def test_fixed_point_spatial_l1_is_a_linear_shift():
    """On R+, mu_s ||X||_1 = mu_s sum X: the solution with mu_s equals the one
    with mu_s = 0 and Y shifted by -mu_s / h_hat(0) (so H^T Y drops by mu_s)."""
    inst = _small_instance()
    pA = O.Params(1e-3, 0.2, 0.1, 1.0, 1.0, 1.0, 1.0)
    probA = O.Problem(inst.psf, inst.dirty, pA)
    h0 = probA.hhat[:, 0, 0].real[:, None, None]
    probB = O.Problem(inst.psf, inst.dirty.astype(np.float64) - pA.mu_s / h0,
                      pA.__class__(**{**pA.__dict__, "mu_s": 0.0}))
    a = _converge(probA, 3000).X
    b = _converge(probB, 3000).X
    np.testing.assert_allclose(a, b, atol=1e-8 * np.abs(a).max())


def test_fixed_point_bands_decouple_into_nnls():
    """mu_s = mu_nu = 0: each band is min ||y - Hx||^2/2 + mu_eps||x||^2/2, x >= 0."""
    rng = np.random.default_rng(8)
    L, n = 3, 8
    psf = _psf(rng, L, n)
    Y = rng.standard_normal((L, n, n))
    p = O.Params(0.05, 0.0, 0.0, 1.0, 1.0, 1.0, 1.0)
    st = _converge(O.Problem(psf, Y, p), 4000)
    for l in range(L):
        Hd = dense_conv_matrix(psf[l])
        A = np.vstack([Hd, np.sqrt(p.mu_eps) * np.eye(n * n)])
        b = np.concatenate([Y[l].ravel(), np.zeros(n * n)])
        x, _ = scipy.optimize.nnls(A, b, maxiter=5000)
        np.testing.assert_allclose(st.P[l].ravel(), x, atol=1e-8)


def test_kkt_certificate_at_convergence(tiny):
    """Stationarity H^T(HX - Y) + mu_eps X - Gamma_P - Gamma_T - Gamma_V W^T = 0
    with Gamma_P >= 0 = Gamma_P * P, Gamma_T = -mu_s sign(T) on T != 0,
    Gamma_V = -mu_nu sign(V) on V != 0 (dense H and W)."""
    prob, Hd, _ = tiny
    p = O.Params(1e-2, 0.05, 0.2, 1.0, 1.0, 1.0, 1.0)
    prob = prob.with_params(p)
    st = _converge(prob, 6000)
    W = dct_matrix(prob.shape[0])
    g = (_apply_dense_T(Hd, _apply_dense(Hd, st.X) - prob.Y) + p.mu_eps * st.X
         - st.GP - st.GT - spec_t(st.GV, W))
    assert np.abs(g).max() < 1e-8
    assert st.GP.min() > -1e-9 and np.abs(st.GP * st.P).max() < 1e-9
    nzT = np.abs(st.T) > 1e-6
    np.testing.assert_allclose(st.GT[nzT], -p.mu_s * np.sign(st.T[nzT]), atol=1e-8)
    assert np.abs(st.GT).max() <= p.mu_s + 1e-9
    nzV = np.abs(st.V) > 1e-6
    np.testing.assert_allclose(st.GV[nzV], -p.mu_nu * np.sign(st.V[nzV]), atol=1e-8)
    assert np.abs(st.GV).max() <= p.mu_nu + 1e-8
    np.testing.assert_allclose(st.X, st.P, atol=1e-9)


# ------------------------------------------------ residuals, E^k and F with dense operators
def test_residuals_energy_objective_against_dense_operators(tiny):
    prob, Hd, rng = tiny
    p = prob.p
    prev = O.run(prob, 3)
    cur = O.admm_iteration(prob, prev)
    L, ny, nx = prob.shape
    n = L * ny * nx
    W = dct_matrix(L)
    Wbig = np.kron(W.T, np.eye(ny * nx))       # vec(C) for C = S W along bands
    I = np.eye(n)
    Z = np.zeros((n, n))
    # constraints stacked: [P - X; T - X; V - S W; S - X] = A x + B z, x = (X, V), z = (P, T, S)
    A = np.block([[-I, Z], [-I, Z], [Z, I], [-I, Z]])
    B = np.block([[I, Z, Z], [Z, I, Z], [Z, Z, -Wbig], [Z, Z, I]])
    rho = np.concatenate([np.full(n, p.rho_P), np.full(n, p.rho_T),
                          np.full(n, p.rho_V), np.full(n, p.rho_S)])
    v = lambda a: a.ravel()
    x = np.concatenate([v(cur.X), v(cur.V)])
    z = np.concatenate([v(cur.P), v(cur.T), v(cur.S)])
    dz = z - np.concatenate([v(prev.P), v(prev.T), v(prev.S)])
    y = np.concatenate([v(cur.GP), v(cur.GT), v(cur.GV), v(cur.GS)])
    dy = y - np.concatenate([v(prev.GP), v(prev.GT), v(prev.GV), v(prev.GS)])
    r = A @ x + B @ z
    s = A.T @ (rho * (B @ dz))
    res = O.residuals(prob, prev, cur, eps_abs=1e-5, eps_rel=1e-4)
    assert res["r"] == pytest.approx(np.linalg.norm(r), rel=1e-12)
    assert res["s"] == pytest.approx(np.linalg.norm(s), rel=1e-12)
    eps_pri = np.sqrt(4 * n) * 1e-5 + 1e-4 * max(np.linalg.norm(A @ x), np.linalg.norm(B @ z))
    eps_dual = np.sqrt(2 * n) * 1e-5 + 1e-4 * np.linalg.norm(A.T @ y)
    assert res["eps_pri"] == pytest.approx(eps_pri, rel=1e-12)
    assert res["eps_dual"] == pytest.approx(eps_dual, rel=1e-12)
    E = np.sum(rho * (B @ dz) ** 2) + np.sum(dy ** 2 / rho)
    assert O.energy(prob, prev, cur) == pytest.approx(E, rel=1e-12)
    P = cur.P
    F = (0.5 * np.sum((prob.Y - _apply_dense(Hd, P)) ** 2) + 0.5 * p.mu_eps * np.sum(P ** 2)
         + p.mu_s * np.sum(np.abs(P)) + p.mu_nu * np.sum(np.abs(spec(P, W))))
    assert O.objective(prob, P) == pytest.approx(F, rel=1e-12)


def test_residuals_vanish_at_convergence():
    inst = _small_instance()
    prob = O.Problem(inst.psf, inst.dirty, O.Params(1e-3, 0.05, 0.05, 1.0, 1.0, 1.0, 1.0))
    prev = O.run(prob, 2000)
    res = O.residuals(prob, prev, O.admm_iteration(prob, prev))
    assert res["r"] < 1e-3 * res["eps_pri"] and res["s"] < 1e-3 * res["eps_dual"]


# ------------------------------------------------ P14: forward-mode gradient
def test_jvp_gradient_matches_central_differences():
    inst = _small_instance()
    base = O.Params(1e-3, 0.05, 0.05, 1.0, 1.0, 1.0, 1.0)
    prob = O.Problem(inst.psf, inst.dirty, base)
    K = 12
    loss, g = O.mse_grad(prob, K, inst.sky)
    h = 1e-6

    def L_at(ms, mn, r):
        q = prob.with_params(O.Params(base.mu_eps, ms, mn, r, r, r, r))
        return O.mse_loss(O.run(q, K).X, inst.sky)
    fd = np.array([
        (L_at(base.mu_s + h, base.mu_nu, 1.0) - L_at(base.mu_s - h, base.mu_nu, 1.0)) / (2 * h),
        (L_at(base.mu_s, base.mu_nu + h, 1.0) - L_at(base.mu_s, base.mu_nu - h, 1.0)) / (2 * h),
        (L_at(base.mu_s, base.mu_nu, 1.0 + h) - L_at(base.mu_s, base.mu_nu, 1.0 - h)) / (2 * h),
    ])
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
    assert loss == pytest.approx(L_at(base.mu_s, base.mu_nu, 1.0), rel=1e-14)


def test_dirty_image_tangent_against_central_differences():
    """The oracle's tangent along a change dY of the dirty images equals
    central differences of K passes in Y (smooth away from the prox kinks)."""
    rng = np.random.default_rng(12)
    L, n = 3, 8
    psf = _psf(rng, L, n)
    Y = rng.uniform(-0.2, 1.5, (L, n, n))
    p = O.Params(1e-3, 0.05, 0.1, 1.0, 1.0, 1.0, 1.0)
    dY = rng.standard_normal((L, n, n))
    _, dX = O.jvp_run(O.Problem(psf, Y, p), 6, (0.0, 0.0, 0.0), dY=dY)
    h = 1e-6
    xp = O.run(O.Problem(psf, Y + h * dY, p), 6).X
    xm = O.run(O.Problem(psf, Y - h * dY, p), 6).X
    fd = (xp - xm) / (2 * h)
    assert np.abs(fd - dX).max() <= 1e-6 * np.abs(dX).max()
