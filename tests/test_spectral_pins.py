"""Pins of the oracle's spectral dictionary (oracle/spectral.py): the
orthonormalised Chebyshev basis against its definition and a library QR,
and Algorithm 1 with W_nu a union of m_nu orthonormal transforms (Section 3:
step V's closed form divides by m_nu rho_V + rho_S) against dense solves,
brute-force proximal steps, a KKT certificate at convergence, closed-form
fixed points, the He-Yuan monotonicity of E^k and dense residual operators."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import oracle as O
from tests.independent import brute_min, dct_matrix, dense_conv_matrix, spec, spec_t

pytestmark = pytest.mark.cpu

UNION = (O.DCT, O.CHEBYSHEV)


def _nodes(L):
    return np.array([0.0]) if L == 1 else -1.0 + 2.0 * np.arange(L) / (L - 1)


def _cheb_qr(L):
    """Orthonormalised Chebyshev columns from a library QR of the Chebyshev
    Vandermonde matrix (numpy's chebvander), degree-k coefficient positive."""
    V = npcheb.chebvander(_nodes(L), L - 1)
    Q, R = np.linalg.qr(V)
    return Q * np.sign(np.diag(R))[None, :]


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 12, 16])
def test_chebyshev_basis_equals_qr_of_the_chebyshev_matrix(L):
    np.testing.assert_allclose(O.chebyshev_basis(L), _cheb_qr(L), atol=1e-11)


@pytest.mark.parametrize("L", [2, 8, 15, 32, 64])
def test_chebyshev_basis_is_orthonormal_and_graded_by_degree(L):
    """W^T W = I; column k is a polynomial of degree k in the band index:
    its (k + 1)-th differences vanish and its k-th differences are a
    positive constant (positive leading coefficient)."""
    W = O.chebyshev_basis(L)
    np.testing.assert_allclose(W.T @ W, np.eye(L), atol=2e-15)
    for k in range(min(L, 10)):
        dk = np.diff(W[:, k], n=k)
        assert np.all(dk > 0) and np.ptp(dk) < 1e-9 * max(1.0, np.abs(dk).max()), (L, k)
        if k + 1 < L:
            assert np.abs(np.diff(W[:, k], n=k + 1)).max() < 1e-9 * max(1.0, np.abs(dk).max()), (L, k)


def test_chebyshev_basis_for_two_bands():
    h = 1.0 / np.sqrt(2.0)
    np.testing.assert_allclose(O.chebyshev_basis(2), [[h, -h], [h, h]], atol=1e-16)


def test_extended_chebyshev_basis_agrees():
    W = O.chebyshev_basis(32)
    Wl = O.chebyshev_basis(32, np.longdouble)
    assert Wl.dtype == np.longdouble
    assert float(np.abs(Wl.T @ Wl - np.eye(32, dtype=np.longdouble)).max()) < 1e-18
    assert float(np.abs(W - Wl).max()) < 1e-16


def _bases(codes, L):
    mats = {O.DCT: dct_matrix(L), O.CHEBYSHEV: _cheb_qr(L), O.SPECTRAL_DIRAC: np.eye(L)}
    return [mats[c] for c in codes]


@pytest.fixture(scope="module")
def tiny_union():
    rng = np.random.default_rng(12)
    L, n = 6, 8
    psf = rng.uniform(0.0, 0.3, size=(L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = rng.standard_normal((L, n, n)) + 1.0
    p = O.Params(mu_eps=1e-3, mu_s=0.3, mu_nu=0.4, rho_P=1.0, rho_T=2.0, rho_V=1.5, rho_S=0.7)
    prob = O.Problem(psf, Y, p, spectral=UNION)
    return prob, psf, rng


def _random_state(rng, shape, m):
    a = {f: rng.standard_normal(shape) for f in ("X", "P", "T", "S", "GP", "GT", "GS")}
    a["V"] = rng.standard_normal((m,) + tuple(shape))
    a["GV"] = rng.standard_normal((m,) + tuple(shape))
    return O.State(**a)


def test_union_steps_IV_V_VI_against_dense_definitions(tiny_union):
    """Step IV per coefficient of every basis by brute-force minimisation;
    step V by a dense solve of S R = C with R = rho_V W_nu W_nu^T + rho_S I
    and W_nu = [W_1 W_2] (L x 2L); step VI as the constraint residual."""
    prob, _, rng = tiny_union
    p = prob.p
    L = prob.shape[0]
    st = _random_state(rng, prob.shape, 2)
    new = O.admm_iteration(prob, st)
    Ws = _bases(UNION, L)
    for j, W in enumerate(Ws):
        SW = spec(st.S, W)
        f = lambda t: (p.mu_nu * np.abs(t) + st.GV[j][..., None] * (t - SW[..., None])
                       + 0.5 * p.rho_V * (t - SW[..., None]) ** 2)
        np.testing.assert_allclose(new.V[j], brute_min(f, SW, 3.0 + np.abs(st.GV[j]) / p.rho_V),
                                   rtol=0, atol=1e-7)
    Wnu = np.hstack(Ws)
    R = p.rho_V * Wnu @ Wnu.T + p.rho_S * np.eye(L)
    C = sum(spec_t(st.GV[j] + p.rho_V * new.V[j], W) for j, W in enumerate(Ws)) - st.GS + p.rho_S * new.X
    Cm = C.reshape(L, -1).T
    Sm = np.linalg.solve(R.T, Cm.T).T
    np.testing.assert_allclose(new.S, Sm.T.reshape(prob.shape), atol=1e-12)
    for j, W in enumerate(Ws):
        np.testing.assert_allclose((new.GV[j] - st.GV[j]) / p.rho_V, new.V[j] - spec(new.S, W), atol=1e-12)


def test_union_step_I_uses_rho_of_eq_Qlsimp(tiny_union):
    """The spectral union does not enter step I: the X-update still zeroes
    the augmented Lagrangian's gradient with rho = mu_eps + rho_S + rho_P + rho_T."""
    prob, psf, rng = tiny_union
    p = prob.p
    st = _random_state(rng, prob.shape, 2)
    new = O.admm_iteration(prob, st)
    L = prob.shape[0]
    for l in range(L):
        Hd = dense_conv_matrix(psf[l])
        x = new.X[l].ravel()
        g = (Hd.T @ (Hd @ x - prob.Y[l].ravel()) + p.mu_eps * x
             - (st.GP[l] + p.rho_P * (st.P[l] - new.X[l])).ravel()
             - (st.GT[l] + p.rho_T * (st.T[l] - new.X[l])).ravel()
             - (st.GS[l] + p.rho_S * (st.S[l] - new.X[l])).ravel())
        assert np.abs(g).max() < 1e-11 * max(1.0, np.abs(x).max())


def test_union_kkt_certificate_at_convergence(tiny_union):
    """At convergence: H^T(HX - Y) + mu_eps X - Gamma_P - Gamma_T
    - sum_j Gamma_V,j W_j^T = 0, |Gamma_V,j| <= mu_nu with equality and the
    opposite sign of V_j where V_j != 0, V_j = X W_j, X = P >= 0."""
    prob, psf, _ = tiny_union
    p = O.Params(1e-2, 0.05, 0.2, 1.0, 1.0, 1.0, 1.0)
    prob = prob.with_params(p)
    st = O.run(prob, 8000)
    L = prob.shape[0]
    Ws = _bases(UNION, L)
    HtHX = np.stack([(dense_conv_matrix(psf[l]).T @ (dense_conv_matrix(psf[l]) @ st.X[l].ravel()
                      - prob.Y[l].ravel())).reshape(st.X[l].shape) for l in range(L)])
    g = HtHX + p.mu_eps * st.X - st.GP - st.GT - sum(spec_t(st.GV[j], W) for j, W in enumerate(Ws))
    assert np.abs(g).max() < 1e-8
    np.testing.assert_allclose(st.X, st.P, atol=1e-9)
    for j, W in enumerate(Ws):
        np.testing.assert_allclose(st.V[j], spec(st.X, W), atol=1e-8)
        nz = np.abs(st.V[j]) > 1e-6
        np.testing.assert_allclose(st.GV[j][nz], -p.mu_nu * np.sign(st.V[j][nz]), atol=1e-8)
        assert np.abs(st.GV[j]).max() <= p.mu_nu + 1e-8


def test_spectral_dirac_fixed_point():
    """H = I, mu_s = 0, W_nu = identity along the bands: per voxel
    min (x - y)^2 / 2 + mu_eps x^2 / 2 + mu_nu |x|, x >= 0:
    X* = max(0, Y - mu_nu) / (1 + mu_eps)."""
    rng = np.random.default_rng(14)
    L, n = 4, 8
    psf = np.zeros((L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = rng.uniform(-0.5, 2.0, (L, n, n))
    p = O.Params(1e-3, 0.0, 0.4, 1.0, 1.0, 1.0, 1.0)
    st = O.run(O.Problem(psf, Y, p, spectral=(O.SPECTRAL_DIRAC,)), 800)
    np.testing.assert_allclose(st.X, np.maximum(0.0, Y - p.mu_nu) / (1 + p.mu_eps), atol=1e-10)


def test_chebyshev_fixed_point_positive_solution():
    """H = I, mu_s = 0, one Chebyshev basis, positive solution:
    X* = W soft(W^T Y, mu_nu) / (1 + mu_eps) per pixel."""
    rng = np.random.default_rng(15)
    L, n = 8, 8
    psf = np.zeros((L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = 5.0 + rng.uniform(-0.5, 0.5, (L, n, n))
    p = O.Params(1e-3, 0.0, 0.3, 1.0, 1.0, 1.0, 1.0)
    W = _cheb_qr(L)
    c = spec(Y, W)
    ref = spec_t(np.sign(c) * np.maximum(np.abs(c) - p.mu_nu, 0.0), W) / (1 + p.mu_eps)
    assert ref.min() > 0
    st = O.run(O.Problem(psf, Y, p, spectral=(O.CHEBYSHEV,)), 800)
    np.testing.assert_allclose(st.X, ref, atol=1e-10)


def test_union_energy_is_non_increasing(tiny_union):
    prob, _, _ = tiny_union
    E = []
    O.run(prob, 60, callback=lambda k, a, b: E.append(O.energy(prob, a, b)))
    E = np.array(E)
    assert np.all(E[1:] <= E[:-1] * (1 + 1e-12)), np.diff(E).max()
    assert E[-1] < 1e-2 * E[0]


def test_union_residuals_energy_objective_against_dense_operators(tiny_union):
    """Residuals, E^k and F(P) for m_nu = 2 against the stacked constraint
    matrices: [P - X; T - X; V_1 - S W_1; V_2 - S W_2; S - X] = A x + B z with
    x = (X, V_1, V_2), z = (P, T, S)."""
    prob, psf, _ = tiny_union
    p = prob.p
    prev = O.run(prob, 3)
    cur = O.admm_iteration(prob, prev)
    L, ny, nx = prob.shape
    n = L * ny * nx
    Ws = _bases(UNION, L)
    Wb = [np.kron(W.T, np.eye(ny * nx)) for W in Ws]
    I = np.eye(n)
    Z = np.zeros((n, n))
    A = np.block([[-I, Z, Z], [-I, Z, Z], [Z, I, Z], [Z, Z, I], [-I, Z, Z]])
    B = np.block([[I, Z, Z], [Z, I, Z], [Z, Z, -Wb[0]], [Z, Z, -Wb[1]], [Z, Z, I]])
    rho = np.concatenate([np.full(n, p.rho_P), np.full(n, p.rho_T), np.full(2 * n, p.rho_V),
                          np.full(n, p.rho_S)])
    v = lambda a: a.ravel()
    x = np.concatenate([v(cur.X), v(cur.V[0]), v(cur.V[1])])
    z = np.concatenate([v(cur.P), v(cur.T), v(cur.S)])
    dz = z - np.concatenate([v(prev.P), v(prev.T), v(prev.S)])
    y = np.concatenate([v(cur.GP), v(cur.GT), v(cur.GV[0]), v(cur.GV[1]), v(cur.GS)])
    dy = y - np.concatenate([v(prev.GP), v(prev.GT), v(prev.GV[0]), v(prev.GV[1]), v(prev.GS)])
    r = A @ x + B @ z
    s = A.T @ (rho * (B @ dz))
    res = O.residuals(prob, prev, cur, eps_abs=1e-5, eps_rel=1e-4)
    assert res["r"] == pytest.approx(np.linalg.norm(r), rel=1e-12)
    assert res["s"] == pytest.approx(np.linalg.norm(s), rel=1e-12)
    eps_pri = np.sqrt(5 * n) * 1e-5 + 1e-4 * max(np.linalg.norm(A @ x), np.linalg.norm(B @ z))
    eps_dual = np.sqrt(3 * n) * 1e-5 + 1e-4 * np.linalg.norm(A.T @ y)
    assert res["eps_pri"] == pytest.approx(eps_pri, rel=1e-12)
    assert res["eps_dual"] == pytest.approx(eps_dual, rel=1e-12)
    E = np.sum(rho * (B @ dz) ** 2) + np.sum(dy ** 2 / rho)
    assert O.energy(prob, prev, cur) == pytest.approx(E, rel=1e-12)
    P = cur.P
    HP = np.stack([(dense_conv_matrix(psf[l]) @ P[l].ravel()).reshape(ny, nx) for l in range(L)])
    F = (0.5 * np.sum((prob.Y - HP) ** 2) + 0.5 * p.mu_eps * np.sum(P ** 2)
         + p.mu_s * np.sum(np.abs(P)) + p.mu_nu * sum(np.sum(np.abs(spec(P, W))) for W in Ws))
    assert O.objective(prob, P) == pytest.approx(F, rel=1e-12)


def test_single_dct_dictionary_is_the_plain_oracle():
    """spectral=(DCT,) is the m_nu = 1 iteration the other pins cover."""
    from synth import make_instance
    inst = make_instance(16, 16, 4, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.01, seed=3)
    p = O.Params(1e-3, 0.1, 0.2, 1.0, 2.0, 1.5, 1.0)
    a = O.run(O.Problem(inst.psf, inst.dirty, p), 20)
    b = O.run(O.Problem(inst.psf, inst.dirty, p, spectral=(O.DCT,)), 20)
    np.testing.assert_array_equal(a.X, b.X)


@pytest.mark.parametrize("basis", [O.CHEBYSHEV, O.SPECTRAL_DIRAC])
def test_tangent_with_one_other_spectral_basis_matches_central_differences(basis):
    """The oracle's forward-mode gradient with the Chebyshev or the identity
    basis as W_nu, against central differences of K passes."""
    from synth import make_instance
    inst = make_instance(16, 16, 4, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.01, seed=21,
                         sigma_range=(1.0, 2.0))
    base = O.Params(1e-3, 0.05, 0.05, 1.0, 1.0, 1.0, 1.0)
    prob = O.Problem(inst.psf, inst.dirty, base, spectral=(basis,))
    K = 12
    loss, g = O.mse_grad(prob, K, inst.sky)
    # the loss curves enough here that h = 1e-6 is 2e-5 off; at 1e-7 the
    # central difference has converged (it agrees with 1e-8 to 3e-7)
    h = 1e-7

    def L_at(ms, mn, r):
        q = prob.with_params(O.Params(base.mu_eps, ms, mn, r, r, r, r))
        return O.mse_loss(O.run(q, K).X, inst.sky)
    fd = np.array([
        (L_at(base.mu_s + h, base.mu_nu, 1.0) - L_at(base.mu_s - h, base.mu_nu, 1.0)) / (2 * h),
        (L_at(base.mu_s, base.mu_nu + h, 1.0) - L_at(base.mu_s, base.mu_nu - h, 1.0)) / (2 * h),
        (L_at(base.mu_s, base.mu_nu, 1.0 + h) - L_at(base.mu_s, base.mu_nu, 1.0 - h)) / (2 * h),
    ])
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())

