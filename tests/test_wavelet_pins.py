"""Pins of the oracle's spatial dictionary (Section 4: W_s = the Dirac basis
and the Daubechies wavelet bases Db1-Db8): the filters against closed forms
and their defining properties, the periodised 2-D transform against a dense
matrix built by loops from its definition, orthonormality, and the ADMM with
a union of bases against special cases and a KKT certificate."""
import math

import numpy as np
import pytest

import oracle as O
from tests.independent import dct_matrix, dense_conv_matrix, dense_dwt_matrix, spec_t

pytestmark = pytest.mark.cpu


def test_db1_db2_db3_closed_forms():
    r2 = math.sqrt(2.0)
    np.testing.assert_allclose(O.daubechies_filter(1), [1 / r2, 1 / r2], atol=1e-15)
    s3 = math.sqrt(3.0)
    db2 = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * r2)
    np.testing.assert_allclose(O.daubechies_filter(2), db2, atol=1e-14)
    s10 = math.sqrt(10.0)
    r = math.sqrt(5 + 2 * s10)
    db3 = np.array([1 + s10 + r, 5 + s10 + 3 * r, 10 - 2 * s10 + 2 * r,
                    10 - 2 * s10 - 2 * r, 5 + s10 - 3 * r, 1 + s10 - r]) / (16 * r2)
    np.testing.assert_allclose(O.daubechies_filter(3), db3, atol=1e-13)


@pytest.mark.parametrize("p", range(1, 9))
def test_filter_properties(p):
    """Length 2p, sum sqrt 2, orthonormal to its even shifts, p vanishing
    moments of the wavelet filter, extra zeros outside the unit circle."""
    h = O.daubechies_filter(p)
    K = len(h)
    assert K == 2 * p
    assert abs(h.sum() - math.sqrt(2.0)) < 1e-13
    for m in range(0, p):
        dot = sum(h[k] * h[k + 2 * m] for k in range(K - 2 * m))
        assert abs(dot - (1.0 if m == 0 else 0.0)) < 1e-12, m
    g = np.array([(-1) ** k * h[K - 1 - k] for k in range(K)])
    k = np.arange(K, dtype=np.float64)
    for m in range(p):
        mom = np.sum(k ** m * g)
        assert abs(mom) < 1e-10 * max(1.0, np.sum(np.abs(k ** m * g))), (p, m, mom)
    # h(z) = (1 + z)^p r(z): the zeros of r lie outside the unit circle
    r = np.array(h[::-1])
    for _ in range(p):
        r, rem = np.polydiv(r, [1.0, 1.0])
        assert np.abs(rem).max() < 1e-9
    if len(r) > 1:
        assert np.abs(np.roots(r)).min() > 1.0 + 1e-6


@pytest.mark.parametrize("p,ny,nx", [(1, 8, 8), (2, 8, 16), (4, 16, 8), (8, 8, 8), (3, 4, 4)])
def test_dwt2_equals_dense_definition_and_is_orthonormal(p, ny, nx):
    h = O.daubechies_filter(p)
    J = O.dwt_levels(nx, ny)
    M = dense_dwt_matrix(list(h), ny, nx, J)
    np.testing.assert_allclose(M @ M.T, np.eye(ny * nx), atol=1e-12)
    rng = np.random.default_rng(p)
    x = rng.standard_normal((2, ny, nx))
    c = O.dwt2(x, h, J)
    for b in range(2):
        np.testing.assert_allclose(c[b].ravel(), M @ x[b].ravel(), atol=1e-12)
        np.testing.assert_allclose(O.idwt2(c, h, J)[b].ravel(), M.T @ c[b].ravel(), atol=1e-12)
    np.testing.assert_allclose(O.idwt2(c, h, J), x, atol=1e-12)


def test_levels_reading_and_constant_image():
    """4 levels, fewer on small images; a constant image keeps only the
    coarsest LL block, scaled by 2 per level ((sum h)^2 = 2)."""
    assert O.dwt_levels(1024, 1024) == 4 and O.dwt_levels(8, 8) == 2 and O.dwt_levels(4, 64) == 1
    for p in (1, 2, 5, 8):
        c = O.dwt2(np.full((1, 32, 32), 3.0), O.daubechies_filter(p), 4)
        np.testing.assert_allclose(c[0, :2, :2], 3.0 * 2 ** 4, atol=1e-11)
        c[0, :2, :2] = 0.0
        assert np.abs(c).max() < 1e-11


def test_dictionary_is_a_union_of_orthonormal_bases():
    rng = np.random.default_rng(3)
    W = O.Dictionary(O.PAPER_DICTIONARY)
    assert W.n_s == 9
    x = rng.standard_normal((2, 16, 32))
    np.testing.assert_allclose(W.adjoint(W.forward(x)), 9 * x, atol=1e-11)
    c = rng.standard_normal((9, 2, 16, 32))
    assert abs(np.sum(W.forward(x) * c) - np.sum(x * W.adjoint(c))) < 1e-10


def test_two_dirac_bases_reach_the_dirac_minimiser_with_twice_mu_s():
    """||[I; I] X||_1 = 2 ||X||_1: the limits agree (the iterates differ:
    rho of eq. Qlsimp counts n_s)."""
    rng = np.random.default_rng(8)
    L, n = 2, 8
    psf = rng.uniform(0.0, 0.3, (L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = rng.uniform(-0.2, 1.5, (L, n, n))
    p = O.Params(1e-2, 0.05, 0.1, 1.0, 1.0, 1.0, 1.0)
    a = O.run(O.Problem(psf, Y, p, bases=(O.DIRAC, O.DIRAC)), 3000).X
    b = O.run(O.Problem(psf, Y, p.with_(mu_s=2 * p.mu_s)), 3000).X
    np.testing.assert_allclose(a, b, atol=1e-9)


def test_kkt_certificate_with_wavelet_dictionary():
    """At the ADMM limit with W_s = (Dirac, Db1, Db2): H^T(HX - Y) + mu_eps X
    - Gamma_P - W_s^T Gamma_T - Gamma_V W_nu^T = 0, Gamma_T = -mu_s sign(T)
    where T != 0 and |Gamma_T| <= mu_s, with dense H, W_s and W_nu."""
    rng = np.random.default_rng(9)
    L, n = 2, 8
    psf = rng.uniform(0.0, 0.3, (L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = rng.uniform(-0.2, 1.5, (L, n, n))
    p = O.Params(1e-2, 0.03, 0.1, 1.0, 1.0, 1.0, 1.0)
    bases = (O.DIRAC, 1, 2)
    prob = O.Problem(psf, Y, p, bases=bases)
    st = O.run(prob, 6000)
    J = O.dwt_levels(n, n)
    Wb = [np.eye(n * n)] + [dense_dwt_matrix(list(O.daubechies_filter(q)), n, n, J) for q in bases[1:]]
    Hd = [dense_conv_matrix(psf[l]) for l in range(L)]
    WsT_GT = np.stack([sum(Wb[i].T @ st.GT[i, l].ravel() for i in range(3)).reshape(n, n)
                       for l in range(L)])
    HtHX = np.stack([(Hd[l].T @ (Hd[l] @ st.X[l].ravel() - Y[l].ravel())).reshape(n, n) for l in range(L)])
    g = HtHX + p.mu_eps * st.X - st.GP - WsT_GT - spec_t(st.GV, dct_matrix(L))
    assert np.abs(g).max() < 1e-8
    for i in range(3):
        WX = np.stack([(Wb[i] @ st.X[l].ravel()).reshape(n, n) for l in range(L)])
        assert np.abs(st.T[i] - WX).max() < 1e-8           # the constraint T = W_s X holds
    nz = np.abs(st.T) > 1e-6
    np.testing.assert_allclose(st.GT[nz], -p.mu_s * np.sign(st.T[nz]), atol=1e-8)
    assert np.abs(st.GT).max() <= p.mu_s + 1e-9


def test_tangent_pass_with_wavelet_bases_against_central_differences():
    """The oracle's forward-mode tangent with wavelet bases in W_s equals
    central differences of K passes along every parameter alone (mu_eps and
    rho_T alone check the n_s rho_T of eq. Qlsimp) and along a change of the
    dirty images (smooth away from the prox kinks at these steps)."""
    rng = np.random.default_rng(33)
    L, n = 3, 16
    psf = np.zeros((L, n, n))
    for l in range(L):
        g = np.exp(-((np.arange(n) - n // 2)[:, None] ** 2 + (np.arange(n) - n // 2)[None, :] ** 2)
                   / (2.0 * (1.2 + 0.3 * l) ** 2))
        psf[l] = g / g.sum()
    Y = rng.uniform(-0.1, 1.0, (L, n, n))
    base = O.Params(1e-3, 0.03, 0.05, 1.1, 0.9, 1.3, 0.8)
    bases = (0, 1, 3)
    prob = O.Problem(psf, Y, base, bases=bases)
    K, h = 5, 1e-6
    names = ("mu_eps", "mu_s", "mu_nu", "rho_P", "rho_T", "rho_V", "rho_S")
    for i, name in enumerate(names):
        d = [0.0] * 7
        d[i] = 1.0
        _, dX = O.jvp_run(prob, K, O.Params(*d))
        xp = O.run(prob.with_params(base.with_(**{name: getattr(base, name) + h})), K).X
        xm = O.run(prob.with_params(base.with_(**{name: getattr(base, name) - h})), K).X
        fd = (xp - xm) / (2 * h)
        assert np.abs(fd - dX).max() <= 1e-6 * max(np.abs(dX).max(), 1e-3), name
    dY = rng.standard_normal((L, n, n))
    _, dX = O.jvp_run(prob, K, (0.0, 0.0, 0.0), dY=dY)
    xp = O.run(O.Problem(psf, Y + h * dY, base, bases=bases), K).X
    xm = O.run(O.Problem(psf, Y - h * dY, base, bases=bases), K).X
    assert np.abs((xp - xm) / (2 * h) - dX).max() <= 1e-6 * np.abs(dX).max()


def test_residuals_energy_objective_with_wavelet_bases_against_dense_operators():
    """The Boyd residuals, their tolerances, E^k and F(P) with a union of
    three spatial bases (Dirac, Db1, Db3), against the stacked constraint
    matrices written out densely: [P - X; T - W_s X; V - S W; S - X] =
    A (X, V) + B (P, T, S), W_s the loop-built DWT matrices stacked under the
    identity (T and Gamma_T hold one cube per basis)."""
    from tests.independent import dense_conv_matrix
    rng = np.random.default_rng(17)
    L, n = 3, 8
    psf = rng.uniform(0.0, 0.3, size=(L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = rng.standard_normal((L, n, n)) + 1.0
    p = O.Params(mu_eps=1e-3, mu_s=0.3, mu_nu=0.7, rho_P=1.0, rho_T=3.0, rho_V=2.0, rho_S=1.5)
    bases = (0, 1, 3)
    prob = O.Problem(psf, Y, p, bases=bases)
    prev = O.run(prob, 3)
    cur = O.admm_iteration(prob, prev)
    N = L * n * n
    J = O.dwt_levels(n, n)
    blocks = [np.eye(N)] + [np.kron(np.eye(L), dense_dwt_matrix(O.daubechies_filter(b), n, n, J))
                            for b in bases[1:]]
    Ws = np.vstack(blocks)                       # (n_s N) x N
    ns = len(bases)
    W = dct_matrix(L)
    Wbig = np.kron(W.T, np.eye(n * n))
    I = np.eye(N)
    Z = np.zeros((N, N))
    ZT = np.zeros((ns * N, N))
    A = np.block([[-I, Z], [-Ws, ZT], [Z, I], [-I, Z]])
    B = np.block([[I, np.zeros((N, ns * N)), Z],
                  [ZT, np.eye(ns * N), ZT],
                  [Z, np.zeros((N, ns * N)), -Wbig],
                  [Z, np.zeros((N, ns * N)), I]])
    rho = np.concatenate([np.full(N, p.rho_P), np.full(ns * N, p.rho_T), np.full(N, p.rho_V),
                          np.full(N, p.rho_S)])
    v = lambda a: np.asarray(a).ravel()
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
    eps_pri = np.sqrt(A.shape[0]) * 1e-5 + 1e-4 * max(np.linalg.norm(A @ x), np.linalg.norm(B @ z))
    eps_dual = np.sqrt(A.shape[1]) * 1e-5 + 1e-4 * np.linalg.norm(A.T @ y)
    assert res["eps_pri"] == pytest.approx(eps_pri, rel=1e-12)
    assert res["eps_dual"] == pytest.approx(eps_dual, rel=1e-12)
    E = np.sum(rho * (B @ dz) ** 2) + np.sum(dy ** 2 / rho)
    assert O.energy(prob, prev, cur) == pytest.approx(E, rel=1e-12)
    P = cur.P
    HP = np.stack([(dense_conv_matrix(psf[l]) @ P[l].ravel()).reshape(n, n) for l in range(L)])
    F = (0.5 * np.sum((Y - HP) ** 2) + 0.5 * p.mu_eps * np.sum(P ** 2)
         + p.mu_s * np.sum(np.abs(Ws @ P.ravel())) + p.mu_nu * np.sum(np.abs(Wbig @ P.ravel())))
    assert O.objective(prob, P) == pytest.approx(F, rel=1e-12)
