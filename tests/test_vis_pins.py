"""Pins of the oracle's visibility-domain model (Section 2: the data as
sampled visibilities, H_l the sky-to-visibility operator; step I by
conjugate gradients on Q_l of eq. Qlsimp): each against a definition
written out independently, a textbook identity or the already-pinned
dirty-image oracle."""
import numpy as np
import pytest

import oracle as O
from oracle.visibility import cg, toeplitz_apply, toeplitz_kernel, vis_adjoint, vis_forward
from synth.visibilities import make_vis_instance


def _dense_H(uv, ny, nx):
    """The operator by its definition, entry by entry."""
    G = np.zeros((len(uv), ny * nx), dtype=np.complex128)
    for j, (u, v) in enumerate(uv):
        for m in range(ny):
            for n in range(nx):
                G[j, m * nx + n] = np.exp(-2j * np.pi * (u * (n - nx // 2) / nx + v * (m - ny // 2) / ny))
    return G


@pytest.fixture
def small():
    rng = np.random.default_rng(5)
    ny, nx = 4, 6
    uv = rng.uniform(-2.7, 2.7, size=(9, 2))
    return rng, ny, nx, uv, _dense_H(uv, ny, nx)


def test_forward_and_adjoint_against_the_dense_operator(small):
    rng, ny, nx, uv, G = small
    x = rng.standard_normal((ny, nx))
    y = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    np.testing.assert_allclose(vis_forward(x, uv), G @ x.ravel(), rtol=0, atol=1e-12)
    np.testing.assert_allclose(vis_adjoint(y, uv, ny, nx).ravel(), np.real(G.conj().T @ y), rtol=0, atol=1e-12)
    # the real adjoint: <H x, y> over C^M as R^(2M) equals <x, H^T y>
    lhs = np.real(np.vdot(y, vis_forward(x, uv)))
    rhs = float(np.sum(x * vis_adjoint(y, uv, ny, nx)))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_toeplitz_product_is_re_HhH(small):
    rng, ny, nx, uv, G = small
    x = rng.standard_normal((ny, nx))
    dense = np.real(G.conj().T @ G) @ x.ravel()
    c = toeplitz_kernel(uv, ny, nx)
    assert c.shape == (2 * ny - 1, 2 * nx - 1)
    # c is even and c(0) counts the visibilities
    np.testing.assert_allclose(c, c[::-1, ::-1], rtol=0, atol=1e-12)
    assert c[ny - 1, nx - 1] == pytest.approx(len(uv))
    np.testing.assert_allclose(toeplitz_apply(c, x).ravel(), dense, rtol=0, atol=1e-11)


def test_cg_reaches_the_direct_solve(small):
    rng, ny, nx, uv, G = small
    rho = 0.7
    Q = np.real(G.conj().T @ G) + rho * np.eye(ny * nx)
    b = rng.standard_normal((ny, nx))
    c = toeplitz_kernel(uv, ny, nx)
    x = cg(lambda z: toeplitz_apply(c, z) + rho * z, b, np.zeros_like(b), 3 * ny * nx)
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(Q, b.ravel()), rtol=0, atol=1e-10)
    # from the exact solution nothing moves (alpha = 0 when r = 0 exactly is
    # not guaranteed in floating point; the step is at rounding level)
    xs = np.linalg.solve(Q, b.ravel()).reshape(ny, nx)
    x1 = cg(lambda z: toeplitz_apply(c, z) + rho * z, b, xs, 2)
    np.testing.assert_allclose(x1, xs, rtol=0, atol=1e-12)


def test_cg_iterates_follow_the_textbook_recursion(small):
    """Two CG steps by hand (Hestenes-Stiefel, dense Q) against cg(., 2)."""
    rng, ny, nx, uv, G = small
    rho = 1.3
    Q = np.real(G.conj().T @ G) + rho * np.eye(ny * nx)
    b = rng.standard_normal(ny * nx)
    x0 = rng.standard_normal(ny * nx)
    x, r = x0.copy(), b - Q @ x0
    p = r.copy()
    for _ in range(2):
        a = (r @ r) / (p @ Q @ p)
        x_new, r_new = x + a * p, r - a * (Q @ p)
        p = r_new + ((r_new @ r_new) / (r @ r)) * p
        x, r = x_new, r_new
    c = toeplitz_kernel(uv, ny, nx)
    got = cg(lambda z: toeplitz_apply(c, z) + rho * z, b.reshape(ny, nx), x0.reshape(ny, nx), 2)
    np.testing.assert_allclose(got.ravel(), x, rtol=0, atol=1e-11)


def test_full_uniform_sampling_gives_a_scaled_identity():
    """Every integer cell sampled once: Re(H^H H) = N^2 I, so one CG step
    solves Q x = b exactly, x = b / (N^2 + rho)."""
    ny, nx = 4, 8
    uv = np.array([(kx, ky) for ky in range(ny) for kx in range(nx)], dtype=np.float64)
    c = toeplitz_kernel(uv, ny, nx)
    x = np.random.default_rng(1).standard_normal((ny, nx))
    np.testing.assert_allclose(toeplitz_apply(c, x), ny * nx * x, rtol=0, atol=1e-10)
    b = np.random.default_rng(2).standard_normal((ny, nx))
    rho = 2.5
    got = cg(lambda z: toeplitz_apply(c, z) + rho * z, b, np.zeros_like(b), 1)
    np.testing.assert_allclose(got, b / (ny * nx + rho), rtol=0, atol=1e-13)


def test_integer_cells_reduce_to_the_dirty_image_model():
    """With the visibilities on integer cells, Re(H^H H) is a circulant
    convolution on the N x N grid (c(d) is N-periodic): the visibility-domain
    iteration with step I solved to convergence equals the dirty-image
    oracle with |h_hat|^2 = FFT2 of the periodic kernel and H^T Y = Re(H^H y)."""
    L, ny, nx = 2, 8, 8
    inst = make_vis_instance(ny, nx, L, n_points=3, n_gauss=1, n_ant=6, noise_sigma=0.05, seed=21, n_time=4,
                             integer_uv=True)
    p = O.Params(1e-3, 0.05, 0.08, 1.0, 1.5, 1.2, 0.8)
    vp = O.VisProblem(inst.uv, inst.vis, inst.shape, p, n_cg=400)
    psf, hty = [], []
    for l in range(L):
        c = toeplitz_kernel(inst.uv[l], ny, nx)
        # the N-periodic kernel on the lags [0, N)^2
        cN = c[ny - 1:, nx - 1:]
        assert cN.shape == (ny, nx)
        chat = np.fft.fft2(cN)
        assert np.abs(chat.imag).max() < 1e-9 * np.abs(chat).max()
        assert chat.real.min() > -1e-9 * chat.real.max()
        hhat = np.sqrt(np.maximum(chat.real, 0.0))
        psf.append(np.fft.fftshift(np.fft.ifft2(hhat).real))
        hty.append(vp.HtY[l])
    dp = O.Problem(np.stack(psf), np.zeros((L, ny, nx)), p)
    for l in range(L):
        cN = toeplitz_kernel(inst.uv[l], ny, nx)[ny - 1:, nx - 1:]
        np.testing.assert_allclose(np.abs(dp.hhat[l]) ** 2, np.fft.fft2(cN).real, rtol=0,
                                   atol=1e-9 * np.abs(np.fft.fft2(cN)).max())
    dp.HtY = np.stack(hty)
    a = O.run(dp, 6)
    b = O.run(vp, 6)
    assert np.abs(a.X - b.X).max() <= 1e-9 * np.abs(a.X).max()
    assert np.abs(a.S - b.S).max() <= 1e-9 * np.abs(a.S).max()


def test_misfit_and_energy_of_the_visibility_model():
    """The objective's data term against the dense operator; E^k
    non-increasing with step I solved to convergence (He and Yuan)."""
    L, ny, nx = 2, 8, 8
    inst = make_vis_instance(ny, nx, L, n_points=3, n_gauss=1, n_ant=7, noise_sigma=0.05, seed=22, n_time=5)
    p = O.Params(1e-3, 0.05, 0.05, 1.0, 1.0, 1.0, 1.0)
    vp = O.VisProblem(inst.uv, inst.vis, inst.shape, p, n_cg=300)
    x = np.random.default_rng(3).standard_normal((L, ny, nx))
    dense = 0.5 * sum(np.sum(np.abs(inst.vis[l] - _dense_H(inst.uv[l], ny, nx) @ x[l].ravel()) ** 2)
                      for l in range(L))
    assert vp.misfit(x) == pytest.approx(dense, rel=1e-12)
    E = []
    O.run(vp, 12, callback=lambda k, prev, cur: E.append(O.energy(vp, prev, cur)))
    E = np.array(E)
    assert np.all(E[2:] <= E[1:-1] * (1 + 1e-9))
    # F(P) at the end below F(P) after the first pass
    st1 = O.run(vp, 1)
    st12 = O.run(vp, 12)
    assert O.objective(vp, st12.P) < O.objective(vp, st1.P)


def test_generator_samples_the_sky_by_the_definition():
    """The generator's visibilities (noise off) equal the dense operator on
    its sky: the data the GPU path and the oracle both read."""
    inst = make_vis_instance(8, 4, 1, n_points=2, n_gauss=1, n_ant=5, noise_sigma=0.0, seed=23, n_time=3)
    G = _dense_H(inst.uv[0], 8, 4)
    np.testing.assert_allclose(inst.vis[0], G @ inst.sky[0].astype(np.float64).ravel(), rtol=0, atol=1e-11)
