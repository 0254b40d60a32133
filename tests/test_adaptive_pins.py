"""Pins of the oracle's residual balancing (Boyd et al. 2011, Sec. 3.4.1):
never triggered it is the plain iteration; triggered it changes the rho's
in the direction that balances the residuals; and it reaches the same
minimiser as a fixed-rho run (the limit does not depend on rho)."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.cpu


def _tiny(seed=3, L=3, n=8):
    rng = np.random.default_rng(seed)
    psf = rng.uniform(0.0, 0.3, (L, n, n))
    psf[:, n // 2, n // 2] = 1.0
    Y = rng.uniform(-0.2, 1.5, (L, n, n))
    return psf, Y


def test_untriggered_balancing_is_the_plain_iteration():
    psf, Y = _tiny()
    prob = O.Problem(psf, Y, O.Params(1e-3, 0.05, 0.1, 1.0, 1.0, 1.0, 1.0))
    st, pr, hist = O.solve_adaptive(prob, 37, 5, 1e300, 2.0, eps_abs=0.0, eps_rel=0.0)
    ref = O.run(prob, 37)
    assert np.array_equal(st.X, ref.X) and pr.p == prob.p
    assert [h[0] for h in hist] == [5, 10, 15, 20, 25, 30, 35, 37]


@pytest.mark.parametrize("rho,direction", [(0.01, +1), (100.0, -1)])
def test_balancing_moves_rho_towards_the_balanced_residuals(rho, direction):
    psf, Y = _tiny(seed=4)
    prob = O.Problem(psf, Y, O.Params(1e-3, 0.05, 0.1, rho, rho, rho, rho))
    _, pr, hist = O.solve_adaptive(prob, 60, 5, 10.0, 2.0, eps_abs=0.0, eps_rel=0.0)
    rhos = [h[1] for h in hist]
    assert (pr.p.rho_P - rho) * direction > 0
    assert all((b - a) * direction >= 0 for a, b in zip(rhos, rhos[1:]))
    # the first check already sees the imbalance the direction comes from
    k, _, r, s = hist[0]
    assert (r > 10.0 * s) if direction > 0 else (s > 10.0 * r)


def test_balancing_reaches_the_fixed_rho_minimiser():
    psf, Y = _tiny(seed=5)
    p = O.Params(1e-2, 0.05, 0.1, 0.05, 0.05, 0.05, 0.05)
    st, pr, _ = O.solve_adaptive(O.Problem(psf, Y, p), 3000, 10, 10.0, 2.0, eps_abs=1e-13, eps_rel=1e-12)
    ref = O.run(O.Problem(psf, Y, p.with_(rho_P=1.0, rho_T=1.0, rho_V=1.0, rho_S=1.0)), 4000)
    np.testing.assert_allclose(st.X, ref.X, atol=1e-8)
