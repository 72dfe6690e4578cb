"""Pins of the polynomial variants of Section 2.5 and of PGD / PPGD (CPU only).

* L-infinity (Chebyshev) design for a known smallest eigenvalue mu: the residual
  ``r(z) = 1 - z p(z)`` equioscillates between +-eps on [mu, 1] at the d+2
  mapped Chebyshev extrema with eps = 1 / T_(d+1)((1+mu)/(1-mu)), agrees with
  NumPy's Chebyshev-series evaluation (an independent route), keeps p > 0 on
  (0, 1] (the positivity theorem) and no small perturbation lowers max |r|.
* Weighted L2 design with w(z) = z^alpha: alpha = 0 is the unweighted fit, and
  the coefficients minimise the weighted cost evaluated by adaptive quadrature.
* PGD / PPGD (Algorithms 1 and 3): lambda = 0 converges to pinv(A') b', the
  lambda > 0 limit satisfies the fixed-point theorem, and the per-eigenvector
  error factor of one PGD step is 1 - mu.
"""

from fractions import Fraction

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest
from scipy.integrate import quad

import oracle as orc
from tests.test_oracle_solve import setup
from tests.tiny import dense_forward, dense_normal, sampled


def residual(coef, z):
    return 1.0 - z * orc.poly_eval(coef, z)


@pytest.mark.parametrize("d,mu", [(1, 0.1), (2, 0.05), (3, 0.05), (4, 0.01), (5, 0.2)])
def test_chebyshev_equioscillation(d, mu):
    c = [float(v) for v in orc.chebyshev_poly_coefficients(d, mu)]
    a = (1 + mu) / (1 - mu)
    eps = 1.0 / np.cosh((d + 1) * np.arccosh(a))          # 1 / T_(d+1)(a)
    k = np.arange(d + 2)
    zk = (1 + mu - (1 - mu) * np.cos(k * np.pi / (d + 1))) / 2
    np.testing.assert_allclose(residual(c, zk), eps * (-1.0) ** k, rtol=0, atol=1e-9 * max(1, eps))
    zz = np.linspace(mu, 1, 20001)
    assert np.max(np.abs(residual(c, zz))) <= eps * (1 + 1e-9)
    assert residual(c, np.array([0.0]))[0] == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("d,mu", [(2, 0.05), (4, 0.01)])
def test_chebyshev_matches_numpy_series(d, mu):
    c = [float(v) for v in orc.chebyshev_poly_coefficients(d, mu)]
    z = np.linspace(0, 1, 101)
    u = (1 + mu - 2 * z) / (1 - mu)
    basis = np.zeros(d + 2)
    basis[-1] = 1.0
    r = npc.chebval(u, basis) / npc.chebval((1 + mu) / (1 - mu), basis)
    np.testing.assert_allclose(residual(c, z), r, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("d,mu", [(1, 0.1), (3, 0.05), (5, 0.02)])
def test_chebyshev_positive_and_minimax(d, mu):
    c = [float(v) for v in orc.chebyshev_poly_coefficients(d, mu)]
    z = np.linspace(1e-6, 1, 100001)
    assert orc.poly_eval(c, z).min() > 0
    zz = np.linspace(mu, 1, 4001)
    best = np.max(np.abs(residual(c, zz)))
    rng = np.random.default_rng(d)
    for _ in range(40):
        pert = np.array(c) + 1e-3 * np.abs(np.array(c)).max() * rng.standard_normal(d + 1)
        assert np.max(np.abs(residual(pert, zz))) > best


def test_weighted_alpha_zero_is_unweighted():
    for d in range(6):
        assert orc.weighted_l2_poly_coefficients(d, 0) == orc.l2_poly_coefficients(d)


@pytest.mark.parametrize("d,alpha", [(1, 0.5), (3, 1.0), (2, 2.5)])
def test_weighted_minimises_quadrature_cost(d, alpha):
    c = np.array([float(v) for v in orc.weighted_l2_poly_coefficients(d, alpha)])

    def cost(cc):
        return quad(lambda z: z ** alpha * (1 - z * orc.poly_eval(cc, z)) ** 2, 0, 1,
                    epsabs=1e-14, epsrel=1e-13)[0]

    base = cost(c)
    for j in range(d + 1):
        for eps in (1e-3, -1e-3):
            cc = c.copy()
            cc[j] += eps
            assert cost(cc) > base
    # weighting towards z = 1 improves the fit there relative to the unweighted design
    u = np.array([float(v) for v in orc.l2_poly_coefficients(d)])
    zz = np.linspace(0.9, 1.0, 101)
    assert np.mean(residual(c, zz) ** 2) < np.mean(residual(u, zz) ** 2)


def test_weighted_rejects_bad_alpha():
    with pytest.raises(ValueError):
        orc.weighted_l2_poly_coefficients(2, Fraction(-1))


@pytest.mark.parametrize("coef", [[1.0], [float(v) for v in orc.l2_poly_coefficients(3)]])
def test_pgd_lambda_zero_least_squares(coef):
    sens, mask, bn, scale = setup()
    a = dense_forward(sens, mask) * np.sqrt(scale)
    x_ls = np.linalg.pinv(a) @ sampled(bn, mask)
    y, _ = orc.pgd(sens, mask, bn, scale, 0.0, coef, 2, 1500)
    assert np.linalg.norm(y.ravel() - x_ls) <= 1e-8 * np.linalg.norm(x_ls)


def test_pgd_fixed_point_and_error_factor():
    sens, mask, bn, scale = setup()
    lam, lv = 2e-3, 2
    y, hist = orc.pgd(sens, mask, bn, scale, lam, [1.0], lv, 3000, history=True)
    ahb = np.sqrt(scale) * orc.adjoint(sens, mask, bn)
    fp = orc.prox_l1_haar(y - (orc.normal(sens, mask, y, scale) - ahb), lam, lv)
    assert np.linalg.norm(fp - y) <= 1e-10 * np.linalg.norm(y)
    # PGD decreases the objective monotonically (unit step <= 1/L)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
    mu, v = np.linalg.eigh(dense_normal(sens, mask, scale))
    e = v[:, 10].reshape(1, 8, 8)
    e1 = e - orc.normal(sens, mask, e, scale)
    np.testing.assert_allclose(e1, (1 - mu[10]) * e, atol=1e-12)
