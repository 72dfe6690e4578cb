"""Pins of the oracle's FISTA / PFISTA iteration (Algorithms 2 and 4), CPU only.

* lambda = 0: both iterations converge to the minimum-norm least-squares
  solution pinv(A') b' (Section 2.8: without regularisation the preconditioner
  changes no solution), checked against a dense pseudo-inverse;
* lambda > 0: the FISTA limit satisfies the fixed-point theorem of PGD, and
  the PFISTA limit the preconditioned fixed point of Section 2.4;
* the error bound of Section 2.6, ||y_inf - x*|| <= delta / (1 - gamma), with
  gamma and delta from a dense eigendecomposition;
* resume: 50 steps equal 25 steps then 25 resumed steps, bit for bit;
* the literal degree-0 fit p = 3/2 with momentum diverges once the top
  eigenvalue of N' exceeds 8/9, which the stability reading relies on.
"""

import numpy as np
import pytest

import oracle as orc
from tests.tiny import dense_forward, dense_normal, sampled, tiny_problem


def setup(n=8, coils=3, accel=1.6, seed=21, sigma=1e-2):
    img, sens, mask, b = tiny_problem(n=n, coils=coils, accel=accel, centre=2, seed=seed,
                                      sigma=sigma)
    lmax = np.linalg.eigvalsh(dense_normal(sens, mask)).max()
    bn, _, scale = orc.normalise(b, 1.01 * lmax)
    return sens, mask, bn, scale


@pytest.mark.parametrize("d", [None, 1, 3])
def test_lambda_zero_converges_to_least_squares(d):
    sens, mask, bn, scale = setup()
    a = dense_forward(sens, mask) * np.sqrt(scale)
    x_ls = np.linalg.pinv(a) @ sampled(bn, mask)
    coef = [1.0] if d is None else orc.l2_poly_coefficients(d)
    x, _, _ = orc.pfista(sens, mask, bn, scale, 0.0, coef, 2, 1000)
    assert np.linalg.norm(x.ravel() - x_ls) <= 1e-8 * np.linalg.norm(x_ls)


def test_fista_limit_satisfies_pgd_fixed_point():
    sens, mask, bn, scale = setup()
    lam, lv = 2e-3, 2
    x, _, _ = orc.pfista(sens, mask, bn, scale, lam, [1.0], lv, 3000)
    ahb = np.sqrt(scale) * orc.adjoint(sens, mask, bn)
    fp = orc.prox_l1_haar(x - (orc.normal(sens, mask, x, scale) - ahb), lam, lv)
    assert np.linalg.norm(fp - x) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("d", [1, 3])
def test_pfista_limit_satisfies_preconditioned_fixed_point(d):
    sens, mask, bn, scale = setup()
    lam, lv = 2e-3, 2
    c = orc.l2_poly_coefficients(d)
    y, _, _ = orc.pfista(sens, mask, bn, scale, lam, c, lv, 1500)
    ahb = np.sqrt(scale) * orc.adjoint(sens, mask, bn)
    g = orc.normal(sens, mask, y, scale) - ahb
    fp = orc.prox_l1_haar(y - orc.poly_apply(sens, mask, scale, c, g), lam, lv)
    assert np.linalg.norm(fp - y) <= 1e-10 * np.linalg.norm(y)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_error_bound_theorem(d):
    sens, mask, bn, scale = setup()
    lam, lv = 2e-3, 2
    nm = dense_normal(sens, mask, scale)
    mu, v = np.linalg.eigh(nm)
    assert mu.min() > 1e-3                         # injective, as the theorem assumes
    c = orc.l2_poly_coefficients(d)
    pmu = orc.poly_eval(c, mu)
    gamma = np.max(np.abs(1 - pmu * mu))
    x_star, _, _ = orc.pfista(sens, mask, bn, scale, lam, [1.0], lv, 3000)
    ahb = np.sqrt(scale) * orc.adjoint(sens, mask, bn)
    r = (orc.normal(sens, mask, x_star, scale) - ahb).ravel()
    i_minus_p = v @ np.diag(1 - pmu) @ v.conj().T
    delta = np.linalg.norm(i_minus_p @ r)
    y_inf, _, _ = orc.pfista(sens, mask, bn, scale, lam, c, lv, 1500)
    assert gamma < 1
    assert np.linalg.norm(y_inf - x_star) <= delta / (1 - gamma)


def test_resume_is_bitwise():
    sens, mask, bn, scale = setup()
    c = orc.l2_poly_coefficients(2)
    x50, z50, _ = orc.pfista(sens, mask, bn, scale, 1e-3, c, 2, 50)
    x25, z25, _ = orc.pfista(sens, mask, bn, scale, 1e-3, c, 2, 25)
    xr, zr, _ = orc.pfista(sens, mask, bn, scale, 1e-3, c, 2, 25, x0=x25, z0=z25, k0=25)
    assert np.array_equal(x50, xr) and np.array_equal(z50, zr)


def test_objective_history_and_minimum():
    # F(0) = 1/2 since ||b'|| = 1; the FISTA limit minimises F, so no PFISTA
    # iterate (whose limit solves the preconditioned problem) goes below it
    sens, mask, bn, scale = setup()
    lam, lv = 2e-3, 2
    _, _, hist = orc.pfista(sens, mask, bn, scale, lam, orc.l2_poly_coefficients(3), lv, 60,
                            history=True)
    f0 = orc.objective(sens, mask, bn, scale, np.zeros_like(sens[:, 0]), lam, lv)
    assert f0 == pytest.approx(0.5, rel=1e-12)
    x_star, _, _ = orc.pfista(sens, mask, bn, scale, lam, [1.0], lv, 3000)
    f_star = orc.objective(sens, mask, bn, scale, x_star, lam, lv)
    assert min(hist) >= f_star * (1 - 1e-12)
    assert hist[-1] < 0.1 * f0 and hist[-1] <= f_star * 1.05   # limits differ (Section 2.6)


def test_literal_degree_zero_fit_diverges_with_momentum():
    sens, mask, bn, _ = setup()
    lmax = np.linalg.eigvalsh(dense_normal(sens, mask)).max()
    scale = 1.0 / lmax                            # top eigenvalue of N' is exactly 1
    _, _, hist = orc.pfista(sens, mask, bn, scale, 1e-3, [1.5], 2, 150, history=True)
    assert not np.isfinite(hist[-1]) or hist[-1] > 10 * 0.5
    _, _, ok = orc.pfista(sens, mask, bn, scale, 1e-3, [1.0], 2, 150, history=True)
    assert ok[-1] < 0.5
