"""Pins of the oracle's reverse-mode derivatives through unrolled PFISTA (CPU).

Every pull-back is checked against central finite differences of the FP64
forward map (the definition of the derivative), on directions and cotangents
drawn at random; the polynomial part also against its closed form for one
step at lambda = 0 (x_1 = p(N') A'^H b', linear in c).
"""

import numpy as np
import pytest

import oracle as orc
from tests.test_oracle_solve import setup


def rdot(a, b):
    return float(np.real(np.vdot(a, b)))


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_soft_threshold_vjp_against_finite_differences():
    rng = np.random.default_rng(1)
    u = crandn(rng, (400,))
    lam = 0.9
    keep = np.abs(u) > lam
    u = np.where(np.abs(np.abs(u) - lam) < 1e-3, u * 1.01, u)   # stay off the kink
    w_bar, du = crandn(rng, u.shape), crandn(rng, u.shape)
    u_bar, lam_bar = orc.soft_threshold_vjp(u, w_bar, lam)
    h = 1e-6
    fd = (orc.soft_threshold(u + h * du, lam) - orc.soft_threshold(u - h * du, lam)) / (2 * h)
    assert rdot(u_bar, du) == pytest.approx(rdot(w_bar, fd), rel=1e-8)
    fdl = (orc.soft_threshold(u, lam + h) - orc.soft_threshold(u, lam - h)) / (2 * h)
    assert lam_bar == pytest.approx(rdot(w_bar, fdl), rel=1e-8)
    assert np.all(u_bar[~keep] == 0) and 0 < keep.sum() < u.size


def test_soft_threshold_vjp_factors():
    # radial component passes with factor 1, tangential with 1 - lam/|u|
    u = np.array([3.0 + 4.0j])
    lam = 1.0
    rad, tan = u / 5.0, 1j * u / 5.0
    assert orc.soft_threshold_vjp(u, rad, lam)[0] == pytest.approx(rad)
    assert orc.soft_threshold_vjp(u, tan, lam)[0] == pytest.approx(tan * (1 - 1 / 5))
    assert orc.soft_threshold_vjp(u, rad, lam)[1] == pytest.approx(-1.0)
    assert orc.soft_threshold_vjp(np.array([0.5j]), rad, lam)[0][0] == 0


def test_prox_vjp_against_finite_differences():
    rng = np.random.default_rng(2)
    v = crandn(rng, (2, 16, 16))
    lam, levels = 0.7, 3
    x_bar, dv = crandn(rng, v.shape), crandn(rng, v.shape)
    v_bar, lam_bar = orc.prox_l1_haar_vjp(v, x_bar, lam, levels)
    h = 1e-6
    fd = (orc.prox_l1_haar(v + h * dv, lam, levels) - orc.prox_l1_haar(v - h * dv, lam, levels)) / (2 * h)
    assert rdot(v_bar, dv) == pytest.approx(rdot(x_bar, fd), rel=1e-7)
    fdl = (orc.prox_l1_haar(v, lam + h, levels) - orc.prox_l1_haar(v, lam - h, levels)) / (2 * h)
    assert lam_bar == pytest.approx(rdot(x_bar, fdl), rel=1e-7)


def test_poly_vjp_is_the_adjoint_of_the_polynomial():
    sens, mask, bn, scale = setup()
    rng = np.random.default_rng(3)
    g, v_bar = crandn(rng, (1, 8, 8)), crandn(rng, (1, 8, 8))
    coef = [float(c) for c in orc.l2_poly_coefficients(3)]
    pv, c_bar = orc.poly_vjp(sens, mask, scale, coef, g, v_bar)
    # <p(N') v_bar, g> = <v_bar, p(N') g>  (p(N') Hermitian)
    assert rdot(pv, g) == pytest.approx(rdot(v_bar, orc.poly_apply(sens, mask, scale, coef, g)), rel=1e-12)
    # v = -p(N') g is linear in c: the derivative is exact
    for i in range(4):
        e = [0.0] * 4
        e[i] = 1.0
        assert c_bar[i] == pytest.approx(-rdot(v_bar, orc.poly_apply(sens, mask, scale, e, g)), rel=1e-12)


def test_one_step_at_lambda_zero_closed_form():
    # K = 1, lam = 0: x_1 = p(N') a with a = A'^H b', so dL/dc_i = Re <x_bar, N'^i a>
    sens, mask, bn, scale = setup()
    rng = np.random.default_rng(4)
    x_bar = crandn(rng, (1, 8, 8))
    coef = [float(c) for c in orc.l2_poly_coefficients(2)]
    _, c_bar = orc.unrolled_vjp(sens, mask, bn, scale, 0.0, coef, 2, 1, x_bar)
    a = np.sqrt(scale) * orc.adjoint(sens, mask, bn)
    q = a
    for i in range(3):
        assert c_bar[i] == pytest.approx(rdot(x_bar, q), rel=1e-10)
        q = orc.normal(sens, mask, q, scale)


def _loss(params, x_bar, momentum, levels, iters):
    sens, mask, bn, scale = setup()
    lam, coef = params[0], list(params[1:])
    x, _ = orc.unrolled_forward(sens, mask, bn, scale, lam, coef, levels, iters, momentum)
    return rdot(x_bar, x)


@pytest.mark.parametrize("degree,momentum,iters", [(3, True, 8), (0, True, 6), (2, False, 7), (1, True, 12)])
def test_unrolled_vjp_against_finite_differences(degree, momentum, iters):
    sens, mask, bn, scale = setup()
    rng = np.random.default_rng(10 + degree)
    x_bar = crandn(rng, (1, 8, 8))
    lam, levels = 3e-3, 2
    coef = [1.0] if degree == 0 else [float(c) for c in orc.l2_poly_coefficients(degree)]
    lam_bar, c_bar = orc.unrolled_vjp(sens, mask, bn, scale, lam, coef, levels, iters, x_bar, momentum)
    theta = np.array([lam] + coef)
    grad = np.concatenate([[lam_bar], c_bar])
    for j in range(theta.size):
        fds = []
        # steps small enough not to cross a threshold kink (the closest
        # coefficient sits ~2e-7 from lambda in these cases), large enough for
        # round-off: lambda moves the threshold directly, c_j only through u
        for rh in ((2e-6, 1e-6) if j == 0 else (2e-8, 1e-8)):
            h = rh * max(abs(theta[j]), 1e-3)
            tp, tm = theta.copy(), theta.copy()
            tp[j] += h
            tm[j] -= h
            fds.append((_loss(tp, x_bar, momentum, levels, iters) - _loss(tm, x_bar, momentum, levels, iters)) / (2 * h))
        scale_g = max(1.0, float(np.abs(grad).max()))
        assert fds[0] == pytest.approx(fds[1], rel=1e-5, abs=1e-8 * scale_g)     # smooth at this point
        assert grad[j] == pytest.approx(fds[1], rel=1e-5, abs=1e-8 * scale_g)


def test_unrolled_forward_is_the_solver():
    sens, mask, bn, scale = setup()
    coef = [float(c) for c in orc.l2_poly_coefficients(3)]
    x, _ = orc.unrolled_forward(sens, mask, bn, scale, 2e-3, coef, 2, 9)
    xs, _, _ = orc.pfista(sens, mask, bn, scale, 2e-3, coef, 2, 9)
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-14)
    y, _ = orc.unrolled_forward(sens, mask, bn, scale, 2e-3, coef, 2, 9, momentum=False)
    ys, _ = orc.pgd(sens, mask, bn, scale, 2e-3, coef, 2, 9)
    np.testing.assert_allclose(y, ys, rtol=0, atol=1e-14)
