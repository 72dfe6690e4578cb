"""Pins of the Haar transform, complex soft-threshold and the l1-Haar prox (CPU).

* Haar: a 4 x 4 two-level example worked by hand from the 2 x 2 block rule
  (LL, x-detail, y-detail, diagonal) = (a+b+c+d, a-b+c-d, a+b-c-d, a-b-c+d)/2;
  the one-level transform equals H x H^T with the textbook orthonormal Haar
  matrix H; perfect reconstruction and Parseval at every level count.
* Soft-threshold: closed-form values, and brute-force minimisation of
  1/2 |u - w|^2 + lam |u| over a grid (the definition of the proximal operator,
  Section 2.1).
* Prox: the optimality (subgradient) condition in the Haar domain and that no
  random perturbation lowers 1/2 ||x - v||^2 + lam ||Psi x||_1.
"""

import numpy as np
import pytest

import oracle as orc


def test_haar_hand_example_two_levels():
    x = np.arange(1, 17, dtype=float).reshape(4, 4)
    want = np.array([[34, -4, -1, -1],
                     [-16, 0, -1, -1],
                     [-4, -4, 0, 0],
                     [-4, -4, 0, 0]], dtype=float)
    np.testing.assert_allclose(orc.haar_fwd(x, 2).real, want, atol=1e-12)
    np.testing.assert_allclose(orc.haar_inv(want.astype(complex), 2).real, x, atol=1e-12)


def test_haar_2x2_block_rule():
    a, b, c, d = 1.0 + 2j, -0.5j, 3.0, 0.25 - 1j
    w = orc.haar_fwd(np.array([[a, b], [c, d]]), 1)
    np.testing.assert_allclose(w, np.array([[a + b + c + d, a - b + c - d],
                                            [a + b - c - d, a - b - c + d]]) / 2, atol=1e-15)


def haar_matrix(n):
    h = np.zeros((n, n))
    for i in range(n // 2):
        h[i, 2 * i] = h[i, 2 * i + 1] = np.sqrt(0.5)
        h[n // 2 + i, 2 * i] = np.sqrt(0.5)
        h[n // 2 + i, 2 * i + 1] = -np.sqrt(0.5)
    return h


@pytest.mark.parametrize("n", [2, 8, 16])
def test_haar_one_level_is_separable_matrix(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    h = haar_matrix(n)
    np.testing.assert_allclose(orc.haar_fwd(x, 1), h @ x @ h.T, atol=1e-12)


def test_haar_multilevel_recurses_on_low_band():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    w = orc.haar_fwd(x, 1)
    w[:8, :8] = orc.haar_fwd(w[:8, :8], 2)
    np.testing.assert_allclose(orc.haar_fwd(x, 3), w, atol=1e-12)


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_haar_orthonormal(levels):
    rng = np.random.default_rng(levels)
    x = rng.standard_normal((2, 32, 32)) + 1j * rng.standard_normal((2, 32, 32))
    w = orc.haar_fwd(x, levels)
    assert np.linalg.norm(w) == pytest.approx(np.linalg.norm(x), rel=1e-13)
    np.testing.assert_allclose(orc.haar_inv(w, levels), x, atol=1e-12)
    y = rng.standard_normal((2, 32, 32)) + 1j * rng.standard_normal((2, 32, 32))
    assert np.vdot(orc.haar_fwd(y, levels), w) == pytest.approx(np.vdot(y, x), rel=1e-12)


def test_soft_threshold_closed_form():
    w = np.array([3 + 4j, 0.5j, 0.0, 1.0, -2.0, 1e-300])
    got = orc.soft_threshold(w, 1.0)
    np.testing.assert_allclose(got, [2.4 + 3.2j, 0, 0, 0, -1.0, 0], atol=1e-15)


def test_soft_threshold_is_prox_by_brute_force():
    lam = 0.7
    g = np.linspace(-3, 3, 1201)
    ur, ui = np.meshgrid(g, g, indexing="ij")
    u = ur + 1j * ui
    for w in (2 + 1j, -0.3 + 0.5j, 0.4 - 2.5j, 0.6j):
        cost = 0.5 * np.abs(u - w) ** 2 + lam * np.abs(u)
        best = u.ravel()[np.argmin(cost)]
        assert abs(best - orc.soft_threshold(np.array([w]), lam)[0]) < 2 * (g[1] - g[0])


def test_prox_optimality_condition_and_no_better_point():
    rng = np.random.default_rng(5)
    v = rng.standard_normal((1, 16, 16)) + 1j * rng.standard_normal((1, 16, 16))
    lam, lv = 0.8, 3
    x = orc.prox_l1_haar(v, lam, lv)
    w, u = orc.haar_fwd(v, lv), orc.haar_fwd(x, lv)
    on = np.abs(u) > 1e-9          # exact zeros come back as round-off
    np.testing.assert_allclose((w - u)[on], lam * u[on] / np.abs(u[on]), atol=1e-12)
    assert np.all(np.abs(w[~on]) <= lam + 1e-12)

    def cost(y):
        return 0.5 * np.linalg.norm(y - v) ** 2 + lam * np.sum(np.abs(orc.haar_fwd(y, lv)))

    base = cost(x)
    for _ in range(50):
        d = 1e-3 * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
        assert cost(x + d) >= base - 1e-12
