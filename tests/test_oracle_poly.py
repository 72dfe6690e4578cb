"""Pins of the L2-optimal polynomial and its Horner application (CPU only).

The coefficients are checked against a second, independent route: the minimiser
of int_0^1 r(z)^2 dz over degree-(d+1) polynomials with r(0) = 1 is the
normalised reproducing kernel of the shifted Legendre basis,
``r(z) = sum_{k<=d+1} (-1)^k (2k+1) P~_k(z) / (d+2)^2``, and ``p = (1 - r) / z``
(Section 2.5, the L2 polynomial cost).  Corollaries: optimal cost 1/(d+2)^2,
``c_0 = (d+1)(d+3)/2`` and ``r(1) = (-1)^(d+1)/(d+2)``.  Positivity on (0, 1] is
the paper's Polynomial Positivity theorem.  The Horner application is checked
against the spectral definition p(N) = V diag(p(mu)) V^H on a dense tiny N, which
also reproduces the per-eigenvalue error factors plotted in the paper's Fig. 1,
and against the permutability lemma A^H p(A A^H) = p(A^H A) A^H.
"""

from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle as orc
from tests.tiny import dense_forward, dense_normal, tiny_problem

DEGREES = range(0, 7)


def shifted_legendre(k):
    # P~_k(z) = sum_j (-1)^(k+j) C(k, j) C(k+j, j) z^j  on [0, 1]
    return [Fraction((-1) ** (k + j) * comb(k, j) * comb(k + j, j)) for j in range(k + 1)]


def legendre_route(d):
    m = d + 1
    r = [Fraction(0)] * (m + 1)
    for k in range(m + 1):
        for j, a in enumerate(shifted_legendre(k)):
            r[j] += (-1) ** k * (2 * k + 1) * a
    r = [v / (d + 2) ** 2 for v in r]
    assert r[0] == 1
    return [-r[j + 1] for j in range(d + 1)]


def exact_cost(c):
    # int_0^1 (1 - z q(z))^2 dz with q = sum c_j z^j, expanded term by term
    d = len(c) - 1
    val = Fraction(1)
    val -= 2 * sum(c[j] / (j + 2) for j in range(d + 1))
    val += sum(c[i] * c[j] / (i + j + 3) for i in range(d + 1) for j in range(d + 1))
    return val


@pytest.mark.parametrize("d", DEGREES)
def test_coefficients_match_legendre_route(d):
    assert orc.l2_poly_coefficients(d) == legendre_route(d)


@pytest.mark.parametrize("d", DEGREES)
def test_coefficient_corollaries(d):
    c = orc.l2_poly_coefficients(d)
    assert c[0] == Fraction((d + 1) * (d + 3), 2)
    assert exact_cost(c) == Fraction(1, (d + 2) ** 2)
    r1 = 1 - sum(c)                                  # r(1) = 1 - p(1)
    assert r1 == Fraction((-1) ** (d + 1), d + 2)


def test_low_degree_values():
    assert orc.l2_poly_coefficients(0) == [Fraction(3, 2)]
    assert orc.l2_poly_coefficients(1) == [Fraction(4), Fraction(-10, 3)]


@pytest.mark.parametrize("d", DEGREES)
def test_cost_is_a_minimum(d):
    c = orc.l2_poly_coefficients(d)
    base = exact_cost(c)
    for j in range(d + 1):
        for eps in (Fraction(1, 1000), Fraction(-1, 1000)):
            cc = list(c)
            cc[j] += eps
            assert exact_cost(cc) > base


@pytest.mark.parametrize("d", DEGREES)
def test_polynomial_positive_on_unit_interval(d):
    z = np.linspace(1e-6, 1.0, 200001)
    assert orc.poly_eval(orc.l2_poly_coefficients(d), z).min() > 0


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_horner_equals_spectral_polynomial(d):
    _, sens, mask, _ = tiny_problem(n=8, coils=2, seed=11)
    scale = 1.0 / 1.01
    nm = dense_normal(sens, mask, scale)
    mu, v = np.linalg.eigh(nm)
    c = orc.l2_poly_coefficients(d)
    pn = v @ np.diag(orc.poly_eval(c, mu)) @ v.conj().T
    rng = np.random.default_rng(d)
    g = rng.standard_normal((1, 8, 8)) + 1j * rng.standard_normal((1, 8, 8))
    got = orc.poly_apply(sens, mask, scale, c, g)
    np.testing.assert_allclose(got.ravel(), pn @ g.ravel(), atol=1e-11 * (1 + np.abs(pn).max()))
    # eigenvalues of p(N)N are p(mu) mu (the abscissa of the paper's Fig. 1)
    pnn = np.stack([orc.poly_apply(sens, mask, scale, c,
                                   orc.normal(sens, mask, e.reshape(1, 8, 8), scale)).ravel()
                    for e in np.eye(64, dtype=np.complex128)], axis=1)
    np.testing.assert_allclose(np.sort(np.linalg.eigvals(pnn).real),
                               np.sort(orc.poly_eval(c, mu) * mu), atol=1e-10)


def test_fig1_error_factors_after_four_applications():
    # With lambda = 0 and b = A x*, PGD contracts the error along eigenvector
    # v_i by (1 - mu_i) per A^H A; PPGD with d = 3 contracts it by
    # (1 - p(mu_i) mu_i) per iteration = per 4 applications.
    img, sens, mask, _ = tiny_problem(n=8, coils=2, seed=13)
    nm = dense_normal(sens, mask)
    mu, v = np.linalg.eigh(nm)
    c = orc.l2_poly_coefficients(3)
    for i in (5, 30, 63):
        e = v[:, i].reshape(1, 8, 8)
        # one PPGD error update: e <- e - p(N) N e
        e1 = e - orc.poly_apply(sens, mask, 1.0, c, orc.normal(sens, mask, e))
        f = 1.0 - float(orc.poly_eval(c, mu[i])) * mu[i]
        np.testing.assert_allclose(e1, f * e, atol=1e-11)
        # four PGD updates: e <- e - N e
        e4 = e
        for _ in range(4):
            e4 = e4 - orc.normal(sens, mask, e4)
        np.testing.assert_allclose(e4, (1 - mu[i]) ** 4 * e, atol=1e-11)


def test_permutability_lemma():
    _, sens, mask, _ = tiny_problem(n=6, coils=2, seed=17)
    a = dense_forward(sens, mask)
    c = [float(v) for v in orc.l2_poly_coefficients(3)]
    aah = a @ a.conj().T
    p_aah = sum(ci * np.linalg.matrix_power(aah, i) for i, ci in enumerate(c))
    rng = np.random.default_rng(3)
    y = rng.standard_normal(a.shape[0]) + 1j * rng.standard_normal(a.shape[0])
    lhs = a.conj().T @ (p_aah @ y)
    ahy = (a.conj().T @ y).reshape(1, 6, 6)
    rhs = orc.poly_apply(sens, mask, 1.0, c, ahy).ravel()
    np.testing.assert_allclose(rhs, lhs, atol=1e-11)
