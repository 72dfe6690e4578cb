"""Pin of the momentum sequence of Algorithms 2 and 4 (and its absence in
Algorithms 1 and 3) with iterates worked out by hand.

The problem is one 2 x 2 image, one coil with S = 1, every k-space point
sampled and ``N' = A'^H A' = I / 4`` (scale 1/4 on a unitary A), one Haar level,
``lambda = 1/10`` and the plain gradient step (``p = 1``).  The data are chosen
so that ``A'^H b' = u / 2`` with Haar coefficients ``Psi u = (3/5, 0, 0, 4i/5)``
(LL, x-detail, y-detail, diagonal; ``||u|| = 1``).  In Haar coordinates the
problem is diagonal: each coefficient follows

    nu_k = zeta_k - (zeta_k / 4 - alpha) = (3/4) zeta_k + alpha
    u_(k+1) = soft(nu_k, 1/10)     (magnitude minus 1/10; both stay above it)
    zeta_(k+1) = u_(k+1) + beta_k (u_(k+1) - u_k),    beta_k = k / (k + 3)

from ``u_0 = zeta_0 = 0``, with alpha = 3/10 for LL and 4i/10 for the diagonal.
Worked by hand in exact fractions (beta = 0, 1/4, 2/5, 1/2, 4/7):

    LL:   1/5, 7/20, 157/320, 781/1280, 7193/10240
    diag: i (3/10, 21/40, 471/640, 2343/2560, 21579/20480)

Without momentum (Algorithms 1 and 3, ``beta = 0``):

    LL:   1/5, 7/20, 37/80, 35/64, 781/1280
    diag: i (3/10, 21/40, 111/160, 105/128, 2343/2560)

A schedule shifted by one step (``(k+1)/(k+4)``) gives LL_2 = 31/80, and the
update printed in the algorithms (``z_(k+1) = x_k + beta_k (x_k - x_(k-1))``)
gives x_2 = x_1; both fail below.  Pixels follow from the 2 x 2 Haar synthesis
``[[ll + d, ll - d], [ll - d, ll + d]] / 2`` (x- and y-details are zero).

Every solver of the oracle is run on this problem: the Cartesian ``pfista``
(also resumed mid-way), ``pgd``, the non-Cartesian ``pfista_nc`` on the integer
grid (where the non-uniform DFT is the unitary DFT), ``pfista_toeplitz`` with
the kernel of that grid, and ``unrolled_forward``.
"""

from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle as orc

LAM = 0.1
SCALE = 0.25
LL_FISTA = [Fr(1, 5), Fr(7, 20), Fr(157, 320), Fr(781, 1280), Fr(7193, 10240)]
DD_FISTA = [Fr(3, 10), Fr(21, 40), Fr(471, 640), Fr(2343, 2560), Fr(21579, 20480)]
LL_PGD = [Fr(1, 5), Fr(7, 20), Fr(37, 80), Fr(35, 64), Fr(781, 1280)]
DD_PGD = [Fr(3, 10), Fr(21, 40), Fr(111, 160), Fr(105, 128), Fr(2343, 2560)]


def pixels(ll, dd):
    """[1, 2, 2] image with Haar coefficients (ll, 0, 0, i dd)."""
    a = (float(ll) + 1j * float(dd)) / 2
    b = (float(ll) - 1j * float(dd)) / 2
    return np.array([[[a, b], [b, a]]])


def problem():
    u = pixels(Fr(3, 5), Fr(4, 5))                 # ||u|| = 1
    sens = np.ones((1, 1, 2, 2), complex)
    mask = np.ones((1, 2, 2), np.uint8)
    bn = orc.fft2u(u)[:, None]                     # b' = F u, ||b'|| = 1
    return u, sens, mask, bn


def test_hand_problem_is_what_the_docstring_says():
    u, sens, mask, bn = problem()
    assert np.linalg.norm(bn) == pytest.approx(1.0, abs=1e-15)
    w = orc.haar_fwd(u, 1)[0]
    np.testing.assert_allclose(w, [[0.6, 0.0], [0.0, 0.8j]], atol=1e-15)
    np.testing.assert_allclose(orc.normal(sens, mask, u, SCALE), u / 4, atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_pfista_iterates_equal_hand_values(k):
    _, sens, mask, bn = problem()
    x, _, _ = orc.pfista(sens, mask, bn, SCALE, LAM, [1.0], 1, k)
    np.testing.assert_allclose(x, pixels(LL_FISTA[k - 1], DD_FISTA[k - 1]), rtol=0, atol=1e-14)


def test_pfista_resumed_mid_way_reaches_the_same_hand_value():
    _, sens, mask, bn = problem()
    x2, z2, _ = orc.pfista(sens, mask, bn, SCALE, LAM, [1.0], 1, 2)
    x5, _, _ = orc.pfista(sens, mask, bn, SCALE, LAM, [1.0], 1, 3, x0=x2, z0=z2, k0=2)
    np.testing.assert_allclose(x5, pixels(LL_FISTA[4], DD_FISTA[4]), rtol=0, atol=1e-14)


@pytest.mark.parametrize("k", [3, 5])
def test_pgd_iterates_equal_hand_values(k):
    _, sens, mask, bn = problem()
    y, _ = orc.pgd(sens, mask, bn, SCALE, LAM, [1.0], 1, k)
    np.testing.assert_allclose(y, pixels(LL_PGD[k - 1], DD_PGD[k - 1]), rtol=0, atol=1e-14)


def _grid_traj():
    return np.array([[kx, ky] for ky in range(2) for kx in range(2)], dtype=np.float64)


def test_noncartesian_solvers_follow_the_same_hand_values():
    u, sens, _, _ = problem()
    traj = _grid_traj()
    bn = orc.nudft_forward(sens, traj[None], u)
    assert np.linalg.norm(bn) == pytest.approx(1.0, abs=1e-14)
    x, _, _ = orc.pfista_nc(sens, traj[None], bn, SCALE, LAM, [1.0], 1, 5)
    np.testing.assert_allclose(x, pixels(LL_FISTA[4], DD_FISTA[4]), rtol=0, atol=1e-14)
    kern = orc.toeplitz_kernel(traj, 2)[None]
    ahb = orc.nudft_adjoint(sens, traj[None], bn)
    x = orc.pfista_toeplitz(sens, kern, ahb, 1.0, SCALE, LAM, [1.0], 1, 4)
    np.testing.assert_allclose(x, pixels(LL_FISTA[3], DD_FISTA[3]), rtol=0, atol=1e-13)


def test_unrolled_forward_follows_the_same_hand_values():
    _, sens, mask, bn = problem()
    x, tape = orc.unrolled_forward(sens, mask, bn, SCALE, LAM, [1.0], 1, 5)
    np.testing.assert_allclose(x, pixels(LL_FISTA[4], DD_FISTA[4]), rtol=0, atol=1e-14)
    assert [t[3] for t in tape] == pytest.approx([0.0, 0.25, 0.4, 0.5, 4.0 / 7.0], abs=1e-15)
    x, _ = orc.unrolled_forward(sens, mask, bn, SCALE, LAM, [1.0], 1, 4, momentum=False)
    np.testing.assert_allclose(x, pixels(LL_PGD[3], DD_PGD[3]), rtol=0, atol=1e-14)


def test_alternative_schedules_would_fail_the_pin():
    """Guards the pin itself: an index shift or the printed lagged update moves x_2."""
    assert Fr(31, 80) != LL_FISTA[1]
    _, sens, mask, bn = problem()
    ahb = SCALE ** 0.5 * orc.adjoint(sens, mask, bn)
    # printed form: z_(k+1) = x_k + beta_k (x_k - x_(k-1)), run with the oracle's prox
    x_prev = x = z = np.zeros_like(ahb)
    xs = []
    for k in range(2):
        x_new = orc.prox_l1_haar(z - (SCALE * z - ahb), LAM, 1)
        beta = k / (k + 3.0)
        z = x + beta * (x - x_prev)
        x_prev, x = x, x_new
        xs.append(x)
    np.testing.assert_allclose(xs[1], xs[0], atol=1e-15)
    assert not np.allclose(xs[1], pixels(LL_FISTA[1], DD_FISTA[1]), atol=1e-6)
