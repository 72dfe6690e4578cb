"""Pins of the non-Cartesian oracle and its Toeplitz normal operator (CPU).

* the Toeplitz embedding (zero-pad to 2n, multiply by K, crop) equals the
  normal operator of the direct non-uniform DFT, with and without weights;
* on integer trajectories the non-uniform DFT is the unitary DFT of the
  Cartesian model, so the normal operator equals the Cartesian one for the
  mask of the same points, and the non-Cartesian PFISTA reproduces the
  Cartesian one;
* K is real, and equals the separable Dirichlet-kernel sum
  ``K(k) = (1/n^2) sum_j w_j D(kx_j/n - kx/2n) D(ky_j/n - ky/2n)``,
  ``D(t) = sin((2n-1) pi t) / sin(pi t)`` (the closed form of the DFT of h).
"""

import numpy as np
import pytest

import oracle as orc
from synth import coil_sensitivities, mask_variable_density, spiral_trajectory
from tests.test_oracle_solve import setup


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def case(n=8, coils=3, J=60, seed=0):
    rng = np.random.default_rng(seed)
    sens = coil_sensitivities(n, coils, rng)[None]
    traj = rng.uniform(-n / 2, n / 2, size=(1, J, 2))
    x = crandn(rng, (1, n, n))
    return sens, traj, x, rng


def test_toeplitz_equals_direct_nudft_normal():
    sens, traj, x, _ = case()
    kern = orc.toeplitz_kernel(traj[0], 8)[None]
    np.testing.assert_allclose(orc.toeplitz_normal(sens, kern, x), orc.nudft_normal(sens, traj, x),
                               rtol=0, atol=1e-12)


def test_weighted_kernel_is_the_weighted_normal_operator():
    sens, traj, x, rng = case(seed=1)
    w = rng.uniform(0.2, 2.0, size=traj.shape[1])
    kern = orc.toeplitz_kernel(traj[0], 8, w)[None]
    e = orc.nudft_matrix(traj[0], 8)
    want = np.sum(np.conj(sens[0]) * (e.conj().T @ (w[:, None] * (e @ (sens[0] * x[0]).reshape(3, 64).T)))
                  .T.reshape(3, 8, 8), axis=0)
    np.testing.assert_allclose(orc.toeplitz_normal(sens, kern, x)[0], want, rtol=0, atol=1e-12)


def test_kernel_is_real_and_the_dirichlet_sum():
    n = 8
    _, traj, _, rng = case(seed=2)
    w = rng.uniform(0.5, 1.5, size=traj.shape[1])
    k = orc.toeplitz_kernel(traj[0], n, w)
    assert np.abs(k.imag).max() <= 1e-12 * np.abs(k.real).max()

    def dirichlet(t):
        s = np.sin(np.pi * t)
        safe = np.where(np.abs(s) < 1e-12, 1.0, s)
        ratio = np.sin((2 * n - 1) * np.pi * t) / safe
        near = np.round(t)
        limit = (2 * n - 1) * np.cos(np.pi * (2 * n - 1) * near) / np.cos(np.pi * near)
        return np.where(np.abs(s) < 1e-12, limit, ratio)

    kk = np.arange(2 * n)
    dy = dirichlet(traj[0][:, 1][:, None] / n - kk[None, :] / (2 * n))       # [J, 2n]
    dx = dirichlet(traj[0][:, 0][:, None] / n - kk[None, :] / (2 * n))
    closed = (dy * w[:, None]).T @ dx / n ** 2
    np.testing.assert_allclose(k.real, closed, rtol=0, atol=1e-11 * np.abs(closed).max())


def test_on_grid_trajectory_is_the_cartesian_model():
    n = 8
    rng = np.random.default_rng(3)
    sens = coil_sensitivities(n, 2, rng)[None]
    mask = mask_variable_density(n, 2.0, 2, rng)[None]
    ky, kx = np.nonzero(mask[0])
    # integer points, some shifted by -n (the same DFT frequency)
    shift = rng.integers(0, 2, size=kx.size) * n
    traj = np.stack([kx - shift, ky], axis=1).astype(np.float64)[None]
    x = crandn(rng, (1, n, n))
    np.testing.assert_allclose(orc.nudft_normal(sens, traj, x), orc.normal(sens, mask, x), rtol=0, atol=1e-12)
    full = np.stack(np.meshgrid(np.arange(n), np.arange(n), indexing="xy"), axis=-1).reshape(-1, 2)
    e = orc.nudft_matrix(full.astype(np.float64), n)
    # full integer grid: E is unitary and matches the 2-D DFT entry by entry
    f = orc.fft2u(x[0])
    np.testing.assert_allclose(e @ x[0].ravel(), f[full[:, 1], full[:, 0]], rtol=0, atol=1e-12)
    np.testing.assert_allclose(e.conj().T @ e, np.eye(n * n), rtol=0, atol=1e-12)


def test_adjoint_identity():
    sens, traj, x, rng = case(seed=4)
    y = crandn(rng, (1, 3, traj.shape[1]))
    lhs = np.vdot(orc.nudft_forward(sens, traj, x), y)
    rhs = np.vdot(x, orc.nudft_adjoint(sens, traj, y))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_noncartesian_pfista_on_grid_matches_cartesian():
    sens, mask, bn, scale = setup()
    n = sens.shape[-1]
    ky, kx = np.nonzero(mask[0])
    traj = np.stack([kx, ky], axis=1).astype(np.float64)[None]
    bnc = bn[:, :, ky, kx]                                   # the same samples in trajectory order
    coef = [float(c) for c in orc.l2_poly_coefficients(2)]
    xc, _, hc = orc.pfista(sens, mask, bn, scale, 2e-3, coef, 2, 10, history=True)
    xn, _, hn = orc.pfista_nc(sens, traj, bnc, scale, 2e-3, coef, 2, 10, history=True)
    np.testing.assert_allclose(xn, xc, rtol=0, atol=1e-12)
    np.testing.assert_allclose(hn, hc, rtol=1e-12)


def test_spiral_trajectory_shape_and_extent():
    rng = np.random.default_rng(5)
    t = spiral_trajectory(64, 4, 100, 3.0, 1.5, rng)
    assert t.shape == (400, 2)
    r = np.hypot(t[:, 0], t[:, 1])
    assert r.max() == pytest.approx(32.0) and r.min() > 0
    # denser near the centre: more samples inside half the radius than its area share
    assert np.mean(r < 16) > 0.25


def test_toeplitz_solver_from_normal_equations_data():
    # the Toeplitz form of the solver (A^H b, ||b||) follows the direct one
    n = 8
    sens, traj, x, rng = case(n=n, coils=2, J=90, seed=6)
    b = orc.nudft_forward(sens, traj, x) + 0.01 * crandn(rng, (1, 2, 90))
    bn = b / np.linalg.norm(b)
    kern = orc.toeplitz_kernel(traj[0], n)[None]
    ahb = orc.nudft_adjoint(sens, traj, b)
    coef = [float(c) for c in orc.l2_poly_coefficients(2)]
    v = crandn(rng, x.shape)
    for _ in range(200):
        v = orc.nudft_normal(sens, traj, v)
        lam_max = np.linalg.norm(v)
        v /= lam_max
    scale = 1.0 / (1.01 * lam_max)
    xd, _, _ = orc.pfista_nc(sens, traj, bn, scale, 1e-3, coef, 2, 12)
    xt = orc.pfista_toeplitz(sens, kern, ahb, np.linalg.norm(b), scale, 1e-3, coef, 2, 12)
    assert np.linalg.norm(xd) > 0.1
    np.testing.assert_allclose(xt, xd, rtol=0, atol=1e-12)
