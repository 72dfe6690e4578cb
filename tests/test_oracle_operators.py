"""Pins of the oracle's forward model against definitions (CPU only).

* the unitary DFT against the DFT matrix written from its definition, at sizes
  that exercise radices 2, 3 and 5;
* the adjoint identity <A x, y> = <x, A^H y>;
* A^H A Hermitian positive semi-definite with spectrum in [0, 1] when the coil
  maps satisfy sum_c |S_c|^2 = 1 (Section 2 assumes unit induced norm);
* full sampling collapses A^H A to the identity (F unitary, sum |S|^2 = 1);
* the phase-encode mask: F^H M F acts only along y, the x-transform pair cancels.
"""

import numpy as np
import pytest

import oracle as orc
from synth import coil_sensitivities, mask_phase_encode_1d
from tests.tiny import dense_forward, dense_normal, sampled, tiny_problem


def dft_matrix(n):
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n) / np.sqrt(n)


@pytest.mark.parametrize("n", [4, 6, 8, 10, 12, 15])
def test_fft2u_is_the_unitary_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    f = dft_matrix(n)
    # 2-D DFT: X[k, l] = sum_{m, q} x[m, q] w^(k m + l q) / n
    ref = np.einsum("km,smq,lq->skl", f, x, f)
    np.testing.assert_allclose(orc.fft2u(x), ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(orc.ifft2u(ref), x, rtol=0, atol=1e-12)


def test_dft_sign_convention():
    # a pure tone exp(+2 pi i k0 m / n) lands in bin k0 under exp(-2 pi i k m / n)
    n, k0 = 8, 3
    m = np.arange(n)
    x = np.exp(2j * np.pi * k0 * m / n)[None, :] * np.ones((n, 1))
    X = orc.fft2u(x[None])[0]
    assert abs(X[0, k0]) == pytest.approx(n, rel=1e-12)
    assert np.sum(np.abs(X) > 1e-9) == 1


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_identity(seed):
    img, sens, mask, b = tiny_problem(n=12, coils=3, seed=seed)
    rng = np.random.default_rng(100 + seed)
    x = rng.standard_normal(img.shape) + 1j * rng.standard_normal(img.shape)
    y = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    lhs = np.vdot(y, orc.forward(sens, mask, x))
    rhs = np.vdot(orc.adjoint(sens, mask, y), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_forward_matches_explicit_sense_sum():
    # b_c[k] = sum_pixels S_c x exp(-2 pi i k.r / n) / n on sampled k only
    img, sens, mask, _ = tiny_problem(n=6, coils=2, seed=3)
    n = 6
    f = dft_matrix(n)
    m = orc.expand_mask(mask, n)[0]
    for c in range(2):
        ref = f @ (sens[0, c] * img[0]) @ f.T
        got = orc.forward(sens, mask, img)[0, c]
        np.testing.assert_allclose(got, np.where(m, ref, 0), atol=1e-13)


def test_normal_is_hermitian_psd_with_unit_bound():
    _, sens, mask, _ = tiny_problem(n=8, coils=2, seed=5)
    nm = dense_normal(sens, mask)
    np.testing.assert_allclose(nm, nm.conj().T, atol=1e-13)
    mu = np.linalg.eigvalsh(nm)
    assert mu.min() > -1e-12 and mu.max() < 1 + 1e-12
    a = dense_forward(sens, mask)
    np.testing.assert_allclose(nm, a.conj().T @ a, atol=1e-13)


def test_full_sampling_gives_identity():
    n, coils = 8, 3
    sens = coil_sensitivities(n, coils, np.random.default_rng(1))[None]
    mask = np.ones((1, n, n), dtype=np.uint8)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))
    np.testing.assert_allclose(orc.normal(sens, mask, x), x, atol=1e-13)


def test_phase_encode_mask_needs_only_column_transforms():
    n, coils = 12, 2
    rng = np.random.default_rng(4)
    sens = coil_sensitivities(n, coils, rng)[None]
    m1 = mask_phase_encode_1d(n, 4, 2, rng)[None]
    x = rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))
    f = dft_matrix(n)
    proj = f.conj().T @ np.diag(m1[0].astype(float)) @ f      # along y only
    ref = sum(np.conj(sens[0, c]) * (proj @ (sens[0, c] * x[0])) for c in range(coils))
    np.testing.assert_allclose(orc.normal(sens, m1, x)[0], ref, atol=1e-13)


def test_kspace_data_is_zero_off_mask_and_noise_on_mask():
    img, sens, mask, b = tiny_problem(n=8, coils=2, seed=9, sigma=0.0)
    m = orc.expand_mask(mask, 8)
    assert np.all(b[:, :, ~m[0]] == 0)
    np.testing.assert_allclose(sampled(b, mask),
                               dense_forward(sens, mask) @ img.ravel(), atol=1e-13)


def test_power_iteration_finds_largest_eigenvalue():
    # one phase-only coil: A^H A = S^H F^H M F S is an orthogonal projection,
    # so from the second iteration on the estimate is exactly 1
    n = 8
    rng = np.random.default_rng(3)
    sens = coil_sensitivities(n, 1, rng)[None]
    _, _, mask, _ = tiny_problem(n=n, coils=1, seed=5)
    v0 = rng.standard_normal((1, n, n)) + 0j
    assert orc.power_iteration(sens, mask, v0, 3) == pytest.approx(1.0, abs=1e-13)
    # general maps: a lower bound of the top eigenvalue that converges to it
    _, sens, mask, _ = tiny_problem(n=8, coils=2, seed=5)
    mu = np.linalg.eigvalsh(dense_normal(sens, mask)).max()
    est = orc.power_iteration(sens, mask, v0, 300)
    assert mu * (1 - 1e-3) <= est <= mu * (1 + 1e-13)
