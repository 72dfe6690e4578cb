"""Tiny dense problems for pinning the oracle (CPU only)."""

import numpy as np

import oracle as orc
from synth import coil_sensitivities, complex_noise, mask_variable_density, phantom


def tiny_problem(n=8, coils=2, accel=2.0, centre=2, seed=7, sigma=1e-2):
    rng = np.random.default_rng(seed)
    img = phantom(n, rng, n_random=3)[None]
    sens = coil_sensitivities(n, coils, rng)[None]
    if accel < 2.0:
        # well-conditioned tiny case: uniform random sampling at rate 1/accel
        keep = rng.permutation(n * n)[: int(round(n * n / accel))]
        mask = np.zeros((1, n * n), dtype=np.uint8)
        mask[0, keep] = 1
        mask = mask.reshape(1, n, n)
    else:
        mask = mask_variable_density(n, accel, centre, rng)[None]
    noise = complex_noise((1, coils, n, n), sigma, rng)
    b = orc.kspace_data(sens, mask, img, noise)
    return img, sens, mask, b


def dense_forward(sens, mask):
    """Matrix of ``orc.forward`` restricted to sampled k-space points."""
    n = sens.shape[-1]
    m = orc.expand_mask(mask, n)[0]
    rows = []
    for j in range(n * n):
        e = np.zeros((1, n, n), dtype=np.complex128)
        e.ravel()[j] = 1.0
        rows.append(orc.forward(sens, mask, e)[0][:, m])
    return np.stack([r.ravel() for r in rows], axis=1)


def dense_normal(sens, mask, scale=1.0):
    n = sens.shape[-1]
    cols = []
    for j in range(n * n):
        e = np.zeros((1, n, n), dtype=np.complex128)
        e.ravel()[j] = 1.0
        cols.append(orc.normal(sens, mask, e, scale).ravel())
    return np.stack(cols, axis=1)


def sampled(b, mask):
    n = b.shape[-1]
    m = orc.expand_mask(mask, n)[0]
    return b[0][:, m].ravel()
