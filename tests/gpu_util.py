"""Helpers shared by the GPU parity tests (inputs, transfers, error metrics)."""

import numpy as np

import oracle as orc
from synth import coil_sensitivities, mask_phase_encode_1d, mask_variable_density

HORNER_PARTIAL_MAX = {0: 1.5, 1: 4.0, 2: 15.0, 3: 56.0, 4: 210.0, 5: 990.0}


def dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a GPU")
    return torch.device("cuda", 0)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def c64(a):
    """Round to complex64 and back: the exact values the GPU sees."""
    return np.asarray(a).astype(np.complex64)


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_case(n, coils, slices, kind, seed):
    """Coil maps (sum |S|^2 = 1), a mask and a random complex image per slice."""
    rng = np.random.default_rng(seed)
    sens = np.stack([coil_sensitivities(n, coils, rng) for _ in range(slices)])
    if kind == "1d":
        mask = np.stack([mask_phase_encode_1d(n, max(2, n // 12), max(1, n // 24), rng)
                         for _ in range(slices)])
    else:
        mask = np.stack([mask_variable_density(n, 4.0, max(2, n // 8), rng) for _ in range(slices)])
    x = rng.standard_normal((slices, n, n)) + 1j * rng.standard_normal((slices, n, n))
    w = rng.standard_normal((slices, n, n)) + 1j * rng.standard_normal((slices, n, n))
    return c64(sens), mask, c64(x), c64(w)


def oracle_normal(sens, mask, x, scale=1.0):
    return orc.normal(sens.astype(np.complex128), mask, x.astype(np.complex128), scale)
