"""Seeded synthetic inputs for SENSE reconstruction problems.

This package builds the *inputs* of the problem ``argmin 1/2 ||A x - b||^2 +
lam ||Psi x||_1`` (phantom image, coil sensitivities, sampling masks or
non-Cartesian trajectories, and measurement noise) and nothing else: it holds no Fourier transform, no forward
model, no wavelet and no solver step.  It is shared by the FP64 test oracle and
by the GPU path so that both see bit-identical inputs.  The k-space data
``b = M (F S x + noise)`` is formed by each side with its own forward model.

The workloads stand in for the paper's knee, spiral and MRF data, which are not
available here; see ``workloads.py`` for the recipes.
"""

from .generators import (  # noqa: F401
    phantom,
    coil_sensitivities,
    mask_variable_density,
    mask_poisson_disc_like,
    mask_phase_encode_1d,
    complex_noise,
    power_start_vector,
    spiral_trajectory,
)
from .workloads import WORKLOADS, Workload, make_slice_inputs, make_inputs  # noqa: F401
