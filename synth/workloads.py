"""The five synthetic workloads (seeded), standing in for the paper's MRI data.

The paper's Cartesian experiment (a 320 x 320, 8-coil knee, about 7.2-fold
Poisson-disc undersampling, Section "Cartesian MRI") cannot be reproduced here;
these workloads keep its structure (multi-coil Cartesian SENSE, variable-density
undersampling with a fully sampled calibration centre, complex Gaussian noise)
with seeded synthetic content.

Seeds: slice ``s`` of workload ``w`` (1-based) uses ``default_rng(1000*w + s)``,
drawing in the order: per-slice shape parameters (batched workload only),
phantom, coil maps, mask (or spiral trajectory), noise.  For the spiral
workload ``mask`` holds the trajectory ``[J, 2]`` and ``noise`` is ``[C, J]``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import generators as g


@dataclass(frozen=True)
class Workload:
    wid: int
    name: str
    n: int | None            # None: drawn per slice
    coils: int | None
    slices: int
    mask: str                # "vd", "poisson", "pe1d"
    accel: float | None
    centre: int | None
    sigma: float
    levels: int
    lam: float | None        # None: drawn per slice
    degree: int
    iters: int | None
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    1: Workload(1, "2-D Cartesian SENSE 64x64, 4 coils", 64, 4, 1, "vd", 4.0, 8,
                1e-3, 3, 1e-3, 3, 50),
    2: Workload(2, "Cartesian SENSE 256x256, 16 coils", 256, 16, 1, "poisson", 6.0, 24,
                5e-3, 4, 5e-4, 3, 200, {"degrees": (0, 1, 2, 3, 4, 5)}),
    3: Workload(3, "slab of 32 slices 384x384, 32 coils, 1-D phase-encode mask", 384, 32, 32,
                "pe1d", 8.0, 32, 5e-3, 4, 5e-4, 4, None, {"n_random_lines": 16}),
    4: Workload(4, "batch of 64 uneven slices", None, None, 64, "vd", None, None,
                5e-3, 4, None, 3, None,
                {"sizes": (128, 160, 192, 256, 320), "coil_counts": (8, 12, 16, 32),
                 "accel_range": (3.0, 8.0), "lam_range": (2e-4, 2e-3)}),
    5: Workload(5, "batch of 8 slices 192x192, 12 coils", 192, 12, 8, "vd", 5.0, 24,
                5e-3, 4, 5e-4, 4, 20),
    7: Workload(7, "knee-like Cartesian SENSE 320x320, 8 coils", 320, 8, 1, "poisson", 7.21, 24,
                5e-3, 4, 1.73e-4, 3, 200),
    6: Workload(6, "non-Cartesian 256x256, 12 coils, variable-density spiral", 256, 12, 1, "spiral",
                None, None, 5e-3, 4, 5e-4, 3, 200,
                {"interleaves": 16, "samples": 1024, "turns": 8.0, "power": 1.5}),
}


def make_slice_inputs(wid: int, s: int) -> dict:
    """Inputs of slice ``s`` of workload ``wid`` (complex128 / uint8 NumPy arrays)."""
    w = WORKLOADS[wid]
    rng = np.random.default_rng(1000 * wid + s)
    n, coils, accel, centre, lam = w.n, w.coils, w.accel, w.centre, w.lam
    if w.n is None:
        n = int(rng.choice(w.extra["sizes"]))
        coils = int(rng.choice(w.extra["coil_counts"]))
        accel = float(rng.uniform(*w.extra["accel_range"]))
        centre = n // 8
        lo, hi = w.extra["lam_range"]
        lam = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    img = g.phantom(n, rng)
    sens = g.coil_sensitivities(n, coils, rng)
    if w.mask == "vd":
        mask = g.mask_variable_density(n, accel, centre, rng)
    elif w.mask == "poisson":
        mask = g.mask_poisson_disc_like(n, accel, centre, rng)
    elif w.mask == "pe1d":
        n_rand = w.extra["n_random_lines"]
        mask = g.mask_phase_encode_1d(n, centre, n_rand, rng)
    elif w.mask == "spiral":
        e = w.extra
        mask = g.spiral_trajectory(n, e["interleaves"], e["samples"], e["turns"], e["power"], rng)
    else:
        raise ValueError(w.mask)
    noise = g.complex_noise((coils, mask.shape[0]) if w.mask == "spiral" else (coils, n, n), w.sigma, rng)
    return {"phantom": img, "sens": sens, "mask": mask, "noise": noise, "n": n,
            "coils": coils, "lam": lam, "accel": accel, "levels": w.levels,
            "degree": w.degree,
            "mask_kind": {"pe1d": "1d", "spiral": "spiral"}.get(w.mask, "2d")}


def make_inputs(wid: int, slices: int | None = None) -> dict:
    """Stacked inputs of a uniform-shape workload: phantom ``[S,n,n]``, sens
    ``[S,C,n,n]``, mask ``[S,n,n]`` or ``[S,n]``, noise ``[S,C,n,n]``."""
    w = WORKLOADS[wid]
    if w.n is None:
        raise ValueError("workload has per-slice shapes; use make_slice_inputs")
    ns = w.slices if slices is None else slices
    parts = [make_slice_inputs(wid, s) for s in range(ns)]
    out = {k: np.stack([p[k] for p in parts]) for k in ("phantom", "sens", "mask", "noise")}
    out.update({k: parts[0][k] for k in ("n", "coils", "lam", "levels", "degree", "mask_kind")})
    out["slices"] = ns
    return out
