"""Seeded generators: phantom, coil maps, k-space masks, noise.

Pure NumPy sampling and geometry.  Every function takes a ``numpy.random.Generator``
so the caller fixes the draw order.  Image coordinates run over [-1, 1) along
each axis (pixel ``i`` sits at ``(i - n/2) / (n/2)``); arrays are indexed
``[y, x]`` with x fastest.

Masks are drawn in centred k-space layout (DC at ``n//2``) and returned in the
natural FFT order (DC at index 0), i.e. ``numpy.fft.ifftshift`` of the centred
mask, because the operator uses the uncentred unitary DFT.
"""

from __future__ import annotations

import numpy as np


def _grid(n: int):
    c = (np.arange(n, dtype=np.float64) - n / 2.0) / (n / 2.0)
    y, x = np.meshgrid(c, c, indexing="ij")
    return y, x


def _ellipse(y, x, cy, cx, ay, ax, theta):
    ct, st = np.cos(theta), np.sin(theta)
    xr = (x - cx) * ct + (y - cy) * st
    yr = -(x - cx) * st + (y - cy) * ct
    return (xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0


def phantom(n: int, rng: np.random.Generator, n_random: int = 12) -> np.ndarray:
    """Piecewise-constant real phantom returned as complex128 ``[n, n]``.

    One outer ellipse (semi-axes 0.9 along x, 0.75 along y, value 1.0) plus
    ``n_random`` ellipses with centres U[-0.6, 0.6]^2, semi-axes U[0.05, 0.5],
    angle U[0, pi) and value U[-0.4, 0.6]; values add and the sum is clipped at 0.
    """
    y, x = _grid(n)
    img = np.where(_ellipse(y, x, 0.0, 0.0, 0.75, 0.9, 0.0), 1.0, 0.0)
    for _ in range(n_random):
        cy, cx = rng.uniform(-0.6, 0.6, size=2)
        ay, ax = rng.uniform(0.05, 0.5, size=2)
        theta = rng.uniform(0.0, np.pi)
        val = rng.uniform(-0.4, 0.6)
        img = img + np.where(_ellipse(y, x, cy, cx, ay, ax, theta), val, 0.0)
    img = np.clip(img, 0.0, None)
    return img.astype(np.complex128)


def coil_sensitivities(n: int, coils: int, rng: np.random.Generator,
                       radius: float = 1.2, width: float = 0.8) -> np.ndarray:
    """Smooth complex coil maps ``[coils, n, n]`` with ``sum_c |S_c|^2 = 1``.

    Coil c is a Gaussian bump of standard deviation ``width`` centred at
    ``radius * (cos 2 pi c / C, sin 2 pi c / C)``, times a random constant phase
    and a random linear phase (slope U[-1, 1] rad per unit length along each
    axis).  The maps are then divided by the root-sum-of-squares so that the
    coil combination is pointwise energy preserving.
    """
    y, x = _grid(n)
    maps = np.empty((coils, n, n), dtype=np.complex128)
    for c in range(coils):
        ang = 2.0 * np.pi * c / coils
        cy, cx = radius * np.sin(ang), radius * np.cos(ang)
        mag = np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * width ** 2))
        phi0 = rng.uniform(0.0, 2.0 * np.pi)
        gy, gx = rng.uniform(-1.0, 1.0, size=2)
        maps[c] = mag * np.exp(1j * (phi0 + gx * x + gy * y))
    rss = np.sqrt(np.sum(np.abs(maps) ** 2, axis=0))
    return maps / rss[None, :, :]


def _centre_box(n: int, centre: int):
    lo = n // 2 - centre // 2
    return lo, lo + centre


def _k_radius(n: int):
    k = np.arange(n, dtype=np.float64) - n // 2
    ky, kx = np.meshgrid(k, k, indexing="ij")
    return np.sqrt(ky ** 2 + kx ** 2) / (n / 2.0)


def mask_variable_density(n: int, accel: float, centre: int,
                          rng: np.random.Generator) -> np.ndarray:
    """2-D variable-density random mask, uint8 ``[n, n]`` in natural order.

    A fully sampled ``centre x centre`` block around DC, plus points drawn
    without replacement with probability proportional to ``(1 - r)^2``
    (r = k-radius over n/2, clipped to 1) until exactly ``round(n*n/accel)``
    points are sampled.
    """
    total = int(round(n * n / accel))
    m = np.zeros((n, n), dtype=bool)
    lo, hi = _centre_box(n, centre)
    m[lo:hi, lo:hi] = True
    need = total - int(m.sum())
    if need > 0:
        dens = (1.0 - np.minimum(_k_radius(n), 1.0)) ** 2
        dens[m] = 0.0
        flat = dens.ravel()
        cand = np.flatnonzero(flat > 0)
        p = flat[cand] / flat[cand].sum()
        pick = rng.choice(cand, size=need, replace=False, p=p)
        m.ravel()[pick] = True
    return np.fft.ifftshift(m).astype(np.uint8)


def _dart_throw(n: int, order: np.ndarray, radius_px: np.ndarray, excluded: np.ndarray,
                scale: float) -> list:
    """Accept candidates in ``order`` unless blocked; an accepted point blocks
    every point closer than ``scale * radius_px`` at the accepted point."""
    blocked = excluded.copy()
    accepted = []
    stencils = {}
    for idx in order:
        ky, kx = divmod(int(idx), n)
        if blocked[ky, kx]:
            continue
        accepted.append(int(idx))
        d = scale * radius_px[ky, kx]
        q = round(d * 4.0) / 4.0
        st = stencils.get(q)
        if st is None:
            rr = int(np.ceil(q))
            off = np.arange(-rr, rr + 1)
            oy, ox = np.meshgrid(off, off, indexing="ij")
            st = (rr, (oy ** 2 + ox ** 2) < q * q)
            stencils[q] = st
        rr, disc = st
        y0, y1 = max(ky - rr, 0), min(ky + rr + 1, n)
        x0, x1 = max(kx - rr, 0), min(kx + rr + 1, n)
        blocked[y0:y1, x0:x1] |= disc[y0 - ky + rr:y1 - ky + rr, x0 - kx + rr:x1 - kx + rr]
    return accepted


def mask_poisson_disc_like(n: int, accel: float, centre: int,
                           rng: np.random.Generator, growth: float = 2.0) -> np.ndarray:
    """Poisson-disc-like variable-density mask, uint8 ``[n, n]`` natural order.

    Dart throwing over a seeded random candidate order: the minimum distance at
    k-radius r is ``s * (1 + growth * r)`` pixels.  The scale ``s`` is bisected
    for the largest value that still yields at least the target count, and the
    accepted list is cut to exactly ``round(n*n/accel)`` samples including the
    fully sampled ``centre x centre`` block (which takes part in no blocking).
    """
    total = int(round(n * n / accel))
    cen = np.zeros((n, n), dtype=bool)
    lo, hi = _centre_box(n, centre)
    cen[lo:hi, lo:hi] = True
    need = total - int(cen.sum())
    m = cen.copy()
    if need > 0:
        radius_px = 1.0 + growth * np.minimum(_k_radius(n), 1.0)
        order = rng.permutation(n * n)
        order = order[~cen.ravel()[order]]
        s_lo, s_hi = 0.0, 8.0
        best = None
        for _ in range(24):
            s_mid = 0.5 * (s_lo + s_hi)
            acc = _dart_throw(n, order, radius_px, cen, s_mid)
            if len(acc) >= need:
                s_lo, best = s_mid, acc
            else:
                s_hi = s_mid
        if best is None:
            best = _dart_throw(n, order, radius_px, cen, 0.0)
        m.ravel()[np.asarray(best[:need], dtype=np.int64)] = True
    return np.fft.ifftshift(m).astype(np.uint8)


def mask_phase_encode_1d(n: int, n_centre: int, n_random: int,
                         rng: np.random.Generator) -> np.ndarray:
    """1-D phase-encode line mask, uint8 ``[n]`` over ky in natural order.

    ``n_centre`` contiguous lines around DC plus ``n_random`` lines drawn
    uniformly without replacement from the rest; every sampled line is fully
    sampled along the readout (x) axis.
    """
    m = np.zeros(n, dtype=bool)
    lo = n // 2 - n_centre // 2
    m[lo:lo + n_centre] = True
    rest = np.flatnonzero(~m)
    m[rng.choice(rest, size=n_random, replace=False)] = True
    return np.fft.ifftshift(m).astype(np.uint8)


def complex_noise(shape, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. complex Gaussian, N(0, sigma^2) on real and imaginary parts."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return sigma * (re + 1j * im)


def spiral_trajectory(n: int, interleaves: int, samples: int, turns: float, power: float,
                      rng: np.random.Generator) -> np.ndarray:
    """Variable-density spiral k-space trajectory, float64 ``[interleaves * samples, 2]``
    (kx, ky) in cycles per field of view (|k| <= n/2).

    Interleave i starts at angle ``2 pi i / interleaves`` plus one random rotation
    shared by all interleaves; sample t = 1..samples of an interleave sits at radius
    ``(n/2) (t/samples)^power`` and angle ``2 pi turns t/samples`` further on, so
    ``power > 1`` samples the centre more densely than the edge.
    """
    rot = rng.uniform(0.0, 2.0 * np.pi)
    t = np.arange(1, samples + 1) / samples
    r = 0.5 * n * t ** power
    out = []
    for i in range(interleaves):
        ang = rot + 2.0 * np.pi * i / interleaves + 2.0 * np.pi * turns * t
        out.append(np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1))
    return np.concatenate(out, axis=0)


def power_start_vector(n: int, slices: int = 1, seed: int = 0) -> np.ndarray:
    """Unit-norm complex Gaussian start vector ``[slices, n, n]`` for power iteration."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((slices, n, n)) + 1j * rng.standard_normal((slices, n, n))
    return v / np.linalg.norm(v)
