"""FP64 oracle of the non-Cartesian SENSE model and its Toeplitz normal operator.

TEST INFRASTRUCTURE: imported only by tests (see the package header).

Non-Cartesian MRI (Section 3.3) replaces the Cartesian ``M F`` by the
non-uniform DFT ``E`` of a k-space trajectory and evaluates the normal operator
through its Toeplitz structure.  Conventions:

* trajectory points ``k_j = (kx_j, ky_j)`` in cycles per field of view (grid
  units, |k| <= n/2); image pixel ``(y, x)`` with x fastest, coordinates 0..n-1;
* ``(E v)_j = (1/n) sum_(y,x) v[y, x] exp(-2 pi i (kx_j x + ky_j y) / n)`` -- on
  the integer grid this is the unitary DFT of the Cartesian model;
* ``E^H E`` has entries ``h(r - r')`` with ``h(m) = (1/n^2) sum_j exp(2 pi i k_j . m / n)``
  for ``m`` in ``[-(n-1), n-1]^2``: a Toeplitz (block-Toeplitz) matrix, applied
  exactly as a circular convolution on a ``2n x 2n`` grid: zero-pad, DFT,
  multiply by ``K = DFT(h wrapped onto the 2n grid)``, inverse DFT, crop.  The
  wrapped entries at index n (no difference reaches it) are set to 0, which
  keeps ``h`` Hermitian-symmetric and ``K`` real.
"""

from __future__ import annotations

import numpy as np

from .pfista_oracle import haar_fwd, iterate

__all__ = ["nudft_matrix", "nudft_forward", "nudft_adjoint", "nudft_normal", "toeplitz_kernel",
           "toeplitz_normal", "nc_data_term", "pfista_nc", "pfista_toeplitz"]


def nudft_matrix(traj: np.ndarray, n: int) -> np.ndarray:
    """``E`` as a dense ``[J, n*n]`` matrix (row-major pixels, x fastest)."""
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ph = np.outer(traj[:, 0], xx.ravel()) + np.outer(traj[:, 1], yy.ravel())
    return np.exp(-2j * np.pi * ph / n) / n


def nudft_forward(sens: np.ndarray, traj: np.ndarray, x: np.ndarray) -> np.ndarray:
    """``A x = E (S_c x)`` per slice and coil: ``[S, n, n] -> [S, C, J]``; traj ``[S, J, 2]``."""
    S, C, n, _ = sens.shape
    out = np.empty((S, C, traj.shape[1]), dtype=np.complex128)
    for s in range(S):
        e = nudft_matrix(traj[s], n)
        out[s] = (e @ (sens[s] * x[s][None]).reshape(C, n * n).T).T
    return out


def nudft_adjoint(sens: np.ndarray, traj: np.ndarray, y: np.ndarray) -> np.ndarray:
    """``A^H y = sum_c conj(S_c) E^H y_c``: ``[S, C, J] -> [S, n, n]``."""
    S, C, n, _ = sens.shape
    out = np.empty((S, n, n), dtype=np.complex128)
    for s in range(S):
        e = nudft_matrix(traj[s], n)
        img = (e.conj().T @ y[s].T).T.reshape(C, n, n)
        out[s] = np.sum(np.conj(sens[s]) * img, axis=0)
    return out


def nudft_normal(sens, traj, x, scale=1.0):
    """``scale A^H A x`` by the direct non-uniform DFT."""
    return scale * nudft_adjoint(sens, traj, nudft_forward(sens, traj, x))


def toeplitz_kernel(traj: np.ndarray, n: int, weights=None) -> np.ndarray:
    """Real ``[2n, 2n]`` kernel ``K`` of one slice's trajectory ``[J, 2]``
    (optional real weights ``w_j`` multiply each sample's term)."""
    w = np.ones(traj.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64)
    m = np.arange(-(n - 1), n)
    ex = np.exp(2j * np.pi * np.outer(traj[:, 0], m) / n)          # [J, 2n-1]
    ey = np.exp(2j * np.pi * np.outer(traj[:, 1], m) / n)
    h = (ey * w[:, None]).T @ ex / n ** 2                            # h[my, mx], m = -(n-1)..n-1
    c = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    idx = np.mod(m, 2 * n)
    c[np.ix_(idx, idx)] = h
    return np.fft.fft2(c)


def toeplitz_normal(sens, kern, x, scale=1.0):
    """``scale sum_c conj(S_c) crop(IDFT_2n(K DFT_2n(pad(S_c x))))``; kern ``[S, 2n, 2n]``."""
    S, C, n, _ = sens.shape
    pad = np.zeros((S, C, 2 * n, 2 * n), dtype=np.complex128)
    pad[:, :, :n, :n] = sens * x[:, None]
    conv = np.fft.ifft2(kern[:, None] * np.fft.fft2(pad, axes=(-2, -1)), axes=(-2, -1))[:, :, :n, :n]
    return scale * np.sum(np.conj(sens) * conv, axis=1)


def nc_data_term(sens, traj, bn, scale, x) -> float:
    """``1/2 ||sqrt(scale) A x - bn||^2`` with the non-uniform model."""
    r = np.sqrt(scale) * nudft_forward(sens, traj, x) - bn
    return 0.5 * float(np.vdot(r, r).real)


def pfista_nc(sens, traj, bn, scale, lam, coef, levels, iters, history=False):
    """Algorithm 4 with the non-Cartesian model ``A = E S`` (direct DFT sums):
    ``iterate`` with ``N' = scale A^H A`` and ``a = sqrt(scale) A^H bn``."""
    a = np.sqrt(scale) * nudft_adjoint(sens, traj, bn)
    hist = []

    def rec(k, z, g, pg, beta, x_new):
        if history:
            hist.append(nc_data_term(sens, traj, bn, scale, x_new)
                        + lam * float(np.sum(np.abs(haar_fwd(x_new, levels)))))

    x, z = iterate(lambda v: nudft_normal(sens, traj, v, scale), a, lam, coef, levels, iters, record=rec)
    return x, z, hist


def pfista_toeplitz(sens, kern, ahb, bnorm, scale, lam, coef, levels, iters):
    """Algorithm 4 from ``A^H b`` and ``||b||`` alone (as a Toeplitz solver
    receives its data): ``iterate`` with ``N' = scale T`` for the Toeplitz
    operator T of ``kern`` and ``a = sqrt(scale) A^H b / ||b||``."""
    a = np.sqrt(scale) * ahb / bnorm
    x, _ = iterate(lambda v: toeplitz_normal(sens, kern, v, scale), a, lam, coef, levels, iters)
    return x
