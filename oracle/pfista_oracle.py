"""FP64 oracle: Cartesian SENSE operators, L2-optimal polynomial, Haar prox, PFISTA.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the CPU
baseline of the benchmark.  complex128 / float64 / exact rationals throughout.

Conventions (one reading of the paper each; the design notes list them):

* Problem: ``argmin_x 1/2 ||A x - b||^2 + lam ||Psi x||_1`` (the unconstrained
  problem of the Introduction), with the Cartesian SENSE model ``A = M F S`` of
  the Cartesian MRI experiment (Section 3.2): S multiplies by each coil map, F
  is the unitary 2-D DFT with forward exponent ``exp(-2 pi i k n / N)`` and DC at
  index 0, M keeps the sampled k-space points.
* Normalisation (Section 3, opening): A is scaled to unit induced norm by a
  scalar ``L`` (an upper estimate of the largest eigenvalue of ``A^H A``), b to
  unit l2 norm: ``A' = A / sqrt(L)``, ``b' = b / ||b||``.
* Psi is the orthonormal 2-D Haar transform with ``levels`` levels in Mallat
  layout; every coefficient is thresholded, the coarsest approximation included.
* Arrays carry a leading slice axis: images ``[S, n, n]``, coil maps and k-space
  ``[S, C, n, n]``, masks ``[S, n, n]`` (2-D) or ``[S, n]`` (one flag per ky
  row, the same for every kx).  Slices are independent blocks of A.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np
import scipy.fft

__all__ = [
    "fft2u", "ifft2u", "expand_mask", "forward", "adjoint", "normal",
    "kspace_data", "l2_poly_coefficients", "poly_eval", "poly_apply",
    "haar_fwd", "haar_inv", "soft_threshold", "prox_l1_haar", "objective",
    "data_term", "power_iteration", "pfista", "pfista_step", "normalise",
    "chebyshev_poly_coefficients", "weighted_l2_poly_coefficients", "pgd",
    "momentum_beta", "horner", "iterate",
]

_SQRT_HALF = np.sqrt(0.5)


# ----------------------------------------------------------------------------
# Forward model (Section 3.2, the Cartesian SENSE model M F S)
# ----------------------------------------------------------------------------

def fft2u(v: np.ndarray) -> np.ndarray:
    """Unitary 2-D DFT over the last two axes, natural (DC-at-0) order."""
    return scipy.fft.fft2(v, axes=(-2, -1), norm="ortho")


def ifft2u(v: np.ndarray) -> np.ndarray:
    """Inverse of ``fft2u`` (its adjoint, since it is unitary)."""
    return scipy.fft.ifft2(v, axes=(-2, -1), norm="ortho")


def expand_mask(mask: np.ndarray, n: int) -> np.ndarray:
    """Boolean k-space mask ``[S, n, n]`` from a 2-D ``[S, n, n]`` or a
    phase-encode ``[S, n]`` mask (row ky sampled for every kx)."""
    m = np.asarray(mask) != 0
    if m.ndim == 2:
        m = np.repeat(m[:, :, None], n, axis=2)
    return m


def forward(sens: np.ndarray, mask: np.ndarray, x: np.ndarray) -> np.ndarray:
    """``A x = M F (S_c x)`` for every coil: ``[S, n, n] -> [S, C, n, n]``."""
    n = x.shape[-1]
    m = expand_mask(mask, n)
    return m[:, None, :, :] * fft2u(sens * x[:, None, :, :])


def adjoint(sens: np.ndarray, mask: np.ndarray, y: np.ndarray) -> np.ndarray:
    """``A^H y = sum_c conj(S_c) F^H (M y_c)``: ``[S, C, n, n] -> [S, n, n]``."""
    n = y.shape[-1]
    m = expand_mask(mask, n)
    return np.sum(np.conj(sens) * ifft2u(m[:, None, :, :] * y), axis=1)


def normal(sens: np.ndarray, mask: np.ndarray, x: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """``scale * A^H A x`` (the normal operator whose spectrum the paper targets)."""
    return scale * adjoint(sens, mask, forward(sens, mask, x))


def kspace_data(sens: np.ndarray, mask: np.ndarray, img: np.ndarray,
                noise: np.ndarray) -> np.ndarray:
    """Simulated measurements ``b = M (F S img + noise)`` (noise only where sampled)."""
    n = img.shape[-1]
    m = expand_mask(mask, n)
    return m[:, None, :, :] * (fft2u(sens * img[:, None, :, :]) + noise)


def normalise(b: np.ndarray, lam_max: float):
    """Scalars of the normalisation: returns ``(b / ||b||, ||b||, 1/L)``."""
    nb = float(np.linalg.norm(b))
    return b / nb, nb, 1.0 / lam_max


def power_iteration(sens: np.ndarray, mask: np.ndarray, v0: np.ndarray, iters: int) -> float:
    """Largest eigenvalue of ``A^H A`` by power iteration (Section 2, the note
    that the maximum eigenvalue can be estimated).

    ``v_{i+1} = N v_i / ||N v_i||`` from the given start vector; returns
    ``||N v_{iters-1}||`` with ``||v_{iters-1}|| = 1`` (all slices form one vector,
    so the result is the maximum over slices).
    """
    v = v0 / np.linalg.norm(v0)
    est = 0.0
    for _ in range(iters):
        w = normal(sens, mask, v)
        est = float(np.linalg.norm(w))
        v = w / est
    return est


# ----------------------------------------------------------------------------
# Polynomial preconditioner (Section 2.5 cost; Section 2.7 evaluation)
# ----------------------------------------------------------------------------

def l2_poly_coefficients(degree: int) -> list:
    """Exact coefficients ``c[0..d]`` (ascending powers) of the polynomial that
    minimises ``int_0^1 (1 - z q(z))^2 dz`` over degree-d polynomials q
    (Section 2.5, the L2 polynomial cost).

    Setting the derivative in ``c_i`` to zero gives the normal equations
    ``sum_j c_j / (i + j + 3) = 1 / (i + 2)`` for ``i = 0..d``, solved here by
    Gaussian elimination over the rationals.
    """
    d = int(degree)
    if d < 0:
        raise ValueError("degree must be >= 0")
    a = [[Fraction(1, i + j + 3) for j in range(d + 1)] + [Fraction(1, i + 2)]
         for i in range(d + 1)]
    return _solve_exact(a)


def _solve_exact(a):
    """Gauss-Jordan elimination over the rationals of an augmented matrix."""
    n = len(a)
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        p = a[col][col]
        a[col] = [v / p for v in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [vr - f * vc for vr, vc in zip(a[r], a[col])]
    return [a[i][n] for i in range(n)]


def weighted_l2_poly_coefficients(degree: int, alpha) -> list:
    """Coefficients of the minimiser of ``int_0^1 z^alpha (1 - z q(z))^2 dz``
    (the weighted cost of Section 2.5 with the weight ``w(z) = z^alpha``,
    alpha > -1).  With moments ``m_k = int_0^1 z^(alpha + k) dz = 1/(alpha+k+1)``
    the normal equations are ``sum_j c_j m_(i+j+2) = m_(i+1)``; solved exactly
    for rational alpha (floats are taken at their exact binary value)."""
    d = int(degree)
    al = Fraction(alpha)
    if al <= -1:
        raise ValueError("alpha must be > -1")
    m = [1 / (al + k + 1) for k in range(2 * d + 3)]
    a = [[m[i + j + 2] for j in range(d + 1)] + [m[i + 1]] for i in range(d + 1)]
    return _solve_exact(a)


def chebyshev_poly_coefficients(degree: int, mu) -> list:
    """Coefficients of ``p(z) = (1 - r(z)) / z`` with the shifted, scaled
    Chebyshev residual ``r(z) = T_(d+1)((1 + mu - 2z)/(1 - mu)) /
    T_(d+1)((1 + mu)/(1 - mu))`` (the L-infinity design of Section 2.5 for a
    known smallest eigenvalue mu in (0, 1)).  Built exactly from the recurrence
    ``T_(n+1)(u) = 2u T_n(u) - T_(n-1)(u)`` in powers of z."""
    d = int(degree)
    m = Fraction(mu)
    if not (0 < m < 1):
        raise ValueError("mu must lie in (0, 1)")
    u = [(1 + m) / (1 - m), -2 / (1 - m)]          # u(z) = u0 + u1 z

    def mul_u(pz):
        out = [Fraction(0)] * (len(pz) + 1)
        for i, c in enumerate(pz):
            out[i] += u[0] * c
            out[i + 1] += u[1] * c
        return out

    t_prev, t_cur = [Fraction(1)], list(u)
    for _ in range(d):
        nxt = [2 * c for c in mul_u(t_cur)]
        for i, c in enumerate(t_prev):
            nxt[i] -= c
        t_prev, t_cur = t_cur, nxt
    r = [c / t_cur[0] for c in t_cur]              # T_(d+1)(u(0)) = t_cur[0]
    return [-r[j + 1] for j in range(d + 1)]


def poly_eval(coef, z):
    """``p(z) = sum_i c[i] z^i`` (the coefficient order of Section 2.7)."""
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros_like(z)
    for c in reversed([float(c) for c in coef]):
        out = out * z + c
    return out


def horner(apply, coef, g: np.ndarray) -> np.ndarray:
    """``p(N') g`` for a normal operator given as the function ``apply``, nested
    as in Listing 1: ``P = c0 I + N'(c1 I + N'(c2 I + ...))``, i.e. ``h = c_d g``
    then ``h = c_i g + N' h`` for ``i = d-1, ..., 0`` (d applications of N')."""
    c = [float(v) for v in coef]
    h = c[-1] * g
    for ci in reversed(c[:-1]):
        h = ci * g + apply(h)
    return h


def poly_apply(sens: np.ndarray, mask: np.ndarray, scale: float, coef, g: np.ndarray) -> np.ndarray:
    """``p(N') g`` with the Cartesian ``N' = scale * A^H A`` (``horner``)."""
    return horner(lambda v: normal(sens, mask, v, scale), coef, g)


# ----------------------------------------------------------------------------
# Regulariser and its proximal operator (Section 2.1 definition)
# ----------------------------------------------------------------------------

def haar_fwd(x: np.ndarray, levels: int) -> np.ndarray:
    """Orthonormal separable 2-D Haar analysis over the last two axes, Mallat
    layout: at each level the current low-pass square is split along x into
    ``(even + odd)/sqrt2 | (even - odd)/sqrt2`` and then likewise along y."""
    w = np.array(x, dtype=np.complex128, copy=True)
    m = w.shape[-1]
    for _ in range(levels):
        blk = w[..., :m, :m]
        lo = (blk[..., :, 0::2] + blk[..., :, 1::2]) * _SQRT_HALF
        hi = (blk[..., :, 0::2] - blk[..., :, 1::2]) * _SQRT_HALF
        blk = np.concatenate([lo, hi], axis=-1)
        lo = (blk[..., 0::2, :] + blk[..., 1::2, :]) * _SQRT_HALF
        hi = (blk[..., 0::2, :] - blk[..., 1::2, :]) * _SQRT_HALF
        w[..., :m, :m] = np.concatenate([lo, hi], axis=-2)
        m //= 2
    return w


def haar_inv(w: np.ndarray, levels: int) -> np.ndarray:
    """Inverse (= adjoint) of ``haar_fwd``."""
    x = np.array(w, dtype=np.complex128, copy=True)
    n = x.shape[-1]
    for lev in reversed(range(levels)):
        m = n >> lev
        h = m // 2
        blk = x[..., :m, :m].copy()
        lo, hi = blk[..., :h, :], blk[..., h:, :]
        cols = np.empty_like(blk)
        cols[..., 0::2, :] = (lo + hi) * _SQRT_HALF
        cols[..., 1::2, :] = (lo - hi) * _SQRT_HALF
        lo, hi = cols[..., :, :h], cols[..., :, h:]
        rows = np.empty_like(blk)
        rows[..., :, 0::2] = (lo + hi) * _SQRT_HALF
        rows[..., :, 1::2] = (lo - hi) * _SQRT_HALF
        x[..., :m, :m] = rows
    return x


def soft_threshold(w: np.ndarray, lam: float) -> np.ndarray:
    """Proximal operator of ``lam |.|`` on complex numbers: ``w (1 - lam/|w|)``
    where ``|w| > lam`` and exactly 0 elsewhere (including w = 0)."""
    mag = np.abs(w)
    keep = mag > lam
    scale = np.zeros_like(mag)
    np.divide(lam, mag, out=scale, where=keep)
    return np.where(keep, w * (1.0 - scale), 0.0)


def prox_l1_haar(v: np.ndarray, lam: float, levels: int) -> np.ndarray:
    """``prox_{lam ||Psi .||_1}(v) = Psi^H soft(Psi v, lam)`` (Psi orthonormal)."""
    return haar_inv(soft_threshold(haar_fwd(v, levels), lam), levels)


# ----------------------------------------------------------------------------
# Objective and the iteration (Algorithms 2 and 4)
# ----------------------------------------------------------------------------

def data_term(sens, mask, bn, scale, x) -> float:
    """``1/2 ||sqrt(scale) A x - bn||^2`` computed from the k-space residual."""
    r = np.sqrt(scale) * forward(sens, mask, x) - bn
    return 0.5 * float(np.vdot(r, r).real)


def objective(sens, mask, bn, scale, x, lam, levels) -> float:
    """``F(x) = 1/2 ||A' x - b'||^2 + lam ||Psi x||_1`` on normalised A', b'."""
    return data_term(sens, mask, bn, scale, x) + lam * float(np.sum(np.abs(haar_fwd(x, levels))))


def pfista_step(z, pg, x_old, lam, levels, beta):
    """One prox + momentum update of Algorithm 4:
    ``x_new = prox(z - P g)``, ``z_new = x_new + beta (x_new - x_old)``."""
    x_new = prox_l1_haar(z - pg, lam, levels)
    z_new = x_new + beta * (x_new - x_old)
    return x_new, z_new


def momentum_beta(k: int) -> float:
    """Momentum weight of step ``k >= 0`` in Algorithms 2 and 4:
    ``beta_k = k / (k + 3)`` (0, 1/4, 2/5, 1/2, 4/7, ...)."""
    return k / (k + 3.0)


def iterate(apply, ahb, lam, coef, levels, iters, x0=None, z0=None, k0=0, momentum=True,
            record=None):
    """The iteration of Algorithm 4 for any normal operator ``apply`` (``N'``)
    and data image ``ahb`` (``A'^H b'``); every solver of the oracle runs it.

    Step k (from ``x_0 = z_0 = 0``, or the given state after ``k0`` steps):
    ``g = N' z_k - A'^H b'``; ``x_{k+1} = prox(z_k - p(N') g)``;
    ``z_{k+1} = x_{k+1} + beta_k (x_{k+1} - x_k)`` with ``beta_k = k/(k+3)``
    (``momentum_beta``), or ``beta_k = 0`` without momentum (Algorithms 1 and 3,
    where ``z = x``).  The momentum uses the newest iterate, the usual FISTA
    form (the printed update names the older pair of iterates).

    ``record(k, z_k, g, pg, beta_k, x_{k+1})`` is called after every step.
    Returns ``(x, z)`` after the last step.
    """
    x = np.zeros_like(ahb) if x0 is None else np.array(x0, dtype=np.complex128)
    z = np.zeros_like(ahb) if z0 is None else np.array(z0, dtype=np.complex128)
    for k in range(k0, k0 + iters):
        g = apply(z) - ahb
        pg = horner(apply, coef, g)
        beta = momentum_beta(k) if momentum else 0.0
        x_new, z_new = pfista_step(z, pg, x, lam, levels, beta)
        if record is not None:
            record(k, z, g, pg, beta, x_new)
        x, z = x_new, z_new
    return x, z


def pgd(sens, mask, bn, scale, lam, coef, levels, iters, x0=None, history=False):
    """Proximal gradient descent with the polynomial preconditioner: Algorithm 3
    (PPGD), or Algorithm 1 (PGD) when coef = [1]:
    ``y_(k+1) = prox(y_k - p(N')(N' y_k - A'^H b'))`` from ``y_0 = 0``
    (``iterate`` without momentum)."""
    ahb = scale ** 0.5 * adjoint(sens, mask, bn)
    hist = []

    def rec(k, z, g, pg, beta, x_new):
        if history:
            hist.append(objective(sens, mask, bn, scale, x_new, lam, levels))

    y, _ = iterate(lambda v: normal(sens, mask, v, scale), ahb, lam, coef, levels, iters,
                   x0=x0, z0=x0, momentum=False, record=rec)
    return y, hist


def pfista(sens, mask, bn, scale, lam, coef, levels, iters, x0=None, z0=None, k0=0,
           history=False):
    """Polynomial-preconditioned FISTA, Algorithm 4 (Algorithm 2 when coef = [1]),
    with the Cartesian ``N' = scale A^H A`` and ``b' = bn`` (already normalised):
    ``iterate`` from ``x_0 = z_0 = 0``.

    Returns ``(x, z, hist)``; ``hist`` holds ``F(x_{k+1})`` per step if asked.
    Passing ``x0, z0, k0`` resumes from the state after ``k0`` steps.
    """
    ahb = scale ** 0.5 * adjoint(sens, mask, bn)
    hist = []

    def rec(k, z, g, pg, beta, x_new):
        if history:
            hist.append(objective(sens, mask, bn, scale, x_new, lam, levels))

    x, z = iterate(lambda v: normal(sens, mask, v, scale), ahb, lam, coef, levels, iters,
                   x0=x0, z0=z0, k0=k0, record=rec)
    return x, z, hist
