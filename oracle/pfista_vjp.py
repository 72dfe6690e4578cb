"""FP64 oracle of reverse-mode derivatives through unrolled PFISTA.

TEST INFRASTRUCTURE: imported only by tests (see the package header).

The iteration is Algorithm 4 run for a fixed count K (``pfista`` of the
operator module, momentum optional as in Algorithms 1/3), seen as a function
of the threshold ``lam`` and the polynomial coefficients ``c``; the output is
``x_K``.  Complex quantities are treated as pairs of reals: the cotangent of a
complex array ``v`` is ``dL/dRe v + i dL/dIm v``, so for a complex-linear map
``y = M v`` the pull-back is ``M^H y_bar`` and a real parameter's derivative is
``sum Re(conj(v_bar) dv/dtheta)``.

Step k (``N' = scale A^H A``, ``a = A'^H b'``):
    g_k = N' z_k - a;   v_k = z_k - p(N') g_k;   u_k = Psi v_k
    x_(k+1) = Psi^H soft(u_k, lam);   z_(k+1) = (1 + beta_k) x_(k+1) - beta_k x_k
Pull-back of step k, from (x_bar_(k+1), z_bar_(k+1)):
    w_bar = Psi (x_bar_(k+1) + (1 + beta_k) z_bar_(k+1))
    u_bar, lam_bar += soft-threshold pull-back at u_k (below)
    v_bar = Psi^H u_bar
    c_bar_i -= Re <N'^i v_bar, g_k>          (N'^i is Hermitian)
    z_bar_k = v_bar - N' p(N') v_bar;   x_bar_k = -beta_k z_bar_(k+1)
Soft threshold ``w = u (1 - lam/|u|)`` on its support ``|u| > lam`` (0 off it):
as a map of R^2 it keeps the radial direction ``u/|u|`` with factor 1 and the
tangential one with factor ``1 - lam/|u|``, a symmetric Jacobian, and
``dw/dlam = -u/|u|``.
"""

from __future__ import annotations

import numpy as np

from .pfista_oracle import adjoint, haar_fwd, haar_inv, iterate, normal

__all__ = ["soft_threshold_vjp", "prox_l1_haar_vjp", "poly_vjp", "unrolled_forward", "unrolled_vjp"]


def soft_threshold_vjp(u: np.ndarray, w_bar: np.ndarray, lam: float):
    """Pull-back of ``w = soft(u, lam)``: returns ``(u_bar, lam_bar)``."""
    mag = np.abs(u)
    keep = mag > lam
    safe = np.where(keep, mag, 1.0)
    dirn = np.where(keep, u / safe, 0.0)                   # u/|u| on the support
    radial = np.real(np.conj(dirn) * w_bar)                 # component of w_bar along u/|u|
    tang = w_bar - radial * dirn
    u_bar = np.where(keep, radial * dirn + (1.0 - lam / safe) * tang, 0.0)
    lam_bar = -float(np.sum(np.where(keep, radial, 0.0)))
    return u_bar, lam_bar


def prox_l1_haar_vjp(v: np.ndarray, x_bar: np.ndarray, lam: float, levels: int):
    """Pull-back of ``x = Psi^H soft(Psi v, lam)``: returns ``(v_bar, lam_bar)``."""
    u = haar_fwd(v, levels)
    u_bar, lam_bar = soft_threshold_vjp(u, haar_fwd(x_bar, levels), lam)
    return haar_inv(u_bar, levels), lam_bar


def poly_vjp(sens, mask, scale, coef, g, v_bar):
    """Pull-back of ``v = z - p(N') g`` through the polynomial, given ``v_bar``:
    returns ``(p(N') v_bar, c_bar)`` with ``c_bar_i = -Re <N'^i v_bar, g>``."""
    q = v_bar
    pv = float(coef[0]) * q
    c_bar = [-float(np.real(np.vdot(q, g)))]
    for ci in coef[1:]:
        q = normal(sens, mask, q, scale)
        pv = pv + float(ci) * q
        c_bar.append(-float(np.real(np.vdot(q, g))))
    return pv, np.array(c_bar)


def unrolled_forward(sens, mask, bn, scale, lam, coef, levels, iters, momentum=True):
    """``x_K`` and the per-step ``(z_k, g_k, pg_k, beta_k)`` of K steps of
    ``iterate`` from zero."""
    a = scale ** 0.5 * adjoint(sens, mask, bn)
    tape = []
    x, _ = iterate(lambda v: normal(sens, mask, v, scale), a, lam, coef, levels, iters, momentum=momentum,
                   record=lambda k, z, g, pg, beta, x_new: tape.append((z, g, pg, beta)))
    return x, tape


def unrolled_vjp(sens, mask, bn, scale, lam, coef, levels, iters, x_bar, momentum=True):
    """``(lam_bar, c_bar)`` of ``L`` given ``x_bar = dL/dx_K`` (pull-back of
    every step in reverse order)."""
    _, tape = unrolled_forward(sens, mask, bn, scale, lam, coef, levels, iters, momentum)
    xb = np.array(x_bar, dtype=np.complex128)
    zb = np.zeros_like(xb)
    lam_bar = 0.0
    c_bar = np.zeros(len(coef))
    for z, g, pg, beta in reversed(tape):
        v_bar, lb = prox_l1_haar_vjp(z - pg, xb + (1.0 + beta) * zb, lam, levels)
        lam_bar += lb
        pv, cb = poly_vjp(sens, mask, scale, coef, g, v_bar)
        c_bar += cb
        xb, zb = -beta * zb, v_bar - normal(sens, mask, pv, scale)
    return lam_bar, c_bar
