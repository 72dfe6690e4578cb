"""GPU parity of the operator calls against the FP64 oracle (through the C-ABI).

Bars: relative l2 error <= 1e-5 per normal / forward / adjoint apply (FP32
complex arithmetic against complex128), <= 1e-5 * H_d for the degree-d
polynomial (H_d = the largest Horner partial sup |q_j| on [0, 1], which bounds
how much the nested evaluation amplifies a rounding error), and <= 1e-5 for
the fused step.  Sizes span every supported radix (2, 3, 5), several coil
and slice counts (ragged against the 16-lane transform groups) and both mask
kinds; the workload shapes (64^2 x 4 coils, 256^2 x 16 coils, 384^2 x 32 coils
with a phase-encode mask) are included.
"""

import numpy as np
import pytest

import oracle as orc
from tests.gpu_util import HORNER_PARTIAL_MAX, c64, oracle_normal, random_case, rel, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    (64, 4, 1, "2d"), (256, 16, 1, "2d"), (128, 3, 3, "2d"), (160, 8, 2, "2d"),
    (192, 12, 1, "2d"), (320, 5, 1, "2d"), (384, 6, 1, "2d"), (512, 2, 1, "2d"),
    (64, 1, 2, "1d"), (128, 2, 1, "1d"), (160, 3, 1, "1d"), (192, 2, 2, "1d"),
    (256, 4, 1, "1d"), (320, 2, 1, "1d"), (384, 32, 2, "1d"), (512, 2, 1, "1d"),
]


def _plan(n, coils, slices, kind, levels=4):
    import paper_2204_10252_amd as pf
    return pf.Plan(n, coils, slices, haar_levels=levels,
                   mask_kind=pf.MASK_1D if kind == "1d" else pf.MASK_2D)


@pytest.mark.parametrize("n,coils,slices,kind", CASES)
def test_normal_apply(n, coils, slices, kind):
    import torch
    import paper_2204_10252_amd as pf
    sens, mask, x, w = random_case(n, coils, slices, kind, seed=n + coils + slices)
    plan = _plan(n, coils, slices, kind)
    ts, tm, tx, tw = to_dev(sens), to_dev(mask), to_dev(x), to_dev(w)
    ty = torch.empty_like(tx)
    alpha, beta = 0.7, -0.3
    pf.normal_apply(plan, ts, tm, tx, ty, alpha, tw, beta)
    ref = alpha * oracle_normal(sens, mask, x) + beta * w.astype(np.complex128)
    got = ty.cpu().numpy()
    assert rel(got, ref) <= 1e-5
    # per-slice check too (a slice mix-up would hide in the global norm)
    for s in range(slices):
        assert rel(got[s], ref[s]) <= 1e-5
    # w == NULL, and w aliasing y
    pf.normal_apply(plan, ts, tm, tx, ty, 1.0)
    assert rel(ty.cpu().numpy(), oracle_normal(sens, mask, x)) <= 1e-5
    ty.copy_(tw)
    pf.normal_apply(plan, ts, tm, tx, ty, alpha, ty, beta)
    assert rel(ty.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("n,coils,slices,kind", [(64, 4, 1, "2d"), (160, 3, 2, "2d"),
                                                 (384, 5, 1, "1d"), (256, 16, 1, "2d")])
def test_forward_adjoint(n, coils, slices, kind):
    import torch
    import paper_2204_10252_amd as pf
    sens, mask, x, _ = random_case(n, coils, slices, kind, seed=3 * n + coils)
    plan = _plan(n, coils, slices, kind)
    ts, tm, tx = to_dev(sens), to_dev(mask), to_dev(x)
    k = torch.empty((slices, coils, n, n), dtype=torch.complex64, device=tx.device)
    pf.forward(plan, ts, tm, tx, k)
    s128 = sens.astype(np.complex128)
    kref = orc.forward(s128, mask, x.astype(np.complex128))
    assert rel(k.cpu().numpy(), kref) <= 1e-5
    rng = np.random.default_rng(n)
    kin = c64(rng.standard_normal(kref.shape) + 1j * rng.standard_normal(kref.shape))
    y = torch.empty_like(tx)
    pf.adjoint(plan, ts, tm, to_dev(kin), y, 0.5)
    assert rel(y.cpu().numpy(), 0.5 * orc.adjoint(s128, mask, kin.astype(np.complex128))) <= 1e-5


@pytest.mark.parametrize("degree", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("n,coils,kind", [(64, 4, "2d"), (256, 16, "2d"), (384, 8, "1d")])
def test_poly_apply(degree, n, coils, kind):
    import torch
    import paper_2204_10252_amd as pf
    sens, mask, g, _ = random_case(n, coils, 1, kind, seed=degree + n)
    plan = _plan(n, coils, 1, kind)
    inv_l = 1.0 / 1.01
    coef = [float(c) for c in orc.l2_poly_coefficients(degree)]
    out = torch.empty_like(to_dev(g))
    pf.poly_apply(plan, to_dev(sens), to_dev(mask), inv_l, coef, to_dev(g), out)
    ref = orc.poly_apply(sens.astype(np.complex128), mask, inv_l, coef, g.astype(np.complex128))
    assert rel(out.cpu().numpy(), ref) <= 1e-5 * HORNER_PARTIAL_MAX[degree]


def test_library_coefficients_match_oracle():
    import paper_2204_10252_amd as pf
    for d in range(9):
        lib = pf.poly_coefficients(d)
        ora = [float(c) for c in orc.l2_poly_coefficients(d)]
        np.testing.assert_allclose(lib, ora, rtol=4e-16, atol=0)


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
@pytest.mark.parametrize("n,slices", [(64, 1), (160, 2)])
def test_step(levels, n, slices):
    import torch
    import paper_2204_10252_amd as pf
    rng = np.random.default_rng(levels * 7 + n)
    shape = (slices, n, n)
    z, pg, xo = (c64(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) for _ in range(3))
    plan = _plan(n, 1, slices, "2d", levels=levels)
    lam, beta = 0.35, 0.6
    tz, tp, to = to_dev(z), to_dev(pg), to_dev(xo)
    xn, zn = torch.empty_like(tz), torch.empty_like(tz)
    red = torch.zeros(3, dtype=torch.float64, device=tz.device)
    pf.step(plan, tz, tp, to, xn, zn, lam, beta, red)
    rx, rz = orc.pfista_step(z.astype(np.complex128), pg.astype(np.complex128),
                             xo.astype(np.complex128), lam, levels, beta)
    assert rel(xn.cpu().numpy(), rx) <= 1e-5
    assert rel(zn.cpu().numpy(), rz) <= 1e-5
    r = red.cpu().numpy()
    l1 = np.sum(np.abs(orc.haar_fwd(rx, levels)))
    assert r[0] == pytest.approx(l1, rel=1e-5)
    assert r[1] == pytest.approx(np.linalg.norm(rx - xo) ** 2, rel=1e-5)
    assert r[2] == pytest.approx(np.linalg.norm(rx) ** 2, rel=1e-5)
    # in place (x_new = x_old, z_new = z) gives the same values
    pf.step(plan, tz, tp, to, to, tz, lam, beta, red)
    assert torch.equal(to, xn) and torch.equal(tz, zn)


def test_step_threshold_edge_cases():
    import torch
    import paper_2204_10252_amd as pf
    n = 64
    plan = _plan(n, 1, 1, "2d", levels=3)
    z = np.zeros((1, n, n), np.complex64)
    z[0, :8, :8] = 1.0 + 1.0j         # one constant 8x8 tile: a single coarse coefficient
    zero = np.zeros_like(z)
    tz, tp, to = to_dev(z), to_dev(zero), to_dev(zero)
    xn, zn = torch.empty_like(tz), torch.empty_like(tz)
    red = torch.zeros(3, dtype=torch.float64, device=tz.device)
    # coarse coefficient of the tile = 8 (1 + i); threshold just above |.| -> all zero
    pf.step(plan, tz, tp, to, xn, zn, float(8 * np.sqrt(2)) * 1.0001, 0.0, red)
    assert float(xn.abs().max()) == 0.0
    pf.step(plan, tz, tp, to, xn, zn, 1.0, 0.0, red)
    rx, _ = orc.pfista_step(z.astype(complex), zero.astype(complex), zero.astype(complex), 1.0, 3, 0.0)
    assert rel(xn.cpu().numpy(), rx) <= 1e-6


def test_deterministic():
    import torch
    import paper_2204_10252_amd as pf
    sens, mask, x, _ = random_case(256, 16, 1, "2d", seed=5)
    plan = _plan(256, 16, 1, "2d")
    ts, tm, tx = to_dev(sens), to_dev(mask), to_dev(x)
    y1, y2 = torch.empty_like(tx), torch.empty_like(tx)
    pf.normal_apply(plan, ts, tm, tx, y1)
    pf.normal_apply(plan, ts, tm, tx, y2)
    assert torch.equal(y1, y2)


def test_power_iteration_and_data_term():
    import torch
    import paper_2204_10252_amd as pf
    sens, mask, x, _ = random_case(128, 4, 1, "2d", seed=11)
    plan = _plan(128, 4, 1, "2d")
    ts, tm = to_dev(sens), to_dev(mask)
    v0 = c64(np.random.default_rng(0).standard_normal((1, 128, 128)) + 0j)
    v = to_dev(v0)
    lam = pf.power_iteration(plan, ts, tm, 40, v=v)
    ref = orc.power_iteration(sens.astype(np.complex128), mask, v0.astype(np.complex128), 40)
    assert lam == pytest.approx(ref, rel=1e-5)
    lam2 = pf.power_iteration(plan, ts, tm, 40)          # internal start vector
    assert 0.9 < lam2 <= 1.0 + 1e-6
    rng = np.random.default_rng(1)
    b = c64(orc.forward(sens.astype(complex), mask, rng.standard_normal((1, 128, 128)) + 0j))
    dt = pf.data_term(plan, ts, tm, to_dev(b), to_dev(x), 0.8, 1.0 / 3.0)
    r = np.sqrt(0.8) * orc.forward(sens.astype(complex), mask, x.astype(complex)) - b / 3.0
    assert dt == pytest.approx(0.5 * np.vdot(r, r).real, rel=1e-5)


def test_validation_errors():
    import torch
    import paper_2204_10252_amd as pf
    with pytest.raises(pf.PfistaError) as e:
        pf.Plan(100, 2, 1)
    assert e.value.code == pf.UNSUPPORTED
    with pytest.raises(pf.PfistaError) as e:
        pf.Plan(64, 2, 1, haar_levels=5)
    assert e.value.code == pf.UNSUPPORTED
    plan = _plan(64, 2, 1, "2d")
    sens, mask, x, _ = random_case(64, 2, 1, "2d", seed=1)
    tx = to_dev(x)
    with pytest.raises(pf.PfistaError) as e:
        pf.normal_apply(plan, to_dev(sens), to_dev(mask), tx, tx)    # y aliases x
    assert e.value.code == pf.EINVAL
    # zero slices is a valid no-op
    p0 = pf.Plan(64, 2, 0)
    empty = torch.empty((0, 64, 64), dtype=torch.complex64, device=tx.device)
    pf.normal_apply(p0, torch.empty((0, 2, 64, 64), dtype=torch.complex64, device=tx.device),
                    torch.empty((0, 64, 64), dtype=torch.uint8, device=tx.device), empty,
                    torch.empty_like(empty))


@pytest.mark.parametrize("n,coils,slices,kind", [(384, 3, 2, "1d"), (160, 2, 3, "2d"), (512, 1, 1, "1d")])
def test_data_term_and_power_iteration_other_shapes(n, coils, slices, kind):
    # the residual column pass of phase-encode masks and of several slices
    import paper_2204_10252_amd as pf
    sens, mask, x, _ = random_case(n, coils, slices, kind, seed=n + slices)
    plan = _plan(n, coils, slices, kind)
    ts, tm = to_dev(sens), to_dev(mask)
    rng = np.random.default_rng(2)
    b = c64(orc.forward(sens.astype(complex), mask, rng.standard_normal((slices, n, n)) + 0j))
    dt = pf.data_term(plan, ts, tm, to_dev(b), to_dev(x), 0.7, 0.5)
    r = np.sqrt(0.7) * orc.forward(sens.astype(complex), mask, x.astype(complex)) - 0.5 * b
    assert dt == pytest.approx(0.5 * np.vdot(r, r).real, rel=1e-5)
    v0 = c64(rng.standard_normal((slices, n, n)) + 1j * rng.standard_normal((slices, n, n)))
    lam = pf.power_iteration(plan, ts, tm, 20, v=to_dev(v0))
    ref = orc.power_iteration(sens.astype(np.complex128), mask, v0.astype(np.complex128), 20)
    assert lam == pytest.approx(ref, rel=1e-5)
