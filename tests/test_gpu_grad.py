"""GPU parity of the derivative of unrolled PFISTA (dL/dlambda, dL/dc_i)
against the FP64 oracle's pull-back, plus the torch autograd wrapper.

Both sides get the same complex64 inputs, the same inv_l (oracle power
iteration) and the same cotangent.  Bars: x_K within 1e-4 (the solve's bar);
every gradient component within 1e-3 of the largest one (a K-step chain of
FP32 applies and thresholds, each within ~1e-5, feeds the pull-back; the FP32
derivative is piecewise smooth: it jumps where a Haar coefficient crosses the
threshold, so the comparison is made at thresholds where no coefficient of the
FP64 path lies within 2e-4 lambda of it), checked separately for dL/dlambda and
for the coefficient gradient.
"""

import numpy as np
import pytest

import oracle as orc
from synth import make_inputs, power_start_vector
from tests.gpu_util import c64, rel, to_dev

pytestmark = pytest.mark.gpu


def problem(wid, power_iters=60):
    inp = make_inputs(wid)
    sens = c64(inp["sens"])
    s128 = sens.astype(np.complex128)
    b = c64(orc.kspace_data(s128, inp["mask"], inp["phantom"], inp["noise"]))
    lam_max = orc.power_iteration(s128, inp["mask"], power_start_vector(inp["n"], inp["slices"]), power_iters)
    inv_l = 1.0 / (1.01 * lam_max)
    bn = b.astype(np.complex128) / np.linalg.norm(b.astype(np.complex128))
    return inp, sens, s128, b, bn, inv_l


@pytest.fixture(scope="module")
def w1():
    return problem(1)


def gpu_unrolled(inp, degree, iters, inv_l, ckpt_every=5, momentum=True, tune=0):
    import paper_2204_10252_amd as pf
    plan = pf.Plan(inp["n"], inp["coils"], inp["slices"], haar_levels=inp["levels"])
    return pf.Unrolled(plan, degree, iters, inv_l, ckpt_every=ckpt_every, momentum=momentum, tune=tune)


def smooth_lambda(inp, s128, bn, inv_l, coef, levels, K, momentum=True, lam0=None):
    """A threshold near lam0 at which no Haar coefficient of the FP64 path comes
    within 2e-4 lambda of the threshold (ten times the FP32 error of a
    coefficient here): the derivative jumps where a coefficient crosses it, so
    FP32 and FP64 runs agree on it only away from such points."""
    lam0 = inp["lam"] if lam0 is None else lam0
    for j in range(80):
        lam = lam0 * (1.0 + 0.013 * j)
        _, tape = orc.unrolled_forward(s128, inp["mask"], bn, inv_l, lam, coef, levels, K, momentum)
        dist = min(float(np.min(np.abs(np.abs(orc.haar_fwd(z - pg, levels)) - lam))) for z, _, pg, _ in tape)
        if dist > 2e-4 * lam:
            return lam
    raise AssertionError("no threshold away from the kinks")


def close(got, want):
    """dL/dlambda within 1e-3 relative; dL/dc within 1e-3 of its largest entry."""
    assert abs(got[0] - want[0]) <= 1e-3 * abs(want[0])
    np.testing.assert_allclose(got[1:], want[1:], rtol=1e-3, atol=1e-3 * np.abs(want[1:]).max())


def coefs(degree):
    return [1.0] if degree == 0 else [float(c) for c in orc.l2_poly_coefficients(degree)]


@pytest.mark.parametrize("degree,momentum", [(3, True), (0, True), (1, True), (2, False)])
def test_gradient_matches_oracle(w1, degree, momentum):
    import torch
    inp, sens, s128, b, bn, inv_l = w1
    K = 12
    coef = coefs(degree)
    lam = smooth_lambda(inp, s128, bn, inv_l, coef, inp["levels"], K, momentum)
    u = gpu_unrolled(inp, degree, K, inv_l, momentum=momentum)
    ts, tm, tb = to_dev(sens), to_dev(inp["mask"]), to_dev(b)
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    u.forward(ts, tm, tb, x, lam, coef)
    xo, _ = orc.unrolled_forward(s128, inp["mask"], bn, inv_l, lam, coef, inp["levels"], K, momentum)
    assert rel(x.cpu().numpy(), xo) <= 1e-4
    rng = np.random.default_rng(5)
    xbar = c64(rng.standard_normal(xo.shape) + 1j * rng.standard_normal(xo.shape))
    gl, gc = u.backward(ts, tm, to_dev(xbar), lam, coef)
    ol, oc = orc.unrolled_vjp(s128, inp["mask"], bn, inv_l, lam, coef, inp["levels"], K,
                              xbar.astype(np.complex128), momentum)
    want = np.concatenate([[ol], oc])
    got = np.concatenate([[gl], gc])
    print("grad gpu", got, "oracle", want, flush=True)
    close(got, want)


@pytest.mark.parametrize("levels", [1, 2, 4])
def test_gradient_every_haar_depth(w1, levels):
    # the pull-back's level recursion at every supported depth (W1 itself uses 3)
    import torch
    inp, sens, s128, b, bn, inv_l = w1
    inp = dict(inp, levels=levels)
    K, coef = 8, coefs(2)
    lam = smooth_lambda(inp, s128, bn, inv_l, coef, levels, K)
    u = gpu_unrolled(inp, 2, K, inv_l)
    ts, tm, tb = to_dev(sens), to_dev(inp["mask"]), to_dev(b)
    x = torch.empty((1, 64, 64), dtype=torch.complex64, device="cuda")
    u.forward(ts, tm, tb, x, lam, coef)
    xo, _ = orc.unrolled_forward(s128, inp["mask"], bn, inv_l, lam, coef, levels, K)
    assert rel(x.cpu().numpy(), xo) <= 1e-4
    rng = np.random.default_rng(20 + levels)
    xbar = c64(rng.standard_normal(xo.shape) + 1j * rng.standard_normal(xo.shape))
    gl, gc = u.backward(ts, tm, to_dev(xbar), lam, coef)
    ol, oc = orc.unrolled_vjp(s128, inp["mask"], bn, inv_l, lam, coef, levels, K, xbar.astype(np.complex128))
    close(np.concatenate([[gl], gc]), np.concatenate([[ol], oc]))


@pytest.mark.parametrize("tune", [2, 6, 12, -1])
def test_gradient_in_other_launch_shapes(w1, tune):
    # forced candidates (second radix schedule, separate row passes, larger
    # coil-combine blocks) and the tuned one give the same iterate and gradient
    import torch
    inp, sens, s128, b, bn, inv_l = w1
    K, coef = 8, coefs(3)
    lam = smooth_lambda(inp, s128, bn, inv_l, coef, inp["levels"], K)
    u = gpu_unrolled(inp, 3, K, inv_l, tune=tune)
    ts, tm, tb = to_dev(sens), to_dev(inp["mask"]), to_dev(b)
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    u.forward(ts, tm, tb, x, lam, coef)
    xo, _ = orc.unrolled_forward(s128, inp["mask"], bn, inv_l, lam, coef, inp["levels"], K)
    assert rel(x.cpu().numpy(), xo) <= 1e-4
    rng = np.random.default_rng(40)
    xbar = c64(rng.standard_normal(xo.shape) + 1j * rng.standard_normal(xo.shape))
    gl, gc = u.backward(ts, tm, to_dev(xbar), lam, coef)
    ol, oc = orc.unrolled_vjp(s128, inp["mask"], bn, inv_l, lam, coef, inp["levels"], K, xbar.astype(np.complex128))
    close(np.concatenate([[gl], gc]), np.concatenate([[ol], oc]))


def test_checkpoint_interval_does_not_change_the_gradient(w1):
    import torch
    inp, sens, s128, b, bn, inv_l = w1
    coef = coefs(2)
    ts, tm, tb = to_dev(sens), to_dev(inp["mask"]), to_dev(b)
    rng = np.random.default_rng(6)
    xbar = to_dev(c64(rng.standard_normal((1, 64, 64)) + 1j * rng.standard_normal((1, 64, 64))))
    res = []
    for ck in (1, 3, 5, 11, 50):
        u = gpu_unrolled(inp, 2, 11, inv_l, ckpt_every=ck)
        x = torch.empty((1, 64, 64), dtype=torch.complex64, device="cuda")
        u.forward(ts, tm, tb, x, inp["lam"], coef)
        res.append((x.cpu().numpy(), u.backward(ts, tm, xbar, inp["lam"], coef)))
    for xr, g in res[1:]:
        assert np.array_equal(xr, res[0][0])
        assert g == res[0][1]


def test_autograd_mse_to_phantom(w1):
    # loss = mean |s x_K - phantom|^2 with s = sqrt(inv_l) ||b|| (x_K in original units)
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = w1
    K, degree = 10, 3
    u = gpu_unrolled(inp, degree, K, inv_l)
    scale = np.sqrt(inv_l) * np.linalg.norm(b.astype(np.complex128))
    lam_v = smooth_lambda(inp, s128, bn, inv_l, coefs(degree), inp["levels"], K)
    lam = torch.tensor(lam_v, dtype=torch.float64, requires_grad=True)
    coef = torch.tensor(coefs(degree), dtype=torch.float64, requires_grad=True)
    ph = to_dev(c64(inp["phantom"]))
    x = pf.unrolled_pfista(lam, coef, u, to_dev(sens), to_dev(inp["mask"]), to_dev(b))
    loss = torch.mean(torch.abs(scale * x - ph) ** 2)
    loss.backward()
    # oracle: the same loss, cotangent dL/dRe x + i dL/dIm x = 2 s (s x - phantom) / M
    xo, _ = orc.unrolled_forward(s128, inp["mask"], bn, inv_l, lam_v, coefs(degree), inp["levels"], K)
    xbar = 2.0 * scale * (scale * xo - inp["phantom"]) / xo.size
    ol, oc = orc.unrolled_vjp(s128, inp["mask"], bn, inv_l, lam_v, coefs(degree), inp["levels"], K, xbar)
    want = np.concatenate([[ol], oc])
    got = np.concatenate([[lam.grad.item()], coef.grad.numpy()])
    print("autograd", got, "oracle", want, flush=True)
    close(got, want)
    assert loss.item() == pytest.approx(float(np.mean(np.abs(scale * xo - inp["phantom"]) ** 2)), rel=1e-4)


def test_autograd_two_forwards_before_their_backwards(w1):
    # two calls on one Unrolled (different thresholds and data scale), then the
    # backward passes in reverse order: each must get its own call's gradient
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = w1
    K, degree = 6, 2
    u = gpu_unrolled(inp, degree, K, inv_l, ckpt_every=3)
    cf = coefs(degree)
    lam_a = smooth_lambda(inp, s128, bn, inv_l, cf, inp["levels"], K)
    lam_b = smooth_lambda(inp, s128, bn, inv_l, cf, inp["levels"], K, lam0=3.0 * inp["lam"])
    ts, tm, tb = to_dev(sens), to_dev(inp["mask"]), to_dev(b)
    xbar_o = np.full(inp["phantom"].shape, 0.5 - 0.25j)
    calls = []
    for lam_v in (lam_a, lam_b):
        lam = torch.tensor(lam_v, dtype=torch.float64, requires_grad=True)
        coef = torch.tensor(cf, dtype=torch.float64, requires_grad=True)
        x = pf.unrolled_pfista(lam, coef, u, ts, tm, tb)
        # L = Re <x_bar, x>: its cotangent is x_bar
        loss = torch.sum(torch.real(torch.conj(to_dev(c64(xbar_o))) * x))
        calls.append((lam_v, lam, coef, loss))
    for lam_v, lam, coef, loss in reversed(calls):
        loss.backward()
        ol, oc = orc.unrolled_vjp(s128, inp["mask"], bn, inv_l, lam_v, cf, inp["levels"], K, xbar_o)
        close(np.concatenate([[lam.grad.item()], coef.grad.numpy()]), np.concatenate([[ol], oc]))


def test_unrolled_rejects_bad_parameters(w1):
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = w1
    with pytest.raises(pf.PfistaError):
        gpu_unrolled(inp, 2, 0, inv_l)
    with pytest.raises(pf.PfistaError):
        gpu_unrolled(inp, 2, 5, 0.0)
    with pytest.raises(pf.PfistaError):
        gpu_unrolled(inp, 2, 5, inv_l, tune=13)


def test_workload5_full_size():
    # 8 slices 192 x 192, 12 coils, R = 5, d = 4, 20 unrolled iterations,
    # checkpoints every 5; MSE to the phantom
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = problem(5, power_iters=30)
    K, degree = 20, 4
    u = gpu_unrolled(inp, degree, K, inv_l, ckpt_every=5)
    scale = np.sqrt(inv_l) * np.linalg.norm(b.astype(np.complex128))
    ts, tm, tb = to_dev(sens), to_dev(inp["mask"]), to_dev(b)
    ph = to_dev(c64(inp["phantom"]))

    def loss_of(lv, cv):
        lam = torch.tensor(lv, dtype=torch.float64, requires_grad=True)
        coef = torch.tensor(cv, dtype=torch.float64, requires_grad=True)
        x = pf.unrolled_pfista(lam, coef, u, ts, tm, tb)
        loss = torch.mean(torch.abs(scale * x - ph) ** 2)
        return loss, lam, coef, x

    c0 = coefs(degree)
    loss, lam, coef, x = loss_of(inp["lam"], c0)
    loss.backward()
    got = np.concatenate([[lam.grad.item()], coef.grad.numpy()])
    xo, _ = orc.unrolled_forward(s128, inp["mask"], bn, inv_l, inp["lam"], c0, inp["levels"], K)
    assert rel(x.detach().cpu().numpy(), xo) <= 1e-4
    xbar = 2.0 * scale * (scale * xo - inp["phantom"]) / xo.size
    ol, oc = orc.unrolled_vjp(s128, inp["mask"], bn, inv_l, inp["lam"], c0, inp["levels"], K, xbar)
    want = np.concatenate([[ol], oc])
    print("W5 grad gpu", got, "oracle", want, flush=True)
    close(got, want)
    # central differences of the FP32 forward: step 1e-3 on each coefficient,
    # 1e-3 relative on lambda (lambda itself is 5e-4)
    theta = np.array([inp["lam"]] + c0)
    for j in range(theta.size):
        h = 1e-3 * abs(theta[j]) if j == 0 else 1e-3
        tp, tm_ = theta.copy(), theta.copy()
        tp[j] += h
        tm_[j] -= h
        with torch.no_grad():
            lp = loss_of(tp[0], list(tp[1:]))[0].item()
            lm = loss_of(tm_[0], list(tm_[1:]))[0].item()
        fd = (lp - lm) / (2 * h)
        print(f"W5 fd[{j}] {fd:.6e} analytic {got[j]:.6e}", flush=True)
        assert fd == pytest.approx(got[j], rel=2e-2)
