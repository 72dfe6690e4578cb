"""GPU parity of the full PFISTA solve (Algorithm 4) against the FP64 oracle.

Both sides get the same complex64 inputs, the same k-space data (formed by
the oracle in FP64, then rounded) and the same normalisation scalar (the
oracle's FP64 power iteration, 100 steps from the seeded start vector, with a
1 % margin).  Bar: relative l2 error of the final iterate <= 1e-4.
"""

import numpy as np
import pytest

import oracle as orc
from synth import make_inputs, power_start_vector
from tests.gpu_util import c64, rel, to_dev

pytestmark = pytest.mark.gpu


def problem(wid, slices=None):
    inp = make_inputs(wid, slices)
    sens = c64(inp["sens"])
    s128 = sens.astype(np.complex128)
    img = inp["phantom"]
    b = c64(orc.kspace_data(s128, inp["mask"], img, inp["noise"]))
    lam_max = orc.power_iteration(s128, inp["mask"], power_start_vector(inp["n"], inp["slices"]), 100)
    inv_l = 1.0 / (1.01 * lam_max)
    bn = b.astype(np.complex128) / np.linalg.norm(b.astype(np.complex128))
    return inp, sens, s128, b, bn, inv_l


def gpu_plan(inp):
    import paper_2204_10252_amd as pf
    return pf.Plan(inp["n"], inp["coils"], inp["slices"], haar_levels=inp["levels"],
                   mask_kind=pf.MASK_1D if inp["mask_kind"] == "1d" else pf.MASK_2D)


@pytest.fixture(scope="module")
def c1():
    return problem(1)


@pytest.mark.parametrize("degree", [None, 1, 3, 5])
def test_solve_workload1(c1, degree):
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    coef = [1.0] if degree is None else [float(c) for c in orc.l2_poly_coefficients(degree)]
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    rep = pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], coef=coef,
                   max_iter=50, inv_l=inv_l, eval_objective=True)
    xo, _, hist = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], 50,
                             history=True)
    assert rel(x.cpu().numpy(), xo) <= 1e-4
    assert rep["objective"] == pytest.approx(hist[-1], rel=1e-5)
    assert rep["iters"] == 50 and rep["normal_applies"] == 50 * len(coef)


def test_solve_workload2_short():
    # the benchmark's launch configuration: graph replay of 10 iterations on a side stream
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = problem(2)
    plan = gpu_plan(inp)
    coef = [float(c) for c in orc.l2_poly_coefficients(3)]
    x = torch.empty((1, 256, 256), dtype=torch.complex64, device="cuda")
    pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], coef=coef,
             max_iter=15, inv_l=inv_l)
    xo, _, _ = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], 20)
    xo15, _, _ = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], 15)
    assert rel(x.cpu().numpy(), xo15) <= 1e-4
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xg = torch.empty_like(x)
        pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), xg, inp["lam"], coef=coef,
                 max_iter=20, inv_l=inv_l, check_every=20, graph_iters=10, stream=s)
    s.synchronize()
    assert rel(xg.cpu().numpy(), xo) <= 1e-4


def test_history_resume_and_graph_are_consistent(c1):
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    ts, tm, tb = to_dev(sens), to_dev(inp["mask"]), to_dev(b)
    shp = (1, inp["n"], inp["n"])
    # per-iteration objective history against the oracle's
    x = torch.empty(shp, dtype=torch.complex64, device="cuda")
    rep = pf.solve(plan, ts, tm, tb, x, inp["lam"], degree=2, max_iter=12, inv_l=inv_l,
                   check_every=1, history=True)
    _, _, hist = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"],
                            orc.l2_poly_coefficients(2), inp["levels"], 12, history=True)
    np.testing.assert_allclose(rep["history"], hist, rtol=1e-5)
    # 20 iterations == 10 + resumed 10, bit for bit
    xa, za = torch.empty(shp, dtype=torch.complex64, device="cuda"), torch.empty(shp, dtype=torch.complex64, device="cuda")
    pf.solve(plan, ts, tm, tb, xa, inp["lam"], degree=2, max_iter=20, inv_l=inv_l, z=za)
    xb, zb = torch.empty_like(xa), torch.empty_like(za)
    pf.solve(plan, ts, tm, tb, xb, inp["lam"], degree=2, max_iter=10, inv_l=inv_l, z=zb)
    pf.solve(plan, ts, tm, tb, xb, inp["lam"], degree=2, max_iter=10, inv_l=inv_l, z=zb, k0=10)
    assert torch.equal(xa, xb) and torch.equal(za, zb)
    # a captured HIP graph replays exactly the launched iterations
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xg = torch.empty_like(xa)
        pf.solve(plan, ts, tm, tb, xg, inp["lam"], degree=2, max_iter=20, inv_l=inv_l,
                 check_every=10, graph_iters=5, stream=s)
    s.synchronize()
    assert torch.equal(xa, xg)


def test_power_iteration_estimate_in_solve(c1):
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    rep = pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], degree=3,
                   max_iter=1, inv_l=0.0, power_iters=100)
    assert rep["inv_l"] == pytest.approx(inv_l, rel=1e-3)
    assert rep["bnorm"] == pytest.approx(np.linalg.norm(b.astype(np.complex128)), rel=1e-6)


def test_literal_degree_zero_fit_is_reported_as_divergence(c1):
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    rep = pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], coef=[1.5],
                   max_iter=400, inv_l=inv_l * 1.01, check_every=20, eval_objective=True,
                   raise_on_diverge=False)
    assert rep["rc"] == pf.DIVERGED and rep["iters"] < 400


def test_lambda_zero_matches_oracle(c1):
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, 0.0, degree=2, max_iter=40,
             inv_l=inv_l)
    xo, _, _ = orc.pfista(s128, inp["mask"], bn, inv_l, 0.0, orc.l2_poly_coefficients(2),
                          inp["levels"], 40)
    assert rel(x.cpu().numpy(), xo) <= 1e-4


@pytest.mark.parametrize("design", ["plain", "l2", "chebyshev", "weighted"])
def test_pgd_ppgd_and_polynomial_designs(c1, design):
    # Algorithms 1 and 3 (no momentum) and the Section 2.5 design variants
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    coef = {"plain": [1.0],
            "l2": [float(c) for c in orc.l2_poly_coefficients(3)],
            "chebyshev": [float(c) for c in orc.chebyshev_poly_coefficients(3, 0.05)],
            "weighted": [float(c) for c in orc.weighted_l2_poly_coefficients(3, 1.0)]}[design]
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], coef=coef,
             max_iter=30, inv_l=inv_l, momentum=False)
    yo, _ = orc.pgd(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], 30)
    assert rel(x.cpu().numpy(), yo) <= 1e-4


@pytest.mark.parametrize("tune", list(range(1, 13)))
def test_every_forced_launch_shape_matches_oracle(c1, tune):
    # every launch-shape candidate computes the same iteration
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    coef = [float(c) for c in orc.l2_poly_coefficients(3)]
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    rep = pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], coef=coef,
                   max_iter=30, inv_l=inv_l, tune=tune)
    assert rep["candidate"] == tune - 1 and rep["tune_us"] == 0.0
    xo, _, _ = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], 30)
    assert rel(x.cpu().numpy(), xo) <= 1e-4


@pytest.mark.parametrize("n", [160, 192, 256, 320, 384, 512])
@pytest.mark.parametrize("tune", [2, 4])
def test_second_radix_schedule_at_every_image_side_matches_oracle(n, tune):
    # candidates 1 and 3 (fused and separate row passes) run the radix schedules
    # with twice the lanes per transform, whose column pass has half as many
    # columns per workgroup; every image side of the library, 2-D masks
    import torch
    import paper_2204_10252_amd as pf
    from tests.gpu_util import random_case
    sens, mask, img, _ = random_case(n, 3, 1, "2d", seed=900 + n + tune)
    s128 = sens.astype(np.complex128)
    noise = 1e-3 * np.random.default_rng(n).standard_normal(s128.shape)
    b = c64(orc.kspace_data(s128, mask, img.astype(np.complex128), noise))
    bn = b.astype(np.complex128) / np.linalg.norm(b.astype(np.complex128))
    inv_l = 1.0 / 1.01   # coil maps with sum |S|^2 = 1 and a 0/1 mask: ||A^H A|| <= 1
    lam, levels, iters = 1e-3, 4, 6
    coef = [float(c) for c in orc.l2_poly_coefficients(2)]
    plan = pf.Plan(n, 3, 1, haar_levels=levels)
    x = torch.empty((1, n, n), dtype=torch.complex64, device="cuda")
    rep = pf.solve(plan, to_dev(sens), to_dev(mask), to_dev(b), x, lam, coef=coef,
                   max_iter=iters, inv_l=inv_l, tune=tune)
    assert rep["candidate"] == tune - 1
    xo, _, _ = orc.pfista(s128, mask, bn, inv_l, lam, coef, levels, iters)
    assert rel(x.cpu().numpy(), xo) <= 1e-4


def test_tuned_solve_workload2_is_cached_and_matches_oracle():
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = problem(2)
    plan = gpu_plan(inp)
    coef = [float(c) for c in orc.l2_poly_coefficients(3)]
    args = (plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b))
    x = torch.empty((1, 256, 256), dtype=torch.complex64, device="cuda")
    r1 = pf.solve(*args, x, inp["lam"], coef=coef, max_iter=15, inv_l=inv_l, tune=-1)
    assert 0 <= r1["candidate"] < pf.TUNE_CANDIDATES and r1["tune_us"] > 0.0
    xo, _, _ = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], 15)
    assert rel(x.cpu().numpy(), xo) <= 1e-4
    x2 = torch.empty_like(x)
    r2 = pf.solve(*args, x2, inp["lam"], coef=coef, max_iter=15, inv_l=inv_l, tune=-1)
    assert (r2["candidate"], r2["tune_us"]) == (r1["candidate"], r1["tune_us"])
    assert torch.equal(x, x2)


def test_phase_encode_plan_ignores_forced_shape():
    # phase-encode masks have one launch shape: a forced candidate runs it
    import torch
    import paper_2204_10252_amd as pf
    inp = make_inputs(3, 1)
    sens = c64(inp["sens"])
    s128 = sens.astype(np.complex128)
    b = c64(orc.kspace_data(s128, inp["mask"], inp["phantom"], inp["noise"]))
    bn = b.astype(np.complex128) / np.linalg.norm(b.astype(np.complex128))
    inv_l = 1.0 / 1.01      # ||A||^2 <= 1 for root-sum-of-squares normalised maps
    plan = gpu_plan(inp)
    coef = [float(c) for c in orc.l2_poly_coefficients(2)]
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    rep = pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], coef=coef,
                   max_iter=5, inv_l=inv_l, tune=6)
    assert rep["candidate"] == 0
    xo, _, _ = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], 5)
    assert rel(x.cpu().numpy(), xo) <= 1e-4


@pytest.mark.parametrize("tune", [-2, 13])
def test_tune_outside_range_is_rejected(c1, tune):
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    x = torch.zeros((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    with pytest.raises(pf.PfistaError) as e:
        pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], degree=1,
                 max_iter=2, inv_l=inv_l, tune=tune)
    assert e.value.code == pf.EINVAL


@pytest.fixture(scope="module")
def w2():
    return problem(2)


@pytest.mark.parametrize("degree", [0, 1, 2, 3, 4, 5])
def test_workload2_fp32_against_fp64_per_degree(w2, degree):
    # the FP32 path against the FP64 oracle at 256 x 256, 16 coils for plain FISTA
    # (degree 0: p = 1) and every fitted degree, the workload's 200 iterations each
    import os
    import scipy.fft
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = w2
    iters = 200
    plan = gpu_plan(inp)
    coef = [1.0] if degree == 0 else [float(c) for c in orc.l2_poly_coefficients(degree)]
    x = torch.empty((1, 256, 256), dtype=torch.complex64, device="cuda")
    args = (plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        # the benchmark's launch configuration: graph replay on a side stream
        rep = pf.solve(*args, inp["lam"], coef=coef, max_iter=iters, inv_l=inv_l, eval_objective=True,
                       graph_iters=10, stream=s)
    s.synchronize()
    # the oracle's FFTs split over the host's cores (independent transforms: same values)
    with scipy.fft.set_workers(min(16, os.cpu_count() or 1)):
        xo, _, _ = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], iters)
        fo = orc.objective(s128, inp["mask"], bn, inv_l, xo, inp["lam"], inp["levels"])
    err = rel(x.cpu().numpy(), xo)
    print(f"W2 degree {degree}: {iters} iterations, final-iterate FP32 vs FP64 relative error {err:.2e}, "
          f"objective {abs(rep['objective'] - fo) / fo:.2e}", flush=True)
    assert err <= 1e-4
    assert rep["objective"] == pytest.approx(fo, rel=1e-5)


def test_fixed_point_residual_of_a_converged_solve(c1):
    # a converged GPU PFISTA run (d = 3) is a fixed point of its own map: the
    # preconditioned fixed-point condition y = prox(y - P(N'y - A'^H b')), here
    # evaluated in FP64 by the oracle on the GPU's final iterate
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    coef = [float(c) for c in orc.l2_poly_coefficients(3)]
    plan = gpu_plan(inp)
    x = torch.empty((inp["slices"], inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], coef=coef, max_iter=800,
             inv_l=inv_l, graph_iters=10)
    y = x.cpu().numpy().astype(np.complex128)
    ahb = np.sqrt(inv_l) * orc.adjoint(s128, inp["mask"], bn)
    g = orc.normal(s128, inp["mask"], y, inv_l) - ahb
    ty = orc.prox_l1_haar(y - orc.poly_apply(s128, inp["mask"], inv_l, coef, g), inp["lam"], inp["levels"])
    res = np.linalg.norm(ty - y) / np.linalg.norm(y)
    print(f"fixed-point residual after 800 iterations: {res:.2e}", flush=True)
    assert res <= 1e-4


@pytest.mark.parametrize("degree,iters", [(0, 2000), (3, 600)])
def test_converged_objective_matches_oracle(c1, degree, iters):
    # the time-to-tolerance reference F_inf is taken from a long GPU run; at the
    # small workload the same long run in the FP64 oracle gives the same value
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    plan = gpu_plan(inp)
    coef = [1.0] if degree == 0 else [float(c) for c in orc.l2_poly_coefficients(degree)]
    x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
    rep = pf.solve(plan, to_dev(sens), to_dev(inp["mask"]), to_dev(b), x, inp["lam"], coef=coef,
                   max_iter=iters, inv_l=inv_l, eval_objective=True, check_every=iters)
    _, _, hist = orc.pfista(s128, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], iters, history=True)
    assert rep["objective"] == pytest.approx(hist[-1], rel=1e-6)
    # and it is converged: the last 10 % of the iterations moved F by less than 1e-6
    assert abs(hist[-1] - hist[int(0.9 * iters)]) <= 1e-6 * hist[-1]


def test_concurrent_solves_from_two_host_threads(c1):
    # two plans solved at once from two host threads on their own streams (the
    # library keeps no shared mutable state besides its locked tuner cache and
    # per-thread error messages); each result equals the same solve run alone
    import threading
    import torch
    import paper_2204_10252_amd as pf
    inp, sens, s128, b, bn, inv_l = c1
    args = (to_dev(sens), to_dev(inp["mask"]), to_dev(b))
    coef = [float(c) for c in orc.l2_poly_coefficients(3)]

    def run(plan, x, stream, tune, out):
        with torch.cuda.stream(stream):
            out.append(pf.solve(plan, *args, x, inp["lam"], coef=coef, max_iter=40, inv_l=inv_l, graph_iters=5,
                                check_every=20, tune=tune, stream=stream))
        stream.synchronize()

    ref = []
    for tune in (0, -1):
        x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda")
        run(gpu_plan(inp), x, torch.cuda.Stream(), tune, [])
        ref.append(x.clone())
    plans = [gpu_plan(inp), gpu_plan(inp)]
    xs = [torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device="cuda") for _ in plans]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [[], []]
    torch.cuda.synchronize()
    threads = [threading.Thread(target=run, args=(plans[i], xs[i], streams[i], (0, -1)[i], outs[i]))
               for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert all(len(o) == 1 and o[0]["rc"] == pf.OK for o in outs)
    for i in range(2):
        assert torch.equal(xs[i], ref[i])


_CACHE_SCRIPT = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
import paper_2204_10252_amd as pf
from synth import make_inputs
inp = make_inputs(1)
dev = torch.device("cuda", 0)
plan = pf.Plan(inp["n"], inp["coils"], 1, haar_levels=inp["levels"])
sens = torch.from_numpy(inp["sens"].astype(np.complex64)).to(dev)
mask = torch.from_numpy(inp["mask"]).to(dev)
b = torch.empty((1, inp["coils"], inp["n"], inp["n"]), dtype=torch.complex64, device=dev)
pf.forward(plan, sens, mask, torch.from_numpy(inp["phantom"].astype(np.complex64)).to(dev), b)
x = torch.empty((1, inp["n"], inp["n"]), dtype=torch.complex64, device=dev)
rep = pf.solve(plan, sens, mask, b, x, inp["lam"], degree=3, max_iter=3, inv_l=0.9, tune=-1)
print("CANDIDATE", rep["candidate"], rep["tune_us"])
"""


def test_tuner_cache_file(tmp_path):
    # a tuned solve writes its choice to $PFISTA_TUNE_CACHE; a later process reads
    # it back (here an entry edited to candidate 6) instead of timing again
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, PFISTA_TUNE_CACHE=str(cache))

    def run():
        out = subprocess.run([sys.executable, "-c", _CACHE_SCRIPT, root], env=env, capture_output=True,
                             text=True, timeout=240)
        assert out.returncode == 0, out.stderr[-2000:]
        line = [ln for ln in out.stdout.splitlines() if ln.startswith("CANDIDATE")][-1].split()
        return int(line[1]), float(line[2])

    cand, us = run()
    lines = cache.read_text().split("\n")
    entry = [ln for ln in lines if "|plan|n64|s1|c4|" in ln]
    assert len(entry) == 1 and int(entry[0].split()[1]) == cand and us > 0
    key = entry[0].split()[0]
    cache.write_text(f"{key} 6 12.5\n")
    assert run() == (6, 12.5)
