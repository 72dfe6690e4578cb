"""GPU parity of the batched solve of uneven slices against the FP64 oracle.

Every slice of a batch is an independent instance of the problem (own coil
count, normalisation and lambda); the oracle runs Algorithm 4 on each slice
alone with the same inputs and the same inv_l.  Bar: relative l2 error of each
slice's final iterate <= 1e-4 (the single-slice solve's bar).
"""

import numpy as np
import pytest

import oracle as orc
from synth import (coil_sensitivities, complex_noise, make_slice_inputs, mask_variable_density, phantom,
                   power_start_vector)
from tests.gpu_util import c64, rel, to_dev

pytestmark = pytest.mark.gpu


def custom_slice(n, coils, levels, lam, seed, accel=4.0):
    """A seeded slice of arbitrary shape from the workload generators."""
    rng = np.random.default_rng(seed)
    img = phantom(n, rng)
    sens = coil_sensitivities(n, coils, rng)
    mask = mask_variable_density(n, accel, max(2, n // 8), rng)
    noise = complex_noise((coils, n, n), 5e-3, rng)
    return {"phantom": img, "sens": sens, "mask": mask, "noise": noise, "n": n, "coils": coils,
            "lam": lam, "levels": levels}


def prepare(sl, inv_l="power"):
    """Rounded inputs of one slice plus its oracle-side normalisation."""
    sens = c64(sl["sens"])[None]
    s128 = sens.astype(np.complex128)
    mask = sl["mask"][None]
    b = c64(orc.kspace_data(s128, mask, sl["phantom"][None], sl["noise"][None]))
    if inv_l == "power":
        lam_max = orc.power_iteration(s128, mask, power_start_vector(sl["n"], 1), 100)
        il = 1.0 / (1.01 * lam_max)
    else:
        il = float(inv_l)
    b128 = b.astype(np.complex128)
    bn = b128 / np.linalg.norm(b128)
    return {"sens": sens, "s128": s128, "mask": mask, "b": b, "bn": bn, "inv_l": il,
            "lam": sl["lam"], "levels": sl["levels"], "n": sl["n"], "coils": sl["coils"]}


def run_batch(slices, coef, iters, chunk_bytes=0, **kw):
    import torch
    import paper_2204_10252_amd as pf
    batch = pf.Batch([(p["n"], p["coils"], p["levels"]) for p in slices], chunk_bytes=chunk_bytes)
    xs = [torch.empty((p["n"], p["n"]), dtype=torch.complex64, device="cuda") for p in slices]
    inv_l = kw.pop("inv_l", [p["inv_l"] for p in slices])
    rep = pf.batch_solve(batch, [to_dev(p["sens"][0]) for p in slices], [to_dev(p["mask"][0]) for p in slices],
                         [to_dev(p["b"][0]) for p in slices], xs, [p["lam"] for p in slices], coef=coef,
                         max_iter=iters, inv_l=inv_l, **kw)
    return [x.cpu().numpy() for x in xs], rep


def oracle_run(p, coef, iters, history=False, momentum=True):
    if momentum:
        return orc.pfista(p["s128"], p["mask"], p["bn"], p["inv_l"], p["lam"], coef, p["levels"], iters,
                          history=history)
    return orc.pgd(p["s128"], p["mask"], p["bn"], p["inv_l"], p["lam"], coef, p["levels"], iters,
                   history=history)


# uneven tiny batch: three coil counts in the (64, L3) group, a (128, L4)
# group and a (64, L2) group
TINY = [(64, 4, 3, 1e-3, 11), (128, 3, 4, 5e-4, 12), (64, 2, 3, 2e-3, 13), (64, 6, 3, 8e-4, 14),
        (64, 3, 2, 1.5e-3, 15)]


@pytest.fixture(scope="module")
def tiny():
    return [prepare(custom_slice(n, c, lv, lam, seed)) for n, c, lv, lam, seed in TINY]


@pytest.fixture(scope="module")
def tiny_oracle(tiny):
    coef = [float(v) for v in orc.l2_poly_coefficients(3)]
    return coef, [oracle_run(p, coef, 20, history=True) for p in tiny]


def test_batch_default_shape_matches_oracle(tiny, tiny_oracle):
    coef, ref = tiny_oracle
    xs, rep = run_batch(tiny, coef, 20, eval_objective=True, check_every=20)
    assert rep["iters"] == 20 and rep["normal_applies"] == 80
    assert len(rep["groups"]) == 3
    assert sorted((g["n"], g["haar_levels"], g["slices"], g["coil_images"]) for g in rep["groups"]) == \
        [(64, 2, 1, 3), (64, 3, 3, 12), (128, 4, 1, 3)]
    for x, p, (xo, _, hist), sr in zip(xs, tiny, ref, rep["slices"]):
        assert rel(x[None], xo) <= 1e-4
        assert sr["objective"] == pytest.approx(hist[-1], rel=1e-5)
        assert sr["inv_l"] == p["inv_l"]
        assert sr["bnorm"] == pytest.approx(np.linalg.norm(p["b"].astype(np.complex128)), rel=1e-6)


@pytest.mark.parametrize("cand", range(12))
def test_every_launch_shape_candidate(tiny, tiny_oracle, cand):
    import paper_2204_10252_amd as pf
    assert pf.TUNE_CANDIDATES == 12
    coef, ref = tiny_oracle
    xs, rep = run_batch(tiny, coef, 20, tune=cand + 1)
    assert all(g["candidate"] == cand for g in rep["groups"])
    for x, (xo, _, _) in zip(xs, ref):
        assert rel(x[None], xo) <= 1e-4


def test_autotune_streams_and_graph(tiny, tiny_oracle):
    import torch
    coef, ref = tiny_oracle
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xs, rep = run_batch(tiny, coef, 20, tune=-1, streams=3, graph_iters=5, check_every=10, stream=s)
    s.synchronize()
    for x, (xo, _, _) in zip(xs, ref):
        assert rel(x[None], xo) <= 1e-4
    assert all(0 <= g["candidate"] < 12 and g["chain_us"] > 0 for g in rep["groups"])
    # a second solve of the same batch reuses the tuner's cached choices
    xs2, rep2 = run_batch(tiny, coef, 20, tune=-1)
    assert [g["candidate"] for g in rep2["groups"]] == [g["candidate"] for g in rep["groups"]]
    assert [g["chain_us"] for g in rep2["groups"]] == [g["chain_us"] for g in rep["groups"]]
    for x, (xo, _, _) in zip(xs2, ref):
        assert rel(x[None], xo) <= 1e-4


def test_chunked_groups(tiny, tiny_oracle):
    # a cap of 5 coil images of 64 x 64 splits the (64, L3) group (4 + 2 + 6 coils) in three
    coef, ref = tiny_oracle
    xs, rep = run_batch(tiny, coef, 20, chunk_bytes=5 * 64 * 64 * 8, tune=-1, streams=2)
    assert sorted((g["n"], g["haar_levels"], g["coil_images"]) for g in rep["groups"]) == \
        [(64, 2, 3), (64, 3, 2), (64, 3, 4), (64, 3, 6), (128, 4, 3)]
    for x, (xo, _, _) in zip(xs, ref):
        assert rel(x[None], xo) <= 1e-4


def test_batch_estimates_inv_l_per_slice(tiny):
    coef = [1.0]
    _, rep = run_batch(tiny, coef, 1, inv_l=None, power_iters=100)
    for p, sr in zip(tiny, rep["slices"]):
        assert sr["inv_l"] == pytest.approx(p["inv_l"], rel=1e-3)


def test_batch_ppgd_and_fista(tiny):
    # momentum off (Algorithm 3) and plain FISTA (Algorithm 2) through the batch
    coef3 = [float(v) for v in orc.l2_poly_coefficients(3)]
    xs, _ = run_batch(tiny, coef3, 15, momentum=False)
    for x, p in zip(xs, tiny):
        yo, _ = oracle_run(p, coef3, 15, momentum=False)
        assert rel(x[None], yo) <= 1e-4
    xs, _ = run_batch(tiny, [1.0], 15)
    for x, p in zip(xs, tiny):
        xo, _, _ = oracle_run(p, [1.0], 15)
        assert rel(x[None], xo) <= 1e-4


def test_batch_tolerance_stop_and_empty():
    import paper_2204_10252_amd as pf
    p = prepare(custom_slice(64, 3, 3, 1e-3, 21))
    _, rep = run_batch([p, p], [1.0], 400, tol=1e-3, check_every=5)
    assert rep["iters"] < 400
    assert all(sr["rel_change"] <= 1e-3 for sr in rep["slices"])
    empty = pf.Batch([])
    rep = pf.batch_solve(empty, [], [], [], [], [], degree=3, max_iter=5)
    assert rep["iters"] == 0 and rep["rc"] == 0


def test_batch_rejects_bad_arguments(tiny):
    import torch
    import paper_2204_10252_amd as pf
    p = tiny[0]
    batch = pf.Batch([(64, 4, 3)])
    x = torch.empty((64, 64), dtype=torch.complex64, device="cuda")
    args = ([to_dev(p["sens"][0])], [to_dev(p["mask"][0])], [to_dev(p["b"][0])], [x])
    with pytest.raises(pf.PfistaError):
        pf.batch_solve(batch, *args, [-1.0], max_iter=2, inv_l=[p["inv_l"]])
    with pytest.raises(pf.PfistaError):
        pf.batch_solve(batch, *args, [1e-3], max_iter=2, inv_l=[p["inv_l"]], tune=13)
    with pytest.raises(pf.PfistaError):
        pf.batch_solve(batch, *args, [1e-3], max_iter=2, inv_l=[p["inv_l"]], streams=0)
    with pytest.raises(ValueError):
        pf.batch_solve(batch, *args, [1e-3, 1e-3], max_iter=2)


# ---- the 64-slice uneven workload at full size, sampled slices against the oracle
SAMPLED = (3, 20, 10, 7, 1)     # one slice of every image side: 128, 160, 192, 256, 320


def test_uneven_workload_full_size_sampled():
    import torch
    import paper_2204_10252_amd as pf
    # inv_l = 1 for every slice: a valid bound (the spectrum of A^H A lies in
    # [0, 1] when sum_c |S_c|^2 = 1) that both sides use without a power iteration
    slices = [make_slice_inputs(4, s) for s in range(64)]
    prep = [prepare(sl, inv_l=1.0) for sl in slices]
    coef = [float(v) for v in orc.l2_poly_coefficients(3)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xs, rep = run_batch(prep, coef, 10, tune=-1, streams=4, graph_iters=5, check_every=10,
                            eval_objective=True, stream=s)
    s.synchronize()
    assert len(rep["groups"]) == 5 and sum(g["slices"] for g in rep["groups"]) == 64
    assert all(np.isfinite(sr["objective"]) for sr in rep["slices"])
    for i in SAMPLED:
        xo, _, hist = oracle_run(prep[i], coef, 10, history=True)
        print(f"slice {i} ({prep[i]['n']}x{prep[i]['coils']}): rel {rel(xs[i][None], xo):.2e}", flush=True)
        assert rel(xs[i][None], xo) <= 1e-4
        assert rep["slices"][i]["objective"] == pytest.approx(hist[-1], rel=1e-5)


def test_batch_extremes():
    # a 512 x 512 single-coil slice, a one-level slice, and a batch of one slice
    coef = [float(v) for v in orc.l2_poly_coefficients(2)]
    sl = [prepare(custom_slice(512, 1, 4, 5e-4, 31), inv_l=1.0), prepare(custom_slice(64, 2, 1, 1e-3, 32))]
    xs, rep = run_batch(sl, coef, 6, tune=-1)
    for x, p in zip(xs, sl):
        xo, _, _ = oracle_run(p, coef, 6)
        assert rel(x[None], xo) <= 1e-4
    xs, _ = run_batch(sl[1:], coef, 6)
    xo, _, _ = oracle_run(sl[1], coef, 6)
    assert rel(xs[0][None], xo) <= 1e-4


def test_batch_zero_data_slice():
    # a slice with b = 0 stays at x = 0 (its normalisation factor is 0) next to a normal one
    coef = [float(v) for v in orc.l2_poly_coefficients(2)]
    p = prepare(custom_slice(64, 3, 3, 1e-3, 33))
    z = dict(p, b=np.zeros_like(p["b"]))
    xs, rep = run_batch([p, z], coef, 8)
    xo, _, _ = oracle_run(p, coef, 8)
    assert rel(xs[0][None], xo) <= 1e-4
    assert np.all(xs[1] == 0) and rep["slices"][1]["bnorm"] == 0.0
