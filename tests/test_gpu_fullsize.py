"""Parity at the full workload sizes, in the launch configuration the benchmark times.

* 256 x 256, 16 coils, Poisson-disc-like mask: the whole output against the
  oracle (it finishes in well under a second at this size).
* slab of 32 slices 384 x 384, 32 coils, phase-encode mask: the GPU applies the
  operator to all 32 slices at once; the oracle recomputes three sampled
  slices (slices are independent blocks of A).
Bar: relative l2 error <= 1e-5 per checked slice.
"""

import numpy as np
import pytest

import oracle as orc
from synth import make_inputs, make_slice_inputs
from tests.gpu_util import c64, rel, to_dev

pytestmark = pytest.mark.gpu


def test_workload2_normal_apply_full():
    import torch
    import paper_2204_10252_amd as pf
    inp = make_inputs(2)
    sens = c64(inp["sens"])
    x = c64(inp["phantom"] + 0.1j * np.roll(inp["phantom"], 7, axis=-1))
    plan = pf.Plan(256, 16, 1, haar_levels=4)
    tx = to_dev(x)
    ty = torch.empty_like(tx)
    pf.normal_apply(plan, to_dev(sens), to_dev(inp["mask"]), tx, ty, 1.0)
    ref = orc.normal(sens.astype(np.complex128), inp["mask"], x.astype(np.complex128))
    assert rel(ty.cpu().numpy(), ref) <= 1e-5


def test_workload3_slab_sampled_slices():
    import torch
    import paper_2204_10252_amd as pf
    n, coils, slices = 384, 32, 32
    dev = torch.device("cuda", 0)
    ts = torch.empty((slices, coils, n, n), dtype=torch.complex64, device=dev)
    tm = torch.empty((slices, n), dtype=torch.uint8, device=dev)
    tx = torch.empty((slices, n, n), dtype=torch.complex64, device=dev)
    keep = {}
    for s in range(slices):
        d = make_slice_inputs(3, s)
        ts[s].copy_(torch.from_numpy(c64(d["sens"])))
        tm[s].copy_(torch.from_numpy(d["mask"]))
        xs = c64(d["phantom"] * np.exp(0.3j))
        tx[s].copy_(torch.from_numpy(xs))
        if s in (0, 17, 31):
            keep[s] = (c64(d["sens"]), d["mask"], xs)
    plan = pf.Plan(n, coils, slices, haar_levels=4, mask_kind=pf.MASK_1D)
    ty = torch.empty_like(tx)
    pf.normal_apply(plan, ts, tm, tx, ty, 1.0)
    got = ty.cpu().numpy()
    for s, (sens, mask, xs) in keep.items():
        ref = orc.normal(sens[None].astype(np.complex128), mask[None], xs[None].astype(np.complex128))
        assert rel(got[s], ref[0]) <= 1e-5, f"slice {s}"
