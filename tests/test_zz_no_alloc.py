"""The allocation-free normal apply (static per-device scratch array) against
the workspace entry point it mirrors, through the C-ABI.

Both run the same kernels in the same launch configuration; only the transform
buffer's location differs, so the outputs must agree bit for bit.  Two calls in
a row, the second on a smaller problem (the array keeps the first call's
contents), then a problem whose transform buffer exceeds the array.
"""

import numpy as np
import pytest

from tests.gpu_util import c64, to_dev

pytestmark = pytest.mark.gpu


def inputs(n, coils, slices, seed, kind=0):
    rng = np.random.default_rng(seed)
    sens = c64(rng.standard_normal((slices, coils, n, n)) + 1j * rng.standard_normal((slices, coils, n, n)))
    x = c64(rng.standard_normal((slices, n, n)) + 1j * rng.standard_normal((slices, n, n)))
    w = c64(rng.standard_normal((slices, n, n)) + 1j * rng.standard_normal((slices, n, n)))
    if kind == 0:
        mask = (rng.random((slices, n, n)) < 0.3).astype(np.uint8)
    else:
        mask = (rng.random((slices, n)) < 0.25).astype(np.uint8)
    return sens, mask, x, w


def both(n, coils, slices, seed, kind=0, levels=3):
    import torch
    import paper_2204_10252_amd as pf
    plan = pf.Plan(n, coils, slices, haar_levels=levels, mask_kind=kind)
    sens, mask, x, w = inputs(n, coils, slices, seed, kind)
    ts, tm, tx, tw = to_dev(sens), to_dev(mask), to_dev(x), to_dev(w)
    y_ws = torch.empty_like(tx)
    y_na = torch.full_like(tx, float("nan"))
    pf.normal_apply(plan, ts, tm, tx, y_ws, 0.7, w=tw, beta=-0.3)
    pf.normal_apply_noalloc(plan, ts, tm, tx, y_na, 0.7, w=tw, beta=-0.3)
    torch.cuda.synchronize()
    return y_ws.cpu().numpy(), y_na.cpu().numpy()


def test_two_calls_in_a_row_second_smaller():
    import paper_2204_10252_amd as pf
    first = both(256, 16, 1, 11)
    second = both(64, 4, 2, 12)
    for y_ws, y_na in (first, second):
        assert np.isfinite(y_na).all()
        assert np.array_equal(y_ws, y_na)
        assert np.linalg.norm(y_ws) > 0


def test_phase_encode_and_toeplitz_plans():
    import torch
    import paper_2204_10252_amd as pf
    y_ws, y_na = both(384, 4, 2, 13, kind=pf.MASK_1D, levels=4)
    assert np.array_equal(y_ws, y_na)
    # Toeplitz plan: the transform buffer holds rows of length 2n
    n, coils = 64, 3
    plan = pf.Plan(n, coils, 1, haar_levels=3, mask_kind=pf.TOEPLITZ)
    rng = np.random.default_rng(14)
    sens, _, x, _ = inputs(n, coils, 1, 14)
    kern = to_dev(rng.standard_normal((1, 2 * n, 2 * n)).astype(np.float32))
    ts, tx = to_dev(sens), to_dev(x)
    y_ws, y_na = torch.empty_like(tx), torch.full_like(tx, float("nan"))
    pf.normal_apply(plan, ts, kern, tx, y_ws, 1.0)
    pf.normal_apply_noalloc(plan, ts, kern, tx, y_na, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(y_ws.cpu().numpy(), y_na.cpu().numpy())


def test_rejects_a_transform_buffer_larger_than_the_array():
    import torch
    import paper_2204_10252_amd as pf
    n, coils = 512, 17      # 512^2 x 17 x 8 bytes = 34 MiB > 32 MiB
    plan = pf.Plan(n, coils, 1, haar_levels=4)
    sens = torch.zeros((1, coils, n, n), dtype=torch.complex64, device="cuda")
    mask = torch.zeros((1, n, n), dtype=torch.uint8, device="cuda")
    x = torch.zeros((1, n, n), dtype=torch.complex64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(pf.PfistaError) as e:
        pf.normal_apply_noalloc(plan, sens, mask, x, y, 1.0)
    assert e.value.code == pf.EINVAL
    assert "static scratch" in str(e.value)
    # the largest buffer that fits: 512^2 x 16 coils = 32 MiB exactly
    plan16 = pf.Plan(n, 16, 1, haar_levels=4)
    s16 = torch.zeros((1, 16, n, n), dtype=torch.complex64, device="cuda")
    pf.normal_apply_noalloc(plan16, s16, mask, x, y, 1.0)
    torch.cuda.synchronize()
    assert float(torch.linalg.vector_norm(y)) == 0.0
