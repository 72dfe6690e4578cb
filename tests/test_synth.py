"""The seeded generators: determinism, exact sample counts, normalisation (CPU)."""

import numpy as np
import pytest

from synth import WORKLOADS, make_slice_inputs


@pytest.mark.parametrize("wid", [1, 3, 5])
def test_deterministic_and_shaped(wid):
    a, b = make_slice_inputs(wid, 0), make_slice_inputs(wid, 0)
    for k in ("phantom", "sens", "mask", "noise"):
        assert np.array_equal(a[k], b[k])
    w = WORKLOADS[wid]
    n = a["n"]
    assert a["sens"].shape == (w.coils, n, n) and a["noise"].shape == (w.coils, n, n)
    assert np.allclose(np.sum(np.abs(a["sens"]) ** 2, axis=0), 1.0, atol=1e-12)
    assert a["phantom"].real.min() >= 0 and np.all(a["phantom"].imag == 0)
    c = make_slice_inputs(wid, 1)
    assert not np.array_equal(a["phantom"], c["phantom"])


@pytest.mark.parametrize("wid,count", [(1, 1024), (2, 10923), (5, 7373)])
def test_mask_counts_and_centre(wid, count):
    d = make_slice_inputs(wid, 0)
    m = np.fft.fftshift(d["mask"])
    assert m.dtype == np.uint8 and int(m.sum()) == count
    n, cen = d["n"], WORKLOADS[wid].centre
    lo = n // 2 - cen // 2
    assert np.all(m[lo:lo + cen, lo:lo + cen] == 1)


def test_phase_encode_mask():
    d = make_slice_inputs(3, 0)
    m = np.fft.fftshift(d["mask"])
    assert m.shape == (384,) and int(m.sum()) == 48
    assert np.all(m[192 - 16:192 + 16] == 1)
    assert not np.array_equal(d["mask"], make_slice_inputs(3, 1)["mask"])


def test_batched_workload_draws_shapes():
    shapes = {(make_slice_inputs(4, s)["n"], make_slice_inputs(4, s)["coils"]) for s in range(8)}
    assert len(shapes) > 2
    for s in range(4):
        d = make_slice_inputs(4, s)
        assert d["n"] in (128, 160, 192, 256, 320) and d["coils"] in (8, 12, 16, 32)
        assert 2e-4 <= d["lam"] <= 2e-3 and 3 <= d["accel"] <= 8
