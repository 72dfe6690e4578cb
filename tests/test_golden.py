"""Stored fixtures under tests/golden/: the paper's printed experiment constants
and the exact L2 coefficients (CPU only)."""

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _coefficients():
    return {int(r[0]): [Fraction(v) for v in r[1:]] for r in _read("l2_coefficients.txt")}


def test_l2_fixture_has_the_optimal_cost():
    # int_0^1 (1 - z q(z))^2 dz expanded exactly: with r(z) = 1 - sum_i c_i z^(i+1),
    # int r^2 = sum_{a,b} r_a r_b / (a + b + 1); the minimum is 1/(d+2)^2
    for d, c in _coefficients().items():
        assert len(c) == d + 1
        r = [Fraction(1)] + [-ci for ci in c]
        cost = sum(r[a] * r[b] / (a + b + 1) for a in range(d + 2) for b in range(d + 2))
        assert cost == Fraction(1, (d + 2) ** 2)


def test_l2_fixture_matches_oracle_and_library():
    fixture = _coefficients()
    for d, c in fixture.items():
        assert orc.l2_poly_coefficients(d) == c
    try:
        import paper_2204_10252_amd as pf
        pf.load_library()
    except (ImportError, RuntimeError, OSError):
        pytest.skip("library not built")
    for d, c in fixture.items():
        got = pf.poly_coefficients(d)
        assert got == pytest.approx([float(v) for v in c], rel=4e-16, abs=0)


def test_knee_like_workload_uses_the_papers_constants():
    from synth import WORKLOADS, make_slice_inputs
    k = {r[0]: float(r[1]) for r in _read("paper_cartesian_experiment.txt")}
    w = WORKLOADS[7]
    assert (w.n, w.coils) == (int(k["matrix_size"]), int(k["coils"]))
    assert w.accel == k["acceleration"] and w.lam == k["fista_lambda"]
    mask = make_slice_inputs(7, 0)["mask"]
    assert mask.size / np.count_nonzero(mask) == pytest.approx(k["acceleration"], rel=2e-3)
