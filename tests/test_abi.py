"""The C-ABI library on the CPU: it loads, exports every function the header
declares, and its host-only parts behave (no GPU is touched here)."""

import ctypes
import os

import pytest

import oracle as orc


@pytest.fixture(scope="module")
def lib():
    import paper_2204_10252_amd as pf
    if not os.path.exists(pf.library_path()):
        from paper_2204_10252_amd import build
        build.build(verbose=False)
    return pf.load_library()


def test_exports_every_declared_function(lib):
    import paper_2204_10252_amd as pf
    names = pf.header_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pf._SIGS)


def test_host_coefficients_match_oracle(lib):
    import paper_2204_10252_amd as pf
    for d in range(9):
        want = [float(c) for c in orc.l2_poly_coefficients(d)]
        got = pf.poly_coefficients(d)
        assert got == pytest.approx(want, rel=4e-16, abs=0)
    with pytest.raises(pf.PfistaError) as e:
        pf.poly_coefficients(9)
    assert e.value.code == pf.UNSUPPORTED


def _desc(n=64, coils=2, slices=1, levels=3, kind=0):
    import paper_2204_10252_amd as pf
    return pf._Desc(n, coils, slices, levels, kind)


@pytest.mark.parametrize("desc,code", [
    (dict(n=100), -2), (dict(n=96), -2), (dict(levels=0), -2), (dict(levels=5), -2),
    (dict(coils=0), -1), (dict(slices=-1), -1), (dict(kind=7), -1),
    (dict(coils=1000, slices=100), -2), (dict(n=320, kind=2), -2), (dict(n=512, kind=2), -2),
    (dict(n=512, coils=1024, slices=1, kind=1), -2), (dict(n=384, coils=1821, slices=1, kind=1), -2),
])
def test_plan_validation_before_any_gpu_call(lib, desc, code):
    h = ctypes.c_void_p()
    d = _desc(**desc)
    rc = lib.pfista_plan_create(ctypes.byref(h), ctypes.byref(d))
    assert rc == code
    assert lib.pfista_last_error().decode()


def test_null_plan_is_rejected(lib):
    rc = lib.pfista_normal_apply(None, None, None, None, None, 1.0, None, 0.0, None, None)
    assert rc == -1
    assert b"plan" in lib.pfista_last_error()
    # the packed-coil-map calls check the plan first too
    assert lib.pfista_pack_coil_maps(None, None, None, None) == -1
    assert b"plan" in lib.pfista_last_error()
    assert lib.pfista_normal_apply_packed(None, None, None, None, None, 1.0, None, 0.0, None, None) == -1
    coef = (ctypes.c_double * 2)(1.0, 0.5)
    assert lib.pfista_poly_apply_packed(None, None, None, 1.0, coef, 1, None, None, None, None) == -1


@pytest.mark.parametrize("d", range(0, 7))
def test_host_weighted_and_chebyshev_coefficients_match_oracle(lib, d):
    import paper_2204_10252_amd as pf
    for alpha in (0.0, 0.7, 2.0):
        want = [float(c) for c in orc.weighted_l2_poly_coefficients(d, alpha)]
        assert pf.poly_coefficients_weighted(d, alpha) == pytest.approx(want, rel=1e-9, abs=0)
    for mu in (0.01, 0.1, 0.5):
        want = [float(c) for c in orc.chebyshev_poly_coefficients(d, mu)]
        assert pf.poly_coefficients_chebyshev(d, mu) == pytest.approx(want, rel=1e-12, abs=0)


def test_host_coefficient_argument_errors(lib):
    import paper_2204_10252_amd as pf
    for bad in ((2, -1.0), (2, float("nan"))):
        with pytest.raises(pf.PfistaError):
            pf.poly_coefficients_weighted(*bad)
    for bad in ((2, 0.0), (2, 1.0), (9, 0.5)):
        with pytest.raises(pf.PfistaError):
            pf.poly_coefficients_chebyshev(*bad)


@pytest.mark.parametrize("sl,code", [
    ((100, 4, 3), -2), ((64, 0, 3), -1), ((64, 4, 0), -2), ((64, 4, 5), -2),
])
def test_batch_validation_before_any_gpu_call(lib, sl, code):
    import paper_2204_10252_amd as pf
    arr = (pf._SliceDesc * 2)(pf._SliceDesc(64, 4, 3), pf._SliceDesc(*sl))
    h = ctypes.c_void_p()
    assert lib.pfista_batch_create(ctypes.byref(h), arr, 2, 0) == code
    assert lib.pfista_last_error().decode()
    assert lib.pfista_batch_create(ctypes.byref(h), arr, -1, 0) == -1


def test_null_batch_is_rejected(lib):
    import paper_2204_10252_amd as pf
    prm = pf._BatchParams(3, None, 10, 10, 0.0, 0, 30, 0, 1, 1, 0)
    rc = lib.pfista_batch_solve(None, None, None, None, None, None, ctypes.byref(prm), None, None, None,
                                None, None, None)
    assert rc == -1 and b"batch" in lib.pfista_last_error()
    assert lib.pfista_batch_workspace_bytes(None) == 0 and lib.pfista_batch_groups(None) == 0


_STRUCTS = {"pfista_desc": "_Desc", "pfista_params": "_Params", "pfista_report": "_Report",
            "pfista_slice_desc": "_SliceDesc", "pfista_batch_params": "_BatchParams",
            "pfista_slice_report": "_SliceReport", "pfista_group_report": "_GroupReport",
            "pfista_batch_report": "_BatchReport", "pfista_unroll_params": "_UnrollParams"}


def _c_field_names(header: str, struct: str):
    """Member names of ``typedef struct { ... } struct;`` in the header text."""
    import re
    end = header.index("} " + struct + ";")
    start = header.rindex("typedef struct {", 0, end)
    body = re.sub(r"/\*.*?\*/", "", header[start + len("typedef struct {"):end], flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            names.append(re.findall(r"[A-Za-z_]\w*", decl)[-1])
    return names


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror has the C struct's size, member names (in order) and
    offsets, as a host C compiler lays out the header's structs."""
    import shutil
    import subprocess
    import paper_2204_10252_amd as pf

    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    header = open(os.path.join(root, "include", "pfista.h")).read()
    fields = {s: _c_field_names(header, s) for s in _STRUCTS}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pfista.h"', "int main(void) {"]
    for s, names in fields.items():
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f in names:
            lines.append(f'  printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c = {}
    for line in out:
        if line:
            s, f, v = line.split()
            c[(s, f)] = int(v)
    for s, py in _STRUCTS.items():
        cls = getattr(pf, py)
        py_names = [n.rstrip("_") for n, _ in cls._fields_]
        assert py_names == fields[s], s
        assert ctypes.sizeof(cls) == c[(s, "size")], s
        for (n, _), f in zip(cls._fields_, fields[s]):
            assert getattr(cls, n).offset == c[(s, f)], (s, f)


def test_image_scale_undoes_the_normalisation():
    # A' = sqrt(inv_l) A and b' = b/||b||: if A' x' = b' then A (s x') = b with
    # s = sqrt(inv_l) ||b||; checked on a dense random A
    import numpy as np
    import paper_2204_10252_amd as pf
    rng = np.random.default_rng(3)
    A = rng.standard_normal((12, 5))
    x = rng.standard_normal(5)
    b = A @ x
    inv_l = 0.37
    xp = np.linalg.lstsq(np.sqrt(inv_l) * A, b / np.linalg.norm(b), rcond=None)[0]
    s = pf.image_scale({"inv_l": inv_l, "bnorm": float(np.linalg.norm(b))})
    assert np.allclose(s * xp, x, rtol=1e-12, atol=1e-12)
