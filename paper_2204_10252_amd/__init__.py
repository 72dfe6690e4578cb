"""Python binding of libpfista (polynomial-preconditioned FISTA on gfx950).

Argument marshalling only: every function forwards device pointers of
``torch`` tensors (complex64 images / coil data, uint8 masks) and the current
HIP stream to the C-ABI of ``include/pfista.h``; all arithmetic runs in the
library's kernels.  Importing needs the built ``libpfista.so`` next to this
file (``python -m paper_2204_10252_amd.build``); there is no fallback.
"""

from __future__ import annotations

import ctypes
import math
import os
import re

__all__ = [
    "Plan", "PfistaError", "load_library", "library_path", "poly_coefficients",
    "poly_coefficients_weighted", "poly_coefficients_chebyshev", "normal_apply", "normal_apply_noalloc", "poly_apply",
    "pack_coil_maps", "normal_apply_packed", "poly_apply_packed", "step", "forward", "adjoint", "data_term",
    "power_iteration", "profile_normal", "solve", "MASK_2D", "MASK_1D", "TOEPLITZ", "header_functions",
    "toeplitz_kernel", "nudft_forward", "nudft_adjoint",
    "Batch", "batch_solve", "TUNE_CANDIDATES", "Unrolled", "unrolled_pfista", "image_scale",
]

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
MASK_2D, MASK_1D, TOEPLITZ = 0, 1, 2
OK, EINVAL, UNSUPPORTED, EHIP, DIVERGED = 0, -1, -2, -3, -4


class PfistaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pfista error {code}: {msg}")
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("coils", ctypes.c_int), ("slices", ctypes.c_int),
                ("haar_levels", ctypes.c_int), ("mask_kind", ctypes.c_int)]


class _Params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("inv_l", ctypes.c_double),
                ("power_iters", ctypes.c_int), ("degree", ctypes.c_int),
                ("coef", ctypes.POINTER(ctypes.c_double)), ("max_iter", ctypes.c_int),
                ("check_every", ctypes.c_int), ("tol", ctypes.c_double),
                ("f_stop", ctypes.c_double), ("eval_objective", ctypes.c_int),
                ("k0", ctypes.c_int), ("graph_iters", ctypes.c_int), ("momentum", ctypes.c_int),
                ("bnorm", ctypes.c_double), ("tune", ctypes.c_int)]


class _Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("objective", ctypes.c_double),
                ("rel_change", ctypes.c_double), ("l1", ctypes.c_double), ("inv_l", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("normal_applies", ctypes.c_longlong),
                ("candidate", ctypes.c_int), ("tune_us", ctypes.c_double), ("loop_ms", ctypes.c_double)]


class _SliceDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("coils", ctypes.c_int), ("haar_levels", ctypes.c_int)]


class _BatchParams(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("coef", ctypes.POINTER(ctypes.c_double)),
                ("max_iter", ctypes.c_int), ("check_every", ctypes.c_int), ("tol", ctypes.c_double),
                ("eval_objective", ctypes.c_int), ("power_iters", ctypes.c_int),
                ("graph_iters", ctypes.c_int), ("momentum", ctypes.c_int), ("streams", ctypes.c_int),
                ("tune", ctypes.c_int)]


class _SliceReport(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_double), ("rel_change", ctypes.c_double), ("l1", ctypes.c_double),
                ("inv_l", ctypes.c_double), ("bnorm", ctypes.c_double)]


class _GroupReport(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("haar_levels", ctypes.c_int), ("slices", ctypes.c_int),
                ("coil_images", ctypes.c_int), ("candidate", ctypes.c_int), ("chain_us", ctypes.c_double)]


class _BatchReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("normal_applies", ctypes.c_longlong)]


class _UnrollParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("inv_l", ctypes.c_double), ("degree", ctypes.c_int),
                ("coef", ctypes.POINTER(ctypes.c_double)), ("iters", ctypes.c_int), ("ckpt_every", ctypes.c_int),
                ("momentum", ctypes.c_int), ("tune", ctypes.c_int)]


TUNE_CANDIDATES = 12

_VP, _I, _F, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
_SIGS = {
    "pfista_plan_create": (_I, [ctypes.POINTER(_VP), ctypes.POINTER(_Desc)]),
    "pfista_plan_destroy": (None, [_VP]),
    "pfista_workspace_bytes": (ctypes.c_size_t, [_VP]),
    "pfista_normal_apply": (_I, [_VP, _VP, _VP, _VP, _VP, _F, _VP, _F, _VP, _VP]),
    "pfista_normal_apply_noalloc": (_I, [_VP, _VP, _VP, _VP, _VP, _F, _VP, _F, _VP]),
    "pfista_poly_apply": (_I, [_VP, _VP, _VP, _D, ctypes.POINTER(_D), _I, _VP, _VP, _VP, _VP]),
    "pfista_pack_coil_maps": (_I, [_VP, _VP, _VP, _VP]),
    "pfista_normal_apply_packed": (_I, [_VP, _VP, _VP, _VP, _VP, _F, _VP, _F, _VP, _VP]),
    "pfista_poly_apply_packed": (_I, [_VP, _VP, _VP, _D, ctypes.POINTER(_D), _I, _VP, _VP, _VP, _VP]),
    "pfista_step": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _F, _F, _VP, _VP, _VP]),
    "pfista_forward": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "pfista_adjoint": (_I, [_VP, _VP, _VP, _VP, _VP, _F, _VP, _VP]),
    "pfista_data_term": (_I, [_VP, _VP, _VP, _VP, _VP, _D, _D, ctypes.POINTER(_D), _VP, _VP]),
    "pfista_power_iteration": (_I, [_VP, _VP, _VP, _VP, _I, ctypes.POINTER(_D), _VP, _VP]),
    "pfista_poly_coefficients": (_I, [_I, ctypes.POINTER(_D)]),
    "pfista_poly_coefficients_weighted": (_I, [_I, _D, ctypes.POINTER(_D)]),
    "pfista_poly_coefficients_chebyshev": (_I, [_I, _D, ctypes.POINTER(_D)]),
    "pfista_solve": (_I, [_VP, _VP, _VP, _VP, ctypes.POINTER(_Params), _VP, _VP,
                          ctypes.POINTER(_D), ctypes.POINTER(_Report), _VP, _VP]),
    "pfista_profile_normal": (_I, [_VP, _VP, _VP, _VP, _VP, _I, ctypes.POINTER(_F),
                                   ctypes.POINTER(_I), _VP, _VP]),
    "pfista_batch_create": (_I, [ctypes.POINTER(_VP), ctypes.POINTER(_SliceDesc), _I, ctypes.c_size_t]),
    "pfista_batch_destroy": (None, [_VP]),
    "pfista_batch_workspace_bytes": (ctypes.c_size_t, [_VP]),
    "pfista_batch_groups": (_I, [_VP]),
    "pfista_batch_solve": (_I, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_BatchParams),
                                ctypes.POINTER(_VP), ctypes.POINTER(_SliceReport),
                                ctypes.POINTER(_GroupReport), ctypes.POINTER(_BatchReport), _VP, _VP]),
    "pfista_unroll_ckpt_bytes": (ctypes.c_size_t, [_VP, ctypes.POINTER(_UnrollParams)]),
    "pfista_unroll_workspace_bytes": (ctypes.c_size_t, [_VP, ctypes.POINTER(_UnrollParams)]),
    "pfista_unroll_forward": (_I, [_VP, _VP, _VP, _VP, ctypes.POINTER(_UnrollParams), _VP, _VP, _VP, _VP]),
    "pfista_unroll_backward": (_I, [_VP, _VP, _VP, ctypes.POINTER(_UnrollParams), _VP, _VP,
                                    ctypes.POINTER(_D), _VP, _VP]),
    "pfista_toeplitz_kernel": (_I, [_VP, _VP, _VP, _I, _VP, _VP]),
    "pfista_nudft_forward": (_I, [_VP, _VP, _VP, _I, _VP, _VP, _VP]),
    "pfista_nudft_adjoint": (_I, [_VP, _VP, _VP, _I, _VP, _VP, _VP]),
    "pfista_last_error": (ctypes.c_char_p, []),
}

_lib = None


def library_path() -> str:
    """The in-tree build; PFISTA_LIBRARY may name another build of the same sources."""
    return os.environ.get("PFISTA_LIBRARY") or os.path.join(HERE, "libpfista.so")


def load_library():
    """Load libpfista.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2204_10252_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype, fn.argtypes = res, args
        _lib = lib
    return _lib


def header_functions() -> list:
    """Names of the functions declared in include/pfista.h."""
    with open(os.path.join(ROOT, "include", "pfista.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfista_\w+)\s*\(", text)))


def _check(rc):
    if rc != OK:
        msg = load_library().pfista_last_error().decode()
        raise PfistaError(rc, msg)
    return rc


# ------------------------------------------------------------------ marshalling

def _ptr(t, name, dtype=None, numel=None, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    # the library launches on the current device (which must be the plan's)
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} is on {t.device}, but the current device is cuda:{torch.cuda.current_device()}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    if s.device.index != torch.cuda.current_device():
        raise ValueError(f"stream is on {s.device}, but the current device is cuda:{torch.cuda.current_device()}")
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Owns a ``pfista_plan`` and a device workspace sized for it."""

    def __init__(self, n, coils, slices, haar_levels=4, mask_kind=MASK_2D, device=None):
        import torch
        lib = load_library()
        self.n, self.coils, self.slices = int(n), int(coils), int(slices)
        self.haar_levels, self.mask_kind = int(haar_levels), int(mask_kind)
        desc = _Desc(self.n, self.coils, self.slices, self.haar_levels, self.mask_kind)
        h = ctypes.c_void_p()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(self.device):
            _check(lib.pfista_plan_create(ctypes.byref(h), ctypes.byref(desc)))
        self._h = h
        nbytes = int(lib.pfista_workspace_bytes(h))
        self.ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)

    @property
    def handle(self):
        return self._h

    @property
    def n_img(self):
        return self.slices * self.n * self.n

    @property
    def n_coil(self):
        return self.slices * self.coils * self.n * self.n

    @property
    def mask_numel(self):
        if self.mask_kind == TOEPLITZ:
            return self.slices * 4 * self.n * self.n
        return self.slices * self.n * (self.n if self.mask_kind == MASK_2D else 1)

    def mask_dtype(self):
        import torch
        return torch.float32 if self.mask_kind == TOEPLITZ else torch.uint8

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.pfista_plan_destroy(h)
            self._h = None


def _cplx():
    import torch
    return torch.complex64


def _u8():
    import torch
    return torch.uint8


def poly_coefficients(degree: int) -> list:
    lib = load_library()
    buf = (ctypes.c_double * (degree + 1))()
    _check(lib.pfista_poly_coefficients(int(degree), buf))
    return list(buf)


def poly_coefficients_weighted(degree: int, alpha: float) -> list:
    """Weighted L2 design with w(z) = z^alpha (Section 2.5)."""
    buf = (ctypes.c_double * (degree + 1))()
    _check(load_library().pfista_poly_coefficients_weighted(int(degree), float(alpha), buf))
    return list(buf)


def poly_coefficients_chebyshev(degree: int, mu: float) -> list:
    """L-infinity design for a known smallest eigenvalue mu (Section 2.5)."""
    buf = (ctypes.c_double * (degree + 1))()
    _check(load_library().pfista_poly_coefficients_chebyshev(int(degree), float(mu), buf))
    return list(buf)


def normal_apply(plan, sens, mask, x, y, alpha=1.0, w=None, beta=0.0, stream=None):
    c = _cplx()
    _check(load_library().pfista_normal_apply(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        _ptr(x, "x", c, plan.n_img), _ptr(y, "y", c, plan.n_img), float(alpha),
        _ptr(w, "w", c, plan.n_img, allow_none=True), float(beta), _ptr(plan.ws, "ws"), _stream(stream)))
    return y


def normal_apply_noalloc(plan, sens, mask, x, y, alpha=1.0, w=None, beta=0.0, stream=None):
    """``normal_apply`` without a workspace: the library's static per-device
    scratch array holds the transform buffer (for callers that cannot allocate;
    calls overlapping on one GPU race)."""
    c = _cplx()
    _check(load_library().pfista_normal_apply_noalloc(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        _ptr(x, "x", c, plan.n_img), _ptr(y, "y", c, plan.n_img), float(alpha),
        _ptr(w, "w", c, plan.n_img, allow_none=True), float(beta), _stream(stream)))
    return y


def poly_apply(plan, sens, mask, inv_l, coef, g, out, stream=None):
    c = _cplx()
    arr = (ctypes.c_double * len(coef))(*[float(v) for v in coef])
    _check(load_library().pfista_poly_apply(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        float(inv_l), arr, len(coef) - 1, _ptr(g, "g", c, plan.n_img), _ptr(out, "out", c, plan.n_img),
        _ptr(plan.ws, "ws"), _stream(stream)))
    return out


def pack_coil_maps(plan, sens, packed=None, stream=None):
    """Coil maps of a phase-encode plan in the layout its operator streams fastest
    (same size as ``sens``; valid only for the ``*_packed`` calls on this plan's shape)."""
    import torch
    c = _cplx()
    if packed is None:
        packed = torch.empty(plan.n_coil, dtype=c, device=sens.device)
    _check(load_library().pfista_pack_coil_maps(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(packed, "packed", c, plan.n_coil), _stream(stream)))
    return packed


def normal_apply_packed(plan, packed, mask, x, y, alpha=1.0, w=None, beta=0.0, stream=None):
    """``normal_apply`` of a phase-encode plan on packed coil maps (bitwise the same result)."""
    c = _cplx()
    _check(load_library().pfista_normal_apply_packed(
        plan.handle, _ptr(packed, "packed", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        _ptr(x, "x", c, plan.n_img), _ptr(y, "y", c, plan.n_img), float(alpha),
        _ptr(w, "w", c, plan.n_img, allow_none=True), float(beta), _ptr(plan.ws, "ws"), _stream(stream)))
    return y


def poly_apply_packed(plan, packed, mask, inv_l, coef, g, out, stream=None):
    """``poly_apply`` of a phase-encode plan on packed coil maps (bitwise the same result)."""
    c = _cplx()
    arr = (ctypes.c_double * len(coef))(*[float(v) for v in coef])
    _check(load_library().pfista_poly_apply_packed(
        plan.handle, _ptr(packed, "packed", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        float(inv_l), arr, len(coef) - 1, _ptr(g, "g", c, plan.n_img), _ptr(out, "out", c, plan.n_img),
        _ptr(plan.ws, "ws"), _stream(stream)))
    return out


def step(plan, z, pg, x_old, x_new, z_new, lam, beta_k, red, stream=None):
    import torch
    c = _cplx()
    _check(load_library().pfista_step(
        plan.handle, _ptr(z, "z", c, plan.n_img), _ptr(pg, "pg", c, plan.n_img),
        _ptr(x_old, "x_old", c, plan.n_img), _ptr(x_new, "x_new", c, plan.n_img),
        _ptr(z_new, "z_new", c, plan.n_img), float(lam), float(beta_k),
        _ptr(red, "red", torch.float64, 3), _ptr(plan.ws, "ws"), _stream(stream)))


def forward(plan, sens, mask, x, kspace, stream=None):
    c = _cplx()
    _check(load_library().pfista_forward(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        _ptr(x, "x", c, plan.n_img), _ptr(kspace, "kspace", c, plan.n_coil), _ptr(plan.ws, "ws"),
        _stream(stream)))
    return kspace


def adjoint(plan, sens, mask, kspace, y, alpha=1.0, stream=None):
    c = _cplx()
    _check(load_library().pfista_adjoint(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        _ptr(kspace, "kspace", c, plan.n_coil), _ptr(y, "y", c, plan.n_img), float(alpha),
        _ptr(plan.ws, "ws"), _stream(stream)))
    return y


def data_term(plan, sens, mask, b, x, inv_l, b_scale, stream=None) -> float:
    c = _cplx()
    out = ctypes.c_double()
    _check(load_library().pfista_data_term(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        _ptr(b, "b", c, plan.n_coil), _ptr(x, "x", c, plan.n_img), float(inv_l), float(b_scale),
        ctypes.byref(out), _ptr(plan.ws, "ws"), _stream(stream)))
    return out.value


def power_iteration(plan, sens, mask, iters, v=None, stream=None) -> float:
    c = _cplx()
    out = ctypes.c_double()
    _check(load_library().pfista_power_iteration(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        _ptr(v, "v", c, plan.n_img, allow_none=True), int(iters), ctypes.byref(out),
        _ptr(plan.ws, "ws"), _stream(stream)))
    return out.value


def profile_normal(plan, sens, mask, x, y, reps=50, stream=None) -> list:
    """Average duration (ms) of each kernel pass of one normal apply."""
    c = _cplx()
    ms = (ctypes.c_float * 4)()
    npass = ctypes.c_int()
    _check(load_library().pfista_profile_normal(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel),
        _ptr(x, "x", c, plan.n_img), _ptr(y, "y", c, plan.n_img), int(reps), ms, ctypes.byref(npass),
        _ptr(plan.ws, "ws"), _stream(stream)))
    return list(ms)[: npass.value]


def solve(plan, sens, mask, b, x, lam, degree=3, coef=None, max_iter=50, inv_l=0.0, power_iters=30,
          check_every=None, tol=0.0, f_stop=0.0, eval_objective=False, z=None, k0=0, graph_iters=0,
          history=False, stream=None, raise_on_diverge=True, momentum=True, bnorm=0.0, tune=0):
    """Algorithm 4 through ``pfista_solve``; returns the report as a dict (with
    ``history`` when asked).  ``tune``: 0 default launch shape, -1 tuned and
    cached, ``k >= 1`` candidate ``k - 1``."""
    c = _cplx()
    lib = load_library()
    ce = max_iter if check_every is None else check_every
    ce = max(1, min(int(ce), 4096))
    carr = None
    if coef is not None:
        carr = (ctypes.c_double * len(coef))(*[float(v) for v in coef])
        degree = len(coef) - 1
    prm = _Params(float(lam), float(inv_l), int(power_iters), int(degree),
                  ctypes.cast(carr, ctypes.POINTER(ctypes.c_double)) if carr is not None else None,
                  int(max_iter), ce, float(tol), float(f_stop), int(bool(eval_objective or history)),
                  int(k0), int(graph_iters), int(bool(momentum)), float(bnorm), int(tune))
    nh = max(1, -(-int(max_iter) // ce))
    hist = (ctypes.c_double * nh)() if history else None
    rep = _Report()
    nb = plan.n_img if plan.mask_kind == TOEPLITZ else plan.n_coil
    rc = lib.pfista_solve(plan.handle, _ptr(sens, "sens", c, plan.n_coil),
                          _ptr(mask, "mask", plan.mask_dtype(), plan.mask_numel), _ptr(b, "b", c, nb),
                          ctypes.byref(prm), _ptr(x, "x", c, plan.n_img),
                          _ptr(z, "z", c, plan.n_img, allow_none=True),
                          ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)) if hist is not None else None,
                          ctypes.byref(rep), _ptr(plan.ws, "ws"), _stream(stream))
    out = {k: getattr(rep, k) for k, _ in _Report._fields_}
    if history:
        nchk = -(-int(rep.iters) // ce) if rep.iters else 0
        out["history"] = list(hist)[:nchk]
    if rc != OK and not (rc == DIVERGED and not raise_on_diverge):
        _check(rc)
    out["rc"] = rc
    return out


def image_scale(report) -> float:
    """Factor that takes a solution from the normalised problem (A' = sqrt(inv_l) A,
    b' = b / ||b||) back to the units of the data: x = image_scale(rep) * x'.
    ``report``: the dict of ``solve`` or one entry of ``batch_solve``'s
    ``slices``."""
    return math.sqrt(float(report["inv_l"])) * float(report["bnorm"])


# ------------------------------------------------------------------ batches

class Batch:
    """Owns a ``pfista_batch`` (slices of uneven shape) and its device workspace.
    ``slices``: sequence of ``(n, coils)`` or ``(n, coils, haar_levels)``;
    ``chunk_bytes``: cap on the coil-map bytes of one group (0: no cap)."""

    def __init__(self, slices, haar_levels=4, chunk_bytes=0, device=None):
        import torch
        lib = load_library()
        sl = [tuple(int(v) for v in t) for t in slices]
        self.slices = [(t[0], t[1], t[2] if len(t) > 2 else int(haar_levels)) for t in sl]
        arr = (_SliceDesc * max(1, len(self.slices)))(*[_SliceDesc(*t) for t in self.slices])
        h = ctypes.c_void_p()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(self.device):
            _check(lib.pfista_batch_create(ctypes.byref(h), arr, len(self.slices), int(chunk_bytes)))
        self._h = h
        self.groups = int(lib.pfista_batch_groups(h))
        nbytes = int(lib.pfista_batch_workspace_bytes(h))
        self.ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)

    @property
    def handle(self):
        return self._h

    def __len__(self):
        return len(self.slices)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.pfista_batch_destroy(h)
            self._h = None


def _ptr_array(tensors, name, dtype, numels):
    arr = (ctypes.c_void_p * max(1, len(tensors)))()
    for i, (t, nel) in enumerate(zip(tensors, numels)):
        arr[i] = _ptr(t, f"{name}[{i}]", dtype, nel).value
    return arr


def batch_solve(batch, sens, mask, b, x, lam, degree=3, coef=None, max_iter=50, inv_l=None,
                power_iters=30, check_every=None, tol=0.0, eval_objective=False, graph_iters=0,
                momentum=True, streams=1, tune=0, stream=None, raise_on_diverge=True):
    """Algorithm 4 on every slice of ``batch`` through ``pfista_batch_solve``.
    ``sens``, ``mask``, ``b``, ``x``: lists of per-slice device tensors; ``lam``
    and ``inv_l`` (None: estimate all): per-slice floats.  Returns a dict with
    the batch report, ``slices`` (per-slice reports) and ``groups``."""
    c = _cplx()
    lib = load_library()
    ns = len(batch)
    for name, v in (("sens", sens), ("mask", mask), ("b", b), ("x", x), ("lam", lam)):
        if len(v) != ns:
            raise ValueError(f"{name} has {len(v)} entries for {ns} slices")
    if inv_l is not None and len(inv_l) != ns:
        raise ValueError("inv_l needs one entry per slice")
    coil_n = [cc * n * n for n, cc, _ in batch.slices]
    img_n = [n * n for n, _, _ in batch.slices]
    ps = _ptr_array(sens, "sens", c, coil_n)
    pm = _ptr_array(mask, "mask", _u8(), img_n)
    pb = _ptr_array(b, "b", c, coil_n)
    px = _ptr_array(x, "x", c, img_n)
    lam_a = (ctypes.c_double * max(1, ns))(*[float(v) for v in lam])
    il_a = (ctypes.c_double * max(1, ns))(*[float(v) for v in inv_l]) if inv_l is not None else None
    ce = max_iter if check_every is None else check_every
    ce = max(1, min(int(ce), 4096))
    carr = None
    if coef is not None:
        carr = (ctypes.c_double * len(coef))(*[float(v) for v in coef])
        degree = len(coef) - 1
    prm = _BatchParams(int(degree), ctypes.cast(carr, ctypes.POINTER(ctypes.c_double)) if carr is not None else None,
                       int(max_iter), ce, float(tol), int(bool(eval_objective)), int(power_iters),
                       int(graph_iters), int(bool(momentum)), int(streams), int(tune))
    srep = (_SliceReport * max(1, ns))()
    grep = (_GroupReport * max(1, batch.groups))()
    rep = _BatchReport()
    rc = lib.pfista_batch_solve(batch.handle, ps, pm, pb, lam_a, il_a, ctypes.byref(prm), px, srep, grep,
                                ctypes.byref(rep), _ptr(batch.ws, "ws"), _stream(stream))
    if rc != OK and not (rc == DIVERGED and not raise_on_diverge):
        _check(rc)
    out = {k: getattr(rep, k) for k, _ in _BatchReport._fields_}
    out["slices"] = [{k: getattr(srep[i], k) for k, _ in _SliceReport._fields_} for i in range(ns)]
    out["groups"] = [{k: getattr(grep[i], k) for k, _ in _GroupReport._fields_} for i in range(batch.groups)]
    out["rc"] = rc
    return out


# ------------------------------------------------------------------ differentiation

class Unrolled:
    """K unrolled iterations of Algorithm 4 on one plan, differentiable in the
    threshold and the polynomial coefficients (``pfista_unroll_forward`` /
    ``pfista_unroll_backward``).  Holds a workspace (scratch of one call: calls
    on different streams must not overlap) and a default checkpoint buffer that
    ``forward`` / ``backward`` use unless given their own ``ckpt`` (from
    ``new_checkpoints``); a backward must read the checkpoints of its own
    forward.  ``tune``: launch shape as in ``solve``."""

    def __init__(self, plan, degree, iters, inv_l, ckpt_every=5, momentum=True, tune=0):
        import torch
        self.plan, self.degree, self.iters = plan, int(degree), int(iters)
        self.inv_l, self.ckpt_every, self.momentum = float(inv_l), int(ckpt_every), bool(momentum)
        self.tune = int(tune)
        lib = load_library()
        prm = self._params(0.0, [0.0] * (self.degree + 1))
        nck = int(lib.pfista_unroll_ckpt_bytes(plan.handle, ctypes.byref(prm)))
        nws = int(lib.pfista_unroll_workspace_bytes(plan.handle, ctypes.byref(prm)))
        if nck == 0 or nws == 0:
            raise PfistaError(EINVAL, lib.pfista_last_error().decode() or "bad unroll parameters")
        self._nck = nck
        self.ckpt = self.new_checkpoints()
        self.ws = torch.empty(nws, dtype=torch.uint8, device=plan.device)

    def new_checkpoints(self):
        """A checkpoint buffer for one forward pass (and its backward pass)."""
        import torch
        return torch.empty(self._nck, dtype=torch.uint8, device=self.plan.device)

    def _params(self, lam, coef):
        self._carr = (ctypes.c_double * len(coef))(*[float(v) for v in coef])
        return _UnrollParams(float(lam), self.inv_l, len(coef) - 1,
                             ctypes.cast(self._carr, ctypes.POINTER(ctypes.c_double)), self.iters,
                             self.ckpt_every, int(self.momentum), self.tune)

    def forward(self, sens, mask, b, x, lam, coef, stream=None, ckpt=None):
        c, pl = _cplx(), self.plan
        if len(coef) != self.degree + 1:
            raise ValueError(f"expected {self.degree + 1} coefficients")
        prm = self._params(lam, coef)
        ck = self.ckpt if ckpt is None else ckpt
        _check(load_library().pfista_unroll_forward(
            pl.handle, _ptr(sens, "sens", c, pl.n_coil), _ptr(mask, "mask", pl.mask_dtype(), pl.mask_numel),
            _ptr(b, "b", c, pl.n_coil), ctypes.byref(prm), _ptr(x, "x", c, pl.n_img),
            _ptr(ck, "ckpt", None, self._nck), _ptr(self.ws, "ws"), _stream(stream)))

    def backward(self, sens, mask, x_bar, lam, coef, stream=None, ckpt=None):
        """(dL/dlambda, [dL/dc_0, ..., dL/dc_d]) for the cotangent x_bar, from
        the checkpoints of the forward pass that wrote ``ckpt`` (default: the
        object's own buffer)."""
        c, pl = _cplx(), self.plan
        prm = self._params(lam, coef)
        g = (ctypes.c_double * (self.degree + 2))()
        ck = self.ckpt if ckpt is None else ckpt
        _check(load_library().pfista_unroll_backward(
            pl.handle, _ptr(sens, "sens", c, pl.n_coil), _ptr(mask, "mask", pl.mask_dtype(), pl.mask_numel),
            ctypes.byref(prm), _ptr(x_bar, "x_bar", c, pl.n_img), _ptr(ck, "ckpt", None, self._nck), g,
            _ptr(self.ws, "ws"), _stream(stream)))
        return g[0], list(g)[1:]


def _unrolled_function():
    import torch

    class _UnrolledPFISTA(torch.autograd.Function):
        @staticmethod
        def forward(ctx, lam, coef, unrolled, sens, mask, b):
            pl = unrolled.plan
            x = torch.empty((pl.slices, pl.n, pl.n), dtype=torch.complex64, device=sens.device)
            lv, cv = float(lam), [float(v) for v in coef.detach().cpu()]
            # every call keeps its own checkpoints, so that two forward passes
            # before their backward passes each get their own gradient
            ck = unrolled.new_checkpoints()
            unrolled.forward(sens, mask, b, x, lv, cv, ckpt=ck)
            ctx.unrolled, ctx.ckpt, ctx.args = unrolled, ck, (sens, mask, lv, cv)
            ctx.dtypes = (lam.dtype, coef.dtype, lam.device, coef.device)
            return x

        @staticmethod
        def backward(ctx, x_bar):
            sens, mask, lv, cv = ctx.args
            gl, gc = ctx.unrolled.backward(sens, mask, x_bar.contiguous(), lv, cv, ckpt=ctx.ckpt)
            ld, cd, ldev, cdev = ctx.dtypes
            return (torch.tensor(gl, dtype=ld, device=ldev), torch.tensor(gc, dtype=cd, device=cdev),
                    None, None, None, None)

    return _UnrolledPFISTA


_UNROLLED_FN = None


def unrolled_pfista(lam, coef, unrolled, sens, mask, b):
    """x_K of ``unrolled`` (an ``Unrolled``) as a differentiable function of the
    real tensors ``lam`` (0-d) and ``coef`` (d + 1), e.g.
    ``loss(unrolled_pfista(lam, coef, u, sens, mask, b)).backward()``.  The
    backward pass runs ``pfista_unroll_backward`` on the checkpoints this call's
    forward pass wrote (each call allocates its own)."""
    global _UNROLLED_FN
    if _UNROLLED_FN is None:
        _UNROLLED_FN = _unrolled_function()
    return _UNROLLED_FN.apply(lam, coef, unrolled, sens, mask, b)


# ------------------------------------------------------------------ non-Cartesian set-up

def toeplitz_kernel(plan, traj, kern, weights=None, stream=None):
    """Toeplitz kernel ``kern`` (float32 [S, 2n, 2n]) of the trajectories
    ``traj`` (float32 [S, J, 2], cycles per field of view) of a Toeplitz plan."""
    import torch
    J = traj.shape[-2]
    _check(load_library().pfista_toeplitz_kernel(
        plan.handle, _ptr(traj, "traj", torch.float32, plan.slices * J * 2),
        _ptr(weights, "weights", torch.float32, plan.slices * J, allow_none=True), int(J),
        _ptr(kern, "kern", torch.float32, plan.mask_numel), _stream(stream)))


def nudft_forward(plan, sens, traj, x, kdata, stream=None):
    """``kdata`` [S, C, J] = non-uniform DFT of the coil images ``S_c x``."""
    import torch
    c, J = _cplx(), traj.shape[-2]
    _check(load_library().pfista_nudft_forward(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(traj, "traj", torch.float32, plan.slices * J * 2),
        int(J), _ptr(x, "x", c, plan.n_img), _ptr(kdata, "kdata", c, plan.slices * plan.coils * J),
        _stream(stream)))


def nudft_adjoint(plan, sens, traj, kdata, y, stream=None):
    """``y`` [S, N, N] = ``sum_c conj(S_c) E^H kdata_c`` (A^H b of a Toeplitz solve)."""
    import torch
    c, J = _cplx(), traj.shape[-2]
    _check(load_library().pfista_nudft_adjoint(
        plan.handle, _ptr(sens, "sens", c, plan.n_coil), _ptr(traj, "traj", torch.float32, plan.slices * J * 2),
        int(J), _ptr(kdata, "kdata", c, plan.slices * plan.coils * J), _ptr(y, "y", c, plan.n_img),
        _stream(stream)))
