"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only, no GPU call): a sanitized build runs the C-ABI validation cases of
test_abi.py (plan and batch descriptors, NULL handles, the host coefficient
solvers) in a child process with the ASan runtime preloaded; any sanitizer
report fails the test."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_validation_paths_are_clean_under_host_sanitizers(tmp_path):
    from paper_2204_10252_amd import build
    try:
        build.hipcc()
    except RuntimeError:
        pytest.skip("no hipcc")
    rt = build.asan_runtime()
    if rt is None:
        pytest.skip("no clang ASan runtime")
    lib = build.build(verbose=False, sanitize=True, out=str(tmp_path / "libpfista_hostsan.so"))
    env = dict(os.environ)
    env.update({
        "PFISTA_LIBRARY": lib,
        "LD_PRELOAD": rt,
        # Python itself is not instrumented: its allocations are not leaks to report
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
        "HIP_VISIBLE_DEVICES": "",
    })
    sel = "validation or null or coefficient or exports"
    res = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                          "-p", "no:cacheprovider", "-k", sel],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert " passed" in res.stdout


def test_sanitized_build_flags_stay_on_the_host():
    # every sanitizer flag of the sanitized build sits behind -Xarch_host (the
    # device code is built exactly as in the normal build)
    from paper_2204_10252_amd import build
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no hipcc")
    cmd = build.command("/dev/null", sanitize=True)
    for i, a in enumerate(cmd):
        if a.startswith("-fsanitize") or a in ("-shared-libasan", "-fno-omit-frame-pointer"):
            assert cmd[i - 1] == "-Xarch_host", a
