"""Host-side consistency of the transform plans and their twiddle tables
(tests/plan_tables_check.cpp, built with hipcc for the host; no GPU): the
stage radices of every plan multiply to its length, the staged twiddle
table blocks tile the table with exponents below the length, the batched
table offsets add up, the cross-lane and row-tile choices hold on known
plans, the XCD pairing of 2-row tiles is a bijection that pairs halves
on one XCD, the padded LDS index of every length is one to one inside its
line, the one-mask pass kernels' static LDS fits a CU, and the library's
twiddle tables equal their definition; a second build runs the same check
under AddressSanitizer and UndefinedBehaviorSanitizer (host code only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def _build_and_run(tmp_path, name, extra):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / name
    src = os.path.join(ROOT, "tests", "plan_tables_check.cpp")
    r = subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *extra,
                        f"-I{os.path.join(ROOT, 'include')}",
                        f"-I{os.path.join(ROOT, 'paper_1302_0120_amd', 'csrc')}", src, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout + run.stderr


def test_plan_tables(tmp_path):
    _build_and_run(tmp_path, "plan_tables_check", [])


def test_plan_tables_sanitized(tmp_path):
    """The same check with the host code built under AddressSanitizer and
    UndefinedBehaviorSanitizer (device code untouched): out-of-bounds table
    writes, leaks and undefined arithmetic in the plan code abort it."""
    _build_and_run(tmp_path, "plan_tables_check_asan",
                   ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"])
