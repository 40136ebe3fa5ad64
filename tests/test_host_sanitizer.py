"""The library's host-side steps under AddressSanitizer and UndefinedBehaviorSanitizer.

The quadrature, the snapped offsets, the lattice classes, the sinc error control, the request
plans (valid and invalid problems) and the autotuner's decision file are compiled with a self-test
driver (``csrc/host_selftest.cpp``) by the host compiler with both sanitizers and run on the CPU:
any out-of-bounds access, use after free, leak or undefined behaviour aborts the run.  Device code
and the HIP runtime's streams are outside this build.
"""
import os
import shutil
import subprocess

import pytest


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_steps_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    import importlib.util
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("lsum_build", os.path.join(here, "paper_1411_1994_amd", "build.py"))
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    exe = build.build_host_selftest(verbose=False)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:detect_leaks=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["TMPDIR"] = str(tmp_path)
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert " 0 failed" in res.stdout, res.stdout
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr
