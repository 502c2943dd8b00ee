"""CPU-only sanitizer check of the host runtime and validation layer: the library built
with AddressSanitizer and UndefinedBehaviorSanitizer on its host code, driven by a C
program (tests/abi_sanitize.c) through the context lifecycle, option defaults, status
strings and every scalar validation path. No GPU is touched."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_runtime_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    import importlib.util
    spec = importlib.util.spec_from_file_location("_b", os.path.join(ROOT, "paper_2512_06143_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    lib = b.build_sanitized()
    exe = str(tmp_path / "abi_sanitize")
    cmd = [hipcc, "-O1", *b.SANITIZE, "-I", os.path.join(ROOT, "include"), "-x", "c",
           os.path.join(ROOT, "tests", "abi_sanitize.c"), "-x", "none", lib, f"-Wl,-rpath,{os.path.dirname(lib)}",
           "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", LSAN_OPTIONS="suppressions=" +
               os.path.join(ROOT, "tests", "lsan_hip.supp"))
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-6000:]
    assert "sanitized host checks passed" in out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
