"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer: the C part
of the oracle (gcc), and the library's host code (hipcc with the sanitizers on
the host side only; the device code is compiled but never run) driven through
its host-only entry points and the argument validation of the device entry
points.  Each driver exits 0 only when every expectation holds and the
sanitizers report nothing."""
import concurrent.futures
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.slow


def _run(exe, env):
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
    return out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["gcc", "-O1", "-g", "-mfma", "-ffp-contract=off", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", exe, os.path.join(ROOT, "oracle", "ps_oracle.c"),
                           os.path.join(HERE, "oracle_driver.c"), "-lm"])
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=1")
    assert "all expectations hold" in _run(exe, env)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_sanitizers(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")] + san
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2312_17396_amd", "csrc", "*.cpp")) +
                  glob.glob(os.path.join(ROOT, "paper_2312_17396_amd", "csrc", "*.hip")) +
                  [os.path.join(HERE, "host_driver.cpp")])

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC, *common, "-c", "-x", "hip", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        return obj

    with concurrent.futures.ThreadPoolExecutor(4) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_asan")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", *san, *objs, "-o", exe])
    assert "all expectations hold" in _run(exe, ENV)
