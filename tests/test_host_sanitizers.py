"""The oracle's C stepper and the library's host code built with the address and
undefined-behaviour sanitizers and driven through their entry points on the CPU (no GPU):
tiny and ragged lattices for every scheme, collision and psi kind in the oracle; parameter
validation, launch rules, EOS helpers, the coexistence solver, the checkpoint reader and the
autotuner cache parser in the library.  Device code is compiled as usual and never run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1412_5170_amd", "csrc")


def _run(cmd, env=None, cwd=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=cwd, timeout=600)
    return r.returncode, r.stdout + r.stderr


def _env(**kw):
    env = dict(os.environ)
    env.update(kw)
    return env


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fopenmp", "-ffp-contract=off", "-o", exe,
                    os.path.join(HERE, "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm"])
    assert rc == 0, out
    rc, out = _run([exe], env=_env(OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1"))
    assert rc == 0 and "oracle driver: ok" in out, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc to compile the library")
def test_library_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    srcs = [os.path.join(CSRC, n) for n in ("lbm_kernels.hip", "lbm_api.cpp", "lbm_batch.cpp",
                                             "lbm_tune.cpp", "lbm_thermo.cpp")]
    cmd = ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # host code only: the sanitizers apply to the host pass, device code is built plain
           "-Xarch_host", "-fsanitize=address,undefined", "-fno-gpu-sanitize",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
           "-x", "hip", *srcs, "-x", "c++", os.path.join(HERE, "host_driver.cpp"), "-o", exe]
    rc, out = _run(cmd)
    assert rc == 0, out
    rc, out = _run(["nm", exe])
    assert "__asan_init" in out and "__ubsan_handle" in out  # the host code is instrumented
    rc, out = _run([exe, str(tmp_path)],
                   env=_env(ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1"))
    assert rc == 0 and "host driver: ok" in out, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
