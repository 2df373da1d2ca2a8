"""AddressSanitizer on the CPU-side code.

* libpond.so's host code (the C ABI's argument checks, layouts, workspace and
  tape sizes, the stream slots) built with AddressSanitizer on the host pass
  only (-Xarch_host -fsanitize=address; the GPU code is built as usual), and
  the ABI tests run against it with the sanitizer runtime preloaded.
* The oracle built with g++ -fsanitize=address, and a set of its pins run
  against it (grid steps with both lattices and edges, the sampled-node
  entry, the complex-step template).
A sanitizer report makes the child process fail; its output is printed.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import build_oracle  # noqa: E402
from paper_1806_05089_amd import build as hip_build  # noqa: E402

ASAN_OPTIONS = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=23"


def _run(cmd, env):
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    print(tail, flush=True)
    assert "AddressSanitizer" not in r.stderr, tail
    assert r.returncode == 0, tail


def test_libpond_host_code_under_asan(tmp_path):
    runtime = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not runtime:
        pytest.skip("no clang AddressSanitizer runtime")
    lib = hip_build.build(extra_flags=("-Xarch_host", "-fsanitize=address", "-Xarch_host",
                                       "-fno-omit-frame-pointer"),
                          out=str(tmp_path / "libpond_asan.so"))
    env = dict(os.environ, POND_LIBRARY=lib, LD_PRELOAD=runtime[-1], ASAN_OPTIONS=ASAN_OPTIONS)
    _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
          "tests/test_abi.py"], env)


def test_oracle_under_asan(tmp_path):
    runtime = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(runtime):
        pytest.skip("no gcc AddressSanitizer runtime")
    lib = build_oracle.build(extra_flags=("-fsanitize=address", "-fno-omit-frame-pointer"),
                             out=str(tmp_path / "libpond_oracle_asan.so"))
    env = dict(os.environ, POND_ORACLE_LIBRARY=lib, LD_PRELOAD=runtime,
               ASAN_OPTIONS=ASAN_OPTIONS, OMP_NUM_THREADS="2")
    _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
          "tests/test_oracle_pins.py", "-k",
          "step_nodes or single_pass or collision or complex_step or uniform_flow or galilean "
          "or seed_independence"], env)
